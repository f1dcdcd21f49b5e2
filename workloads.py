"""Seeded synthetic planning problems (input generator only).

This module is shared by the oracle, the GPU tests and the benchmark.  It
holds no arithmetic of the planning method: it only draws maps, start/goal
pairs and robot parameters, samples analytic signed-distance fields onto
grids, and writes down the linear dynamics of the robot models that the
paper's experiments name (the LTI point robot / double integrator of
Sec. 7.1 and the planar quadrotor of Sec. 7.3, eq. planar_quad).

All randomness comes from numpy's PCG64 generator seeded per problem, so the
oracle and the GPU path always see identical arrays.

Problem dictionaries use these keys (shapes in brackets):
  n, m, N, dt            state dim, noise-input dim, support states, step
  A [n,n] | [N-1,n,n]    drift matrix (LTI: one copy; LTV: one per interval)
  a [n]   | [N-1,n]      drift offset
  B [n,m] | [N-1,n,m]    noise input matrix
  ltv                    True when A, a, B are given per interval
  Qc [m,m]               white-noise spectral density
  mu_start, Sig_start, mu_goal, Sig_goal   Gaussian boundary factors
  temperature, beta_max, kl_bound, max_bisect, n_iters
  coll_kind              'point2d' | 'point3d' | 'arm3d' | 'none'
  coll_index [d]         state components that are configuration coords
  gh_points              Gauss-Hermite points per dimension
  sdf                    float32 [gy,gx] or [gz,gy,gx], node-sampled
  origin [3], cell       grid geometry (node (ix,iy,iz) at origin+idx*cell)
  hinge_eps, obs_weight  hinge margin and scalar weight
  sphere_radius [S]      collision sphere radii (point robots: one, r=0)
  fk                     arm chain parameters (arm3d only), see arm_problem
"""
from __future__ import annotations

import math

import numpy as np

GRAVITY = 9.81
# Step-size rule of App. C: KL(q_{k+1} || q_k) <= epsilon.  The paper prints no
# epsilon; 10 nats keeps the proximal iteration stable on these workloads.
KL_BOUND = 10.0


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# --------------------------------------------------------------------------
# analytic shape distances sampled onto grids (input data, not the method)
# --------------------------------------------------------------------------
def _disc_dist(px, py, cx, cy, r):
    return np.hypot(px - cx, py - cy) - r


def _box_dist(pts, c, h):
    """Exact signed distance to an axis-aligned box (any dimension)."""
    q = np.abs(pts - c) - h
    outside = np.sqrt(np.sum(np.maximum(q, 0.0) ** 2, axis=-1))
    inside = np.minimum(np.max(q, axis=-1), 0.0)
    return outside + inside


def sdf_grid_2d(shapes, gx, gy, cell, origin=(0.0, 0.0)):
    """float32 [gy,gx] grid of min over shape distances, computed in FP64."""
    xs = origin[0] + cell * np.arange(gx, dtype=np.float64)
    ys = origin[1] + cell * np.arange(gy, dtype=np.float64)
    X, Y = np.meshgrid(xs, ys)  # [gy,gx]
    d = np.full(X.shape, np.inf)
    pts = np.stack([X, Y], axis=-1)
    for s in shapes:
        if s[0] == "disc":
            _, cx, cy, r = s
            d = np.minimum(d, _disc_dist(X, Y, cx, cy, r))
        else:
            _, cx, cy, hx, hy = s
            d = np.minimum(d, _box_dist(pts, np.array([cx, cy]), np.array([hx, hy])))
    return d.astype(np.float32)


def sdf_grid_3d(boxes, g, cell, origin=(0.0, 0.0, 0.0)):
    """float32 [gz,gy,gx] grid for axis-aligned boxes (centre, half-extent)."""
    ax = [origin[k] + cell * np.arange(g, dtype=np.float64) for k in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    pts = np.stack([X, Y, Z], axis=-1)
    d = np.full(X.shape, np.inf)
    for c, h in boxes:
        d = np.minimum(d, _box_dist(pts, np.asarray(c), np.asarray(h)))
    return d.astype(np.float32)


def _shapes_min_dist(shapes, p):
    """Distance from point p to the nearest shape (for clearance redraws)."""
    best = np.inf
    for s in shapes:
        if s[0] == "disc":
            best = min(best, float(_disc_dist(p[0], p[1], s[1], s[2], s[3])))
        else:
            best = min(best, float(_box_dist(np.asarray(p), np.array(s[1:3]), np.array(s[3:5]))))
    return best


def random_shapes_2d(rng, count, extent, keep_clear, clearance, boxes=False):
    """Discs (and, if boxes, axis-aligned boxes with prob. 1/2) in [0,extent]^2.

    A shape is redrawn while any point in keep_clear lies within its size
    plus clearance (same rule for discs and boxes: the bounding radius).
    """
    shapes = []
    while len(shapes) < count:
        cx, cy = rng.uniform(0.0, extent, size=2)
        if boxes and rng.uniform() < 0.5:
            hx, hy = rng.uniform(0.5, 1.5, size=2)
            s = ("box", float(cx), float(cy), float(hx), float(hy))
            reach = math.hypot(hx, hy)
        else:
            r = rng.uniform(0.5, 1.5)
            s = ("disc", float(cx), float(cy), float(r))
            reach = r
        if all(math.hypot(cx - p[0], cy - p[1]) > reach + clearance for p in keep_clear):
            shapes.append(s)
    return shapes


# --------------------------------------------------------------------------
# robot models named by the paper (problem statement, no solver arithmetic)
# --------------------------------------------------------------------------
def double_integrator(dof):
    """LTI model of Sec. 7.1: A=[[0,I],[0,0]], a=0, B=[0;I]."""
    n = 2 * dof
    A = np.zeros((n, n))
    A[:dof, dof:] = np.eye(dof)
    B = np.zeros((n, dof))
    B[dof:, :] = np.eye(dof)
    return A, np.zeros(n), B


def quadrotor_params(rng):
    """Planar quadrotor constants of Sec. 7.3, with seeded mass and inertia.

    The paper fixes m=1/sqrt(2), l=sqrt(2), J=1; the seeded variants scale
    m and J by U[0.8,1.2].  Gravity is not printed; 9.81 is used.
    """
    return {
        "mass": (1.0 / math.sqrt(2.0)) * float(rng.uniform(0.8, 1.2)),
        "inertia": float(rng.uniform(0.8, 1.2)),
        "length": math.sqrt(2.0),
        "gravity": GRAVITY,
    }


def quadrotor_B(params):
    """Input matrix of eq. planar_quad (rows x, z, phi, vx, vz, phidot)."""
    m, l, J = params["mass"], params["length"], params["inertia"]
    B = np.zeros((6, 2))
    B[4, :] = [1.0 / m, 1.0 / m]
    B[5, :] = [l / J, -l / J]
    return B


# --------------------------------------------------------------------------
# problem constructors
# --------------------------------------------------------------------------
def _base(n, m, N, dt, A, a, B, Qc, mu_s, mu_g, sig_end=1e-4):
    return {
        "n": n, "m": m, "N": N, "dt": dt,
        "A": np.asarray(A, dtype=np.float64), "a": np.asarray(a, dtype=np.float64),
        "B": np.asarray(B, dtype=np.float64), "ltv": False,
        "Qc": np.asarray(Qc, dtype=np.float64),
        "mu_start": np.asarray(mu_s, dtype=np.float64),
        "Sig_start": sig_end * np.eye(n),
        "mu_goal": np.asarray(mu_g, dtype=np.float64),
        "Sig_goal": sig_end * np.eye(n),
        "temperature": 1.0, "beta_max": 1.0, "kl_bound": KL_BOUND,
        "max_bisect": 20, "n_iters": 20,
    }


def point2d_problem(seed, N=50, grid=100, cell=0.1, n_shapes=6, boxes=False,
                    start=(1.0, 1.0), goal=(9.0, 9.0), gh_points=3, dt=0.1,
                    qc=0.8, hinge_eps=0.5, sigma_obs=0.01, n_iters=20):
    """Planar point robot (state x, y, vx, vy) over a seeded disc/box map."""
    rng = _rng(seed)
    extent = grid * cell
    shapes = random_shapes_2d(rng, n_shapes, extent, [start, goal], 1.0, boxes=boxes)
    A, a, B = double_integrator(2)
    p = _base(4, 2, N, dt, A, a, B, qc * np.eye(2),
              [start[0], start[1], 0.0, 0.0], [goal[0], goal[1], 0.0, 0.0])
    p.update({
        "coll_kind": "point2d", "coll_index": np.array([0, 1], dtype=np.int32),
        "gh_points": gh_points,
        "sdf": sdf_grid_2d(shapes, grid, grid, cell), "origin": np.zeros(3),
        "cell": cell, "hinge_eps": hinge_eps, "obs_weight": 1.0 / sigma_obs ** 2,
        "sphere_radius": np.zeros(1), "n_iters": n_iters, "shapes": shapes,
        "seed": seed,
    })
    return p


def config0_problem(seed=0):
    """Point robot, N=50, 100x100 grid (0.1 m), 6 discs, GH p=3, 20 iterations."""
    return point2d_problem(seed)


def config1_problem(seed=0, N=750):
    """Point robot, N=750, 500x500 grid (0.1 m), 40 discs/boxes, GH p=5."""
    return point2d_problem(seed, N=N, grid=500, cell=0.1, n_shapes=40, boxes=True,
                           start=(2.0, 2.0), goal=(48.0, 48.0), gh_points=5)


def point3d_problem(seed, N=50, grid=64, cell=0.1, n_boxes=8, gh_points=3,
                    start=(0.6, 0.6, 0.6), goal=(5.6, 5.6, 5.6), hinge_eps=0.5,
                    sigma_obs=0.01, n_iters=20):
    """3-D point robot (state x,y,z,vx,vy,vz) over a seeded box map."""
    rng = _rng(seed)
    extent = grid * cell
    boxes = []
    while len(boxes) < n_boxes:
        c = rng.uniform(0.0, extent, size=3)
        h = rng.uniform(0.2, 0.6, size=3)
        reach = float(np.linalg.norm(h))
        if all(np.linalg.norm(c - np.asarray(q)) > reach + 0.5 for q in (start, goal)):
            boxes.append((c, h))
    A, a, B = double_integrator(3)
    p = _base(6, 3, N, 0.1, A, a, B, 0.8 * np.eye(3),
              list(start) + [0.0] * 3, list(goal) + [0.0] * 3)
    p.update({
        "coll_kind": "point3d", "coll_index": np.array([0, 1, 2], dtype=np.int32),
        "gh_points": gh_points, "sdf": sdf_grid_3d(boxes, grid, cell),
        "origin": np.zeros(3), "cell": cell, "hinge_eps": hinge_eps,
        "obs_weight": 1.0 / sigma_obs ** 2, "sphere_radius": np.zeros(1),
        "n_iters": n_iters, "seed": seed,
    })
    return p


ARM_DOF = 7
ARM_BASE = (1.28, 1.28, 0.2)


def arm_chain(rng):
    """Synthetic 7-joint serial chain (the paper's WAM model is not given).

    Joint k rotates about its local z axis (k even) or y axis (k odd); link k
    then extends along the rotated local z by length l_k ~ U[0.1,0.4].  Twenty
    spheres: three on each of links 0..5 at 1/3, 2/3 and 1 of the link, two on
    link 6 at 1/2 and 1.
    """
    lengths = rng.uniform(0.1, 0.4, size=ARM_DOF)
    axes = np.array([2 if k % 2 == 0 else 1 for k in range(ARM_DOF)], dtype=np.int32)
    sph_link, sph_frac = [], []
    for k in range(6):
        for f in (1.0 / 3.0, 2.0 / 3.0, 1.0):
            sph_link.append(k)
            sph_frac.append(f)
    for f in (0.5, 1.0):
        sph_link.append(6)
        sph_frac.append(f)
    return {
        "base": np.array(ARM_BASE), "link_len": lengths, "axes": axes,
        "sphere_link": np.array(sph_link, dtype=np.int32),
        "sphere_frac": np.array(sph_frac),
    }


def arm_problem(seed, N=100, grid=128, cell=0.02, n_boxes=15, gh_points=2,
                radius=0.06, hinge_eps=0.15, sigma_obs=0.01, n_iters=20):
    """7-DOF arm, state (q, qdot) in R^14, double-integrator GP prior.

    Start and goal joint angles are drawn from U[-1.5,1.5]^7 with zero
    velocity; they are not checked for collision (that check needs forward
    kinematics, which belongs to the method, not to this generator).
    """
    rng = _rng(seed)
    chain = arm_chain(rng)
    extent = grid * cell
    base = np.array(ARM_BASE)
    boxes = []
    while len(boxes) < n_boxes:
        c = rng.uniform(0.0, extent, size=3)
        h = rng.uniform(0.05, 0.25, size=3)
        if _box_dist(base, c, h) > 0.3:
            boxes.append((c, h))
    q0 = rng.uniform(-1.5, 1.5, size=ARM_DOF)
    q1 = rng.uniform(-1.5, 1.5, size=ARM_DOF)
    A, a, B = double_integrator(ARM_DOF)
    p = _base(14, 7, N, 0.1, A, a, B, 0.8 * np.eye(7),
              np.concatenate([q0, np.zeros(7)]), np.concatenate([q1, np.zeros(7)]))
    p.update({
        "coll_kind": "arm3d", "coll_index": np.arange(7, dtype=np.int32),
        "gh_points": gh_points, "sdf": sdf_grid_3d(boxes, grid, cell),
        "origin": np.zeros(3), "cell": cell, "hinge_eps": hinge_eps,
        "obs_weight": 1.0 / sigma_obs ** 2,
        "sphere_radius": np.full(20, radius), "fk": chain, "n_iters": n_iters,
        "seed": seed,
    })
    return p


def config2_problem(seed=0):
    return arm_problem(seed)


def quadrotor_problem(seed, N=None, gh_points=3, slr_points=3, n_rounds=10,
                      n_iters=15, qc=0.8, hinge_eps=0.5, sigma_obs=0.01, span=None,
                      diffusion=0.01):
    """Nonlinear planar quadrotor (x, z, phi, vx, vz, phidot) over a 10x10 m
    map of 6 seeded discs.  N ~ U{100..300} unless given, over a time span
    T ~ U[4, 6] s (Sec. 7.3's range) unless given, so dt = T / (N - 1).  The
    LTI fields (A, a) hold the model's hover linearisation (phi = 0, zero
    velocity: xdot = vx, zdot = vz, vxdot = -g phi, vzdot = -g) until the
    first statistical linearisation replaces them; the nominal trajectory is
    the straight line with covariance 1e-2 I.

    Noise: the thrusts' white noise (Qc = qc I through the input matrix of
    eq. planar_quad) plus an isotropic diffusion floor diffusion^2 I on every
    state, handed over as the square factor B = chol(B_u Qc B_u^T +
    diffusion^2 I) with Qc = I.  Through the rank-2 input matrix alone the
    position is a fourfold integral of the noise and cond(K^-1) grows like
    2 N^7 (numerically singular in FP64 from N ~ 100); the floor bounds it
    near 1e9 at N = 300.  diffusion=0 gives the plain rank-2 model."""
    rng = _rng(seed)
    if N is None:
        N = int(rng.integers(100, 301))
    shapes = random_shapes_2d(rng, 6, 10.0, [], 0.0)
    sdf = sdf_grid_2d(shapes, 100, 100, 0.1)

    def free_point():
        while True:
            q = rng.uniform(0.5, 9.4, size=2)
            if _shapes_min_dist(shapes, q) >= 1.0:
                return q

    s, g = free_point(), free_point()
    while np.linalg.norm(s - g) < 4.0:
        g = free_point()
    params = quadrotor_params(rng)
    T = float(rng.uniform(4.0, 6.0)) if span is None else float(span)
    B_u = quadrotor_B(params)
    if diffusion > 0.0:
        B = np.linalg.cholesky(qc * B_u @ B_u.T + diffusion ** 2 * np.eye(6))
        Qc = np.eye(6)
    else:
        B, Qc = B_u, qc * np.eye(2)
    mu_s = np.array([s[0], s[1], 0.0, 0.0, 0.0, 0.0])
    mu_g = np.array([g[0], g[1], 0.0, 0.0, 0.0, 0.0])
    A_hover = np.zeros((6, 6))
    A_hover[0, 3] = A_hover[1, 4] = A_hover[2, 5] = 1.0
    A_hover[3, 2] = -params["gravity"]
    a_hover = np.array([0.0, 0.0, 0.0, 0.0, -params["gravity"], 0.0])
    p = _base(6, B.shape[1], N, T / max(N - 1, 1), A_hover, a_hover, B, Qc, mu_s, mu_g)
    ts = np.linspace(0.0, 1.0, N)[:, None]
    nominal = (1.0 - ts) * mu_s[None, :] + ts * mu_g[None, :]
    p.update({
        "coll_kind": "point2d", "coll_index": np.array([0, 1], dtype=np.int32),
        "gh_points": gh_points, "sdf": sdf, "origin": np.zeros(3), "cell": 0.1,
        "hinge_eps": hinge_eps, "obs_weight": 1.0 / sigma_obs ** 2,
        "sphere_radius": np.zeros(1), "n_iters": n_iters,
        "quad": params, "slr_points": slr_points, "n_rounds": n_rounds,
        "nominal_mean": nominal, "nominal_cov": np.repeat(1e-2 * np.eye(6)[None], N, axis=0),
        "seed": seed,
    })
    return p


def config3_problem(seed=0, N=None):
    return quadrotor_problem(seed, N=N)


def free_problem(n_dof=2, N=12, dt=0.1, qc=0.8, seed=0, temperature=1.0, beta_max=1.0):
    """Obstacle-free double integrator with a constant far-away SDF value.

    Every hinge term is zero, so the collision cost vanishes identically.
    """
    rng = _rng(seed)
    A, a, B = double_integrator(n_dof)
    n = 2 * n_dof
    s = np.concatenate([rng.uniform(0, 1, n_dof), np.zeros(n_dof)])
    g = np.concatenate([rng.uniform(4, 5, n_dof), np.zeros(n_dof)])
    p = _base(n, n_dof, N, dt, A, a, B, qc * np.eye(n_dof), s, g)
    p["temperature"] = temperature
    p["beta_max"] = beta_max
    kind = {2: "point2d", 3: "point3d"}[n_dof]
    shape = (16,) * n_dof
    p.update({
        "coll_kind": kind, "coll_index": np.arange(n_dof, dtype=np.int32),
        "gh_points": 3, "sdf": np.full(shape, 1000.0, dtype=np.float32),
        "origin": np.zeros(3), "cell": 1.0, "hinge_eps": 0.5, "obs_weight": 1e4,
        "sphere_radius": np.zeros(1), "seed": seed,
    })
    return p


def affine_sdf_problem(slope=(0.25, -0.125), offset=2.0, N=10, kappa_eps=10.0,
                       weight=1.0, gh_points=3, seed=0, temperature=1.0, beta_max=1.0):
    """Point robot over an affine SDF sampled exactly on a dyadic grid.

    sdf(x,y) = s0*x + s1*y + offset on a 256x256 grid with cell 0.125, so
    every FP32 grid value is exact and bilinear interpolation reproduces the
    field.  With a huge hinge margin every hinge term is active, making the
    collision cost an exact quadratic in the position.
    """
    rng = _rng(seed)
    g, cell = 256, 0.125
    xs = cell * np.arange(g, dtype=np.float64)
    X, Y = np.meshgrid(xs, xs)
    sdf = (slope[0] * X + slope[1] * Y + offset).astype(np.float32)
    assert np.array_equal(sdf.astype(np.float64), slope[0] * X + slope[1] * Y + offset)
    A, a, B = double_integrator(2)
    s = np.array([rng.uniform(8, 10), rng.uniform(8, 10), 0.0, 0.0])
    t = np.array([rng.uniform(20, 22), rng.uniform(20, 22), 0.0, 0.0])
    p = _base(4, 2, N, 0.1, A, a, B, 0.8 * np.eye(2), s, t)
    p["temperature"] = temperature
    p["beta_max"] = beta_max
    p.update({
        "coll_kind": "point2d", "coll_index": np.array([0, 1], dtype=np.int32),
        "gh_points": gh_points, "sdf": sdf, "origin": np.zeros(3), "cell": cell,
        "hinge_eps": kappa_eps, "obs_weight": weight, "sphere_radius": np.zeros(1),
        "affine": (np.array(slope, dtype=np.float64), float(offset)), "seed": seed,
    })
    return p


def affine_grid_3d(slope, offset, g, cell):
    """float32 [g,g,g] grid (z, y, x) of the affine field slope . x + offset at
    nodes cell * (ix, iy, iz); dyadic slope, offset and cell keep every value
    exact in FP32, and trilinear interpolation reproduces the field."""
    xs = cell * np.arange(g, dtype=np.float64)
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    f = slope[0] * X + slope[1] * Y + slope[2] * Z + offset
    grid = f.astype(np.float32)
    assert np.array_equal(grid.astype(np.float64), f)
    return grid


def affine_sdf3_problem(slope=(0.25, -0.125, 0.5), offset=2.0, N=10, kappa_eps=10.0,
                        weight=1.0, gh_points=3, seed=0):
    """3-D point robot (n = 6) over an affine SDF on a 64^3 dyadic grid
    (cell 0.125, an 8 m cube).  With a huge hinge margin every hinge term is
    active and the collision cost is an exact quadratic in the position."""
    rng = _rng(seed)
    A, a, B = double_integrator(3)
    s = np.concatenate([rng.uniform(2.0, 2.5, size=3), np.zeros(3)])
    t = np.concatenate([rng.uniform(5.5, 6.0, size=3), np.zeros(3)])
    p = _base(6, 3, N, 0.1, A, a, B, 0.8 * np.eye(3), s, t)
    p.update({
        "coll_kind": "point3d", "coll_index": np.array([0, 1, 2], dtype=np.int32),
        "gh_points": gh_points, "sdf": affine_grid_3d(slope, offset, 64, 0.125),
        "origin": np.zeros(3), "cell": 0.125, "hinge_eps": kappa_eps,
        "obs_weight": weight, "sphere_radius": np.zeros(1),
        "affine": (np.array(slope, dtype=np.float64), float(offset)), "seed": seed,
    })
    return p


def arm_affine_problem(slope=(0.25, -0.125, 0.5), offset=2.0, N=6, kappa_eps=10.0,
                       weight=1.0, gh_points=2, seed=0):
    """7-DOF arm over an affine SDF on a 48^3 dyadic grid (cell 0.125, a 6 m
    cube), base at its centre, seven links of 0.25 m (reach 1.75 m, so every
    sphere stays inside the grid for any joint angles), twenty spheres of
    distinct radii 0.02 + 0.01 s.  Every hinge is active."""
    rng = _rng(seed)
    chain = arm_chain(rng)
    chain["base"] = np.array([3.0, 3.0, 3.0])
    chain["link_len"] = np.full(ARM_DOF, 0.25)
    q0 = rng.uniform(-1.0, 1.0, size=ARM_DOF)
    q1 = rng.uniform(-1.0, 1.0, size=ARM_DOF)
    A, a, B = double_integrator(ARM_DOF)
    p = _base(14, 7, N, 0.1, A, a, B, 0.8 * np.eye(7),
              np.concatenate([q0, np.zeros(7)]), np.concatenate([q1, np.zeros(7)]))
    p.update({
        "coll_kind": "arm3d", "coll_index": np.arange(7, dtype=np.int32),
        "gh_points": gh_points, "sdf": affine_grid_3d(slope, offset, 48, 0.125),
        "origin": np.zeros(3), "cell": 0.125, "hinge_eps": kappa_eps,
        "obs_weight": weight, "sphere_radius": 0.02 + 0.01 * np.arange(20),
        "fk": chain, "affine": (np.array(slope, dtype=np.float64), float(offset)), "seed": seed,
    })
    return p


def serving_mix(seed=0, count=100, qps=50.0, n_range=(50, 1000), map_pool=None):
    """Request stream: Poisson arrivals, each drawing a config 0..3 shape
    and N ~ U{n_range}.

    With map_pool = P, the point-robot and arm requests draw their map (and
    with it their start and goal) from P seeded maps per kind, so that long
    streams are generated quickly and share device copies of their maps;
    the quadrotor's nominal trajectory depends on N, so it is drawn anew.
    Returns a list of (arrival_time_s, problem) sorted by arrival.
    """
    rng = _rng(seed)
    t = 0.0
    out = []
    cache = {}
    for k in range(count):
        t += float(rng.exponential(1.0 / qps))
        kind = int(rng.integers(0, 4))
        N = int(rng.integers(n_range[0], n_range[1] + 1))
        s = int(rng.integers(0, 1 << 30))
        if map_pool and kind < 3:
            s = s % map_pool
        if kind < 3 and map_pool and (kind, s) in cache:
            prob = dict(cache[(kind, s)], N=N)
        elif kind == 0:
            prob = point2d_problem(s, N=N)
        elif kind == 1:
            prob = point2d_problem(s, N=N, grid=500, cell=0.1, n_shapes=40, boxes=True,
                                   start=(2.0, 2.0), goal=(48.0, 48.0), gh_points=5)
        elif kind == 2:
            prob = arm_problem(s, N=N)
        else:
            prob = quadrotor_problem(s, N=N)
        if kind < 3 and map_pool:
            cache.setdefault((kind, s), prob)
        prob["mix_kind"] = kind
        out.append((t, prob))
    return out
