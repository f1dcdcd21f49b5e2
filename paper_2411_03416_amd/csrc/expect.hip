// Collision-factor expectations (Sec. 4.1 eq. gradients_psid, Sec. 4.3).
//
// For the factor of state s with configuration marginal N(mu, Sigma)
// (d-dim, Sigma = L L^T), the tensor Gauss-Hermite rule with p points per
// axis gives x_j = mu + L xi_j, weights W_j, and
//   s0 = sum_j W_j psi_j,  s1 = sum_j W_j psi_j xi_j,
//   S2 = sum_j W_j psi_j xi_j xi_j^T,
// from which, since x - mu = L xi,
//   E[psi] = s0,
//   grad_mu = Sigma^-1 E[(x-mu) psi] = L^-T s1,
//   2 grad_Sigma = Sigma^-1 (E[(x-mu)(x-mu)^T psi] - E[psi] Sigma) Sigma^-1
//                = L^-T (S2 - s0 I) L^-1.
// The derivative-free (Stein) form needs no SDF gradient, so the hinge's
// kinks are harmless.
//
// One workgroup serves F factors of one plan in three stages:
//   A. thread f loads factor f's marginal (coalesced SoA rows), factors it
//      in FP64 and puts mu and L (type R) into LDS;
//   B. the workgroup evaluates the cost at every (factor, node) pair of a
//      chunk, consecutive threads taking consecutive nodes of one factor
//      (no idle lanes whatever p^d is, and the nodes of one gather
//      instruction fall in a few neighbouring SDF cells); psi goes to LDS;
//   C. thread f sums W_j (psi_j - c) xi_j ... over its nodes in node order
//      (the node loop is uniform, so nodes and weights are scalar loads),
//      then runs the FP64 epilogue and stores E, g and H (coalesced).
// Chunks of nodes repeat B and C when p^d nodes of F factors exceed the
// LDS budget.  Every factor's arithmetic is independent of F, the chunk
// size and the rest of the launch, so results do not depend on the batch.
//
// Node math, SDF lookups, forward kinematics and the cost run in type R
// (float in mixed mode, double in FP64 mode); the Cholesky factor and the
// epilogue are always FP64.  In mixed mode (p >= 2) the cost is centred by
// c = psi(mu) before the FP32 sums: the rule integrates constants and the
// first two moments of xi exactly, so only E[psi] needs c added back.
//
// Plan q always runs on XCD q mod 8 (one L2 per XCD): neighbouring states
// of a plan share SDF cache lines, and an XCD's L2 holds only its own
// plans' maps.
#include <algorithm>

#include "ctx.h"

namespace pg {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }
constexpr int cmin(int a, int b) { return a < b ? a : b; }
// LDS bytes of node values per workgroup: the arm's nodes are costly, so
// small chunks of them leave room for more resident workgroups
constexpr int expect_lds(int kind) { return kind == PGVIMP_COLL_ARM3D ? 8 * 1024 : 40 * 1024; }

template <typename R>
struct Tab;
template <>
struct Tab<double> {
    static __device__ const double* x(const DevState& st) { return st.gh_x64; }
    static __device__ const double* w(const DevState& st) { return st.gh_w64; }
};
template <>
struct Tab<float> {
    static __device__ const float* x(const DevState& st) { return st.gh_x32; }
    static __device__ const float* w(const DevState& st) { return st.gh_w32; }
};

__device__ __forceinline__ double clamp_axis(double u, double top) { return fmin(fmax(u, 0.0), top); }
__device__ __forceinline__ float clamp_axis(float u, float top) { return fminf(fmaxf(u, 0.0f), top); }

// Cell index and offset along one axis: u = x * (1/cell) - origin/cell,
// clamped to [0, g-1]; the cell is min(floor(u), g-2) and t = u - cell.
// fmax/fmin return the non-NaN operand, so a NaN coordinate lands on the
// grid's first node instead of producing an undefined index.
template <typename R>
__device__ __forceinline__ void axis_cell(R x, R o_ic, R inv_cell, R top, R last, uint32_t& i, R& t) {
    const R u = clamp_axis(x * inv_cell - o_ic, top);
    const R k = fmin(floor(u), last);
    i = (uint32_t)(int)k;
    t = u - k;
}

// Grid values are read through global (not flat) address-space pointers.
typedef const __attribute__((address_space(1))) float gfloat;
// Two horizontally adjacent grid values (the cell's corners along x) in one
// 8-byte load: the cell index is at most g - 2, so both lie in the row.
typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));
typedef const __attribute__((address_space(1))) f2u gf2u;
__device__ __forceinline__ f2u row2(gfloat* grid, uint32_t off) { return *(gf2u*)(grid + off); }

// Per-axis constants of a grid lookup in type R.
template <typename R>
struct Axis {
    R o_ic, top, last;
    __device__ void init(double origin, double inv_cell, int g) {
        o_ic = (R)(origin * inv_cell);
        top = R(g - 1);
        last = R(g - 2);
    }
};

template <typename R>
__device__ __forceinline__ R sdf2(gfloat* grid, uint32_t gx, const Axis<R>& ax, const Axis<R>& ay, R ic, R x, R y) {
    uint32_t ix, iy;
    R tx, ty;
    axis_cell<R>(x, ax.o_ic, ic, ax.top, ax.last, ix, tx);
    axis_cell<R>(y, ay.o_ic, ic, ay.top, ay.last, iy, ty);
    const uint32_t o0 = iy * gx + ix;
    const f2u r0 = row2(grid, o0), r1 = row2(grid, o0 + gx);
    const R v00 = (R)r0.x, v01 = (R)r0.y, v10 = (R)r1.x, v11 = (R)r1.y;
    const R a = v00 + tx * (v01 - v00);
    const R b = v10 + tx * (v11 - v10);
    return a + ty * (b - a);
}

template <typename R>
__device__ __forceinline__ R sdf3(gfloat* grid, uint32_t gx, uint32_t gxy, const Axis<R>& ax, const Axis<R>& ay,
                                  const Axis<R>& az, R ic, R x, R y, R z) {
    uint32_t ix, iy, iz;
    R tx, ty, tz;
    axis_cell<R>(x, ax.o_ic, ic, ax.top, ax.last, ix, tx);
    axis_cell<R>(y, ay.o_ic, ic, ay.top, ay.last, iy, ty);
    axis_cell<R>(z, az.o_ic, ic, az.top, az.last, iz, tz);
    const uint32_t o = iz * gxy + iy * gx + ix;
    const f2u r00 = row2(grid, o), r01 = row2(grid, o + gx), r10 = row2(grid, o + gxy),
              r11 = row2(grid, o + gxy + gx);
    const R a0 = (R)r00.x + tx * ((R)r00.y - (R)r00.x);
    const R a1 = (R)r01.x + tx * ((R)r01.y - (R)r01.x);
    const R a2 = (R)r10.x + tx * ((R)r10.y - (R)r10.x);
    const R a3 = (R)r11.x + tx * ((R)r11.y - (R)r11.x);
    const R b0 = a0 + ty * (a1 - a0);
    const R b1 = a2 + ty * (a3 - a2);
    return b0 + tz * (b1 - b0);
}

template <typename R>
__device__ __forceinline__ R hinge2(R eps_r, R dist) {
    R h = eps_r - dist;
    h = h > R(0) ? h : R(0);
    return h * h;
}

__device__ __forceinline__ void dsincos(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ void dsincos(float x, float* s, float* c) { sincosf(x, s, c); }

// Cost of one configuration x[D] for the plan's collision model.
template <typename R, int D, int KIND>
struct Cost;

template <typename R, int D>
struct Cost<R, D, PGVIMP_COLL_POINT2D> {
    gfloat* grid;
    uint32_t gx;
    Axis<R> ax, ay;
    R ic, er, w;
    __device__ void init(const PlanDev& p) {
        grid = (gfloat*)p.sdf;
        gx = (uint32_t)p.gx;
        ax.init(p.origin[0], p.inv_cell, p.gx);
        ay.init(p.origin[1], p.inv_cell, p.gy);
        ic = (R)p.inv_cell;
        er = (R)(p.hinge_eps + p.radius[0]);
        w = (R)p.obs_weight;
    }
    __device__ R operator()(const R* x) const { return w * hinge2<R>(er, sdf2<R>(grid, gx, ax, ay, ic, x[0], x[1])); }
};

template <typename R, int D>
struct Cost<R, D, PGVIMP_COLL_POINT3D> {
    gfloat* grid;
    uint32_t gx, gxy;
    Axis<R> ax, ay, az;
    R ic, er, w;
    __device__ void init(const PlanDev& p) {
        grid = (gfloat*)p.sdf;
        gx = (uint32_t)p.gx;
        gxy = (uint32_t)p.gx * (uint32_t)p.gy;
        ax.init(p.origin[0], p.inv_cell, p.gx);
        ay.init(p.origin[1], p.inv_cell, p.gy);
        az.init(p.origin[2], p.inv_cell, p.gz);
        ic = (R)p.inv_cell;
        er = (R)(p.hinge_eps + p.radius[0]);
        w = (R)p.obs_weight;
    }
    __device__ R operator()(const R* x) const {
        return w * hinge2<R>(er, sdf3<R>(grid, gx, gxy, ax, ay, az, ic, x[0], x[1], x[2]));
    }
};

// Serial chain of PGVIMP_ARM_DOF revolute joints; spheres sorted by link.
template <typename R, int D>
struct Cost<R, D, PGVIMP_COLL_ARM3D> {
    gfloat* grid;
    const double* fk;
    const double* rad;
    uint32_t gx, gxy;
    int ns;
    Axis<R> ax, ay, az;
    R ic, eps, w;
    __device__ void init(const PlanDev& p) {
        grid = (gfloat*)p.sdf;
        gx = (uint32_t)p.gx;
        gxy = (uint32_t)p.gx * (uint32_t)p.gy;
        ax.init(p.origin[0], p.inv_cell, p.gx);
        ay.init(p.origin[1], p.inv_cell, p.gy);
        az.init(p.origin[2], p.inv_cell, p.gz);
        ic = (R)p.inv_cell;
        eps = (R)p.hinge_eps;
        w = (R)p.obs_weight;
        fk = p.fk;
        rad = p.radius;
        ns = p.n_spheres;
    }
    __device__ R operator()(const R* q) const {
        // fk layout: base[3], len[7], frac[ns], axes[7], link[ns]
        const double* len = fk + 3;
        const double* frac = fk + 3 + PGVIMP_ARM_DOF;
        const double* axes = frac + ns;
        const double* link = axes + PGVIMP_ARM_DOF;
        R c0[3] = {R(1), R(0), R(0)}, c1[3] = {R(0), R(1), R(0)}, c2[3] = {R(0), R(0), R(1)};
        R o[3] = {(R)fk[0], (R)fk[1], (R)fk[2]};
        R acc = R(0);
        int s = 0;
#pragma unroll
        for (int k = 0; k < PGVIMP_ARM_DOF; ++k) {
            R sn, cs;
            dsincos(q[k], &sn, &cs);
            const int axis = (int)axes[k];
            if (axis == 2) {
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const R a = c0[r], b = c1[r];
                    c0[r] = a * cs + b * sn;
                    c1[r] = b * cs - a * sn;
                }
            } else if (axis == 1) {
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const R a = c0[r], b = c2[r];
                    c0[r] = a * cs - b * sn;
                    c2[r] = a * sn + b * cs;
                }
            } else {
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const R a = c1[r], b = c2[r];
                    c1[r] = a * cs + b * sn;
                    c2[r] = b * cs - a * sn;
                }
            }
            const R L = (R)len[k];
            for (; s < ns && (int)link[s] == k; ++s) {
                const R f = (R)frac[s] * L;
                const R px = o[0] + f * c2[0], py = o[1] + f * c2[1], pz = o[2] + f * c2[2];
                const R dist = sdf3<R>(grid, gx, gxy, ax, ay, az, ic, px, py, pz);
                acc += hinge2<R>(eps + (R)rad[s], dist);
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) o[r] += L * c2[r];
        }
        return w * acc;
    }
};

// Lower Cholesky factor of the symmetric D x D matrix whose lower triangle
// is A (packed by rows: A[a(a+1)/2 + c], c <= a); false if not PD.
template <int D>
__device__ __forceinline__ bool chol_packed(const double* A, double* L) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        double dd = A[j * (j + 1) / 2 + j];
#pragma unroll
        for (int k = 0; k < j; ++k) dd = fma(-L[j * (j + 1) / 2 + k], L[j * (j + 1) / 2 + k], dd);
        ok = ok && dd > 0.0 && dd < INFINITY;
        const double l = sqrt(ok ? dd : 1.0);
        L[j * (j + 1) / 2 + j] = l;
        const double il = 1.0 / l;
#pragma unroll
        for (int i = j + 1; i < D; ++i) {
            double s = A[i * (i + 1) / 2 + j];
#pragma unroll
            for (int k = 0; k < j; ++k) s = fma(-L[i * (i + 1) / 2 + k], L[j * (j + 1) / 2 + k], s);
            L[i * (i + 1) / 2 + j] = s * il;
        }
    }
    return ok;
}

// Shape of one instantiation: F factors per workgroup of T = 256 threads
// (F < T at small batches: more threads per factor shorten each thread's
// chain of dependent node evaluations), node
// evaluations per factor NE (the centre first in mixed mode), chunks of CH
// evaluations whose LDS rows have an odd stride CHS (no bank conflicts when
// thread f walks its row).
template <typename R, int D, int P, int F, int KIND>
struct ExpectShape {
    static constexpr int T = 256;
    static constexpr int NODES = ipow(P, D);
    static constexpr bool CENTRE = sizeof(R) == 4 && P >= 2;
    static constexpr int NE = NODES + (CENTRE ? 1 : 0);
    static constexpr int PS = D + D * (D + 1) / 2;  // mu, then L packed by rows
    static constexpr int CHMAX = ((expect_lds(KIND) / (int)sizeof(R)) / F - 1) | 1;  // odd, < budget
    static constexpr int CH = cmin(NE, CHMAX);
    static constexpr int CHS = CH | 1;
    static constexpr int NCH = (NE + CH - 1) / CH;
    // rule points of every evaluation in an LDS table when it is small
    static constexpr bool TAB = NE * D <= 1024;
};

template <typename R, int D, int P, int KIND, int F>
__global__ void __launch_bounds__((ExpectShape<R, D, P, F, KIND>::T))
    expect_kernel(DevState st, int plan_lo, int plan_hi, int tiles, int respect_budget) {
    using Sh = ExpectShape<R, D, P, F, KIND>;
    constexpr int T = Sh::T, NE = Sh::NE, PS = Sh::PS, CH = Sh::CH, CHS = Sh::CHS, NCH = Sh::NCH;
    constexpr bool CENTRE = Sh::CENTRE;
    constexpr int NS2 = D * (D + 1) / 2;
    __shared__ R psi[F * CHS];
    __shared__ R par[F * PS];
    __shared__ R xs[P], ws[P];
    __shared__ R xtab[Sh::TAB ? NE * D : 1];  // xi of evaluation e at [e * D + a]

    const int b = blockIdx.x;
    const int k = b / kNumXcd;
    const int pid = plan_lo + (k / tiles) * kNumXcd + b % kNumXcd;
    if (pid >= plan_hi) return;
    const PlanDev& p = st.plans[pid];
    if (!p.active || p.coll_kind != KIND || p.gh_points != P) return;
    if (respect_budget && p.iters_left <= 0) return;
    const int tid = threadIdx.x;
    const int N = p.N;
    const int lo = p.coll_states == 1 ? 1 : 0;
    const int hi = p.coll_states == 1 ? N - 1 : N;
    const int64_t S = st.S;
    const int n = st.n;
    const R* xg = Tab<R>::x(st) + P * kMaxGH;
    if (tid < P) {
        xs[tid] = xg[tid];
        ws[tid] = Tab<R>::w(st)[P * kMaxGH + tid];
    }
    // rule point of evaluation e (the centre, then the tensor nodes with
    // coordinate 0 varying fastest)
    auto point = [&](const R* x1, uint32_t e, R* xi) {
        uint32_t node = CENTRE ? (e == 0 ? 0u : e - 1u) : e;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const uint32_t q = node % (uint32_t)P;
            node /= (uint32_t)P;
            xi[a] = (CENTRE && e == 0) ? R(0) : x1[q];
        }
    };
    if (Sh::TAB)
        for (int e = tid; e < NE; e += T) point(xg, (uint32_t)e, xtab + e * D);
    Cost<R, D, KIND> cost;
    cost.init(p);

    for (int i0 = (k % tiles) * F; i0 < N; i0 += tiles * F) {
        // A: marginal of factor i0 + tid, its FP64 Cholesky factor, mu and L to LDS
        const int i = i0 + tid;
        const bool mine = tid < F && i >= lo && i < hi;
        const int64_t s = p.off + i;
        // the factor's covariance (lower triangle) and its FP64 Cholesky factor
        auto factor = [&](double* L) {
            double A[NS2];
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int c = 0; c <= a; ++c)
                    A[a * (a + 1) / 2 + c] = st.SD[(int64_t)(p.coll_index[a] * n + p.coll_index[c]) * S + s];
            return chol_packed<D>(A, L);
        };
        if (tid < F) {
            double L[NS2];
            if (mine) {
                factor(L);
#pragma unroll
                for (int a = 0; a < D; ++a) par[tid * PS + a] = (R)st.mu[(int64_t)p.coll_index[a] * S + s];
            } else {
#pragma unroll
                for (int e = 0; e < NS2; ++e) L[e] = 0.0;
#pragma unroll
                for (int a = 0; a < D; ++a) par[tid * PS + a] = R(0);
            }
#pragma unroll
            for (int e = 0; e < NS2; ++e) par[tid * PS + D + e] = (R)L[e];
        }
        R s0 = R(0), s1[D], S2[NS2], centre = R(0);
#pragma unroll
        for (int a = 0; a < D; ++a) s1[a] = R(0);
#pragma unroll
        for (int e = 0; e < NS2; ++e) S2[e] = R(0);
        const int nf = min(F, hi - i0);  // factors of this round (those below lo are skipped)

        for (int ch = 0; ch < NCH; ++ch) {
            __syncthreads();
            // B: cost at every (factor, evaluation) pair of the chunk.  The
            // body has no branch: pairs past the last factor or evaluation
            // run on zeroed or clamped inputs and their values are never read,
            // so the loads of several pairs can be in flight at once.
            constexpr int ITEMS = F * CH;
#pragma unroll 4
            for (int it = tid; it < ITEMS; it += T) {
                const uint32_t f = (uint32_t)it / (uint32_t)CH;
                const uint32_t jj = (uint32_t)it - f * (uint32_t)CH;
                const uint32_t e = min((uint32_t)(ch * CH) + jj, (uint32_t)(NE - 1));
                R xi[D];
                if (Sh::TAB) {
#pragma unroll
                    for (int a = 0; a < D; ++a) xi[a] = xtab[e * D + a];
                } else {
                    point(xs, e, xi);
                }
                const R* pf = par + f * PS;
                R x[D];
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    R v = pf[a];
#pragma unroll
                    for (int c = 0; c <= a; ++c) v += pf[D + a * (a + 1) / 2 + c] * xi[c];
                    x[a] = v;
                }
                psi[f * CHS + jj] = cost(x);
            }
            __syncthreads();
            // C: thread tid accumulates its factor's moments in node order
            if (mine) {
                const R* row = psi + tid * CHS;
#pragma unroll 4
                for (int jj = 0; jj < CH; ++jj) {
                    const int e = ch * CH + jj;
                    if (NE % CH != 0 && e >= NE) break;
                    const R v = row[jj];
                    if (CENTRE && e == 0) {
                        centre = v;
                        continue;
                    }
                    int node = CENTRE ? e - 1 : e;
                    R xi[D], W = R(1);
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        const int q = node % P;
                        node /= P;
                        xi[a] = xs[q];
                        W *= ws[q];
                    }
                    const R wp = W * (v - centre);
                    s0 += wp;
                    int t = 0;
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        const R wa = wp * xi[a];
                        s1[a] += wa;
#pragma unroll
                        for (int c = a; c < D; ++c) S2[t++] += wa * xi[c];
                    }
                }
            }
        }
        // FP64 epilogue: Li = L^-1 (lower), g = Li^T s1, H = Li^T (S2 - s0 I) Li
        // (the factor is formed again: cheaper than holding it through B and C)
        if (mine) {
            double L[NS2];
            if (!factor(L)) {
                st.Ecol[s] = NAN;
#pragma unroll
                for (int a = 0; a < D; ++a) st.gcol[a * S + s] = NAN;
#pragma unroll
                for (int a = 0; a < D * D; ++a) st.Hcol[a * S + s] = NAN;
            } else {
                // Li packed by rows like L: Li[a(a+1)/2 + c], c <= a
                double Li[NS2];
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    const double inv = 1.0 / L[a * (a + 1) / 2 + a];
                    Li[a * (a + 1) / 2 + a] = inv;
#pragma unroll
                    for (int c = 0; c < a; ++c) {
                        double v = 0.0;
#pragma unroll
                        for (int q = c; q < a; ++q) v = fma(L[a * (a + 1) / 2 + q], Li[q * (q + 1) / 2 + c], v);
                        Li[a * (a + 1) / 2 + c] = -v * inv;
                    }
                }
                const double e0 = (double)s0;
                // M = S2 - s0 I from the upper-triangle accumulators
                auto M = [&](int a, int c) {
                    const int lo2 = a < c ? a : c, hi2 = a < c ? c : a;
                    const int t = lo2 * D - lo2 * (lo2 - 1) / 2 + (hi2 - lo2);
                    return (double)S2[t] - (a == c ? e0 : 0.0);
                };
                st.Ecol[s] = e0 + (double)centre;
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    double v = 0.0;
#pragma unroll
                    for (int q = a; q < D; ++q) v = fma(Li[q * (q + 1) / 2 + a], (double)s1[q], v);
                    st.gcol[a * S + s] = v;
                }
                // row a of H: t = (Li^T M)_a = sum_q Li[q][a] M[q][.], then H_ac = t Li[.][c]
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    double t[D];
#pragma unroll
                    for (int r = 0; r < D; ++r) {
                        double v = 0.0;
#pragma unroll
                        for (int q = a; q < D; ++q) v = fma(Li[q * (q + 1) / 2 + a], M(q, r), v);
                        t[r] = v;
                    }
#pragma unroll
                    for (int c = a; c < D; ++c) {
                        double v = 0.0;
#pragma unroll
                        for (int r = c; r < D; ++r) v = fma(t[r], Li[r * (r + 1) / 2 + c], v);
                        st.Hcol[(a * D + c) * S + s] = v;
                        st.Hcol[(c * D + a) * S + s] = v;
                    }
                }
            }
        }
        __syncthreads();  // LDS rows are rewritten by the next round
    }
}

// Grid: per XCD, `slots` plan slots of `tiles` blocks each.  Block b runs on
// XCD b mod 8 and serves plan plan_lo + 8*slot + (b mod 8), so the plan and
// its fields are wave-uniform (scalar loads) and each XCD's L2 caches the
// maps of its own plans only.  A block strides over its plan's states in
// steps of `tiles` rounds of F factors, so any plan length is covered
// whatever the grid.
template <typename R, int D, int P, int KIND, int F>
static hipError_t launch_one(const DevState& st, int plo, int phi, int maxN, int respect, hipStream_t s) {
    const int tiles = std::max(1, (maxN + F - 1) / F);
    const int64_t slots = (phi - plo + kNumXcd - 1) / kNumXcd;
    const int64_t blocks = slots * tiles * kNumXcd;
    if (blocks <= 0) return hipSuccess;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((expect_kernel<R, D, P, KIND, F>), dim3((unsigned)blocks),
                       dim3(ExpectShape<R, D, P, F, KIND>::T), 0, s, st, plo, phi, tiles, respect);
    return hipGetLastError();
}

// Factors per workgroup: the requested group (32, 64, 128 or 256) or, for
// 0, the largest that still gives every compute unit four workgroups.
// Results do not depend on it.
static int pick_group(int group, int plans, int maxN, int cus) {
    if (group == 32 || group == 64 || group == 128 || group == 256) return group;
    const int64_t slots = (plans + kNumXcd - 1) / kNumXcd;
    for (int f = 256; f > 32; f /= 2)
        if (slots * kNumXcd * ((maxN + f - 1) / f) >= 4 * (int64_t)cus) return f;
    return 32;
}

#define PG_GROUPS(R, D, P, KIND)                                                              \
    switch (f) {                                                                              \
        case 256: return launch_one<R, D, P, KIND, 256>(st, plo, phi, maxN, respect, s);    \
        case 128: return launch_one<R, D, P, KIND, 128>(st, plo, phi, maxN, respect, s);    \
        case 64: return launch_one<R, D, P, KIND, 64>(st, plo, phi, maxN, respect, s);      \
        default: return launch_one<R, D, P, KIND, 32>(st, plo, phi, maxN, respect, s);      \
    }

template <typename R>
static hipError_t dispatch(const DevState& st, int kind, int d, int p, int f, int plo, int phi, int maxN, int respect,
                           hipStream_t s) {
    if (kind == PGVIMP_COLL_POINT2D && d == 2) {
        switch (p) {
            case 1: PG_GROUPS(R, 2, 1, PGVIMP_COLL_POINT2D);
            case 2: PG_GROUPS(R, 2, 2, PGVIMP_COLL_POINT2D);
            case 3: PG_GROUPS(R, 2, 3, PGVIMP_COLL_POINT2D);
            case 4: PG_GROUPS(R, 2, 4, PGVIMP_COLL_POINT2D);
            case 5: PG_GROUPS(R, 2, 5, PGVIMP_COLL_POINT2D);
            case 6: PG_GROUPS(R, 2, 6, PGVIMP_COLL_POINT2D);
            case 7: PG_GROUPS(R, 2, 7, PGVIMP_COLL_POINT2D);
            case 8: PG_GROUPS(R, 2, 8, PGVIMP_COLL_POINT2D);
            case 10: PG_GROUPS(R, 2, 10, PGVIMP_COLL_POINT2D);
            default: return hipErrorInvalidValue;
        }
    }
    if (kind == PGVIMP_COLL_POINT3D && d == 3) {
        switch (p) {
            case 2: PG_GROUPS(R, 3, 2, PGVIMP_COLL_POINT3D);
            case 3: PG_GROUPS(R, 3, 3, PGVIMP_COLL_POINT3D);
            case 4: PG_GROUPS(R, 3, 4, PGVIMP_COLL_POINT3D);
            case 5: PG_GROUPS(R, 3, 5, PGVIMP_COLL_POINT3D);
            default: return hipErrorInvalidValue;
        }
    }
    if (kind == PGVIMP_COLL_ARM3D && d == PGVIMP_ARM_DOF) {
        // the arm's nodes are costly and many: 32 factors per workgroup
        switch (p) {
            case 2: return launch_one<R, PGVIMP_ARM_DOF, 2, PGVIMP_COLL_ARM3D, 32>(st, plo, phi, maxN, respect, s);
            case 3: return launch_one<R, PGVIMP_ARM_DOF, 3, PGVIMP_COLL_ARM3D, 32>(st, plo, phi, maxN, respect, s);
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}
#undef PG_GROUPS

int expect_group_for(int group, int plans, int maxN, int cus) { return pick_group(group, plans, maxN, cus); }

bool expect_supported(int kind, int d, int p, int group) {
    if (group != 0 && group != 32 && group != 64 && group != 128 && group != 256) return false;
    if (kind == PGVIMP_COLL_POINT2D) return d == 2 && p >= 1 && p <= 10 && p != 9;
    if (kind == PGVIMP_COLL_POINT3D) return d == 3 && p >= 2 && p <= 5;
    if (kind == PGVIMP_COLL_ARM3D) return d == PGVIMP_ARM_DOF && (p == 2 || p == 3);
    return kind == PGVIMP_COLL_NONE;
}

hipError_t launch_expect(const DevState& st, int kind, int d, int p, int precision, int group, int plo, int phi,
                         int maxN, int respect, hipStream_t s) {
    if (kind == PGVIMP_COLL_NONE) return hipSuccess;
    const int f = pick_group(group, phi - plo, maxN, st.wbudget);
    if (precision == PGVIMP_MIXED) return dispatch<float>(st, kind, d, p, f, plo, phi, maxN, respect, s);
    return dispatch<double>(st, kind, d, p, f, plo, phi, maxN, respect, s);
}

}  // namespace pg
