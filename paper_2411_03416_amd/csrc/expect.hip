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
__device__ __forceinline__ void axis_cell(double x, double o_ic, double inv_cell, double top, double last,
                                          uint32_t& i, double& t) {
    const double u = clamp_axis(x * inv_cell - o_ic, top);
    const double k = fmin(floor(u), last);
    i = (uint32_t)(int)k;
    t = u - k;
}
// FP32: the same cell and offset with two median-of-three clamps, the cell
// floor(u) clamped to [0, g-2] and t = u - cell clamped to [0, 1], which
// equals clamping u to [0, g-1] first, bit for bit, for every non-NaN u.
// A NaN coordinate gives cell 0 (the float-to-integer conversion of NaN is
// 0), so the index stays in the grid.
__device__ __forceinline__ void axis_cell(float x, float o_ic, float inv_cell, float top, float last, uint32_t& i,
                                          float& t) {
    (void)top;
    const float u = x * inv_cell - o_ic;
    const float k = __builtin_amdgcn_fmed3f(floorf(u), 0.0f, last);
    i = (uint32_t)(int)k;
    t = __builtin_amdgcn_fmed3f(u - k, 0.0f, 1.0f);
}

// Grid tables are read by raw buffer loads through a resource that spans
// exactly the table: 32-bit byte offsets (one VGPR per address), and an
// offset past the table reads 0 instead of faulting.
struct Grid {
    __amdgpu_buffer_rsrc_t rsrc;
    __device__ void init(const float* g, int64_t count) {
        // word 3 = 0x00020000: 32-bit data format, as raw dword loads need on CDNA
        rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)g, (short)0, (int)(count * 4), 0x00020000);
    }
};
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

// 2-D lookup from the cell-corner table: the four values of cell (ix, iy)
// in one 16-byte load, bilinear in x then y.
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
template <typename R>
__device__ __forceinline__ R sdf2q(const Grid& quad, uint32_t cx, const Axis<R>& ax, const Axis<R>& ay, R ic, R x,
                                   R y) {
    uint32_t ix, iy;
    R tx, ty;
    axis_cell(x, ax.o_ic, ic, ax.top, ax.last, ix, tx);
    axis_cell(y, ay.o_ic, ic, ay.top, ay.last, iy, ty);
    const u4v q = __builtin_amdgcn_raw_buffer_load_b128(quad.rsrc, (iy * cx + ix) * 16u, 0, 0);
    const R v00 = (R)__uint_as_float(q.x), v01 = (R)__uint_as_float(q.y), v10 = (R)__uint_as_float(q.z),
            v11 = (R)__uint_as_float(q.w);
    const R a = v00 + tx * (v01 - v00);
    const R b = v10 + tx * (v11 - v10);
    return a + ty * (b - a);
}

// Cell-corner table of each z-slice of a grid [gz][gy][gx]: entry
// (iz, iy, ix) holds v[iz][iy][ix], v[iz][iy][ix+1], v[iz][iy+1][ix],
// v[iz][iy+1][ix+1] (a 2-D grid is one slice).
__global__ void build_quads_kernel(const float* __restrict__ sdf, int gx, int gy, int gz, float* __restrict__ quad) {
    const int64_t per = (int64_t)(gx - 1) * (gy - 1), cells = per * gz;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t iz = c / per, r = c - iz * per, iy = r / (gx - 1), ix = r - iy * (gx - 1);
        const float* r0 = sdf + (iz * gy + iy) * gx + ix;
        quad[4 * c + 0] = r0[0];
        quad[4 * c + 1] = r0[1];
        quad[4 * c + 2] = r0[gx];
        quad[4 * c + 3] = r0[gx + 1];
    }
}

hipError_t launch_build_quads(const float* sdf, int gx, int gy, int gz, float* quad, hipStream_t s) {
    const int64_t cells = (int64_t)(gx - 1) * (gy - 1) * gz;
    if (cells <= 0) return hipSuccess;
    const int threads = 256;
    const int blocks = (int)std::min<int64_t>((cells + threads - 1) / threads, 65536);
    hipLaunchKernelGGL(build_quads_kernel, dim3(blocks), dim3(threads), 0, s, sdf, gx, gy, gz, quad);
    return hipGetLastError();
}

// 3-D lookup from the per-slice corner tables: two 16-byte loads (slices
// iz and iz + 1), trilinear in x, then y, then z.
template <typename R>
__device__ __forceinline__ R sdf3q(const Grid& quad, uint32_t cx, uint32_t cxy, const Axis<R>& ax, const Axis<R>& ay,
                                   const Axis<R>& az, R ic, R x, R y, R z) {
    uint32_t ix, iy, iz;
    R tx, ty, tz;
    axis_cell(x, ax.o_ic, ic, ax.top, ax.last, ix, tx);
    axis_cell(y, ay.o_ic, ic, ay.top, ay.last, iy, ty);
    axis_cell(z, az.o_ic, ic, az.top, az.last, iz, tz);
    const uint32_t o = iz * cxy + iy * cx + ix;
    const u4v q0 = __builtin_amdgcn_raw_buffer_load_b128(quad.rsrc, o * 16u, 0, 0);
    const u4v q1 = __builtin_amdgcn_raw_buffer_load_b128(quad.rsrc, (o + cxy) * 16u, 0, 0);
    const R a0 = (R)__uint_as_float(q0.x) + tx * ((R)__uint_as_float(q0.y) - (R)__uint_as_float(q0.x));
    const R a1 = (R)__uint_as_float(q0.z) + tx * ((R)__uint_as_float(q0.w) - (R)__uint_as_float(q0.z));
    const R a2 = (R)__uint_as_float(q1.x) + tx * ((R)__uint_as_float(q1.y) - (R)__uint_as_float(q1.x));
    const R a3 = (R)__uint_as_float(q1.z) + tx * ((R)__uint_as_float(q1.w) - (R)__uint_as_float(q1.z));
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
    Grid quad;
    uint32_t cx;
    Axis<R> ax, ay;
    R ic, er, w;
    __device__ void init(const PlanDev& p) {
        quad.init(p.sdfq, (int64_t)(p.gx - 1) * (p.gy - 1) * 4);
        cx = (uint32_t)(p.gx - 1);
        ax.init(p.origin[0], p.inv_cell, p.gx);
        ay.init(p.origin[1], p.inv_cell, p.gy);
        ic = (R)p.inv_cell;
        er = (R)(p.hinge_eps + p.radius[0]);
        w = (R)p.obs_weight;
    }
    __device__ R operator()(const R* x) const { return w * hinge2<R>(er, sdf2q<R>(quad, cx, ax, ay, ic, x[0], x[1])); }
};

template <typename R, int D>
struct Cost<R, D, PGVIMP_COLL_POINT3D> {
    Grid quad;
    uint32_t cx, cxy;
    Axis<R> ax, ay, az;
    R ic, er, w;
    __device__ void init(const PlanDev& p) {
        quad.init(p.sdfq, (int64_t)(p.gx - 1) * (p.gy - 1) * p.gz * 4);
        cx = (uint32_t)(p.gx - 1);
        cxy = (uint32_t)(p.gx - 1) * (uint32_t)(p.gy - 1);
        ax.init(p.origin[0], p.inv_cell, p.gx);
        ay.init(p.origin[1], p.inv_cell, p.gy);
        az.init(p.origin[2], p.inv_cell, p.gz);
        ic = (R)p.inv_cell;
        er = (R)(p.hinge_eps + p.radius[0]);
        w = (R)p.obs_weight;
    }
    __device__ R operator()(const R* x) const {
        return w * hinge2<R>(er, sdf3q<R>(quad, cx, cxy, ax, ay, az, ic, x[0], x[1], x[2]));
    }
};

// Serial chain of PGVIMP_ARM_DOF revolute joints; spheres sorted by link.
template <typename R, int D>
struct Cost<R, D, PGVIMP_COLL_ARM3D> {
    Grid quad;
    const double* fk;
    const double* rad;
    uint32_t cx, cxy;
    int ns;
    Axis<R> ax, ay, az;
    R ic, eps, w;
    __device__ void init(const PlanDev& p) {
        quad.init(p.sdfq, (int64_t)(p.gx - 1) * (p.gy - 1) * p.gz * 4);
        cx = (uint32_t)(p.gx - 1);
        cxy = (uint32_t)(p.gx - 1) * (uint32_t)(p.gy - 1);
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
                const R dist = sdf3q<R>(quad, cx, cxy, ax, ay, az, ic, px, py, pz);
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

// Shape of one instantiation: F factors per workgroup of T = 256 threads,
// node evaluations per factor NE (the centre first in mixed mode), chunks
// of CH evaluations whose LDS rows have an odd stride CHS (no bank
// conflicts when thread f walks its row).
template <typename R, int D, int P, int F, int KIND>
struct ExpectShape {
    static constexpr int T = 256;
    // P = 0: the plan's sparse rule (Smolyak), whose size is known at run time
    static constexpr bool SPARSE = P == 0;
    static constexpr int NODES = SPARSE ? 0 : ipow(P, D);
    static constexpr bool CENTRE = sizeof(R) == 4 && (SPARSE || P >= 2);
    static constexpr int NE = NODES + (CENTRE ? 1 : 0);
    static constexpr int NS2 = D * (D + 1) / 2;
    static constexpr int PS = D + NS2;  // mu, then L packed by rows
    static constexpr int CHMAX = ((expect_lds(KIND) / (int)sizeof(R)) / F - 1) | 1;  // odd, < budget
    static constexpr int CH = SPARSE ? CHMAX : cmin(NE, CHMAX);
    static constexpr int CHS = CH | 1;
    static constexpr int NCH = (NE + CH - 1) / CH;
    // rule points and weights of every evaluation in an LDS table when small
    static constexpr bool TAB = !SPARSE && NE * D <= 1024;
    static constexpr int TS = D + 1;  // table row: xi[0..D-1], W
};

// Rule point xi and weight W of evaluation e: the centre (xi = 0) first in
// mixed mode, then the tensor nodes with coordinate 0 varying fastest.  x1
// and w1 are the 1-D rule of p points.
template <typename R, int D, int P, bool CENTRE>
__device__ __forceinline__ void rule_point(const R* x1, const R* w1, uint32_t e, R* xi, R& W) {
    uint32_t node = CENTRE ? (e == 0 ? 0u : e - 1u) : e;
    W = R(1);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const uint32_t q = node % (uint32_t)P;
        node /= (uint32_t)P;
        xi[a] = (CENTRE && e == 0) ? R(0) : x1[q];
        W *= w1[q];
    }
}

// Rule point and weight of evaluation e of a sparse rule: the centre first
// (when cen), then the plan's rows (xi[0..D-1], W).
template <typename R, int D>
__device__ __forceinline__ void sparse_point(const R* __restrict__ rows, bool cen, uint32_t e, R* xi, R& W) {
    const uint32_t r = cen ? (e == 0 ? 0u : e - 1u) : e;
#pragma unroll
    for (int a = 0; a < D; ++a) xi[a] = (cen && e == 0) ? R(0) : rows[r * (D + 1) + a];
    W = rows[r * (D + 1) + D];
}
__device__ __forceinline__ const double* rule_rows(const PlanDev& p, double) { return p.rule64; }
__device__ __forceinline__ const float* rule_rows(const PlanDev& p, float) { return p.rule32; }

// x = mu + L xi (L lower, packed by rows), with explicit FMAs
template <typename R, int D>
__device__ __forceinline__ void node_point(const R* mu, const R* L, const R* xi, R* x) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
        R v = mu[a];
#pragma unroll
        for (int c = 0; c <= a; ++c) v = fma(L[a * (a + 1) / 2 + c], xi[c], v);
        x[a] = v;
    }
}

// Running moments of one factor: s0 = sum W (psi - c), s1 = sum W (psi - c)
// xi, S2 = sum W (psi - c) xi xi^T (upper triangle by rows), added in node
// order by both kernels with the same operations (this file is built with
// contraction within expressions only, so psi - c is never fused with the
// product that formed psi: that product is in registers in one kernel and
// behind an LDS store in the other); the FMAs are explicit.
template <typename R, int D>
struct Moments {
    static constexpr int NS2 = D * (D + 1) / 2;
    R s0, s1[D], S2[NS2];
    __device__ void zero() {
        s0 = R(0);
#pragma unroll
        for (int a = 0; a < D; ++a) s1[a] = R(0);
#pragma unroll
        for (int e = 0; e < NS2; ++e) S2[e] = R(0);
    }
    __device__ __forceinline__ void add(R v, R centre, R W, const R* xi) {
        const R wp = W * (v - centre);
        s0 = s0 + wp;
        int t = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const R wa = wp * xi[a];
            s1[a] = s1[a] + wa;
#pragma unroll
            for (int c = a; c < D; ++c, ++t) S2[t] = fma(wa, xi[c], S2[t]);
        }
    }
};

// The factor's covariance (lower triangle, configuration coordinates) from
// the marginals and its FP64 Cholesky factor; false if it is not PD.
template <int D>
__device__ __forceinline__ bool factor_chol(const DevState& st, const PlanDev& p, int64_t s, double* L) {
    constexpr int NS2 = D * (D + 1) / 2;
    double A[NS2];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int c = 0; c <= a; ++c)
            A[a * (a + 1) / 2 + c] = st.SD[(int64_t)(p.coll_index[a] * st.n + p.coll_index[c]) * st.S + s];
    return chol_packed<D>(A, L);
}

// FP64 epilogue: Li = L^-1 (lower), E = s0 + c, g = Li^T s1,
// H = Li^T (S2 - s0 I) Li; NaN outputs for a factor that is not PD.
template <typename R, int D>
__device__ __forceinline__ void store_factor(const DevState& st, int64_t s, bool ok, const double* L,
                                             const Moments<R, D>& m, R centre) {
    const int64_t S = st.S;
    if (!ok) {
        st.Ecol[s] = NAN;
#pragma unroll
        for (int a = 0; a < D; ++a) st.gcol[a * S + s] = NAN;
#pragma unroll
        for (int a = 0; a < D * D; ++a) st.Hcol[a * S + s] = NAN;
        return;
    }
    constexpr int NS2 = D * (D + 1) / 2;
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
    const double e0 = (double)m.s0;
    // M = S2 - s0 I from the upper-triangle accumulators
    auto M = [&](int a, int c) {
        const int lo2 = a < c ? a : c, hi2 = a < c ? c : a;
        const int t = lo2 * D - lo2 * (lo2 - 1) / 2 + (hi2 - lo2);
        return (double)m.S2[t] - (a == c ? e0 : 0.0);
    };
    st.Ecol[s] = e0 + (double)centre;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double v = 0.0;
#pragma unroll
        for (int q = a; q < D; ++q) v = fma(Li[q * (q + 1) / 2 + a], (double)m.s1[q], v);
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

// Block b of a launch serves plan plan_lo + 8*slot + (b mod 8) (slot =
// (b / 8) / tiles) and its rounds of F factors starting at tile (b / 8) mod
// tiles; false if the block has nothing to do.
__device__ __forceinline__ bool expect_block_plan(const DevState& st, int plan_lo, int plan_hi, int tiles,
                                                  int respect_budget, int kind, int gh, int& pid, int& tile) {
    // gh = 0: plans with a sparse rule (any level); else tensor plans of gh points
    const int b = blockIdx.x;
    const int k = b / kNumXcd;
    pid = plan_lo + (k / tiles) * kNumXcd + b % kNumXcd;
    tile = k % tiles;
    if (pid >= plan_hi) return false;
    const PlanDev& p = st.plans[pid];
    if (!p.active || p.coll_kind != kind) return false;
    if (gh == 0 ? p.quadrature != PGVIMP_QUAD_SPARSE : (p.quadrature != PGVIMP_QUAD_TENSOR || p.gh_points != gh))
        return false;
    return !(respect_budget && p.iters_left <= 0);
}

// Small batches: F factors per workgroup of 256 threads in three stages
// (see the top of this file).
template <typename R, int D, int P, int KIND, int F>
__global__ void __launch_bounds__(256) expect_kernel(DevState st, int plan_lo, int plan_hi, int tiles,
                                                     int respect_budget) {
    using Sh = ExpectShape<R, D, P, F, KIND>;
    constexpr int T = Sh::T, PS = Sh::PS, CH = Sh::CH, CHS = Sh::CHS, TS = Sh::TS;
    constexpr bool SPARSE = Sh::SPARSE;
    constexpr int NS2 = Sh::NS2;
    constexpr int PX = P > 0 ? P : 1;
    __shared__ R psi[F * CHS];
    __shared__ R par[F * PS];
    __shared__ R xs[PX], ws[PX];
    __shared__ R ntab[Sh::TAB ? Sh::NE * TS : 1];  // row e: xi of evaluation e, then its weight

    int pid, tile;
    if (!expect_block_plan(st, plan_lo, plan_hi, tiles, respect_budget, KIND, P, pid, tile)) return;
    const PlanDev& p = st.plans[pid];
    const int tid = threadIdx.x;
    const int N = p.N;
    const int lo = p.coll_states == 1 ? 1 : 0;
    const int hi = p.coll_states == 1 ? N - 1 : N;
    const int64_t S = st.S;
    // evaluations per factor (the centre first in mixed mode, when the rule
    // integrates xi xi^T: a sparse rule of level k >= 2)
    const bool CENTRE = SPARSE ? Sh::CENTRE && p.gh_points >= 2 : Sh::CENTRE;
    const int NE = SPARSE ? p.rule_n + (CENTRE ? 1 : 0) : Sh::NE;
    const int NCH = (NE + CH - 1) / CH;
    const R* __restrict__ rows = rule_rows(p, R(0));
    if (!SPARSE && tid < P) {
        xs[tid] = Tab<R>::x(st)[P * kMaxGH + tid];
        ws[tid] = Tab<R>::w(st)[P * kMaxGH + tid];
    }
    if (Sh::TAB) {
        __syncthreads();
        for (int e = tid; e < NE; e += T)
            rule_point<R, D, PX, Sh::CENTRE>(xs, ws, (uint32_t)e, ntab + e * TS, ntab[e * TS + D]);
    }
    Cost<R, D, KIND> cost;
    cost.init(p);

    for (int i0 = tile * F; i0 < N; i0 += tiles * F) {
        // A: marginal of factor i0 + tid, its FP64 Cholesky factor, mu and L to LDS
        const int i = i0 + tid;
        const bool mine = tid < F && i >= lo && i < hi;
        const int64_t s = p.off + i;
        if (tid < F) {
            double L[NS2];
            if (mine) {
                factor_chol<D>(st, p, s, L);
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
        Moments<R, D> m;
        m.zero();
        R centre = R(0);

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
                R xi[D], W;
                if (SPARSE) {
                    sparse_point<R, D>(rows, CENTRE, e, xi, W);
                } else if (Sh::TAB) {
#pragma unroll
                    for (int a = 0; a < D; ++a) xi[a] = ntab[e * TS + a];
                } else {
                    rule_point<R, D, PX, Sh::CENTRE>(xs, ws, e, xi, W);
                }
                const R* pf = par + f * PS;
                R x[D];
                node_point<R, D>(pf, pf + D, xi, x);
                psi[f * CHS + jj] = cost(x);
            }
            __syncthreads();
            // C: thread tid accumulates its factor's moments in node order
            if (mine) {
                const R* row = psi + tid * CHS;
#pragma unroll 4
                for (int jj = 0; jj < CH; ++jj) {
                    const int e = ch * CH + jj;
                    if (e >= NE) break;
                    const R v = row[jj];
                    if (CENTRE && e == 0) {
                        centre = v;
                        continue;
                    }
                    R xi[D], W;
                    if (SPARSE) {
                        sparse_point<R, D>(rows, CENTRE, (uint32_t)e, xi, W);
                    } else if (Sh::TAB) {
#pragma unroll
                        for (int a = 0; a < D; ++a) xi[a] = ntab[e * TS + a];
                        W = ntab[e * TS + D];
                    } else {
                        rule_point<R, D, PX, Sh::CENTRE>(xs, ws, (uint32_t)e, xi, W);
                    }
                    m.add(v, centre, W, xi);
                }
            }
        }
        // the factor is formed again: cheaper than holding it through B and C
        if (mine) {
            double L[NS2];
            const bool ok = factor_chol<D>(st, p, s, L);
            store_factor<R, D>(st, s, ok, L, m, centre);
        }
        __syncthreads();  // LDS rows are rewritten by the next round
    }
}

// Large batches: one factor per thread, 256 per workgroup; every lane
// walks the same evaluation at the same time (weights and points are
// uniform LDS reads), and the moments stay in registers.  Node values,
// their order and the moment updates are those of expect_kernel, so both
// give the same bits.
template <typename R, int D, int P, int KIND>
__global__ void __launch_bounds__(256) expect_lane_kernel(DevState st, int plan_lo, int plan_hi, int tiles,
                                                          int respect_budget) {
    using Sh = ExpectShape<R, D, P, 256, KIND>;
    constexpr int T = 256, NE = Sh::NE, TS = Sh::TS;
    constexpr bool CENTRE = Sh::CENTRE;
    constexpr int NS2 = Sh::NS2;
    static_assert(Sh::TAB, "the lane kernel needs the rule table");
    __shared__ R xs[P], ws[P];
    __shared__ R ntab[NE * TS];

    int pid, tile;
    if (!expect_block_plan(st, plan_lo, plan_hi, tiles, respect_budget, KIND, P, pid, tile)) return;
    const PlanDev& p = st.plans[pid];
    const int tid = threadIdx.x;
    const int N = p.N;
    const int lo = p.coll_states == 1 ? 1 : 0;
    const int hi = p.coll_states == 1 ? N - 1 : N;
    const int64_t S = st.S;
    if (tid < P) {
        xs[tid] = Tab<R>::x(st)[P * kMaxGH + tid];
        ws[tid] = Tab<R>::w(st)[P * kMaxGH + tid];
    }
    __syncthreads();
    for (int e = tid; e < NE; e += T) rule_point<R, D, P, CENTRE>(xs, ws, (uint32_t)e, ntab + e * TS, ntab[e * TS + D]);
    __syncthreads();
    Cost<R, D, KIND> cost;
    cost.init(p);

    for (int i0 = tile * T; i0 < N; i0 += tiles * T) {
        const int i = i0 + tid;
        const bool mine = i >= lo && i < hi;
        const int64_t s = p.off + i;
        double L64[NS2];
        bool ok = false;
        R mu[D], L[NS2];
        if (mine) {
            ok = factor_chol<D>(st, p, s, L64);
#pragma unroll
            for (int a = 0; a < D; ++a) mu[a] = (R)st.mu[(int64_t)p.coll_index[a] * S + s];
        } else {
#pragma unroll
            for (int e = 0; e < NS2; ++e) L64[e] = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) mu[a] = R(0);
        }
#pragma unroll
        for (int e = 0; e < NS2; ++e) L[e] = (R)L64[e];
        Moments<R, D> m;
        m.zero();
        R centre = R(0);
        if (CENTRE) {
            R x[D];
            node_point<R, D>(mu, L, ntab, x);  // row 0: xi = 0
            centre = cost(x);
        }
#pragma unroll 4
        for (int e = CENTRE ? 1 : 0; e < NE; ++e) {
            R xi[D];
#pragma unroll
            for (int a = 0; a < D; ++a) xi[a] = ntab[e * TS + a];
            R x[D];
            node_point<R, D>(mu, L, xi, x);
            m.add(cost(x), centre, ntab[e * TS + D], xi);
        }
        if (mine) store_factor<R, D>(st, s, ok, L64, m, centre);
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
    if constexpr (F == 256 && ExpectShape<R, D, P, 256, KIND>::TAB)
        hipLaunchKernelGGL((expect_lane_kernel<R, D, P, KIND>), dim3((unsigned)blocks), dim3(256), 0, s, st, plo,
                           phi, tiles, respect);
    else
        hipLaunchKernelGGL((expect_kernel<R, D, P, KIND, F>), dim3((unsigned)blocks), dim3(256), 0, s, st, plo,
                           phi, tiles, respect);
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

// P = 0 launches the plans' own sparse rules.
template <typename R>
static hipError_t dispatch(const DevState& st, int kind, int d, int p, int f, int plo, int phi, int maxN, int respect,
                           hipStream_t s) {
    if (kind == PGVIMP_COLL_POINT2D && d == 2) {
        switch (p) {
            case 0: PG_GROUPS(R, 2, 0, PGVIMP_COLL_POINT2D);
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
            case 0: PG_GROUPS(R, 3, 0, PGVIMP_COLL_POINT3D);
            case 2: PG_GROUPS(R, 3, 2, PGVIMP_COLL_POINT3D);
            case 3: PG_GROUPS(R, 3, 3, PGVIMP_COLL_POINT3D);
            case 4: PG_GROUPS(R, 3, 4, PGVIMP_COLL_POINT3D);
            case 5: PG_GROUPS(R, 3, 5, PGVIMP_COLL_POINT3D);
            default: return hipErrorInvalidValue;
        }
    }
    if (kind == PGVIMP_COLL_ARM3D && d == PGVIMP_ARM_DOF) {
        // the arm's nodes are costly and many: 32 factors per workgroup, or
        // 8 (f < 32, see launch_expect) when 32 would leave most compute
        // units idle
        if (f < 32) {
            switch (p) {
                case 0: return launch_one<R, PGVIMP_ARM_DOF, 0, PGVIMP_COLL_ARM3D, 8>(st, plo, phi, maxN, respect, s);
                case 2: return launch_one<R, PGVIMP_ARM_DOF, 2, PGVIMP_COLL_ARM3D, 8>(st, plo, phi, maxN, respect, s);
                case 3: return launch_one<R, PGVIMP_ARM_DOF, 3, PGVIMP_COLL_ARM3D, 8>(st, plo, phi, maxN, respect, s);
                default: return hipErrorInvalidValue;
            }
        }
        switch (p) {
            case 0: return launch_one<R, PGVIMP_ARM_DOF, 0, PGVIMP_COLL_ARM3D, 32>(st, plo, phi, maxN, respect, s);
            case 2: return launch_one<R, PGVIMP_ARM_DOF, 2, PGVIMP_COLL_ARM3D, 32>(st, plo, phi, maxN, respect, s);
            case 3: return launch_one<R, PGVIMP_ARM_DOF, 3, PGVIMP_COLL_ARM3D, 32>(st, plo, phi, maxN, respect, s);
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}
#undef PG_GROUPS

int expect_group_for(int group, int plans, int maxN, int cus) { return pick_group(group, plans, maxN, cus); }

// Sparse rules (p = level k) are built on the host from the 1-D rules of up
// to k points, for any level the host accepts; tensor rules need a compiled
// shape.
bool expect_supported(int kind, int d, int p, int group, int quadrature) {
    if (group != 0 && group != 32 && group != 64 && group != 128 && group != 256) return false;
    if (kind == PGVIMP_COLL_NONE) return true;
    if (quadrature == PGVIMP_QUAD_SPARSE) {
        const bool shape = (kind == PGVIMP_COLL_POINT2D && d == 2) || (kind == PGVIMP_COLL_POINT3D && d == 3) ||
                           (kind == PGVIMP_COLL_ARM3D && d == PGVIMP_ARM_DOF);
        return shape && p >= 1 && p <= kMaxGH;
    }
    if (quadrature != PGVIMP_QUAD_TENSOR) return false;
    if (kind == PGVIMP_COLL_POINT2D) return d == 2 && p >= 1 && p <= 10 && p != 9;
    if (kind == PGVIMP_COLL_POINT3D) return d == 3 && p >= 2 && p <= 5;
    if (kind == PGVIMP_COLL_ARM3D) return d == PGVIMP_ARM_DOF && (p == 2 || p == 3);
    return false;
}

hipError_t launch_expect(const DevState& st, int kind, int d, int p, int quadrature, int precision, int group, int plo,
                         int phi, int maxN, int respect, hipStream_t s) {
    if (kind == PGVIMP_COLL_NONE) return hipSuccess;
    int f = pick_group(group, phi - plo, maxN, st.wbudget);
    if (kind == PGVIMP_COLL_ARM3D) {
        // the arm: 32 factors per workgroup, or 8 when the batch gives fewer
        // than two workgroups of 32 per compute unit (f = 8 then)
        const int64_t slots = (phi - plo + kNumXcd - 1) / kNumXcd;
        const bool small = group == 0 && slots * kNumXcd * ((maxN + 31) / 32) < 2 * (int64_t)st.wbudget;
        f = small ? 8 : 32;
    }
    const int shape = quadrature == PGVIMP_QUAD_SPARSE ? 0 : p;
    if (precision == PGVIMP_MIXED) return dispatch<float>(st, kind, d, shape, f, plo, phi, maxN, respect, s);
    return dispatch<double>(st, kind, d, shape, f, plo, phi, maxN, respect, s);
}

}  // namespace pg
