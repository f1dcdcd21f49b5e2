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
// Launch shape: G lanes of a wavefront share one factor; lane l evaluates
// nodes l, l+G, ...; partial sums are combined by a butterfly of xor
// shuffles in a fixed order, so a factor's result does not depend on what
// else is in the launch.  Node math, SDF lookups, forward kinematics and
// the cost run in type R (float in mixed mode, double in FP64 mode); the
// Cholesky factor and the epilogue are always FP64.  In mixed mode the cost
// is centred by psi(mu) before the FP32 sums (the rule integrates constants
// and the first two moments exactly, so only E[psi] needs it added back).
//
// Each block serves one plan, and plan q always runs on XCD q mod 8 (one L2
// per XCD): neighbouring states of a plan share SDF cache lines, and an
// XCD's L2 holds only its own plans' maps.
#include <algorithm>

#include "ctx.h"

namespace pg {

constexpr int kExpectThreads = 256;
constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

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

// Cell index and offset along one axis.  fmax/fmin return the non-NaN
// operand, so a NaN coordinate lands on the grid's first node instead of
// producing an undefined index.
template <typename R>
__device__ __forceinline__ void axis_cell(R x, R o, R inv_cell, int g, int& i, R& t) {
    const R u = clamp_axis((x - o) * inv_cell, R(g - 1));
    int k = (int)floor(u);
    k = k > g - 2 ? g - 2 : k;
    i = k;
    t = u - R(k);
}

template <typename R>
__device__ __forceinline__ R sdf2(const float* __restrict__ grid, int gx, int gy, R ox, R oy, R ic, R x, R y) {
    int ix, iy;
    R tx, ty;
    axis_cell<R>(x, ox, ic, gx, ix, tx);
    axis_cell<R>(y, oy, ic, gy, iy, ty);
    const float* r0 = grid + (int64_t)iy * gx + ix;
    const float* r1 = r0 + gx;
    const R v00 = (R)r0[0], v01 = (R)r0[1], v10 = (R)r1[0], v11 = (R)r1[1];
    const R a = v00 + tx * (v01 - v00);
    const R b = v10 + tx * (v11 - v10);
    return a + ty * (b - a);
}

template <typename R>
__device__ __forceinline__ R sdf3(const float* __restrict__ grid, int gx, int gy, int gz, R ox, R oy, R oz, R ic,
                                  R x, R y, R z) {
    int ix, iy, iz;
    R tx, ty, tz;
    axis_cell<R>(x, ox, ic, gx, ix, tx);
    axis_cell<R>(y, oy, ic, gy, iy, ty);
    axis_cell<R>(z, oz, ic, gz, iz, tz);
    const int64_t sy = gx, sz = (int64_t)gx * gy;
    const float* c = grid + iz * sz + iy * sy + ix;
    const R v000 = (R)c[0], v001 = (R)c[1], v010 = (R)c[sy], v011 = (R)c[sy + 1];
    const R v100 = (R)c[sz], v101 = (R)c[sz + 1], v110 = (R)c[sz + sy], v111 = (R)c[sz + sy + 1];
    const R a0 = v000 + tx * (v001 - v000);
    const R a1 = v010 + tx * (v011 - v010);
    const R a2 = v100 + tx * (v101 - v100);
    const R a3 = v110 + tx * (v111 - v110);
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
    const float* grid;
    int gx, gy;
    R ox, oy, ic, er, w;
    __device__ void init(const PlanDev& p) {
        grid = p.sdf;
        gx = p.gx;
        gy = p.gy;
        ox = (R)p.origin[0];
        oy = (R)p.origin[1];
        ic = (R)p.inv_cell;
        er = (R)(p.hinge_eps + p.radius[0]);
        w = (R)p.obs_weight;
    }
    __device__ R operator()(const R* x) const { return w * hinge2<R>(er, sdf2<R>(grid, gx, gy, ox, oy, ic, x[0], x[1])); }
};

template <typename R, int D>
struct Cost<R, D, PGVIMP_COLL_POINT3D> {
    const float* grid;
    int gx, gy, gz;
    R ox, oy, oz, ic, er, w;
    __device__ void init(const PlanDev& p) {
        grid = p.sdf;
        gx = p.gx;
        gy = p.gy;
        gz = p.gz;
        ox = (R)p.origin[0];
        oy = (R)p.origin[1];
        oz = (R)p.origin[2];
        ic = (R)p.inv_cell;
        er = (R)(p.hinge_eps + p.radius[0]);
        w = (R)p.obs_weight;
    }
    __device__ R operator()(const R* x) const {
        return w * hinge2<R>(er, sdf3<R>(grid, gx, gy, gz, ox, oy, oz, ic, x[0], x[1], x[2]));
    }
};

// Serial chain of PGVIMP_ARM_DOF revolute joints; spheres sorted by link.
template <typename R, int D>
struct Cost<R, D, PGVIMP_COLL_ARM3D> {
    const float* grid;
    const double* fk;
    const double* rad;
    int gx, gy, gz, ns;
    R ox, oy, oz, ic, eps, w;
    __device__ void init(const PlanDev& p) {
        grid = p.sdf;
        gx = p.gx;
        gy = p.gy;
        gz = p.gz;
        ox = (R)p.origin[0];
        oy = (R)p.origin[1];
        oz = (R)p.origin[2];
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
            const int ax = (int)axes[k];
            if (ax == 2) {
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const R a = c0[r], b = c1[r];
                    c0[r] = a * cs + b * sn;
                    c1[r] = b * cs - a * sn;
                }
            } else if (ax == 1) {
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
                const R dist = sdf3<R>(grid, gx, gy, gz, ox, oy, oz, ic, px, py, pz);
                acc += hinge2<R>(eps + (R)rad[s], dist);
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) o[r] += L * c2[r];
        }
        return w * acc;
    }
};

template <int D>
__device__ __forceinline__ bool chol_d(const double* A, double* L) {
    bool ok = true;
#pragma unroll
    for (int e = 0; e < D * D; ++e) L[e] = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        double dd = A[j * D + j];
#pragma unroll
        for (int k = 0; k < j; ++k) dd = fma(-L[j * D + k], L[j * D + k], dd);
        ok = ok && dd > 0.0 && dd < INFINITY;
        const double l = sqrt(ok ? dd : 1.0);
        L[j * D + j] = l;
        const double il = 1.0 / l;
#pragma unroll
        for (int i = j + 1; i < D; ++i) {
            double s = A[i * D + j];
#pragma unroll
            for (int k = 0; k < j; ++k) s = fma(-L[i * D + k], L[j * D + k], s);
            L[i * D + j] = s * il;
        }
    }
    return ok;
}

// One factor: state s (index i within its plan), evaluated by the G lanes
// that share it.
template <typename R, int D, int P, int G, int KIND>
__device__ __forceinline__ void expect_factor(const DevState& st, const PlanDev& p, const Cost<R, D, KIND>& cost,
                                              int64_t s, int lane) {
    constexpr int NODES = ipow(P, D);
    constexpr int NS2 = D * (D + 1) / 2;
    constexpr int STEPS = (NODES + G - 1) / G;  // nodes per lane, rounded up
    const int64_t S = st.S;
    const int n = st.n;

    // marginal of the configuration coordinates (FP64) and its Cholesky factor
    double mu[D], Sg[D * D], L[D * D];
#pragma unroll
    for (int a = 0; a < D; ++a) mu[a] = st.mu[(int64_t)p.coll_index[a] * S + s];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int c = 0; c < D; ++c) Sg[a * D + c] = st.SD[(int64_t)(p.coll_index[a] * n + p.coll_index[c]) * S + s];
    const bool ok = chol_d<D>(Sg, L);

    R muR[D], LR[D * D];
#pragma unroll
    for (int a = 0; a < D; ++a) muR[a] = (R)mu[a];
#pragma unroll
    for (int e = 0; e < D * D; ++e) LR[e] = (R)L[e];
    const R centre = (sizeof(R) == 4) ? cost(muR) : R(0);

    const R* xi1 = Tab<R>::x(st) + P * kMaxGH;
    const R* w1 = Tab<R>::w(st) + P * kMaxGH;
    R s0 = R(0), s1[D], S2[NS2];
#pragma unroll
    for (int a = 0; a < D; ++a) s1[a] = R(0);
#pragma unroll
    for (int a = 0; a < NS2; ++a) S2[a] = R(0);
    // a fixed trip count lets the compiler overlap several nodes' SDF gathers
#pragma unroll 4
    for (int k = 0; k < STEPS; ++k) {
        const int j = lane + k * G;
        if (NODES % G != 0 && j >= NODES) break;
        R xi[D], x[D];
        R W = R(1);
        int r = j;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int q = r % P;
            r /= P;
            xi[a] = xi1[q];
            W *= w1[q];
        }
#pragma unroll
        for (int a = 0; a < D; ++a) {
            R v = muR[a];
#pragma unroll
            for (int c = 0; c <= a; ++c) v += LR[a * D + c] * xi[c];
            x[a] = v;
        }
        const R wp = W * (cost(x) - centre);
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
    // butterfly over the G lanes of this factor
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) {
        s0 += __shfl_xor(s0, o, G);
#pragma unroll
        for (int a = 0; a < D; ++a) s1[a] += __shfl_xor(s1[a], o, G);
#pragma unroll
        for (int a = 0; a < NS2; ++a) S2[a] += __shfl_xor(S2[a], o, G);
    }
    if (lane != 0) return;
    if (!ok) {
        st.Ecol[s] = NAN;
        for (int a = 0; a < D; ++a) st.gcol[a * S + s] = NAN;
        for (int a = 0; a < D * D; ++a) st.Hcol[a * S + s] = NAN;
        return;
    }
    // FP64 epilogue: Li = L^-1 (lower), g = Li^T s1, H = Li^T (S2 - s0 I) Li
    double Li[D * D];
#pragma unroll
    for (int e = 0; e < D * D; ++e) Li[e] = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double inv = 1.0 / L[a * D + a];
        Li[a * D + a] = inv;
#pragma unroll
        for (int c = 0; c < a; ++c) {
            double v = 0.0;
#pragma unroll
            for (int k = c; k < a; ++k) v = fma(L[a * D + k], Li[k * D + c], v);
            Li[a * D + c] = -v * inv;
        }
    }
    const double e0 = (double)s0;
    double M[D * D];
    {
        int t = 0;
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int c = a; c < D; ++c) {
                const double v = (double)S2[t++] - (a == c ? e0 : 0.0);
                M[a * D + c] = v;
                M[c * D + a] = v;
            }
    }
    st.Ecol[s] = e0 + (double)centre;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double v = 0.0;
#pragma unroll
        for (int k = a; k < D; ++k) v = fma(Li[k * D + a], (double)s1[k], v);
        st.gcol[a * S + s] = v;
    }
    // T = M Li, H = Li^T T
    double Tm[D * D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int c = 0; c < D; ++c) {
            double v = 0.0;
#pragma unroll
            for (int k = c; k < D; ++k) v = fma(M[a * D + k], Li[k * D + c], v);
            Tm[a * D + c] = v;
        }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int c = a; c < D; ++c) {
            double v = 0.0;
#pragma unroll
            for (int k = a; k < D; ++k) v = fma(Li[k * D + a], Tm[k * D + c], v);
            st.Hcol[(a * D + c) * S + s] = v;
            st.Hcol[(c * D + a) * S + s] = v;
        }
}

// Grid: per XCD, `slots` plan slots of `tiles` blocks each.  Block b runs on
// XCD b mod 8 and serves plan plan_lo + 8*slot + (b mod 8), so the plan and
// its fields are wave-uniform (scalar loads) and each XCD's L2 caches the
// maps of its own plans only.  A block strides over its plan's states in
// steps of `tiles` tiles, so any plan length is covered whatever the grid.
template <typename R, int D, int P, int G, int KIND>
__global__ void __launch_bounds__(kExpectThreads) expect_kernel(DevState st, int plan_lo, int plan_hi, int tiles,
                                                                int respect_budget) {
    constexpr int FPB = kExpectThreads / G;  // factors per block
    const int b = blockIdx.x;
    const int k = b / kNumXcd;
    const int pid = plan_lo + (k / tiles) * kNumXcd + b % kNumXcd;
    if (pid >= plan_hi) return;
    const PlanDev& p = st.plans[pid];
    if (!p.active || p.coll_kind != KIND || p.gh_points != P) return;
    if (respect_budget && p.iters_left <= 0) return;
    const int lane = threadIdx.x % G;
    const int N = p.N;
    const int lo = p.coll_states == 1 ? 1 : 0;
    const int hi = p.coll_states == 1 ? N - 1 : N;
    Cost<R, D, KIND> cost;
    cost.init(p);
    for (int i0 = (k % tiles) * FPB; i0 < N; i0 += tiles * FPB) {
        const int i = i0 + (int)threadIdx.x / G;
        if (i < lo || i >= hi) continue;  // all G lanes of a factor agree
        expect_factor<R, D, P, G, KIND>(st, p, cost, p.off + i, lane);
    }
}

template <typename R, int D, int P, int G, int KIND>
static hipError_t launch_one(const DevState& st, int plo, int phi, int maxN, int respect, hipStream_t s) {
    constexpr int FPB = kExpectThreads / G;
    const int tiles = std::max(1, (maxN + FPB - 1) / FPB);
    const int64_t slots = (phi - plo + kNumXcd - 1) / kNumXcd;
    const int64_t blocks = slots * tiles * kNumXcd;
    if (blocks <= 0) return hipSuccess;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((expect_kernel<R, D, P, G, KIND>), dim3((unsigned)blocks), dim3(kExpectThreads), 0, s, st,
                       plo, phi, tiles, respect);
    return hipGetLastError();
}

// Instantiated shapes: (kind, d, p) x lanes per factor (1, 2 and 4 lanes
// for the point robots only).
#define PG_LANES_SMALL(R, D, P, KIND)                                            \
    switch (lanes) {                                                             \
        case 1: return launch_one<R, D, P, 1, KIND>(st, plo, phi, maxN, respect, s);     \
        case 2: return launch_one<R, D, P, 2, KIND>(st, plo, phi, maxN, respect, s);     \
        case 4: return launch_one<R, D, P, 4, KIND>(st, plo, phi, maxN, respect, s);     \
        default: break;                                                          \
    }                                                                            \
    PG_LANES(R, D, P, KIND)
#define PG_LANES(R, D, P, KIND)                                                  \
    switch (lanes) {                                                             \
        case 8: return launch_one<R, D, P, 8, KIND>(st, plo, phi, maxN, respect, s);     \
        case 16: return launch_one<R, D, P, 16, KIND>(st, plo, phi, maxN, respect, s);   \
        case 32: return launch_one<R, D, P, 32, KIND>(st, plo, phi, maxN, respect, s);   \
        case 64: return launch_one<R, D, P, 64, KIND>(st, plo, phi, maxN, respect, s);   \
        default: return hipErrorInvalidValue;                                    \
    }

template <typename R>
static hipError_t dispatch(const DevState& st, int kind, int d, int p, int lanes, int plo, int phi, int maxN,
                           int respect, hipStream_t s) {
    if (kind == PGVIMP_COLL_POINT2D && d == 2) {
        switch (p) {
            case 1: PG_LANES_SMALL(R, 2, 1, PGVIMP_COLL_POINT2D);
            case 2: PG_LANES_SMALL(R, 2, 2, PGVIMP_COLL_POINT2D);
            case 3: PG_LANES_SMALL(R, 2, 3, PGVIMP_COLL_POINT2D);
            case 4: PG_LANES_SMALL(R, 2, 4, PGVIMP_COLL_POINT2D);
            case 5: PG_LANES_SMALL(R, 2, 5, PGVIMP_COLL_POINT2D);
            case 6: PG_LANES_SMALL(R, 2, 6, PGVIMP_COLL_POINT2D);
            case 7: PG_LANES_SMALL(R, 2, 7, PGVIMP_COLL_POINT2D);
            case 8: PG_LANES_SMALL(R, 2, 8, PGVIMP_COLL_POINT2D);
            case 10: PG_LANES_SMALL(R, 2, 10, PGVIMP_COLL_POINT2D);
            default: return hipErrorInvalidValue;
        }
    }
    if (kind == PGVIMP_COLL_POINT3D && d == 3) {
        switch (p) {
            case 2: PG_LANES_SMALL(R, 3, 2, PGVIMP_COLL_POINT3D);
            case 3: PG_LANES_SMALL(R, 3, 3, PGVIMP_COLL_POINT3D);
            case 4: PG_LANES_SMALL(R, 3, 4, PGVIMP_COLL_POINT3D);
            case 5: PG_LANES_SMALL(R, 3, 5, PGVIMP_COLL_POINT3D);
            default: return hipErrorInvalidValue;
        }
    }
    if (kind == PGVIMP_COLL_ARM3D && d == PGVIMP_ARM_DOF) {
        switch (p) {
            case 2: PG_LANES(R, 7, 2, PGVIMP_COLL_ARM3D);
            case 3: PG_LANES(R, 7, 3, PGVIMP_COLL_ARM3D);
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}
#undef PG_LANES
#undef PG_LANES_SMALL

bool expect_supported(int kind, int d, int p, int lanes) {
    const bool small = lanes == 1 || lanes == 2 || lanes == 4;
    if (!small && lanes != 8 && lanes != 16 && lanes != 32 && lanes != 64) return false;
    if (small && kind == PGVIMP_COLL_ARM3D) return false;
    if (kind == PGVIMP_COLL_POINT2D) return d == 2 && p >= 1 && p <= 10 && p != 9;
    if (kind == PGVIMP_COLL_POINT3D) return d == 3 && p >= 2 && p <= 5;
    if (kind == PGVIMP_COLL_ARM3D) return d == PGVIMP_ARM_DOF && (p == 2 || p == 3);
    return kind == PGVIMP_COLL_NONE;
}

// Lanes per factor chosen so that the nodes fill the lanes with little
// idling; the autotuner's table overrides these through the engine config.
int default_lanes(int kind, int d, int p) {
    int nodes = 1;
    for (int k = 0; k < d; ++k) nodes *= p;
    if (kind == PGVIMP_COLL_ARM3D) return 64;
    if (nodes <= 8) return 8;
    if (nodes <= 16) return 16;
    if (nodes <= 32) return 32;
    return 64;
}

hipError_t launch_expect(const DevState& st, int kind, int d, int p, int precision, int lanes, int plo, int phi,
                         int maxN, int respect, hipStream_t s) {
    if (kind == PGVIMP_COLL_NONE) return hipSuccess;
    if (precision == PGVIMP_MIXED) return dispatch<float>(st, kind, d, p, lanes, plo, phi, maxN, respect, s);
    return dispatch<double>(st, kind, d, p, lanes, plo, phi, maxN, respect, s);
}

}  // namespace pg
