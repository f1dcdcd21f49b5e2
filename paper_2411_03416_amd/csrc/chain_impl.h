// Chain kernels: marginal covariances of the block-tridiagonal precision
// (Gaussian belief propagation on the chain, Sec. 5.1), the block-
// tridiagonal mean solve of Theorem 1, and the fused step-size loop of
// Alg. 1 / App. C.  One workgroup of one wavefront serves one plan.
//
// Parallel form.  GBP on a chain is exact and equals the block-tridiagonal
// selected inverse (Sigma_ii, Sigma_{i,i+1}).  Instead of one sequential
// sweep of N dependent n x n steps, the chain is cut into nseg segments;
// the last state of each segment but the last is a separator.  Each lane
// eliminates the interior states of its segment (a forward sweep that
// carries the fill towards the segment's left separator), producing the
// Schur-complement contribution of the segment to its two separators.  The
// reduced chain of the m = nseg - 1 separators is then factored by block
// cyclic reduction across the lanes: lane j owns separator j, which is
// eliminated at level ctz(j + 1) with neighbours j -/+ 2^level, so the
// reduced chain takes floor(log2 m) + 1 levels forward and as many back.
// Each lane finally recovers its interior marginals by a backward sweep
// conditioned on the joint covariance of its two separators.  Depth:
// 2 N / nseg block steps plus about 2 log2(nseg) levels, instead of 2 N.
// log det Lambda is the sum of the log determinants of all pivots
// (interior Schur complements and reduced-chain pivots), and Lambda is
// positive definite iff every pivot is.
//
// The same elimination with a right-hand side solves
// (K^-1 + Lambda_k / beta) mu' = eta - g + Lambda_k mu_k / beta.
//
// Step-size selection.  Halving from beta_max accepts the first trial step
// that passes (Alg. 1, App. C), so the trials are independent of each
// other: one iteration evaluates a window of W consecutive trial step sizes
// at once, one workgroup per (plan, trial), and a select kernel takes the
// first passing trial of the window in order.  Plans still pending after a
// window continue with the next W step sizes.  The chosen step and every
// result are the same as trying the step sizes one after another.
#pragma once
#include "blockmath.h"
#include "ctx.h"

namespace pg {

// Entry offsets in the per-segment scratch (stride DevState::seg_stride).
// Slot j holds segment j's contributions to its separators and, for the
// reduced chain, the data of separator j (node j).
template <int n>
struct SegLayout {
    static constexpr int DL = 0;              // Schur contribution to left separator
    static constexpr int DR = n * n;          // ... to right separator
    static constexpr int CLR = 2 * n * n;     // coupling block (left sep, right sep)
    // node j; NGL/NGR reuse DL/DR, which are consumed when the nodes are assembled
    static constexpr int NGL = 0;             // pivot^-1 M(j, left neighbour)
    static constexpr int NGR = n * n;         // pivot^-1 M(j, right neighbour)
    static constexpr int NA = 3 * n * n;      // current diagonal block; Sigma_jj after the backward pass
    static constexpr int NC = 4 * n * n;      // coupling M(j, right neighbour at the current level)
    static constexpr int NP = 5 * n * n;      // pivot inverse at elimination
    static constexpr int NX = 6 * n * n;      // Cov(j, right neighbour at j's level); Cov(j, j+1) at the end
    static constexpr int RL = 7 * n * n;      // rhs contribution to left separator
    static constexpr int RR = 7 * n * n + n;  // ... to right separator
    static constexpr int NR = 7 * n * n + 2 * n;  // current rhs of node j
    static constexpr int NZ = 7 * n * n + 3 * n;  // pivot^-1 rhs at elimination
    static constexpr int XS = 7 * n * n + 4 * n;  // solution at separator j
    static constexpr int STRIDE = 7 * n * n + 5 * n;
};

// Entry offsets in the per-state scratch (stride DevState::ws_stride).
template <int n>
struct WsLayout {
    static constexpr int PINV = 0;      // inverse of the interior pivot
    static constexpr int GU = n * n;    // pivot^-1 U_i
    static constexpr int HX = 2 * n * n;  // pivot^-1 X_i (fill towards left sep)
    static constexpr int YV = 3 * n * n;  // pivot^-1 y_i
    static constexpr int STRIDE = 3 * n * n + n;
};

// Blocks of the matrix being factored: D_i = a0 D0_i + a1 D1_i, U likewise
// (D1/U1 may be null), right-hand side r_i = a0 R0_i + a1 R1_i.  Inputs are
// SoA with stride S; the element for output index s is read at s + shift
// (outputs of trial slot t live t * S further on).
struct BlockSrc {
    const double* D0;
    const double* D1;
    const double* U0;
    const double* U1;
    const double* R0;
    const double* R1;
    double a0, a1;
    int64_t S, shift;
};

// Entry e of a matrix built as a0 X0 + a1 X1 (the same expression is used
// when the accepted trial precision is written back).
__device__ __forceinline__ double lin2(double a0, double x0, double a1, double x1) { return fma(a1, x1, a0 * x0); }

template <int n>
__device__ __forceinline__ void ld_soa(const double* __restrict__ X, int64_t S, int64_t s, double* M) {
PG_UNROLL
    for (int e = 0; e < n * n; ++e) M[e] = X[e * S + s];
}
template <int n>
__device__ __forceinline__ void st_soa(double* __restrict__ X, int64_t S, int64_t s, const double* M) {
PG_UNROLL
    for (int e = 0; e < n * n; ++e) X[e * S + s] = M[e];
}
template <int n>
__device__ __forceinline__ void st_soa_sym(double* __restrict__ X, int64_t S, int64_t s, const double* M) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j < n; ++j) X[(i * n + j) * S + s] = 0.5 * (M[i * n + j] + M[j * n + i]);
}
template <int n>
__device__ __forceinline__ void ld_vec(const double* __restrict__ X, int64_t S, int64_t s, double* v) {
PG_UNROLL
    for (int e = 0; e < n; ++e) v[e] = X[e * S + s];
}
template <int n>
__device__ __forceinline__ void st_vec(double* __restrict__ X, int64_t S, int64_t s, const double* v) {
PG_UNROLL
    for (int e = 0; e < n; ++e) X[e * S + s] = v[e];
}
template <int n>
__device__ __forceinline__ void ld_aos(const double* __restrict__ p, double* M, int cnt) {
    for (int e = 0; e < cnt; ++e) M[e] = p[e];
}

template <int n>
__device__ __forceinline__ void src_D(const BlockSrc& b, int64_t s, double* M) {
    s += b.shift;
PG_UNROLL
    for (int e = 0; e < n * n; ++e)
        M[e] = b.D1 ? lin2(b.a0, b.D0[e * b.S + s], b.a1, b.D1[e * b.S + s]) : b.a0 * b.D0[e * b.S + s];
}
template <int n>
__device__ __forceinline__ void src_U(const BlockSrc& b, int64_t s, double* M) {
    s += b.shift;
PG_UNROLL
    for (int e = 0; e < n * n; ++e)
        M[e] = b.U1 ? lin2(b.a0, b.U0[e * b.S + s], b.a1, b.U1[e * b.S + s]) : b.a0 * b.U0[e * b.S + s];
}
template <int n>
__device__ __forceinline__ void src_r(const BlockSrc& b, int64_t s, double* v) {
    s += b.shift;
PG_UNROLL
    for (int e = 0; e < n; ++e)
        v[e] = b.R1 ? lin2(b.a0, b.R0[e * b.S + s], b.a1, b.R1[e * b.S + s]) : b.a0 * b.R0[e * b.S + s];
}

__device__ __forceinline__ void seg_bounds(int N, int nseg, int j, int& a, int& b, bool& hasL, bool& hasR) {
    const int st = (int)(((int64_t)j * N) / nseg);
    const int en = (int)(((int64_t)(j + 1) * N) / nseg);
    hasL = j > 0;
    hasR = j < nseg - 1;
    a = st;
    b = hasR ? en - 2 : en - 1;
}
__device__ __forceinline__ int sep_state(int N, int nseg, int j) {
    return (int)(((int64_t)(j + 1) * N) / nseg) - 1;
}

// Forward elimination of the interior states of segment j.
template <int n, bool RHS>
__device__ __forceinline__ bool seg_forward(const BlockSrc& M, int64_t off, int N, int nseg, int j, double* ws, int wsst,
                            double* sg, double* logdet, TS ts) {
    using W = WsLayout<n>;
    using G = SegLayout<n>;
    int a, b;
    bool hasL, hasR;
    seg_bounds(N, nseg, j, a, b, hasL, hasR);
    PG_MAT(P, ts);
    PG_MAT(X, ts);
    PG_MAT(Z, ts);
    PG_MAT(U, ts);   // U_i of the current step
    PG_MAT(Dn, ts);  // D_{i+1} and U_{i+1}, loaded one step ahead so the
    PG_MAT(Un, ts);  // loads overlap the current step's arithmetic
    PG_MAT(Pinv, ts);
    PG_MAT(GU, ts);
    PG_MAT(HX, ts);
    PG_VEC(y, ts); PG_VEC(yv, ts); PG_VEC(rL, ts); PG_VEC(rn, ts);
    src_D<n>(M, off + a, P);
    if (hasL) {
        src_U<n>(M, off + a - 1, Un);
PG_UNROLL
        for (int r = 0; r < n; ++r)
PG_UNROLL
            for (int c = 0; c < n; ++c) X[r * n + c] = Un[c * n + r];
        mzero<n>(Z);
    }
    if (a < b || hasR) src_U<n>(M, off + a, U);
    if (RHS) {
        src_r<n>(M, off + a, y);
PG_UNROLL
        for (int e = 0; e < n; ++e) rL[e] = 0.0;
    }
    bool ok = true;
    for (int i = a; i <= b; ++i) {
        TS lt = ts;
        const bool hasNext = (i < b) || hasR;
        if (i < b) {
            src_D<n>(M, off + i + 1, Dn);
            if (i + 1 < b || hasR) src_U<n>(M, off + i + 1, Un);
            if (RHS) src_r<n>(M, off + i + 1, rn);
        }
        ok = spd_inverse<n>(P, Pinv, RHS ? nullptr : logdet, lt) && ok;
        double* w = ws + (off + i) * (int64_t)wsst;
PG_UNROLL
        for (int e = 0; e < n * n; ++e) w[W::PINV + e] = Pinv[e];
        if (hasNext) {
            mmul<n>(Pinv, U, GU);
PG_UNROLL
            for (int e = 0; e < n * n; ++e) w[W::GU + e] = GU[e];
        }
        if (hasL) {
            mmul<n>(Pinv, X, HX);
PG_UNROLL
            for (int e = 0; e < n * n; ++e) w[W::HX + e] = HX[e];
            msub_tn<n>(X, HX, Z);
        }
        if (RHS) {
            mvec<n>(Pinv, y, yv);
PG_UNROLL
            for (int e = 0; e < n; ++e) w[W::YV + e] = yv[e];
            if (hasL) mvec_tn_sub<n>(X, yv, rL);
        }
        if (i < b) {
            mcopy<n>(Dn, P);
            msub_tn<n>(U, GU, P);
            if (hasL) {
                PG_MAT(T, lt);
                mmul_tn<n>(U, HX, T);
PG_UNROLL
                for (int e = 0; e < n * n; ++e) X[e] = -T[e];
            }
            if (RHS) {
PG_UNROLL
                for (int e = 0; e < n; ++e) y[e] = rn[e];
                mvec_tn_sub<n>(U, yv, y);
            }
            if (i + 1 < b || hasR) mcopy<n>(Un, U);
        } else {
            double* g = sg + (int64_t)j * G::STRIDE;
            if (hasR) {
                PG_MAT(T, lt);
                mmul_tn<n>(U, GU, T);
PG_UNROLL
                for (int e = 0; e < n * n; ++e) g[G::DR + e] = -T[e];
                if (RHS) {
                    PG_VEC(t, lt);
PG_UNROLL
                    for (int e = 0; e < n; ++e) t[e] = 0.0;
                    mvec_tn_sub<n>(U, yv, t);
PG_UNROLL
                    for (int e = 0; e < n; ++e) g[G::RR + e] = t[e];
                }
            }
            if (hasL) {
PG_UNROLL
                for (int e = 0; e < n * n; ++e) g[G::DL + e] = Z[e];
                if (RHS) {
PG_UNROLL
                    for (int e = 0; e < n; ++e) g[G::RL + e] = rL[e];
                }
            }
            if (hasL && hasR) {
                PG_MAT(T, lt);
                mmul_tn<n>(X, GU, T);
PG_UNROLL
                for (int e = 0; e < n * n; ++e) g[G::CLR + e] = -T[e];
            }
        }
    }
    return ok;
}

// Reduced chain of the m = nseg - 1 separators by block cyclic reduction.
// Lane j < m owns separator j; it is eliminated at level lv(j) = ctz(j + 1),
// where its neighbours are j - 2^lv and j + 2^lv (when inside [0, m)).
// Every lane of the calling half must call these (they contain workgroup
// barriers; the count depends on m only).
__device__ __forceinline__ int cr_levels(int m) { return m > 0 ? 32 - __clz(m) : 0; }

template <int n>
__device__ __forceinline__ void ld_blk(const double* p, double* M) {
PG_UNROLL
    for (int e = 0; e < n * n; ++e) M[e] = p[e];
}
template <int n>
__device__ __forceinline__ void st_blk(double* p, const double* M) {
PG_UNROLL
    for (int e = 0; e < n * n; ++e) p[e] = M[e];
}

// Node j's diagonal block, right coupling and rhs from its separator state
// and the two adjacent segments.
template <int n, bool RHS>
__device__ __forceinline__ void cr_assemble(const BlockSrc& M, int64_t off, int N, int nseg, int j, double* sg, TS ts) {
    using G = SegLayout<n>;
    const int m = nseg - 1;
    const int s = sep_state(N, nseg, j);
    double* gj = sg + (int64_t)j * G::STRIDE;
    const double* gn = sg + (int64_t)(j + 1) * G::STRIDE;
    PG_MAT(A, ts);
    src_D<n>(M, off + s, A);
PG_UNROLL
    for (int e = 0; e < n * n; ++e) A[e] += gj[G::DR + e] + gn[G::DL + e];
    st_blk<n>(gj + G::NA, A);
    if (j + 1 < m) {
PG_UNROLL
        for (int e = 0; e < n * n; ++e) gj[G::NC + e] = gn[G::CLR + e];
    }
    if (RHS) {
        PG_VEC(r, ts);
        src_r<n>(M, off + s, r);
PG_UNROLL
        for (int e = 0; e < n; ++e) gj[G::NR + e] = r[e] + gj[G::RR + e] + gn[G::RL + e];
    }
}

// Forward elimination.  Level l: the nodes eliminated at l store their pivot
// inverse P, G_L = P M(k, L), G_R = P M(k, R) and z = P r (barrier); the
// surviving nodes then take the Schur updates of their eliminated
// neighbours and their new right coupling -M(j, k) P M(k, R) (barrier).
template <int n, bool RHS>
__device__ __forceinline__ bool cr_forward(int m, int j, double* sg, double* logdet, TS ts) {
    using G = SegLayout<n>;
    const int levels = cr_levels(m);
    const bool own = j < m;
    const int lv = own ? __builtin_ctz(j + 1) : -1;
    double* gj = sg + (int64_t)(own ? j : 0) * G::STRIDE;
    bool ok = true;
    for (int l = 0; l < levels; ++l) {
        const int h = 1 << l;
        if (own && lv == l) {
            TS lt = ts;
            PG_MAT(A, lt);
            PG_MAT(P, lt);
            PG_MAT(C, lt);
            PG_MAT(T, lt);
            ld_blk<n>(gj + G::NA, A);
            ok = spd_inverse<n>(A, P, RHS ? nullptr : logdet, lt) && ok;
            st_blk<n>(gj + G::NP, P);
            if (j - h >= 0) {
                ld_blk<n>(sg + (int64_t)(j - h) * G::STRIDE + G::NC, C);  // M(L, k)
                mmul_nt<n>(P, C, T);
                st_blk<n>(gj + G::NGL, T);
            }
            if (j + h < m) {
                ld_blk<n>(gj + G::NC, C);  // M(k, R)
                mmul<n>(P, C, T);
                st_blk<n>(gj + G::NGR, T);
            }
            if (RHS) {
                PG_VEC(r, lt);
                PG_VEC(z, lt);
PG_UNROLL
                for (int e = 0; e < n; ++e) r[e] = gj[G::NR + e];
                mvec<n>(P, r, z);
PG_UNROLL
                for (int e = 0; e < n; ++e) gj[G::NZ + e] = z[e];
            }
        }
        __syncthreads();
        if (own && lv > l && ((j + 1) & (h - 1)) == 0) {
            TS lt = ts;
            PG_MAT(A, lt);
            PG_MAT(C, lt);
            PG_MAT(Gk, lt);
            PG_VEC(r, lt);
            PG_VEC(z, lt);
            ld_blk<n>(gj + G::NA, A);
            if (RHS) {
PG_UNROLL
                for (int e = 0; e < n; ++e) r[e] = gj[G::NR + e];
            }
            if (j + h < m) {
                // right neighbour k = j + h: A -= M(j,k) G_L(k), r -= M(j,k) z_k,
                // new coupling to k + h: -M(j,k) G_R(k)
                const double* gk = sg + (int64_t)(j + h) * G::STRIDE;
                ld_blk<n>(gj + G::NC, C);
                ld_blk<n>(gk + G::NGL, Gk);
                msub<n>(C, Gk, A);
                if (RHS) {
PG_UNROLL
                    for (int e = 0; e < n; ++e) z[e] = gk[G::NZ + e];
                    mvec_sub<n>(C, z, r);
                }
                if (j + 2 * h < m) {
                    PG_MAT(T, lt);
                    ld_blk<n>(gk + G::NGR, Gk);
                    mmul<n>(C, Gk, T);
PG_UNROLL
                    for (int e = 0; e < n * n; ++e) gj[G::NC + e] = -T[e];
                }
            }
            if (j - h >= 0) {
                // left neighbour k = j - h: A -= M(k,j)^T G_R(k), r -= M(k,j)^T z_k
                const double* gk = sg + (int64_t)(j - h) * G::STRIDE;
                ld_blk<n>(gk + G::NC, C);
                ld_blk<n>(gk + G::NGR, Gk);
                msub_tn<n>(C, Gk, A);
                if (RHS) {
PG_UNROLL
                    for (int e = 0; e < n; ++e) z[e] = gk[G::NZ + e];
                    mvec_tn_sub<n>(C, z, r);
                }
            }
            st_blk<n>(gj + G::NA, A);
            if (RHS) {
PG_UNROLL
                for (int e = 0; e < n; ++e) gj[G::NR + e] = r[e];
            }
        }
        __syncthreads();
    }
    return ok;
}

// Backward selected inversion, top level first: node k eliminated at level l
// with neighbours L, R (whose covariances are known from higher levels):
//   Cov(k, L) = -(G_L S_LL + G_R S_RL),  Cov(k, R) = -(G_L S_LR + G_R S_RR),
//   S_kk = P - Cov(k, L) G_L^T - Cov(k, R) G_R^T.
// Writes S_kk (node and SDo) and the cross-covariances of the two new
// adjacent pairs (L, k) and (k, R).  run = false keeps the barriers only.
template <int n>
__device__ __forceinline__ void cr_backward_cov(int m, int j, bool run, int64_t off, int N, int nseg, double* sg,
                                                double* SDo, int64_t S, TS ts) {
    using G = SegLayout<n>;
    const int levels = cr_levels(m);
    const bool own = run && j < m;
    const int lv = own ? __builtin_ctz(j + 1) : -1;
    double* gj = sg + (int64_t)(own ? j : 0) * G::STRIDE;
    for (int l = levels - 1; l >= 0; --l) {
        const int h = 1 << l;
        if (own && lv == l) {
            TS lt = ts;
            const bool hasL = j - h >= 0, hasR = j + h < m;
            double* gl = sg + (int64_t)(hasL ? j - h : j) * G::STRIDE;
            const double* gr = sg + (int64_t)(hasR ? j + h : j) * G::STRIDE;
            PG_MAT(Sk, lt);
            PG_MAT(GL, lt);
            PG_MAT(GR, lt);
            PG_MAT(CL, lt);
            PG_MAT(CR, lt);
            PG_MAT(X, lt);
            PG_MAT(T, lt);
            ld_blk<n>(gj + G::NP, Sk);
            if (hasL) ld_blk<n>(gj + G::NGL, GL);
            if (hasR) ld_blk<n>(gj + G::NGR, GR);
            if (hasL && hasR) ld_blk<n>(gl + G::NX, X);  // Cov(L, R)
            if (hasL) {
                ld_blk<n>(gl + G::NA, T);  // S_LL
                mmul<n>(GL, T, CL);
                if (hasR) {
                    // + G_R S_RL, S_RL = X^T
                    PG_MAT(U, lt);
                    mmul_nt<n>(GR, X, U);
PG_UNROLL
                    for (int e = 0; e < n * n; ++e) CL[e] += U[e];
                }
PG_UNROLL
                for (int e = 0; e < n * n; ++e) CL[e] = -CL[e];
                msub_nt<n>(CL, GL, Sk);
            }
            if (hasR) {
                ld_blk<n>(gr + G::NA, T);  // S_RR
                mmul<n>(GR, T, CR);
                if (hasL) {
                    PG_MAT(U, lt);
                    mmul<n>(GL, X, U);
PG_UNROLL
                    for (int e = 0; e < n * n; ++e) CR[e] += U[e];
                }
PG_UNROLL
                for (int e = 0; e < n * n; ++e) CR[e] = -CR[e];
                msub_nt<n>(CR, GR, Sk);
            }
            st_blk<n>(gj + G::NA, Sk);
            st_soa_sym<n>(SDo, S, off + sep_state(N, nseg, j), Sk);
            if (hasL) {
PG_UNROLL
                for (int r = 0; r < n; ++r)
PG_UNROLL
                    for (int c = 0; c < n; ++c) gl[G::NX + r * n + c] = CL[c * n + r];  // Cov(L, k)
            }
            if (hasR) st_blk<n>(gj + G::NX, CR);  // Cov(k, R)
        }
        __syncthreads();
    }
}

// Backward substitution: x_k = z_k - G_L x_L - G_R x_R, top level first.
template <int n>
__device__ __forceinline__ void cr_backward_rhs(int m, int j, bool run, int64_t off, int N, int nseg, double* sg,
                                                double* xo, int64_t S, TS ts) {
    using G = SegLayout<n>;
    const int levels = cr_levels(m);
    const bool own = run && j < m;
    const int lv = own ? __builtin_ctz(j + 1) : -1;
    double* gj = sg + (int64_t)(own ? j : 0) * G::STRIDE;
    for (int l = levels - 1; l >= 0; --l) {
        const int h = 1 << l;
        if (own && lv == l) {
            TS lt = ts;
            PG_VEC(x, lt);
            PG_VEC(y, lt);
            PG_MAT(Gk, lt);
PG_UNROLL
            for (int e = 0; e < n; ++e) x[e] = gj[G::NZ + e];
            if (j - h >= 0) {
                const double* gl = sg + (int64_t)(j - h) * G::STRIDE;
                ld_blk<n>(gj + G::NGL, Gk);
PG_UNROLL
                for (int e = 0; e < n; ++e) y[e] = gl[G::XS + e];
                mvec_sub<n>(Gk, y, x);
            }
            if (j + h < m) {
                const double* gr = sg + (int64_t)(j + h) * G::STRIDE;
                ld_blk<n>(gj + G::NGR, Gk);
PG_UNROLL
                for (int e = 0; e < n; ++e) y[e] = gr[G::XS + e];
                mvec_sub<n>(Gk, y, x);
            }
PG_UNROLL
            for (int e = 0; e < n; ++e) gj[G::XS + e] = x[e];
            st_vec<n>(xo, S, off + sep_state(N, nseg, j), x);
        }
        __syncthreads();
    }
}

// Backward recovery of segment j's interior marginals.
template <int n>
__device__ __forceinline__ void seg_backward_cov(int64_t off, int N, int nseg, int j, const double* ws, int wsst,
                                 const double* sg, double* SDo, double* SUo, int64_t S, TS ts) {
    using W = WsLayout<n>;
    using G = SegLayout<n>;
    int a, b;
    bool hasL, hasR;
    seg_bounds(N, nseg, j, a, b, hasL, hasR);
    PG_MAT(SLL, ts);
    PG_MAT(Snn, ts);
    PG_MAT(SnL, ts);
    if (hasL) ld_soa<n>(SDo, S, off + a - 1, SLL);
    if (hasR) {
        ld_soa<n>(SDo, S, off + b + 1, Snn);
        if (hasL) {
            const double* cr = sg + (int64_t)(j - 1) * G::STRIDE + G::NX;  // Cov(L, R)
PG_UNROLL
            for (int r = 0; r < n; ++r)
PG_UNROLL
                for (int c = 0; c < n; ++c) SnL[r * n + c] = cr[c * n + r];
        }
    }
    // blocks of the forward sweep for the current state (c) and, loaded one
    // step ahead, for the next state down the segment (n)
    PG_MAT(Pc, ts);
    PG_MAT(Gc, ts);
    PG_MAT(Hc, ts);
    PG_MAT(Pn, ts);
    PG_MAT(Gn, ts);
    PG_MAT(Hn, ts);
    {
        const double* w = ws + (off + b) * (int64_t)wsst;
PG_UNROLL
        for (int e = 0; e < n * n; ++e) Pc[e] = w[W::PINV + e];
        if (hasR) {
PG_UNROLL
            for (int e = 0; e < n * n; ++e) Gc[e] = w[W::GU + e];
        }
        if (hasL) {
PG_UNROLL
            for (int e = 0; e < n * n; ++e) Hc[e] = w[W::HX + e];
        }
    }
    for (int i = b; i >= a; --i) {
        TS lt = ts;
        const bool hasNext = (i < b) || hasR;
        if (i > a) {
            const double* w = ws + (off + i - 1) * (int64_t)wsst;
PG_UNROLL
            for (int e = 0; e < n * n; ++e) Pn[e] = w[W::PINV + e];
PG_UNROLL
            for (int e = 0; e < n * n; ++e) Gn[e] = w[W::GU + e];
            if (hasL) {
PG_UNROLL
                for (int e = 0; e < n * n; ++e) Hn[e] = w[W::HX + e];
            }
        }
        // Pc becomes Sigma_ii in place
        PG_MAT(SiL, lt);
        PG_MAT(Sin, lt);
        PG_MAT(T, lt);
        if (hasNext) {
            // Cov(i, next) = -GU Snn - HX SnL^T
            mmul<n>(Gc, Snn, Sin);
            if (hasL) {
                mmul_nt<n>(Hc, SnL, T);
PG_UNROLL
                for (int e = 0; e < n * n; ++e) Sin[e] += T[e];
                // Cov(i, L) = -GU SnL - HX SLL
                mmul<n>(Gc, SnL, SiL);
                mmul<n>(Hc, SLL, T);
PG_UNROLL
                for (int e = 0; e < n * n; ++e) SiL[e] = -(SiL[e] + T[e]);
                // Sigma_ii = Pinv + G Sin^T + Hh SiL^T with G = -GU, Hh = -HX
                mmul_nt<n>(Hc, SiL, T);
PG_UNROLL
                for (int e = 0; e < n * n; ++e) Pc[e] -= T[e];
            }
PG_UNROLL
            for (int e = 0; e < n * n; ++e) Sin[e] = -Sin[e];
            mmul_nt<n>(Gc, Sin, T);
PG_UNROLL
            for (int e = 0; e < n * n; ++e) Pc[e] -= T[e];
            st_soa<n>(SUo, S, off + i, Sin);
        } else if (hasL) {
            mmul<n>(Hc, SLL, SiL);
PG_UNROLL
            for (int e = 0; e < n * n; ++e) SiL[e] = -SiL[e];
            mmul_nt<n>(Hc, SiL, T);
PG_UNROLL
            for (int e = 0; e < n * n; ++e) Pc[e] -= T[e];
        }
        st_soa_sym<n>(SDo, S, off + i, Pc);
        mcopy<n>(Pc, Snn);
        if (hasL) mcopy<n>(SiL, SnL);
        if (i > a) {
            mcopy<n>(Pn, Pc);
            mcopy<n>(Gn, Gc);
            if (hasL) mcopy<n>(Hn, Hc);
        }
    }
    if (hasL) {
        // Cov(L, a) = Cov(a, L)^T
        PG_MAT(T, ts);
PG_UNROLL
        for (int r = 0; r < n; ++r)
PG_UNROLL
            for (int c = 0; c < n; ++c) T[r * n + c] = SnL[c * n + r];
        st_soa<n>(SUo, S, off + a - 1, T);
    }
}

template <int n>
__device__ __forceinline__ void seg_backward_rhs(int64_t off, int N, int nseg, int j, const double* ws, int wsst,
                                 const double* sg, double* xo, int64_t S, TS ts) {
    using W = WsLayout<n>;
    using G = SegLayout<n>;
    int a, b;
    bool hasL, hasR;
    seg_bounds(N, nseg, j, a, b, hasL, hasR);
    PG_VEC(xL, ts); PG_VEC(xn, ts);
    if (hasL) {
        const double* p = sg + (int64_t)(j - 1) * G::STRIDE + G::XS;
PG_UNROLL
        for (int e = 0; e < n; ++e) xL[e] = p[e];
    }
    if (hasR) {
        const double* p = sg + (int64_t)j * G::STRIDE + G::XS;
PG_UNROLL
        for (int e = 0; e < n; ++e) xn[e] = p[e];
    }
    for (int i = b; i >= a; --i) {
        TS lt = ts;
        const double* w = ws + (off + i) * (int64_t)wsst;
        const bool hasNext = (i < b) || hasR;
        PG_VEC(x, lt);
        PG_VEC(t, lt);
PG_UNROLL
        for (int e = 0; e < n; ++e) x[e] = w[W::YV + e];
        if (hasNext) {
            PG_MAT(GUi, lt);
PG_UNROLL
            for (int e = 0; e < n * n; ++e) GUi[e] = w[W::GU + e];
            mvec<n>(GUi, xn, t);
PG_UNROLL
            for (int e = 0; e < n; ++e) x[e] -= t[e];
        }
        if (hasL) {
            PG_MAT(HXi, lt);
PG_UNROLL
            for (int e = 0; e < n * n; ++e) HXi[e] = w[W::HX + e];
            mvec<n>(HXi, xL, t);
PG_UNROLL
            for (int e = 0; e < n; ++e) x[e] -= t[e];
        }
        st_vec<n>(xo, S, off + i, x);
PG_UNROLL
        for (int e = 0; e < n; ++e) xn[e] = x[e];
    }
}

// Workgroup-wide GBP: marginals of (D, U) from src into (SDo, SUo).  Called
// by every lane of the half (tid = lane); sh_ld / sh_ok hold
// kChainThreads + 1 entries.
template <int n>
__device__ __forceinline__ bool wg_gbp(const BlockSrc& M, const DevState& st, double* ws, int tid, int64_t off,
                                       int64_t So, int N, int nseg, double* sg, double* SDo, double* SUo,
                                       double* logdet_out, double* sh_ld, int* sh_ok, TS ts) {
    const int m = nseg - 1;
    double ld = 0.0;
    bool ok = true;
    if (tid < nseg) ok = seg_forward<n, false>(M, off, N, nseg, tid, ws, st.ws_stride, sg, &ld, ts);
    __syncthreads();
    if (tid < m) cr_assemble<n, false>(M, off, N, nseg, tid, sg, ts);
    __syncthreads();
    ok = cr_forward<n, false>(m, tid, sg, &ld, ts) && ok;
    sh_ld[tid] = ld;
    sh_ok[tid] = ok ? 1 : 0;
    __syncthreads();
    if (tid == 0) {
        double tot = 0.0;
        int all = 1;
        for (int t = 0; t < kChainThreads; ++t) {
            tot += sh_ld[t];
            all &= sh_ok[t];
        }
        sh_ld[kChainThreads] = tot;
        sh_ok[kChainThreads] = all;
    }
    __syncthreads();
    const bool okall = sh_ok[kChainThreads] != 0;
    *logdet_out = sh_ld[kChainThreads];
    cr_backward_cov<n>(m, tid, okall, off, N, nseg, sg, SDo, So, ts);
    if (okall && tid < nseg) seg_backward_cov<n>(off, N, nseg, tid, ws, st.ws_stride, sg, SDo, SUo, So, ts);
    __syncthreads();
    return okall;
}

// Workgroup-wide solve of (D, U) x = r into xo (same barriers as wg_gbp).
template <int n>
__device__ __forceinline__ bool wg_solve(const BlockSrc& M, const DevState& st, double* ws, int tid, int64_t off,
                                         int64_t So, int N, int nseg, double* sg, double* xo, int* sh_ok, TS ts) {
    const int m = nseg - 1;
    double ld = 0.0;
    bool ok = true;
    if (tid < nseg) ok = seg_forward<n, true>(M, off, N, nseg, tid, ws, st.ws_stride, sg, &ld, ts);
    __syncthreads();
    if (tid < m) cr_assemble<n, true>(M, off, N, nseg, tid, sg, ts);
    __syncthreads();
    ok = cr_forward<n, true>(m, tid, sg, &ld, ts) && ok;
    sh_ok[tid] = ok ? 1 : 0;
    __syncthreads();
    if (tid == 0) {
        int all = 1;
        for (int t = 0; t < kChainThreads; ++t) all &= sh_ok[t];
        sh_ok[kChainThreads] = all;
    }
    __syncthreads();
    const bool okall = sh_ok[kChainThreads] != 0;
    cr_backward_rhs<n>(m, tid, okall, off, N, nseg, sg, xo, So, ts);
    if (okall && tid < nseg) seg_backward_rhs<n>(off, N, nseg, tid, ws, st.ws_stride, sg, xo, So, ts);
    __syncthreads();
    return okall;
}

// Collision contributions of state i embedded into the n-dim state.
template <int n>
__device__ __forceinline__ bool coll_active(const PlanDev& p, int i) {
    if (p.coll_kind == PGVIMP_COLL_NONE) return false;
    if (p.coll_states == 1 && (i == 0 || i == p.N - 1)) return false;
    return true;
}

// Closed-form expected prior-factor costs touching state i: the transition
// starting at i (i < N-1), plus the start factor (i = 0) and the goal
// factor (i = N-1).  Each is 1/2 (tr(W Cov r) + rbar^T W rbar).
template <int n>
__device__ __forceinline__ double prior_cost_state(const DevState& st, const PlanDev& p, int i, double* trans_out,
                                   double* start_out, double* goal_out, TS ts) {
    const int64_t S = st.S;
    const int64_t s = p.off + i;
    double tot = 0.0;
    PG_MAT(Si, ts);
    PG_VEC(mi, ts);
    ld_soa<n>(st.SD, S, s, Si);
    ld_vec<n>(st.mu, S, s, mi);
    if (i < p.N - 1) {
        PG_MAT(Phi, ts);
        PG_MAT(Wq, ts);
        PG_MAT(Sn, ts);
        PG_MAT(Sx, ts);
        PG_VEC(mn, ts); PG_VEC(ab, ts);
        ld_soa<n>(st.Phi, S, s, Phi);
        ld_soa<n>(st.Qinv, S, s, Wq);
        ld_soa<n>(st.SD, S, s + 1, Sn);
        ld_soa<n>(st.SU, S, s, Sx);
        ld_vec<n>(st.mu, S, s + 1, mn);
        ld_vec<n>(st.abar, S, s, ab);
        PG_VEC(rb, ts);
        mvec<n>(Phi, mi, rb);
PG_UNROLL
        for (int e = 0; e < n; ++e) rb[e] = mn[e] - rb[e] - ab[e];
        // C = Sn - Sx^T Phi^T - Phi Sx + Phi Si Phi^T
        PG_MAT(PS, ts);
        PG_MAT(C, ts);
        PG_MAT(T, ts);
        mmul<n>(Phi, Sx, PS);
        mmul<n>(Phi, Si, T);
        mmul_nt<n>(T, Phi, C);
PG_UNROLL
        for (int r = 0; r < n; ++r)
PG_UNROLL
            for (int c = 0; c < n; ++c) C[r * n + c] += Sn[r * n + c] - PS[r * n + c] - PS[c * n + r];
        double tr = 0.0, q = 0.0;
PG_UNROLL
        for (int r = 0; r < n; ++r) {
            double wr = 0.0;
PG_UNROLL
            for (int c = 0; c < n; ++c) {
                tr = fma(Wq[r * n + c], C[c * n + r], tr);
                wr = fma(Wq[r * n + c], rb[c], wr);
            }
            q = fma(rb[r], wr, q);
        }
        const double v = 0.5 * (tr + q);
        if (trans_out) *trans_out = v;
        tot += v;
    }
    for (int endf = 0; endf < 2; ++endf) {
        if ((endf == 0 && i != 0) || (endf == 1 && i != p.N - 1)) continue;
        const double* Wm = endf == 0 ? p.Wstart : p.Wgoal;
        const double* m0 = endf == 0 ? p.mu_start : p.mu_goal;
        TS et = ts;
        PG_VEC(r, et);
PG_UNROLL
        for (int e = 0; e < n; ++e) r[e] = mi[e] - m0[e];
        double tr = 0.0, q = 0.0;
        for (int a = 0; a < n; ++a) {
            double wr = 0.0;
            for (int c = 0; c < n; ++c) {
                tr = fma(Wm[a * n + c], Si[c * n + a], tr);
                wr = fma(Wm[a * n + c], r[c], wr);
            }
            q = fma(r[a], wr, q);
        }
        const double v = 0.5 * (tr + q);
        if (endf == 0 && start_out) *start_out = v;
        if (endf == 1 && goal_out) *goal_out = v;
        tot += v;
    }
    return tot;
}

// Sum over the workgroup in a fixed order (sh holds blockDim.x + 1 doubles).
__device__ __forceinline__ double wg_sum(double v, double* sh) {
    const int tid = threadIdx.x, nt = blockDim.x;
    sh[tid] = v;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int k = 0; k < nt; ++k) t += sh[k];
        sh[nt] = t;
    }
    __syncthreads();
    const double r = sh[nt];
    __syncthreads();
    return r;
}

// Scratch of (plan, trial slot, half): half 0 serves the marginals, half 1
// the mean solve of the same trial, which run side by side.
template <int n>
__device__ __forceinline__ double* seg_scratch(const DevState& st, int pid, int t, int half) {
    return st.seg + ((((int64_t)pid * st.W + t) * 2 + half) * kMaxSeg) * st.seg_stride;
}
template <int n>
__device__ __forceinline__ TS thread_ws(const DevState& st, int pid, int t) {
    return TS{st.tws + (((int64_t)pid * st.W + t) * kTrialThreads + threadIdx.x) * st.tws_stride};
}
__device__ __forceinline__ double* state_ws(const DevState& st, int half) {
    return st.ws + (int64_t)half * st.W * st.S * st.ws_stride;
}

// Set-up and marginals of a plan (trial slot 0 of its scratch):
// CHAIN_INIT: Lambda = K^-1, mean = solve(K^-1, eta), marginals, budget reset;
// CHAIN_REINIT: Lambda = K^-1 (mean kept), marginals;
// CHAIN_MARGINALS: marginals of the current Lambda.
template <int n>
__global__ void __launch_bounds__(kChainThreads) chain_kernel(DevState st, int mode, int plan_lo) {
    __shared__ double sh_d[kChainThreads + 1];
    __shared__ int sh_i[kChainThreads + 1];
    const int pid = plan_lo + blockIdx.x;
    PlanDev& p = st.plans[pid];
    if (!p.active) return;
    const int tid = threadIdx.x;
    const int N = p.N;
    const int64_t off = p.off;
    const int64_t S = st.S;
    const int nseg = p.nseg;
    double* sg = seg_scratch<n>(st, pid, 0, 0);
    double* ws = state_ws(st, 0);
    TS ts = thread_ws<n>(st, pid, 0);
    const int n2 = n * n;
    if (mode == CHAIN_INIT || mode == CHAIN_REINIT) {
        for (int i = tid; i < N; i += kChainThreads) {
            for (int e = 0; e < n2; ++e) {
                st.LD[e * S + off + i] = st.KD[e * S + off + i];
                st.LU[e * S + off + i] = st.KU[e * S + off + i];
            }
        }
        __syncthreads();
        if (mode == CHAIN_INIT) {
            BlockSrc M{st.KD, nullptr, st.KU, nullptr, st.eta, nullptr, 1.0, 0.0, S, 0};
            wg_solve<n>(M, st, ws, tid, off, S, N, nseg, sg, st.mu, sh_i, ts);
            if (tid == 0) {
                p.iters_left = p.n_iters;
                p.iters_done = 0;
                p.trials_total = 0;
            }
        }
    }
    BlockSrc M{st.LD, nullptr, st.LU, nullptr, nullptr, nullptr, 1.0, 0.0, S, 0};
    double ld = 0.0;
    const bool ok = wg_gbp<n>(M, st, ws, tid, off, S, N, nseg, sg, st.SD, st.SU, &ld, sh_d, sh_i, ts);
    if (tid == 0) {
        p.logdet = ok ? ld : NAN;
        p.status = ok ? 0 : PGVIMP_ENOTPD;
    }
}

// Sum over the block in a fixed order (sh holds blockDim.x + 1 doubles).
__device__ __forceinline__ double block_sum(double v, double* sh) { return wg_sum(v, sh); }

// One proximal iteration (Alg. 1), part 1: per-state quantities shared by all
// trial step sizes -- KH = K^-1 + H (collision Hessians on the diagonal
// blocks), rb = eta - g, Lmu = Lambda_k mu_k -- and the expected costs
// (per-block partial sums; the select kernel adds them in block order).
// Grid (plans, iter_blocks), kIterThreads threads, grid-stride over states.
template <int n>
__global__ void __launch_bounds__(kIterThreads) prep_kernel(DevState st) {
    __shared__ double sh_d[kIterThreads + 1];
    const int pid = blockIdx.x, y = blockIdx.y, nb = gridDim.y;
    PlanDev& p = st.plans[pid];
    if (!p.active) return;
    const int tid = threadIdx.x;
    if (p.iters_left <= 0) {
        if (y == 0 && tid == 0) p.phase = 1;
        return;
    }
    const int N = p.N, d = p.d;
    const int64_t off = p.off, S = st.S;
    const int n2 = n * n;
    TS ts = thread_ws<n>(st, pid, y);
    double ecol = 0.0, epri = 0.0;
    for (int i = y * kIterThreads + tid; i < N; i += nb * kIterThreads) {
        TS lt = ts;
        const int64_t s = off + i;
        const bool act = coll_active<n>(p, i);
        for (int e = 0; e < n2; ++e) st.KH[e * S + s] = st.KD[e * S + s];
        PG_VEC(r, lt);
        ld_vec<n>(st.eta, S, s, r);
        if (act) {
            ecol += st.Ecol[s];
            for (int a = 0; a < d; ++a) {
                r[p.coll_index[a]] -= st.gcol[a * S + s];
                for (int b2 = 0; b2 < d; ++b2) {
                    const int e = p.coll_index[a] * n + p.coll_index[b2];
                    st.KH[e * S + s] = st.KD[e * S + s] + st.Hcol[(a * d + b2) * S + s];
                }
            }
        }
        st_vec<n>(st.rb, S, s, r);
        PG_MAT(Dm, lt);
        PG_VEC(m, lt);
        PG_VEC(t, lt);
        PG_VEC(acc, lt);
        ld_soa<n>(st.LD, S, s, Dm);
        ld_vec<n>(st.mu, S, s, m);
        mvec<n>(Dm, m, acc);
        if (i < N - 1) {
            ld_soa<n>(st.LU, S, s, Dm);
            ld_vec<n>(st.mu, S, s + 1, m);
            mvec<n>(Dm, m, t);
PG_UNROLL
            for (int e = 0; e < n; ++e) acc[e] += t[e];
        }
        if (i > 0) {
            ld_soa<n>(st.LU, S, s - 1, Dm);
            ld_vec<n>(st.mu, S, s - 1, m);
PG_UNROLL
            for (int e = 0; e < n; ++e) t[e] = 0.0;
            mvec_tn_sub<n>(Dm, m, t);
PG_UNROLL
            for (int e = 0; e < n; ++e) acc[e] -= t[e];
        }
        st_vec<n>(st.Lmu, S, s, acc);
        epri += prior_cost_state<n>(st, p, i, nullptr, nullptr, nullptr, lt);
    }
    ecol = block_sum(ecol, sh_d);
    epri = block_sum(epri, sh_d);
    if (tid == 0) {
        st.psum[((int64_t)pid * nb + y) * 2 + 0] = ecol;
        st.psum[((int64_t)pid * nb + y) * 2 + 1] = epri;
        if (y == 0) p.phase = 0;
    }
}

// Part 2: trial step size number round * W + blockIdx.y for plan blockIdx.x:
//   Lambda' = (beta (K^-1 + H) + Lambda_k) / (beta T + 1)  -> marginals, log det, PD
//   (K^-1 + Lambda_k / beta) mu' = eta - g + Lambda_k mu_k / beta
//   KL(q' || q_k) = 1/2 [beta (T dim - tr((K^-1 + H) Sigma')) + dmu^T Lambda_k dmu
//                        + log det Lambda' - log det Lambda_k]
// (the trace term uses Lambda_k = (beta T + 1) Lambda' - beta (K^-1 + H) and
// tr(Lambda' Sigma') = dim).  Results go to the trial slot and st.tres.
template <int n>
__global__ void __launch_bounds__(kTrialThreads) trial_kernel(DevState st, int round) {
    __shared__ double sh_d[kTrialThreads + 1];
    __shared__ int sh_i[kChainThreads + 1];
    __shared__ int sh_j[kChainThreads + 1];
    const int pid = blockIdx.x, t = blockIdx.y;
    const PlanDev& p = st.plans[pid];
    if (!p.active || p.phase != 0) return;
    const int tt = round * st.W + t;
    if (tt >= p.max_bisect) return;
    const int tid = threadIdx.x;
    const int half = tid / kChainThreads, lane = tid % kChainThreads;
    const int N = p.N, nseg = p.nseg;
    const int64_t S = st.S, off = p.off;
    const int64_t SW = S * st.W, offt = (int64_t)t * S + off, shift = -(int64_t)t * S;
    double* sg = seg_scratch<n>(st, pid, t, half);
    double* ws = state_ws(st, half);
    TS ts = thread_ws<n>(st, pid, t);
    double* res = st.tres + ((int64_t)pid * st.W + t) * 4;
    const double beta = ldexp(p.beta_max, -tt);
    const double T = p.temperature;
    const double c = 1.0 / fma(beta, T, 1.0);
    // wave 0: marginals and PD test of the trial precision; wave 1: trial mean.
    // Both helpers pass the same three workgroup barriers.
    double ldt = 0.0;
    if (half == 0) {
        BlockSrc MT{st.KH, st.LD, st.KU, st.LU, nullptr, nullptr, c * beta, c, S, shift};
        wg_gbp<n>(MT, st, ws, lane, offt, SW, N, nseg, sg, st.TSD, st.TSU, &ldt, sh_d, sh_i, ts);
    } else {
        BlockSrc MM{st.KD, st.LD, st.KU, st.LU, st.rb, st.Lmu, 1.0, 1.0 / beta, S, shift};
        wg_solve<n>(MM, st, ws, lane, offt, SW, N, nseg, sg, st.Tmu, sh_j, ts);
    }
    __syncthreads();
    const bool pd = sh_i[kChainThreads] != 0;
    ldt = sh_d[kChainThreads];
    __syncthreads();
    if (!pd) {
        if (tid == 0) {
            res[0] = 0.0;
            res[1] = NAN;
            res[2] = NAN;
            res[3] = beta;
        }
        return;
    }
    double trKH = 0.0, quad = 0.0;
    const int n2 = n * n;
    for (int i = tid; i < N; i += kTrialThreads) {
        TS lt = ts;
        const int64_t s = off + i, q = offt + i;
        PG_MAT(Sg, lt);
        PG_MAT(Dm, lt);
        PG_VEC(dm, lt);
        PG_VEC(tv, lt);
        ld_soa<n>(st.TSD, SW, q, Sg);
        for (int r = 0; r < n; ++r)
            for (int k = 0; k < n; ++k) trKH = fma(st.KH[(r * n + k) * S + s], Sg[k * n + r], trKH);
        for (int e = 0; e < n; ++e) dm[e] = st.Tmu[e * SW + q] - st.mu[e * S + s];
        ld_soa<n>(st.LD, S, s, Dm);
        mvec<n>(Dm, dm, tv);
        for (int e = 0; e < n; ++e) quad = fma(dm[e], tv[e], quad);
        if (i < N - 1) {
            PG_MAT(Su, lt);
            PG_VEC(dn, lt);
            ld_soa<n>(st.TSU, SW, q, Su);
            for (int e = 0; e < n2; ++e) trKH = fma(2.0 * st.KU[e * S + s], Su[e], trKH);
            for (int e = 0; e < n; ++e) dn[e] = st.Tmu[e * SW + q + 1] - st.mu[e * S + s + 1];
            ld_soa<n>(st.LU, S, s, Dm);
            mvec<n>(Dm, dn, tv);
            for (int e = 0; e < n; ++e) quad = fma(2.0 * dm[e], tv[e], quad);
        }
    }
    trKH = wg_sum(trKH, sh_d);
    quad = wg_sum(quad, sh_d);
    if (tid == 0) {
        res[0] = 1.0;
        res[1] = 0.5 * (beta * (T * (double)N * n - trKH) + quad + ldt - p.logdet);
        res[2] = ldt;
        res[3] = beta;
    }
}

// Part 3: take the first passing trial of this window (in step-size order)
// and write it back as the new iterate; finish the iteration of plans whose
// step sizes are exhausted (state unchanged, ENOCONV).  Grid (plans,
// iter_blocks): every block finds the same pick from the trial results and
// copies its share of the states; block 0 does the bookkeeping and tags
// the plan with phase 2 + round, which the other blocks of this launch still
// read as pending.
template <int n>
__global__ void __launch_bounds__(kIterThreads) select_kernel(DevState st, int round) {
    const int pid = blockIdx.x, y = blockIdx.y, nb = gridDim.y;
    PlanDev& p = st.plans[pid];
    if (!p.active) return;
    const int ph = p.phase;
    if (ph != 0 && ph != 2 + round) return;
    const int tid = threadIdx.x;
    const int W = st.W;
    int pick = -1;
    int tried = 0;
    double last_kl = NAN;
    for (int t = 0; t < W; ++t) {
        const int tt = round * W + t;
        if (tt >= p.max_bisect) break;
        const double* res = st.tres + ((int64_t)pid * W + t) * 4;
        tried = tt + 1;
        last_kl = res[1];
        if (res[0] != 0.0 && res[1] <= p.kl_bound) {
            pick = t;
            break;
        }
    }
    const bool exhausted = (round + 1) * W >= p.max_bisect;
    if (pick < 0 && !exhausted) return;  // next window
    const int N = p.N;
    const int64_t S = st.S, off = p.off, SW = S * W;
    const int n2 = n * n;
    double beta = 0.0, kl = last_kl, ld = 0.0;
    if (pick >= 0) {
        const double* res = st.tres + ((int64_t)pid * W + pick) * 4;
        beta = res[3];
        kl = res[1];
        ld = res[2];
        const double c = 1.0 / fma(beta, p.temperature, 1.0);
        const double a0 = c * beta, a1 = c;
        const int64_t tq = (int64_t)pick * S;
        for (int i = y * kIterThreads + tid; i < N; i += nb * kIterThreads) {
            const int64_t s = off + i, q = tq + s;
            for (int e = 0; e < n2; ++e) {
                st.LD[e * S + s] = lin2(a0, st.KH[e * S + s], a1, st.LD[e * S + s]);
                st.SD[e * S + s] = st.TSD[e * SW + q];
                if (i < N - 1) {
                    st.LU[e * S + s] = lin2(a0, st.KU[e * S + s], a1, st.LU[e * S + s]);
                    st.SU[e * S + s] = st.TSU[e * SW + q];
                }
            }
            for (int e = 0; e < n; ++e) st.mu[e * S + s] = st.Tmu[e * SW + q];
        }
    }
    if (y == 0 && tid == 0) {
        double ecol = 0.0, epri = 0.0;
        for (int k = 0; k < nb; ++k) {
            ecol += st.psum[((int64_t)pid * nb + k) * 2 + 0];
            epri += st.psum[((int64_t)pid * nb + k) * 2 + 1];
        }
        p.E_coll = ecol;
        p.E_prior = epri;
        p.trials = pick >= 0 ? round * W + pick + 1 : tried;
        p.trials_total += p.trials;
        p.kl = kl;
        if (pick >= 0) {
            p.logdet = ld;
            p.beta = beta;
            p.status = 0;
        } else {
            p.beta = 0.0;
            p.status = PGVIMP_ENOCONV;
        }
        p.entropy = 0.5 * (double)N * n * (1.0 + 1.8378770664093453) - 0.5 * p.logdet;
        p.iters_left -= 1;
        p.iters_done += 1;
        p.phase = 2 + round;
    }
}

// per-factor prior costs for output: trans at off+i, goal at off+N-1, start at S+plan
template <int n>
__global__ void __launch_bounds__(kChainThreads) prior_cost_kernel(DevState st, int plan) {
    const PlanDev& p = st.plans[plan];
    const TS ts = thread_ws<n>(st, plan, 0);
    for (int i = threadIdx.x; i < p.N; i += kChainThreads) {
        double tr = 0.0, s0 = 0.0, g0 = 0.0;
        prior_cost_state<n>(st, p, i, &tr, &s0, &g0, ts);
        if (i < p.N - 1) st.Epri[p.off + i] = tr;
        if (i == p.N - 1) st.Epri[p.off + i] = g0;
        if (i == 0) st.Epri[st.S + plan] = s0;
    }
}

template <int n>
hipError_t launch_chain_n(const DevState& st, int mode, int lo, int hi, hipStream_t s) {
    if (hi <= lo) return hipSuccess;
    hipLaunchKernelGGL(chain_kernel<n>, dim3(hi - lo), dim3(kChainThreads), 0, s, st, mode, lo);
    return hipGetLastError();
}

// part: 0 = prep, 1 = trial window `round`, 2 = select for window `round`
template <int n>
hipError_t launch_iteration_n(const DevState& st, int phw, int part, int round, hipStream_t s) {
    if (phw <= 0) return hipSuccess;
    const dim3 it(phw, st.iter_blocks);
    if (part == 0) hipLaunchKernelGGL(prep_kernel<n>, it, dim3(kIterThreads), 0, s, st);
    if (part == 1) hipLaunchKernelGGL(trial_kernel<n>, dim3(phw, st.W), dim3(kTrialThreads), 0, s, st, round);
    if (part == 2) hipLaunchKernelGGL(select_kernel<n>, it, dim3(kIterThreads), 0, s, st, round);
    return hipGetLastError();
}

template <int n>
hipError_t launch_prior_costs_n(const DevState& st, int plan, int N, hipStream_t s) {
    (void)N;
    hipLaunchKernelGGL(prior_cost_kernel<n>, dim3(1), dim3(kChainThreads), 0, s, st, plan);
    return hipGetLastError();
}

}  // namespace pg
