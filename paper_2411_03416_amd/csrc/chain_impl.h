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
// Schur-complement contribution of the segment to its two separators.  Lane
// 0 solves the reduced chain of separators sequentially (forward
// elimination, backward selected inversion).  Each lane then recovers its
// interior marginals by a backward sweep conditioned on the separators'
// joint covariance.  Depth: N/nseg + 2 nseg + N/nseg dependent block steps
// instead of 2N.  log det Lambda is the sum of the log determinants of all
// pivots (interior Schur complements and reduced-chain pivots), and Lambda
// is positive definite iff every pivot is.
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
template <int n>
struct SegLayout {
    static constexpr int DL = 0;             // Schur contribution to left separator
    static constexpr int DR = n * n;         // ... to right separator
    static constexpr int CLR = 2 * n * n;    // coupling block (left sep, right sep)
    static constexpr int CROSS = 3 * n * n;  // Cov(left sep, right sep)
    static constexpr int RPINV = 4 * n * n;  // reduced-chain pivot inverse (right sep)
    static constexpr int RG = 5 * n * n;     // reduced-chain pivot^-1 * coupling
    static constexpr int RL = 6 * n * n;     // rhs contribution to left separator
    static constexpr int RR = 6 * n * n + n;
    static constexpr int RZ = 6 * n * n + 2 * n;  // reduced-chain pivot^-1 * rhs
    static constexpr int XS = 6 * n * n + 3 * n;  // solution at right separator
    static constexpr int STRIDE = 6 * n * n + 4 * n;
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

// Reduced chain over the nseg-1 separators (run by one lane).  COV: write
// the separators' marginals into SDo and their cross-covariances into the
// segment scratch.  RHS: solve and write the separator solutions into xo
// and the segment scratch.
template <int n, bool RHS, bool COV>
__device__ __forceinline__ bool reduced_chain(const BlockSrc& M, int64_t off, int N, int nseg, double* sg, double* SDo,
                              double* xo, int64_t S, double* logdet, TS ts) {
    using G = SegLayout<n>;
    const int nsep = nseg - 1;
    if (nsep <= 0) return true;
    bool ok = true;
    PG_MAT(P, ts);
    PG_MAT(Pinv, ts);
    PG_MAT(Ut, ts);
    PG_MAT(Gt, ts);
    PG_MAT(Dn, ts);  // next separator's assembled diagonal block, one step ahead
    PG_MAT(Un, ts);  // next coupling block
    PG_VEC(y, ts); PG_VEC(z, ts); PG_VEC(rn, ts);
    // assembled diagonal block (and rhs) of separator j into Dd, rd
    auto assemble = [&](int j, double* Dd, double* rd) {
        const int s = sep_state(N, nseg, j);
        const double* gj = sg + (int64_t)j * G::STRIDE;
        const double* gn = sg + (int64_t)(j + 1) * G::STRIDE;
        src_D<n>(M, off + s, Dd);
PG_UNROLL
        for (int e = 0; e < n * n; ++e) Dd[e] += gj[G::DR + e] + gn[G::DL + e];
        if (RHS) {
            src_r<n>(M, off + s, rd);
PG_UNROLL
            for (int e = 0; e < n; ++e) rd[e] += gj[G::RR + e] + gn[G::RL + e];
        }
    };
    assemble(0, P, y);
    if (nsep > 1) {
        const double* g1 = sg + (int64_t)1 * G::STRIDE;
PG_UNROLL
        for (int e = 0; e < n * n; ++e) Ut[e] = g1[G::CLR + e];
    }
    for (int j = 0; j < nsep; ++j) {
        TS lt = ts;
        double* gj = sg + (int64_t)j * G::STRIDE;
        if (j + 1 < nsep) {
            assemble(j + 1, Dn, rn);
            if (j + 2 < nsep) {
                const double* g2 = sg + (int64_t)(j + 2) * G::STRIDE;
PG_UNROLL
                for (int e = 0; e < n * n; ++e) Un[e] = g2[G::CLR + e];
            }
        }
        ok = spd_inverse<n>(P, Pinv, RHS ? nullptr : logdet, lt) && ok;
PG_UNROLL
        for (int e = 0; e < n * n; ++e) gj[G::RPINV + e] = Pinv[e];
        if (RHS) {
            mvec<n>(Pinv, y, z);
PG_UNROLL
            for (int e = 0; e < n; ++e) gj[G::RZ + e] = z[e];
        }
        if (j + 1 < nsep) {
            // coupling between separator j and j+1 lives in segment j+1;
            // next pivot P = D_{j+1} - Ut^T Pinv Ut, next rhs y = r_{j+1} - Ut^T z
            mmul<n>(Pinv, Ut, Gt);
PG_UNROLL
            for (int e = 0; e < n * n; ++e) gj[G::RG + e] = Gt[e];
            mcopy<n>(Dn, P);
            msub_tn<n>(Ut, Gt, P);
            if (RHS) {
PG_UNROLL
                for (int e = 0; e < n; ++e) y[e] = rn[e];
                mvec_tn_sub<n>(Ut, z, y);
            }
            if (j + 2 < nsep) mcopy<n>(Un, Ut);
        }
    }
    if (!ok) return false;
    if (COV) {
        PG_MAT(Sn, ts);
        {
            const int j = nsep - 1;
            double* gj = sg + (int64_t)j * G::STRIDE;
PG_UNROLL
            for (int e = 0; e < n * n; ++e) Sn[e] = gj[G::RPINV + e];
            st_soa_sym<n>(SDo, S, off + sep_state(N, nseg, j), Sn);
        }
        for (int j = nsep - 2; j >= 0; --j) {
            TS lt = ts;
            double* gj = sg + (int64_t)j * G::STRIDE;
            double* gn = sg + (int64_t)(j + 1) * G::STRIDE;
            PG_MAT(Gj, lt);
            PG_MAT(C, lt);
            PG_MAT(Sj, lt);
PG_UNROLL
            for (int e = 0; e < n * n; ++e) Gj[e] = gj[G::RG + e];
            mmul<n>(Gj, Sn, C);  // C = Gj Sn ; Cov(j, j+1) = -C
PG_UNROLL
            for (int e = 0; e < n * n; ++e) gn[G::CROSS + e] = -C[e];
            // Sj = Pinv_j + C Gj^T
            mmul_nt<n>(C, Gj, Sj);
PG_UNROLL
            for (int e = 0; e < n * n; ++e) Sj[e] += gj[G::RPINV + e];
            st_soa_sym<n>(SDo, S, off + sep_state(N, nseg, j), Sj);
            mcopy<n>(Sj, Sn);
        }
    }
    if (RHS) {
        PG_VEC(x, ts);
        {
            const int j = nsep - 1;
            double* gj = sg + (int64_t)j * G::STRIDE;
PG_UNROLL
            for (int e = 0; e < n; ++e) x[e] = gj[G::RZ + e];
PG_UNROLL
            for (int e = 0; e < n; ++e) gj[G::XS + e] = x[e];
            st_vec<n>(xo, S, off + sep_state(N, nseg, j), x);
        }
        for (int j = nsep - 2; j >= 0; --j) {
            TS lt = ts;
            double* gj = sg + (int64_t)j * G::STRIDE;
            PG_MAT(Gj, lt);
            PG_VEC(t, lt);
PG_UNROLL
            for (int e = 0; e < n * n; ++e) Gj[e] = gj[G::RG + e];
            mvec<n>(Gj, x, t);
PG_UNROLL
            for (int e = 0; e < n; ++e) x[e] = gj[G::RZ + e] - t[e];
PG_UNROLL
            for (int e = 0; e < n; ++e) gj[G::XS + e] = x[e];
            st_vec<n>(xo, S, off + sep_state(N, nseg, j), x);
        }
    }
    return true;
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
            const double* cr = sg + (int64_t)j * G::STRIDE + G::CROSS;  // Cov(L, R)
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

// Workgroup-wide GBP: marginals of (D, U) from src into (SDo, SUo).
template <int n>
__device__ __forceinline__ bool wg_gbp(const BlockSrc& M, const DevState& st, double* ws, int tid, int64_t off,
                                       int64_t So, int N, int nseg, double* sg, double* SDo, double* SUo,
                                       double* logdet_out, double* sh_ld, int* sh_ok, TS ts) {
    double ld = 0.0;
    bool ok = true;
    if (tid < nseg) ok = seg_forward<n, false>(M, off, N, nseg, tid, ws, st.ws_stride, sg, &ld, ts);
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
        double ldr = 0.0;
        bool okr = all ? reduced_chain<n, false, true>(M, off, N, nseg, sg, SDo, nullptr, So, &ldr, ts) : false;
        sh_ld[kChainThreads] = tot + ldr;
        sh_ok[kChainThreads] = (all && okr) ? 1 : 0;
    }
    __syncthreads();
    const bool okall = sh_ok[kChainThreads] != 0;
    *logdet_out = sh_ld[kChainThreads];
    if (okall && tid < nseg) seg_backward_cov<n>(off, N, nseg, tid, ws, st.ws_stride, sg, SDo, SUo, So, ts);
    __syncthreads();
    return okall;
}

// Workgroup-wide solve of (D, U) x = r into xo.
template <int n>
__device__ __forceinline__ bool wg_solve(const BlockSrc& M, const DevState& st, double* ws, int tid, int64_t off,
                                         int64_t So, int N, int nseg, double* sg, double* xo, int* sh_ok, TS ts) {
    double ld = 0.0;
    bool ok = true;
    if (tid < nseg) ok = seg_forward<n, true>(M, off, N, nseg, tid, ws, st.ws_stride, sg, &ld, ts);
    sh_ok[tid] = ok ? 1 : 0;
    __syncthreads();
    if (tid == 0) {
        int all = 1;
        for (int t = 0; t < kChainThreads; ++t) all &= sh_ok[t];
        double ldr = 0.0;
        bool okr = all ? reduced_chain<n, true, false>(M, off, N, nseg, sg, nullptr, xo, So, &ldr, ts) : false;
        sh_ok[kChainThreads] = (all && okr) ? 1 : 0;
    }
    __syncthreads();
    const bool okall = sh_ok[kChainThreads] != 0;
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

// One proximal iteration (Alg. 1), part 1: per-state quantities shared by all
// trial step sizes -- KH = K^-1 + H (collision Hessians on the diagonal
// blocks), rb = eta - g, Lmu = Lambda_k mu_k -- and the expected costs.
template <int n>
__global__ void __launch_bounds__(kChainThreads) prep_kernel(DevState st) {
    __shared__ double sh_d[kChainThreads + 1];
    const int pid = blockIdx.x;
    PlanDev& p = st.plans[pid];
    if (!p.active) return;
    const int tid = threadIdx.x;
    if (p.iters_left <= 0) {
        if (tid == 0) p.phase = 1;
        return;
    }
    const int N = p.N, d = p.d;
    const int64_t off = p.off, S = st.S;
    const int n2 = n * n;
    TS ts = thread_ws<n>(st, pid, 0);
    double ecol = 0.0, epri = 0.0;
    for (int i = tid; i < N; i += kChainThreads) {
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
    ecol = wg_sum(ecol, sh_d);
    epri = wg_sum(epri, sh_d);
    if (tid == 0) {
        p.E_coll = ecol;
        p.E_prior = epri;
        p.phase = 0;
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
// step sizes are exhausted (state unchanged, ENOCONV).
template <int n>
__global__ void __launch_bounds__(kChainThreads) select_kernel(DevState st, int round) {
    const int pid = blockIdx.x;
    PlanDev& p = st.plans[pid];
    if (!p.active || p.phase != 0) return;
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
    __syncthreads();
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
        for (int i = tid; i < N; i += kChainThreads) {
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
    if (tid == 0) {
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
        p.phase = 1;
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
    if (part == 0) hipLaunchKernelGGL(prep_kernel<n>, dim3(phw), dim3(kChainThreads), 0, s, st);
    if (part == 1) hipLaunchKernelGGL(trial_kernel<n>, dim3(phw, st.W), dim3(kTrialThreads), 0, s, st, round);
    if (part == 2) hipLaunchKernelGGL(select_kernel<n>, dim3(phw), dim3(kChainThreads), 0, s, st, round);
    return hipGetLastError();
}

template <int n>
hipError_t launch_prior_costs_n(const DevState& st, int plan, int N, hipStream_t s) {
    (void)N;
    hipLaunchKernelGGL(prior_cost_kernel<n>, dim3(1), dim3(kChainThreads), 0, s, st, plan);
    return hipGetLastError();
}

}  // namespace pg
