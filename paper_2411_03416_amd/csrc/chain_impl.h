// Chain kernels: marginal covariances of the block-tridiagonal precision
// (Gaussian belief propagation on the chain, Sec. 5.1), the block-
// tridiagonal mean solve of Theorem 1, and the fused step-size loop of
// Alg. 1 / App. C.  One wavefront (64 lanes, one per segment) factors one
// matrix of one plan.
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
// Chain order.  The lanes of a wavefront walk their segments in lock step,
// so the blocks they touch at one step belong to nseg different segments.
// The data the sweeps read and write is therefore kept in chain order:
// state i of segment j (local index il = i - start_j) sits at position
// il * nseg + j of the plan's chain range, which makes every per-step load
// and store of a wavefront contiguous.  The prep kernel writes the
// iteration's inputs in chain order, the sweeps' temporaries and the trial
// results stay in chain order, and the select kernel writes the accepted
// trial back in state order.
//
// The same elimination with a right-hand side solves
// (K^-1 + Lambda_k / beta) mu' = eta - g + Lambda_k mu_k / beta, or for the
// natural-gradient step (Sec. 3.1(d)) Lambda' mu' / beta =
// eta - g + H mu_k + (1 / beta - T) Lambda_k mu_k with
// Lambda' / beta = K^-1 + H + (1 / beta - T) Lambda_k.
//
// Step-size selection.  Halving from beta_max accepts the first trial step
// that passes (Alg. 1, App. C), so the trials are independent of each
// other: one launch evaluates a window of consecutive trial step sizes at
// once, one workgroup per (plan, trial).  A plan with a passing step in an
// earlier window skips the later ones; after the last window a select
// kernel takes the first passing step size in order.  The chosen step and
// every result are the same as trying the step sizes one after another.
#pragma once
#include "blockmath.h"
#include "ctx.h"

namespace pg {

// Entry offsets in the per-segment scratch, stored field-major:
// sg[f * kMaxSeg + j] is field f of slot j.  Slot j holds the data of
// separator j (node j) of the reduced chain; before the nodes are
// assembled, the first fields hold segment j's contributions to its two
// separators (they are read into registers before the node fields are
// written).  The covariance half (selected inversion, RHS = false) and the
// mean half (solve, RHS = true) keep only the fields they use.  For small
// blocks the scratch lives in LDS.
template <int n, bool RHS>
struct SegLayout;
template <int n>
struct SegLayout<n, false> {
    static constexpr int NA = 0;          // current diagonal block; Sigma_jj after the backward pass
    static constexpr int NC = n * n;      // coupling M(j, right neighbour at the current level)
    static constexpr int NP = 2 * n * n;  // pivot inverse at elimination
    static constexpr int NGL = 3 * n * n; // pivot^-1 M(j, left neighbour)
    static constexpr int NGR = 4 * n * n; // pivot^-1 M(j, right neighbour)
    // Cov(j, right neighbour at j's level), Cov(j, j+1) at the end.  It
    // shares the coupling's entries: the backward pass reads no coupling.
    static constexpr int NX = NC;
    static constexpr int STRIDE = 5 * n * n;
    // segment j's contributions before assembly (aliases)
    static constexpr int DL = NA;   // Schur contribution to the left separator
    static constexpr int DR = NC;   // ... to the right separator
    static constexpr int CLR = NP;  // coupling block (left sep, right sep)
};
template <int n>
struct SegLayout<n, true> {
    static constexpr int NA = 0;
    static constexpr int NC = n * n;
    static constexpr int NGL = 2 * n * n;
    static constexpr int NGR = 3 * n * n;
    static constexpr int NR = 4 * n * n;          // current rhs of node j
    static constexpr int NZ = 4 * n * n + n;      // pivot^-1 rhs at elimination
    static constexpr int XS = 4 * n * n + 2 * n;  // solution at separator j
    static constexpr int STRIDE = 4 * n * n + 3 * n;
    static constexpr int DL = NA;
    static constexpr int DR = NC;
    static constexpr int CLR = NGL;
    static constexpr int RL = NR;  // rhs contribution to the left separator
    static constexpr int RR = NZ;  // ... to the right separator
};
constexpr unsigned kTrialLdsPad = 4096;
// Node scratch in LDS (both halves of a workgroup) for small blocks.
template <int n>
struct NodeLds {
    static constexpr bool value = RegBlocks<n>::value;
    static constexpr int size = value ? kMaxSeg * (SegLayout<n, false>::STRIDE + SegLayout<n, true>::STRIDE) : 1;
};

// Field f of slot j of the segment scratch.
__device__ __forceinline__ double& sgv(double* sg, int j, int f) { return sg[(uint32_t)(f * kMaxSeg + j)]; }

// Chain-order arrays are tiled in groups of kTile positions, with entries
// paired: entry e of position q (E entries per position, E even) is element
// ((q >> 5) * E + (e & ~1)) * 32 + (q & 31) * 2 + (e & 1).  Entries 2k and
// 2k + 1 of a position are adjacent, so a lane moves them with one 16-byte
// access, and a wave doing so for 32 consecutive positions touches 512
// contiguous bytes.  All entries of one position share one per-lane byte
// offset (entry e adds the constant (e >> 1) * 512 + (e & 1) * 8).  Views
// (plan range, trial slot) start at a multiple of kTile positions.
constexpr int kTile = 32;
template <int E>
__device__ __forceinline__ uint32_t toff(uint32_t pl) {
    static_assert(E % 2 == 0, "paired tiles need an even entry count");
    return ((pl >> 5) * (uint32_t)(E * kTile) + (pl & 31u) * 2u) * 8u;
}
template <int E>
__device__ __forceinline__ int64_t tidx(int64_t q, int e) {
    static_assert(E % 2 == 0, "paired tiles need an even entry count");
    return ((q >> 5) * E + (e & ~1)) * kTile + (q & 31) * 2 + (e & 1);
}
__device__ __forceinline__ constexpr uint32_t tent(int e) { return (uint32_t)((e >> 1) * (2 * kTile * 8) + (e & 1) * 8); }
__device__ __forceinline__ double ldo(const double* base, uint32_t off, int e) {
    return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + off + tent(e));
}
__device__ __forceinline__ void sto(double* base, uint32_t off, int e, double v) {
    *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + off + tent(e)) = v;
}

// Per-state temporaries of one sweep (views over the same positions): the
// interior pivot inverse, pivot^-1 U_i, pivot^-1 X_i (fill towards the left
// separator) and pivot^-1 y_i.
struct Ws {
    double *P, *G, *H, *Y;
};

// Blocks of the matrix being factored: D_i = a0 D0_i + a1 D1_i, U likewise,
// right-hand side r_i = a0 R0_i + a1 R1_i (a single source is passed twice
// with a1 = 0).  All are chain-order views of the plan's range.
struct BlockSrc {
    const double* D0;
    const double* D1;
    const double* U0;
    const double* U1;
    const double* R0;
    const double* R1;
    double a0, a1;
};

// Entry e of a matrix built as a0 X0 + a1 X1 (the same expression is used
// when the accepted trial precision is written back).
__device__ __forceinline__ double lin2(double a0, double x0, double a1, double x1) { return fma(a1, x1, a0 * x0); }

// SoA blocks and vectors at 64-bit state indices (per-state kernels).
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
__device__ __forceinline__ void ld_vec(const double* __restrict__ X, int64_t S, int64_t s, double* v) {
PG_UNROLL
    for (int e = 0; e < n; ++e) v[e] = X[e * S + s];
}
template <int n>
__device__ __forceinline__ void st_vec(double* __restrict__ X, int64_t S, int64_t s, const double* v) {
PG_UNROLL
    for (int e = 0; e < n; ++e) X[e * S + s] = v[e];
}

// Blocks (CNT = n*n) and vectors (CNT = n) of a chain-order view at the
// per-lane byte offset off (toff<CNT> of the position).
template <int n, int CNT>
__device__ __forceinline__ void ldt(const double* X, uint32_t off, double* M) {
PG_UNROLL
    for (int e = 0; e < CNT; ++e) M[e] = ldo(X, off, e);
}
template <int n, int CNT>
__device__ __forceinline__ void stt(double* X, uint32_t off, const double* M) {
PG_UNROLL
    for (int e = 0; e < CNT; ++e) sto(X, off, e, M[e]);
}
template <int n>
__device__ __forceinline__ void stt_sym(double* X, uint32_t off, const double* M) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j < n; ++j) sto(X, off, i * n + j, 0.5 * (M[i * n + j] + M[j * n + i]));
}
// Raw loads of the two sources of a block (or vector) and their combination,
// split so that loads issued one step ahead are combined one step later.
template <int n, int CNT>
__device__ __forceinline__ void ld2(const double* X0, const double* X1, uint32_t off, double* M0, double* M1) {
PG_UNROLL
    for (int e = 0; e < CNT; ++e) {
        M0[e] = ldo(X0, off, e);
        M1[e] = ldo(X1, off, e);
    }
}
template <int n, int CNT>
__device__ __forceinline__ void comb(double a0, const double* M0, double a1, const double* M1, double* M) {
PG_UNROLL
    for (int e = 0; e < CNT; ++e) M[e] = lin2(a0, M0[e], a1, M1[e]);
}
// Lower triangles (j <= i) of symmetric blocks: raw loads of both sources,
// their combination, a block built directly, and stores / loads of a
// symmetric block's lower triangle (the loads fill the upper one).
template <int n>
__device__ __forceinline__ void ld2_lo(const double* X0, const double* X1, uint32_t off, double* M0, double* M1) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j <= i; ++j) {
            M0[i * n + j] = ldo(X0, off, i * n + j);
            M1[i * n + j] = ldo(X1, off, i * n + j);
        }
}
template <int n>
__device__ __forceinline__ void comb_lo(double a0, const double* M0, double a1, const double* M1, double* M) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j <= i; ++j) M[i * n + j] = lin2(a0, M0[i * n + j], a1, M1[i * n + j]);
}
template <int n>
__device__ __forceinline__ void src_D_lo(const BlockSrc& b, uint32_t off, double* M) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j <= i; ++j)
            M[i * n + j] = lin2(b.a0, ldo(b.D0, off, i * n + j), b.a1, ldo(b.D1, off, i * n + j));
}
template <int n>
__device__ __forceinline__ void stt_lo(double* X, uint32_t off, const double* M) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j <= i; ++j) sto(X, off, i * n + j, M[i * n + j]);
}
template <int n>
__device__ __forceinline__ void ldt_sym(const double* X, uint32_t off, double* M) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j <= i; ++j) {
            const double v = ldo(X, off, i * n + j);
            M[i * n + j] = v;
            M[j * n + i] = v;
        }
}
template <int n>
__device__ __forceinline__ void src_D(const BlockSrc& b, uint32_t off, double* M) {
PG_UNROLL
    for (int e = 0; e < n * n; ++e) M[e] = lin2(b.a0, ldo(b.D0, off, e), b.a1, ldo(b.D1, off, e));
}
template <int n>
__device__ __forceinline__ void src_U(const BlockSrc& b, uint32_t off, double* M) {
PG_UNROLL
    for (int e = 0; e < n * n; ++e) M[e] = lin2(b.a0, ldo(b.U0, off, e), b.a1, ldo(b.U1, off, e));
}
template <int n>
__device__ __forceinline__ void src_r(const BlockSrc& b, uint32_t off, double* v) {
PG_UNROLL
    for (int e = 0; e < n; ++e) v[e] = lin2(b.a0, ldo(b.R0, off, e), b.a1, ldo(b.R1, off, e));
}

__device__ __forceinline__ void seg_bounds(int N, int nseg, int j, int& a, int& b, bool& hasL, bool& hasR) {
    const int st = (int)(((int64_t)j * N) / nseg);
    const int en = (int)(((int64_t)(j + 1) * N) / nseg);
    hasL = j > 0;
    hasR = j < nseg - 1;
    a = st;
    b = hasR ? en - 2 : en - 1;
}

__device__ __forceinline__ int seg_start(int N, int nseg, int j) { return (int)(((int64_t)j * N) / nseg); }
__device__ __forceinline__ int sep_state(int N, int nseg, int j) { return seg_start(N, nseg, j + 1) - 1; }
// Segment of state i: the largest j with seg_start(j) <= i.
__device__ __forceinline__ int seg_of(int N, int nseg, int i) {
    return (int)((((int64_t)i + 1) * nseg + N - 1) / N) - 1;
}
// Plan-local position of state i in the plan's chain range.
__device__ __forceinline__ int64_t chain_pos(int N, int nseg, int i) {
    const int j = seg_of(N, nseg, i);
    return (int64_t)(i - seg_start(N, nseg, j)) * nseg + j;
}
// Length of the chain range: nseg columns of the longest segment's length.
__device__ __forceinline__ int chain_len(int N, int nseg) { return (N + nseg - 1) / nseg * nseg; }

// Plan-local positions of the states of segment j.
struct SegPos {
    int nseg, j, a0;
    __device__ __forceinline__ uint32_t at(int i) const { return (uint32_t)((i - a0) * nseg + j); }
};
__device__ __forceinline__ SegPos seg_pos(int N, int nseg, int j) { return SegPos{nseg, j, seg_start(N, nseg, j)}; }
// Position of separator j (the last state of segment j).
__device__ __forceinline__ uint32_t sep_pos(int N, int nseg, int j) {
    return seg_pos(N, nseg, j).at(sep_state(N, nseg, j));
}

// Forward elimination of the interior states of segment j.  Matrix blocks
// come from M, temporaries go to ws; both are chain-order views indexed
// by plan-local positions.  The loop body has no branches: a missing left
// separator is a zero fill X, and the coupling stored after the chain's last
// state is a zero block; the blocks of state i + 1 are loaded at the top of
// step i and combined at its end.  The pivot P and the fill contribution Z
// are symmetric: only their lower triangles are formed (P is read only by
// the inverse; Z is completed once, after the sweep).
template <int n, bool RHS>
__device__ __forceinline__ bool seg_forward(const BlockSrc& M, int N, int nseg, int j, const Ws& ws, double* sg,
                                            double* logdet, TS ts) {
    using G = SegLayout<n, RHS>;
    constexpr int NN = n * n;
    int a, b;
    bool hasL, hasR;
    seg_bounds(N, nseg, j, a, b, hasL, hasR);
    const SegPos ps = seg_pos(N, nseg, j);
    PG_MAT(P, ts);
    PG_MAT(X, ts);
    PG_MAT(Z, ts);
    PG_MAT(U, ts);
    PG_MAT(Pinv, ts);
    PG_MAT(GU, ts);
    PG_MAT(HX, ts);
    PG_MAT(D0n, ts);  // raw blocks of the next state, loaded one step ahead
    PG_MAT(D1n, ts);
    PG_MAT(U0n, ts);
    PG_MAT(U1n, ts);
    PG_VEC(y, ts); PG_VEC(yv, ts); PG_VEC(rL, ts); PG_VEC(R0n, ts); PG_VEC(R1n, ts);
    src_D_lo<n>(M, toff<NN>(ps.at(a)), P);
    src_U<n>(M, toff<NN>(ps.at(a)), U);  // every segment has >= 2 states, so U_a exists
    {
        TS ut = ts;
        PG_MAT(UL, ut);
        src_U<n>(M, toff<NN>(hasL ? sep_pos(N, nseg, j - 1) : ps.at(a)), UL);
PG_UNROLL
        for (int r = 0; r < n; ++r)
PG_UNROLL
            for (int c = 0; c < n; ++c) X[r * n + c] = hasL ? UL[c * n + r] : 0.0;
    }
    mzero<n>(Z);
    if constexpr (RHS) {
        src_r<n>(M, toff<n>(ps.at(a)), y);
PG_UNROLL
        for (int e = 0; e < n; ++e) rL[e] = 0.0;
    }
    bool ok = true;
    DetAcc det;
    for (int i = a; i < b; ++i) {
        TS lt = ts;
        const uint32_t q = ps.at(i), qn = ps.at(i + 1);
        const uint32_t oB = toff<NN>(q), oV = toff<n>(q), oBn = toff<NN>(qn), oVn = toff<n>(qn);
        ld2_lo<n>(M.D0, M.D1, oBn, D0n, D1n);
        ld2<n, NN>(M.U0, M.U1, oBn, U0n, U1n);
        if constexpr (RHS) ld2<n, n>(M.R0, M.R1, oVn, R0n, R1n);
        double dblk;
        ok = spd_inverse<n>(P, Pinv, &dblk, lt) && ok;
        if constexpr (!RHS) {
            det.mul(dblk);
            stt_lo<n>(ws.P, oB, Pinv);
        }
        mmul<n>(Pinv, U, GU);
        stt<n, NN>(ws.G, oB, GU);
        mmul<n>(Pinv, X, HX);
        stt<n, NN>(ws.H, oB, HX);
        // the next state's blocks, combined as soon as the pivot is used up
        // (shorter live ranges for the raw loads)
        comb_lo<n>(M.a0, D0n, M.a1, D1n, P);
        PG_MAT(Un, lt);
        comb<n, n * n>(M.a0, U0n, M.a1, U1n, Un);
        msub_tn_lo<n>(X, HX, Z);
        if constexpr (RHS) {
            mvec<n>(Pinv, y, yv);
            stt<n, n>(ws.Y, oV, yv);
            mvec_tn_sub<n>(X, yv, rL);
        }
        // X_{i+1} = -U^T HX, P_{i+1} = D_{i+1} - U^T GU, y_{i+1} = r_{i+1} - U^T yv
        mmul_tn_neg<n>(U, HX, X);
        msub_tn_lo<n>(U, GU, P);
        if constexpr (RHS) {
            comb<n, n>(M.a0, R0n, M.a1, R1n, y);
            mvec_tn_sub<n>(U, yv, y);
        }
        mcopy<n>(Un, U);
    }
    {
        // last interior state b: its Schur contributions to the separators
        TS lt = ts;
        const uint32_t q = ps.at(b), oB = toff<NN>(q), oV = toff<n>(q);
        double dblk;
        ok = spd_inverse<n>(P, Pinv, &dblk, lt) && ok;
        if constexpr (!RHS) {
            det.mul(dblk);
            stt_lo<n>(ws.P, oB, Pinv);
            *logdet += det.log_value();
        }
        mmul<n>(Pinv, U, GU);
        stt<n, NN>(ws.G, oB, GU);
        mmul<n>(Pinv, X, HX);
        stt<n, NN>(ws.H, oB, HX);
        msub_tn_lo<n>(X, HX, Z);
        sym_from_lo<n>(Z);
        if constexpr (RHS) {
            mvec<n>(Pinv, y, yv);
            stt<n, n>(ws.Y, oV, yv);
            mvec_tn_sub<n>(X, yv, rL);
        }
        PG_MAT(T, lt);
        if (hasR) {
            mmul_tn<n>(U, GU, T);
PG_UNROLL
            for (int e = 0; e < n * n; ++e) sgv(sg, j, G::DR + e) = -T[e];
            if constexpr (RHS) {
                PG_VEC(t, lt);
PG_UNROLL
                for (int e = 0; e < n; ++e) t[e] = 0.0;
                mvec_tn_sub<n>(U, yv, t);
PG_UNROLL
                for (int e = 0; e < n; ++e) sgv(sg, j, G::RR + e) = t[e];
            }
        }
        if (hasL) {
PG_UNROLL
            for (int e = 0; e < n * n; ++e) sgv(sg, j, G::DL + e) = Z[e];
            if constexpr (RHS) {
PG_UNROLL
                for (int e = 0; e < n; ++e) sgv(sg, j, G::RL + e) = rL[e];
            }
        }
        if (hasL && hasR) {
            mmul_tn<n>(X, GU, T);
PG_UNROLL
            for (int e = 0; e < n * n; ++e) sgv(sg, j, G::CLR + e) = -T[e];
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
__device__ __forceinline__ void ld_node(double* sg, int j, int f, double* M) {
PG_UNROLL
    for (int e = 0; e < n * n; ++e) M[e] = sgv(sg, j, f + e);
}
template <int n>
__device__ __forceinline__ void st_node(double* sg, int j, int f, const double* M) {
PG_UNROLL
    for (int e = 0; e < n * n; ++e) sgv(sg, j, f + e) = M[e];
}

// Node j's diagonal block, right coupling and rhs from its separator state
// and the two adjacent segments: read into registers (A, C, r) ...
template <int n, bool RHS>
__device__ __forceinline__ void cr_assemble_read(const BlockSrc& M, int N, int nseg, int j, double* sg, double* A,
                                                 double* C, double* r) {
    using G = SegLayout<n, RHS>;
    const int m = nseg - 1;
    const uint32_t q = sep_pos(N, nseg, j);
    src_D<n>(M, toff<n * n>(q), A);
PG_UNROLL
    for (int e = 0; e < n * n; ++e) {
        A[e] += sgv(sg, j, G::DR + e) + sgv(sg, j + 1, G::DL + e);
        C[e] = j + 1 < m ? sgv(sg, j + 1, G::CLR + e) : 0.0;
    }
    if constexpr (RHS) {
        src_r<n>(M, toff<n>(q), r);
PG_UNROLL
        for (int e = 0; e < n; ++e) r[e] += sgv(sg, j, G::RR + e) + sgv(sg, j + 1, G::RL + e);
    }
}
// ... and, after a barrier, written as the node's fields.
template <int n, bool RHS>
__device__ __forceinline__ void cr_assemble_write(int j, double* sg, const double* A, const double* C,
                                                  const double* r) {
    using G = SegLayout<n, RHS>;
    st_node<n>(sg, j, G::NA, A);
    st_node<n>(sg, j, G::NC, C);
    if constexpr (RHS) {
PG_UNROLL
        for (int e = 0; e < n; ++e) sgv(sg, j, G::NR + e) = r[e];
    }
}

// Forward elimination.  Level l: the nodes eliminated at l store their pivot
// inverse P, G_L = P M(k, L), G_R = P M(k, R) and z = P r (barrier); the
// surviving nodes then take the Schur updates of their eliminated
// neighbours and their new right coupling -M(j, k) P M(k, R) (barrier).
template <int n, bool RHS>
__device__ __forceinline__ bool cr_forward(int m, int j, double* sg, double* logdet, TS ts) {
    using G = SegLayout<n, RHS>;
    const int levels = cr_levels(m);
    const bool own = j < m;
    const int lv = own ? __builtin_ctz(j + 1) : -1;
    bool ok = true;
    for (int l = 0; l < levels; ++l) {
        const int h = 1 << l;
        if (own && lv == l) {
            TS lt = ts;
            PG_MAT(A, lt);
            PG_MAT(P, lt);
            PG_MAT(C, lt);
            PG_MAT(T, lt);
            ld_node<n>(sg, j, G::NA, A);
            double dblk;
            ok = spd_inverse<n>(A, P, &dblk, lt) && ok;
            if constexpr (!RHS) *logdet += log(dblk);
            if constexpr (!RHS) st_node<n>(sg, j, G::NP, P);
            if (j - h >= 0) {
                ld_node<n>(sg, j - h, G::NC, C);  // M(L, k)
                mmul_nt<n>(P, C, T);
                st_node<n>(sg, j, G::NGL, T);
            }
            if (j + h < m) {
                ld_node<n>(sg, j, G::NC, C);  // M(k, R)
                mmul<n>(P, C, T);
                st_node<n>(sg, j, G::NGR, T);
            }
            if constexpr (RHS) {
                PG_VEC(r, lt);
                PG_VEC(z, lt);
PG_UNROLL
                for (int e = 0; e < n; ++e) r[e] = sgv(sg, j, G::NR + e);
                mvec<n>(P, r, z);
PG_UNROLL
                for (int e = 0; e < n; ++e) sgv(sg, j, G::NZ + e) = z[e];
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
            ld_node<n>(sg, j, G::NA, A);
            if constexpr (RHS) {
PG_UNROLL
                for (int e = 0; e < n; ++e) r[e] = sgv(sg, j, G::NR + e);
            }
            if (j + h < m) {
                // right neighbour k = j + h: A -= M(j,k) G_L(k), r -= M(j,k) z_k,
                // new coupling to k + h: -M(j,k) G_R(k)
                const int k = j + h;
                ld_node<n>(sg, j, G::NC, C);
                ld_node<n>(sg, k, G::NGL, Gk);
                msub<n>(C, Gk, A);
                if constexpr (RHS) {
PG_UNROLL
                    for (int e = 0; e < n; ++e) z[e] = sgv(sg, k, G::NZ + e);
                    mvec_sub<n>(C, z, r);
                }
                if (j + 2 * h < m) {
                    PG_MAT(T, lt);
                    ld_node<n>(sg, k, G::NGR, Gk);
                    mmul<n>(C, Gk, T);
PG_UNROLL
                    for (int e = 0; e < n * n; ++e) sgv(sg, j, G::NC + e) = -T[e];
                }
            }
            if (j - h >= 0) {
                // left neighbour k = j - h: A -= M(k,j)^T G_R(k), r -= M(k,j)^T z_k
                const int k = j - h;
                ld_node<n>(sg, k, G::NC, C);
                ld_node<n>(sg, k, G::NGR, Gk);
                msub_tn<n>(C, Gk, A);
                if constexpr (RHS) {
PG_UNROLL
                    for (int e = 0; e < n; ++e) z[e] = sgv(sg, k, G::NZ + e);
                    mvec_tn_sub<n>(C, z, r);
                }
            }
            st_node<n>(sg, j, G::NA, A);
            if constexpr (RHS) {
PG_UNROLL
                for (int e = 0; e < n; ++e) sgv(sg, j, G::NR + e) = r[e];
            }
        }
        __syncthreads();
    }
    return ok;
}

// Contributions to the KL terms of a trial (Theorem 1 step, App. C), added
// where the blocks they need are produced:
//   trace: tr(KH_i Sigma'_ii) with Sigma'_ii symmetrised, and
//          2 tr(KU_i^T Sigma'_{i,i+1});
//   quad:  d_i^T LD_i d_i and 2 d_i^T LU_i d_{i+1}, d = mu' - mu_k.
template <int n>
__device__ __forceinline__ double tr_diag(const double* K, const double* Sg) {
    double t = 0.0;
PG_UNROLL
    for (int r = 0; r < n; ++r)
PG_UNROLL
        for (int k = 0; k < n; ++k) t = fma(K[r * n + k], 0.5 * (Sg[k * n + r] + Sg[r * n + k]), t);
    return t;
}
template <int n>
__device__ __forceinline__ double tr_off(const double* K, const double* So) {
    double t = 0.0;
PG_UNROLL
    for (int e = 0; e < n * n; ++e) t = fma(K[e], So[e], t);
    return 2.0 * t;
}
template <int n>
__device__ __forceinline__ double quad_form(const double* L, const double* u, const double* v) {
    double t = 0.0;
PG_UNROLL
    for (int r = 0; r < n; ++r) {
        double w = 0.0;
PG_UNROLL
        for (int c = 0; c < n; ++c) w = fma(L[r * n + c], v[c], w);
        t = fma(u[r], w, t);
    }
    return t;
}

// Backward selected inversion, top level first: node k eliminated at level l
// with neighbours L, R (whose covariances are known from higher levels):
//   Cov(k, L) = -(G_L S_LL + G_R S_RL),  Cov(k, R) = -(G_L S_LR + G_R S_RR),
//   S_kk = P - Cov(k, L) G_L^T - Cov(k, R) G_R^T.
// Writes S_kk (node and SDo) and the cross-covariances of the two new
// adjacent pairs (L, k) and (k, R).  run = false keeps the barriers only.
template <int n, bool TRACE>
__device__ __forceinline__ void cr_backward_cov(int m, int j, bool run, int N, int nseg, double* sg, double* SDo,
                                                const double* KH, double* trace, TS ts) {
    using G = SegLayout<n, false>;
    const int levels = cr_levels(m);
    const bool own = run && j < m;
    const int lv = own ? __builtin_ctz(j + 1) : -1;
    for (int l = levels - 1; l >= 0; --l) {
        const int h = 1 << l;
        if (own && lv == l) {
            TS lt = ts;
            const bool hasL = j - h >= 0, hasR = j + h < m;
            const int L = j - h, R = j + h;
            PG_MAT(Sk, lt);
            PG_MAT(GL, lt);
            PG_MAT(GR, lt);
            PG_MAT(CL, lt);
            PG_MAT(CR, lt);
            PG_MAT(X, lt);
            PG_MAT(T, lt);
            ld_node<n>(sg, j, G::NP, Sk);
            if (hasL) ld_node<n>(sg, j, G::NGL, GL);
            if (hasR) ld_node<n>(sg, j, G::NGR, GR);
            if (hasL && hasR) ld_node<n>(sg, L, G::NX, X);  // Cov(L, R)
            if (hasL) {
                ld_node<n>(sg, L, G::NA, T);  // S_LL
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
                ld_node<n>(sg, R, G::NA, T);  // S_RR
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
            st_node<n>(sg, j, G::NA, Sk);
            const uint32_t oS = toff<n * n>(sep_pos(N, nseg, j));
            stt_sym<n>(SDo, oS, Sk);
            if (TRACE) {
                ldt<n, n * n>(KH, oS, T);
                *trace += tr_diag<n>(T, Sk);
            }
            if (hasL) {
PG_UNROLL
                for (int r = 0; r < n; ++r)
PG_UNROLL
                    for (int c = 0; c < n; ++c) sgv(sg, L, G::NX + r * n + c) = CL[c * n + r];  // Cov(L, k)
            }
            if (hasR) st_node<n>(sg, j, G::NX, CR);  // Cov(k, R)
        }
        __syncthreads();
    }
}

// Backward substitution: x_k = z_k - G_L x_L - G_R x_R, top level first.
template <int n, bool QUAD>
__device__ __forceinline__ void cr_backward_rhs(int m, int j, bool run, int N, int nseg, double* sg, double* xo,
                                                const double* LD, const double* mu0, double* quad, TS ts) {
    using G = SegLayout<n, true>;
    const int levels = cr_levels(m);
    const bool own = run && j < m;
    const int lv = own ? __builtin_ctz(j + 1) : -1;
    for (int l = levels - 1; l >= 0; --l) {
        const int h = 1 << l;
        if (own && lv == l) {
            TS lt = ts;
            PG_VEC(x, lt);
            PG_VEC(y, lt);
            PG_MAT(Gk, lt);
PG_UNROLL
            for (int e = 0; e < n; ++e) x[e] = sgv(sg, j, G::NZ + e);
            if (j - h >= 0) {
                ld_node<n>(sg, j, G::NGL, Gk);
PG_UNROLL
                for (int e = 0; e < n; ++e) y[e] = sgv(sg, j - h, G::XS + e);
                mvec_sub<n>(Gk, y, x);
            }
            if (j + h < m) {
                ld_node<n>(sg, j, G::NGR, Gk);
PG_UNROLL
                for (int e = 0; e < n; ++e) y[e] = sgv(sg, j + h, G::XS + e);
                mvec_sub<n>(Gk, y, x);
            }
PG_UNROLL
            for (int e = 0; e < n; ++e) sgv(sg, j, G::XS + e) = x[e];
            const uint32_t q = sep_pos(N, nseg, j);
            stt<n, n>(xo, toff<n>(q), x);
            if (QUAD) {
                ldt<n, n * n>(LD, toff<n * n>(q), Gk);
                ldt<n, n>(mu0, toff<n>(q), y);
PG_UNROLL
                for (int e = 0; e < n; ++e) y[e] = x[e] - y[e];
                *quad += quad_form<n>(Gk, y, y);
            }
        }
        __syncthreads();
    }
}

// Backward recovery of segment j's interior marginals, top state first.
// With x_i = P_i^-1 y_i - GU_i x_next - HX_i x_L:
//   Cov(i, next) = -(GU S_nn + HX S_Ln),  Cov(i, L) = -(GU S_nL + HX S_LL),
//   Sigma_ii = P_i^-1 - Cov(i, next) GU^T - Cov(i, L) HX^T.
// Branch-free: the forward sweep stored zero GU after the chain's last state
// and zero HX where there is no left separator; missing separator
// covariances are zero blocks.
template <int n, bool TRACE>
__device__ __forceinline__ void seg_backward_cov(int N, int nseg, int j, const Ws& ws, double* sg, double* SDo,
                                                 double* SUo, const double* KH, const double* KU, double* trace,
                                                 TS ts) {
    using G = SegLayout<n, false>;
    constexpr int NN = n * n;
    int a, b;
    bool hasL, hasR;
    seg_bounds(N, nseg, j, a, b, hasL, hasR);
    const SegPos ps = seg_pos(N, nseg, j);
    const uint32_t qL = hasL ? sep_pos(N, nseg, j - 1) : ps.at(a);
    const uint32_t qR = hasR ? ps.at(b + 1) : ps.at(b);
    PG_MAT(SLL, ts);
    PG_MAT(Snn, ts);
    PG_MAT(SnL, ts);
    ldt<n, NN>(SDo, toff<NN>(qL), SLL);
    ldt<n, NN>(SDo, toff<NN>(qR), Snn);
PG_UNROLL
    for (int e = 0; e < n * n; ++e) {
        SLL[e] = hasL ? SLL[e] : 0.0;
        Snn[e] = hasR ? Snn[e] : 0.0;
    }
    // Cov(R, L) = Cov(L, R)^T, Cov(L, R) = Cov(sep j-1, sep j)
PG_UNROLL
    for (int r = 0; r < n; ++r)
PG_UNROLL
        for (int c = 0; c < n; ++c) SnL[r * n + c] = (hasL && hasR) ? sgv(sg, j - 1, G::NX + c * n + r) : 0.0;
    // forward-sweep blocks of the current state (c) and, loaded one step
    // ahead, of the state below it (n)
    PG_MAT(Pc, ts);
    PG_MAT(Gc, ts);
    PG_MAT(Hc, ts);
    PG_MAT(Pn, ts);
    PG_MAT(Gn, ts);
    PG_MAT(Hn, ts);
    PG_MAT(Kd, ts);  // trace blocks KH_i, KU_i (loaded at the top of step i, used at its end)
    PG_MAT(Ku, ts);
    {
        const uint32_t ob = toff<NN>(ps.at(b));
        ldt_sym<n>(ws.P, ob, Pc);
        ldt<n, NN>(ws.G, ob, Gc);
        ldt<n, NN>(ws.H, ob, Hc);
    }
    for (int i = b; i >= a; --i) {
        TS lt = ts;
        const uint32_t oB = toff<NN>(ps.at(i)), oBp = toff<NN>(ps.at(i > a ? i - 1 : a));
        const bool hasNext = i < b || hasR;
        ldt_sym<n>(ws.P, oBp, Pn);
        ldt<n, NN>(ws.G, oBp, Gn);
        ldt<n, NN>(ws.H, oBp, Hn);
        if (TRACE) {
            ldt<n, NN>(KH, oB, Kd);
            ldt<n, NN>(KU, oB, Ku);
        }
        PG_MAT(Sin, lt);
        PG_MAT(SiL, lt);
        // Sin = -(GU S_nn + HX S_nL^T), SiL = -(GU S_nL + HX S_LL)
        mmul_neg<n>(Gc, Snn, Sin);
        msub_nt<n>(Hc, SnL, Sin);
        mmul_neg<n>(Gc, SnL, SiL);
        msub<n>(Hc, SLL, SiL);
        // Sigma_ii is symmetric: its lower triangle, then the upper one
        msub_nt_lo<n>(Sin, Gc, Pc);
        msub_nt_lo<n>(SiL, Hc, Pc);
        sym_from_lo<n>(Pc);
        stt<n, NN>(SUo, oB, Sin);
        stt<n, NN>(SDo, oB, Pc);
        if (TRACE) {
            const double to = tr_off<n>(Ku, Sin);
            *trace += tr_diag<n>(Kd, Pc) + (hasNext ? to : 0.0);
        }
        mcopy<n>(Pc, Snn);
        mcopy<n>(SiL, SnL);
        mcopy<n>(Pn, Pc);
        mcopy<n>(Gn, Gc);
        mcopy<n>(Hn, Hc);
    }
    if (hasL) {
        // Cov(L, a) = Cov(a, L)^T
        TS lt = ts;
        PG_MAT(T, lt);
PG_UNROLL
        for (int r = 0; r < n; ++r)
PG_UNROLL
            for (int c = 0; c < n; ++c) T[r * n + c] = SnL[c * n + r];
        stt<n, NN>(SUo, toff<NN>(qL), T);
        if (TRACE) {
            ldt<n, NN>(KU, toff<NN>(qL), Ku);
            *trace += tr_off<n>(Ku, T);
        }
    }
}

// Backward substitution of segment j: x_i = P_i^-1 y_i - GU_i x_next - HX_i x_L.
template <int n, bool QUAD>
__device__ __forceinline__ void seg_backward_rhs(int N, int nseg, int j, const Ws& ws, double* sg, double* xo,
                                                 const double* LD, const double* LU, const double* mu0, double* quad,
                                                 TS ts) {
    using G = SegLayout<n, true>;
    constexpr int NN = n * n;
    int a, b;
    bool hasL, hasR;
    seg_bounds(N, nseg, j, a, b, hasL, hasR);
    const SegPos ps = seg_pos(N, nseg, j);
    PG_VEC(xL, ts); PG_VEC(xn, ts);
PG_UNROLL
    for (int e = 0; e < n; ++e) {
        xL[e] = hasL ? sgv(sg, j - 1, G::XS + e) : 0.0;
        xn[e] = hasR ? sgv(sg, j, G::XS + e) : 0.0;
    }
    PG_MAT(Gc, ts);
    PG_MAT(Hc, ts);
    PG_VEC(yc, ts);
    PG_MAT(Gn, ts);
    PG_MAT(Hn, ts);
    PG_VEC(yn, ts);
    ldt<n, NN>(ws.G, toff<NN>(ps.at(b)), Gc);
    ldt<n, NN>(ws.H, toff<NN>(ps.at(b)), Hc);
    ldt<n, n>(ws.Y, toff<n>(ps.at(b)), yc);
    // d of the state after the current one (the right separator first)
    PG_VEC(dn, ts);
    if (QUAD) {
        ldt<n, n>(mu0, toff<n>(hasR ? ps.at(b + 1) : ps.at(b)), dn);
PG_UNROLL
        for (int e = 0; e < n; ++e) dn[e] = hasR ? xn[e] - dn[e] : 0.0;
    }
    PG_MAT(Ld, ts);  // quadratic-term blocks (loaded at the top of step i, used at its end)
    PG_MAT(Lu, ts);
    PG_VEC(m0, ts);
    for (int i = b; i >= a; --i) {
        TS lt = ts;
        const uint32_t q = ps.at(i), qp = ps.at(i > a ? i - 1 : a);
        const uint32_t oBp = toff<NN>(qp), oVp = toff<n>(qp);
        const bool hasNext = i < b || hasR;
        ldt<n, NN>(ws.G, oBp, Gn);
        ldt<n, NN>(ws.H, oBp, Hn);
        ldt<n, n>(ws.Y, oVp, yn);
        if (QUAD) {
            ldt<n, NN>(LD, toff<NN>(q), Ld);
            ldt<n, NN>(LU, toff<NN>(q), Lu);
            ldt<n, n>(mu0, toff<n>(q), m0);
        }
        PG_VEC(x, lt);
PG_UNROLL
        for (int e = 0; e < n; ++e) x[e] = yc[e];
        mvec_sub<n>(Gc, xn, x);
        mvec_sub<n>(Hc, xL, x);
        stt<n, n>(xo, toff<n>(q), x);
        if (QUAD) {
            PG_VEC(d, lt);
PG_UNROLL
            for (int e = 0; e < n; ++e) d[e] = x[e] - m0[e];
            const double cross = 2.0 * quad_form<n>(Lu, d, dn);
            *quad += quad_form<n>(Ld, d, d) + (hasNext ? cross : 0.0);
PG_UNROLL
            for (int e = 0; e < n; ++e) dn[e] = d[e];
        }
PG_UNROLL
        for (int e = 0; e < n; ++e) xn[e] = x[e];
        mcopy<n>(Gn, Gc);
        mcopy<n>(Hn, Hc);
PG_UNROLL
        for (int e = 0; e < n; ++e) yc[e] = yn[e];
    }
    if (QUAD && hasL) {
        // 2 d_L^T LU_L d_a, L = left separator, a = first state (d_a in dn)
        const uint32_t qL = sep_pos(N, nseg, j - 1);
        TS lt = ts;
        PG_VEC(dL, lt);
        ldt<n, NN>(LU, toff<NN>(qL), Lu);
        ldt<n, n>(mu0, toff<n>(qL), dL);
PG_UNROLL
        for (int e = 0; e < n; ++e) dL[e] = xL[e] - dL[e];
        *quad += 2.0 * quad_form<n>(Lu, dL, dn);
    }
}

// Workgroup-wide GBP of the matrix in M into (SDo, SUo), log det
// and PD flag; all arrays offset to the plan's chain range.  Called by every
// lane of the half (tid = lane); sh_ld / sh_ok hold kChainThreads + 1 entries.
template <int n, bool TRACE>
__device__ __forceinline__ bool wg_gbp(const BlockSrc& M, const Ws& ws, int tid, int N, int nseg, double* sg,
                                       double* SDo, double* SUo, double* logdet_out, double* sh_ld, int* sh_ok,
                                       double* trace, TS ts) {
    const int m = nseg - 1;
    double ld = 0.0;
    bool ok = true;
    if (tid < nseg) ok = seg_forward<n, false>(M, N, nseg, tid, ws, sg, &ld, ts);
    __syncthreads();
    {
        TS at = ts;
        PG_MAT(A, at);
        PG_MAT(C, at);
        PG_VEC(r, at);
        if (tid < m) cr_assemble_read<n, false>(M, N, nseg, tid, sg, A, C, r);
        __syncthreads();
        if (tid < m) cr_assemble_write<n, false>(tid, sg, A, C, r);
    }
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
    cr_backward_cov<n, TRACE>(m, tid, okall, N, nseg, sg, SDo, M.D0, trace, ts);
    if (okall && tid < nseg) seg_backward_cov<n, TRACE>(N, nseg, tid, ws, sg, SDo, SUo, M.D0, M.U0, trace, ts);
    __syncthreads();
    return okall;
}

// Workgroup-wide solve of (D, U) x = r into xo (same barriers as wg_gbp).
template <int n, bool QUAD>
__device__ __forceinline__ bool wg_solve(const BlockSrc& M, const Ws& ws, int tid, int N, int nseg, double* sg,
                                         double* xo, int* sh_ok, const double* mu0, double* quad, TS ts) {
    const int m = nseg - 1;
    double ld = 0.0;
    bool ok = true;
    if (tid < nseg) ok = seg_forward<n, true>(M, N, nseg, tid, ws, sg, &ld, ts);
    __syncthreads();
    {
        TS at = ts;
        PG_MAT(A, at);
        PG_MAT(C, at);
        PG_VEC(r, at);
        if (tid < m) cr_assemble_read<n, true>(M, N, nseg, tid, sg, A, C, r);
        __syncthreads();
        if (tid < m) cr_assemble_write<n, true>(tid, sg, A, C, r);
    }
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
    cr_backward_rhs<n, QUAD>(m, tid, okall, N, nseg, sg, xo, M.D1, mu0, quad, ts);
    if (okall && tid < nseg) seg_backward_rhs<n, QUAD>(N, nseg, tid, ws, sg, xo, M.D1, M.U1, mu0, quad, ts);
    __syncthreads();
    return okall;
}

// Entries per staged chunk of the per-state copies (all loads of a chunk,
// then its stores).
template <int NN>
constexpr int kCopyChunk = NN < 16 ? NN : 16;

// Position of state coordinate r among the plan's collision coordinates, or -1.
__device__ __forceinline__ int coll_slot(const PlanDev& p, int r) {
    int a = -1;
    for (int t = 0; t < p.d; ++t) a = p.coll_index[t] == r ? t : a;
    return a;
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
    double* base = st.tws + (((int64_t)pid * st.W + t) * kTrialThreads + threadIdx.x) * st.tws_stride;
    return TS{base, base + st.tws_stride, st.flags};
}
}  // namespace pg
#include "coop.h"
namespace pg {

// Block temporaries of the chain and trial kernels in LDS (n = 6, plans of
// at most kLdsWsSegments segments): a slice of STRIDE doubles per lane of
// both halves, the stride odd so that the lanes of a wave spread over the
// banks.  Lanes past the slices (they run no sweep and no reduced-chain
// work) and plans of more segments keep their workspace slices in HBM.
template <int n>
struct LdsWs {
    static constexpr bool value = n == 6 && !Coop<n>::value;
    static constexpr int STRIDE = (kTwsBlocks * n * n + kTwsVecs * n) | 1;
    static constexpr int size = value ? 2 * kLdsWsSegments * STRIDE : 1;
};
template <int n>
__device__ __forceinline__ TS chain_ws(const DevState& st, double* lds, int pid, int t, int half, int lane,
                                       int nseg) {
    if (LdsWs<n>::value && nseg <= kLdsWsSegments && lane < kLdsWsSegments) {
        double* base = lds + (half * kLdsWsSegments + lane) * LdsWs<n>::STRIDE;
        return TS{base, base + LdsWs<n>::STRIDE, st.flags};
    }
    return thread_ws<n>(st, pid, t);
}

// Sweep temporaries of one half for the chain range starting at position c0
// (trial slot included): four tiled arrays of W * Sc positions each.
template <int n>
__device__ __forceinline__ Ws sweep_ws(const DevState& st, int half, int64_t c0) {
    const int64_t cap = (int64_t)st.W * st.Sc;
    double* base = st.ws + (int64_t)half * (3 * n * n + n) * cap;
    return Ws{base + c0 * n * n, base + cap * n * n + c0 * n * n, base + 2 * cap * n * n + c0 * n * n,
              base + 3 * cap * n * n + c0 * n};
}

// Set-up and marginals of a plan (trial slot 0 of its scratch):
// CHAIN_INIT: Lambda = K^-1, mean = solve(K^-1, eta), marginals, budget reset;
// CHAIN_REINIT: Lambda = K^-1 (mean kept), marginals;
// CHAIN_MARGINALS: marginals of the current Lambda.
// The inputs are first copied into chain order, the results (trial slot 0)
// are copied back in state order.  CHAIN_INIT runs with two wavefronts:
// wave 0 computes the marginals while wave 1 solves for the mean; the other
// modes run with one.
template <int n>
__global__ void __launch_bounds__(Coop<n>::value ? Coop<n>::THREADS : kTrialThreads)
    chain_kernel(DevState st, int mode, int plan_lo) {
    __shared__ double sh_d[kChainThreads + 1];
    __shared__ int sh_i[kChainThreads + 1];
    __shared__ int sh_j[kChainThreads + 1];
    constexpr int NN = n * n;
    const int pid = plan_lo + blockIdx.x;
    PlanDev& p = st.plans[pid];
    if (!p.active) return;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int half = tid / kChainThreads, lane = tid % kChainThreads;
    const int N = p.N, nseg = p.nseg;
    const int64_t off = p.off, S = st.S, coff = p.coff;
    __shared__ double sg_lds[NodeLds<n>::size];
    __shared__ double ws_lds[LdsWs<n>::size];
    double* sg = NodeLds<n>::value ? sg_lds + half * kMaxSeg * SegLayout<n, false>::STRIDE : seg_scratch<n>(st, pid, 0, half);
    const Ws ws = sweep_ws<n>(st, half, coff);
    TS ts = chain_ws<n>(st, ws_lds, pid, 0, half, lane, nseg);
    const bool prior = mode == CHAIN_INIT || mode == CHAIN_REINIT;
    // precision to factor (K^-1 or the current Lambda) in chain order
    double* cD = prior ? st.cKD : st.cLD;
    double* cU = prior ? st.cKU : st.cLU;
    const double* sD = prior ? st.KD : st.LD;
    const double* sU = prior ? st.KU : st.LU;
    for (int i = tid; i < N; i += nt) {
        const int64_t s = off + i, q = coff + chain_pos(N, nseg, i);
        const bool notlast = i < N - 1;
        for (int e0 = 0; e0 < NN; e0 += kCopyChunk<NN>) {
            // every load of the chunk before its stores (see prep_kernel)
            constexpr int CH = kCopyChunk<NN>;
            double dv[CH], uv[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int e = min(e0 + k, NN - 1);
                dv[k] = sD[e * S + s];
                // the coupling after the chain's last state is a zero block
                uv[k] = notlast ? sU[e * S + s] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int e = e0 + k;
                if (e >= NN) break;
                cD[tidx<NN>(q, e)] = dv[k];
                cU[tidx<NN>(q, e)] = uv[k];
                if (prior) {
                    // K^-1 + H outside the collision blocks: K^-1 until the
                    // next prior build (prep writes the collision blocks)
                    st.cKH[tidx<NN>(q, e)] = dv[k];
                    st.LD[e * S + s] = dv[k];
                    if (notlast) st.LU[e * S + s] = uv[k];
                }
            }
        }
        if (mode == CHAIN_INIT) {
            double r[n];
#pragma unroll
            for (int e = 0; e < n; ++e) r[e] = st.eta[e * S + s];
#pragma unroll
            for (int e = 0; e < n; ++e) st.crb[tidx<n>(q, e)] = r[e];
        }
    }
    __syncthreads();
    if constexpr (Coop<n>::value) {
        // one wavefront per matrix: marginals on wave 0, the mean on wave 1
        __shared__ double c_lds[2 * Coop<n>::WAVE_LDS];
        __shared__ double c_sh[Coop<n>::THREADS + 4];
        const double *d = cD + coff * NN, *u = cU + coff * NN;
        const BlockSrc MT{d, d, u, u, d, d, 1.0, 0.0};
        const double *kd = st.cKD + coff * NN, *ku = st.cKU + coff * NN, *r = st.crb + coff * n;
        const BlockSrc MM{kd, kd, ku, ku, r, r, 1.0, 0.0};
        coop_chain<n>(MT, MM, mode == CHAIN_INIT, N, sweep_ws<n>(st, 0, coff), sweep_ws<n>(st, 1, coff),
                      st.TSD + coff * NN, st.TSU + coff * NN, st.Tmu + coff * n, nullptr, nullptr, nullptr, c_lds,
                      c_sh);
        if (tid == 0) {
            sh_d[kChainThreads] = c_sh[0];
            sh_i[kChainThreads] = c_sh[1] != 0.0 ? 1 : 0;
        }
    } else if (half == 0) {
        const double *d = cD + coff * NN, *u = cU + coff * NN;
        BlockSrc M{d, d, u, u, d, d, 1.0, 0.0};
        double ld = 0.0;
        wg_gbp<n, false>(M, ws, lane, N, nseg, sg, st.TSD + coff * NN, st.TSU + coff * NN, &ld, sh_d, sh_i, nullptr,
                         ts);
    } else {
        const double *kd = st.cKD + coff * NN, *ku = st.cKU + coff * NN, *r = st.crb + coff * n;
        BlockSrc M{kd, kd, ku, ku, r, r, 1.0, 0.0};
        wg_solve<n, false>(M, ws, lane, N, nseg, sg, st.Tmu + coff * n, sh_j, nullptr, nullptr, ts);
    }
    __syncthreads();
    const bool ok = sh_i[kChainThreads] != 0;
    if (tid == 0) {
        p.logdet = ok ? sh_d[kChainThreads] : NAN;
        p.status = ok ? 0 : PGVIMP_ENOTPD;
        if (mode == CHAIN_INIT) {
            p.iters_left = p.n_iters;
            p.iters_done = 0;
            p.trials_total = 0;
            p.evals_total = 0;
        }
    }
    for (int i = tid; i < N; i += nt) {
        const int64_t s = off + i, q = coff + chain_pos(N, nseg, i);
        const bool notlast = i < N - 1;
        if (ok) {
            for (int e0 = 0; e0 < NN; e0 += kCopyChunk<NN>) {
                constexpr int CH = kCopyChunk<NN>;
                double dv[CH], uv[CH];
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const int e = min(e0 + k, NN - 1);
                    dv[k] = st.TSD[tidx<NN>(q, e)];
                    uv[k] = notlast ? st.TSU[tidx<NN>(q, e)] : 0.0;
                }
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const int e = e0 + k;
                    if (e >= NN) break;
                    st.SD[e * S + s] = dv[k];
                    if (notlast) st.SU[e * S + s] = uv[k];
                }
            }
        }
        if (mode == CHAIN_INIT) {
            double m[n];
#pragma unroll
            for (int e = 0; e < n; ++e) m[e] = st.Tmu[tidx<n>(q, e)];
#pragma unroll
            for (int e = 0; e < n; ++e) st.mu[e * S + s] = m[e];
        }
    }
}

// Sum over the block in a fixed order (sh holds blockDim.x + 1 doubles).
__device__ __forceinline__ double block_sum(double v, double* sh) { return wg_sum(v, sh); }

// Row e of state i's right-hand side eta - g (eta - g + H mu_k for the
// natural-gradient step), of mu_k and of Lambda_k mu_k = D_i mu_i + U_i
// mu_{i+1} + U_{i-1}^T mu_{i-1}, the blocks read straight from memory (for
// n >= 6, one thread per (state, row)).
template <int n>
__device__ __forceinline__ void prep_rhs_row(const DevState& st, const PlanDev& p, int i, int e, int64_t s,
                                             int64_t q, bool act) {
    const int64_t S = st.S;
    const int N = p.N, d = p.d;
    double r = st.eta[e * S + s];
    if (act) {
        for (int a = 0; a < d; ++a) {
            const double ga = st.gcol[a * S + s];
            const int ca = p.coll_index[a];
            double h = 0.0;
            if (p.update == PGVIMP_UPDATE_NGD) {
                for (int b = 0; b < d; ++b)
                    h = fma(st.Hcol[(a * d + b) * S + s], st.mu[(int64_t)p.coll_index[b] * S + s], h);
            }
            r += e == ca ? h - ga : 0.0;
        }
    }
    double m[n];
#pragma unroll
    for (int c = 0; c < n; ++c) m[c] = st.mu[c * S + s];
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < n; ++c) acc = fma(st.LD[(e * n + c) * S + s], m[c], acc);
    if (i < N - 1) {
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < n; ++c) t = fma(st.LU[(e * n + c) * S + s], st.mu[c * S + s + 1], t);
        acc += t;
    }
    if (i > 0) {
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < n; ++c) t = fma(st.LU[(c * n + e) * S + s - 1], st.mu[c * S + s - 1], t);
        acc += t;
    }
    st.crb[tidx<n>(q, e)] = r;
    st.cmu[tidx<n>(q, e)] = m[e];
    st.cLmu[tidx<n>(q, e)] = acc;
}

// One proximal iteration (Alg. 1), part 1: per-state quantities shared by all
// trial step sizes, written in chain order -- KH = K^-1 + H (collision
// Hessians on the diagonal blocks), rb = eta - g (eta - g + H mu_k for the
// natural-gradient step), Lmu = Lambda_k mu_k, and
// copies of K^-1, Lambda_k and mu_k -- and the expected costs (per-block
// partial sums; the select kernel adds them in block order).
// Grid (plans, iter_blocks), kIterThreads threads, grid-stride over states.
template <int n>
__global__ void __launch_bounds__(kIterThreads) prep_kernel(DevState st) {
    __shared__ double sh_d[kIterThreads + 1];
    constexpr int NN = n * n;
    const int pid = blockIdx.x, y = blockIdx.y, nb = gridDim.y;
    PlanDev& p = st.plans[pid];
    if (!p.active) return;
    const int tid = threadIdx.x;
    if (p.iters_left <= 0) {
        if (y == 0 && tid == 0) p.phase = 1;
        return;
    }
    const int N = p.N, d = p.d, nseg = p.nseg;
    const int64_t off = p.off, S = st.S, coff = p.coff;
    TS ts = thread_ws<n>(st, pid, y);
    double ecol = 0.0, epri = 0.0;
    // Each group's loads come before its stores (the stores go to other
    // arrays, but the compiler cannot know that): Lambda_k's blocks and the
    // collision blocks of K^-1 + H, then the right-hand side eta - g and
    // Lambda_k mu_k, then the prior costs.  K^-1 itself and K^-1 + H outside
    // the collision blocks are written by the set-up chain kernel after every
    // prior build (K^-1 does not change between builds).  For n >= 6 the
    // copies are spread over (state, chunk of entries) and the right-hand
    // sides over (state, row), states fastest, so a state's many loads are
    // not one thread's chain of waits.
    constexpr int CPS = Coop<n>::value ? (NN + kCopyChunk<NN> - 1) / kCopyChunk<NN> : 1;
    for (int w = y * kIterThreads + tid; w < N * CPS; w += nb * kIterThreads) {
        const int i = w % N;
        const int64_t s = off + i, q = coff + chain_pos(N, nseg, i);
        const bool act = coll_active<n>(p, i);
        const bool notlast = i < N - 1;
        const int c_lo = Coop<n>::value ? (w / N) * kCopyChunk<NN> : 0;
        const int c_hi = Coop<n>::value ? c_lo + kCopyChunk<NN> : NN;
        for (int e0 = c_lo; e0 < c_hi && e0 < NN; e0 += kCopyChunk<NN>) {
            constexpr int CH = kCopyChunk<NN>;
            double kh[CH], ld[CH], lu[CH];
            bool ce[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int e = min(e0 + k, NN - 1);
                ld[k] = st.LD[e * S + s];
                // the coupling after the chain's last state is a zero block
                lu[k] = notlast ? st.LU[e * S + s] : 0.0;
                // collision Hessian on the collision coordinates
                const int a = coll_slot(p, e / n), b2 = coll_slot(p, e % n);
                ce[k] = act && a >= 0 && b2 >= 0;
                kh[k] = ce[k] ? st.KD[e * S + s] + st.Hcol[(a * d + b2) * S + s] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int e = e0 + k;
                if (e >= NN) break;
                const int64_t qe = tidx<NN>(q, e);
                if (ce[k]) st.cKH[qe] = kh[k];
                st.cLD[qe] = ld[k];
                st.cLU[qe] = lu[k];
            }
        }
        if constexpr (Coop<n>::value) continue;
        TS lt = ts;
        PG_VEC(r, lt);
        ld_vec<n>(st.eta, S, s, r);
        if (act) {
            ecol += st.Ecol[s];
            for (int a = 0; a < d; ++a) {
                const double ga = st.gcol[a * S + s];
                const int ca = p.coll_index[a];
PG_UNROLL
                for (int e = 0; e < n; ++e) r[e] -= e == ca ? ga : 0.0;  // static indexing keeps r in registers
            }
        }
        PG_MAT(Dm, lt);
        PG_MAT(Um, lt);
        PG_MAT(Up, lt);
        PG_VEC(m, lt);
        PG_VEC(mn, lt);
        PG_VEC(mp, lt);
        PG_VEC(t, lt);
        PG_VEC(acc, lt);
        ld_soa<n>(st.LD, S, s, Dm);
        ld_vec<n>(st.mu, S, s, m);
        if (p.update == PGVIMP_UPDATE_NGD && act) {
            // natural-gradient step: H mu_k on the collision coordinates
            for (int a = 0; a < d; ++a) {
                double h = 0.0;
                for (int b = 0; b < d; ++b) {
                    const int cb = p.coll_index[b];
                    double mb = 0.0;
PG_UNROLL
                    for (int e = 0; e < n; ++e) mb = e == cb ? m[e] : mb;
                    h = fma(st.Hcol[(a * d + b) * S + s], mb, h);
                }
                const int ca = p.coll_index[a];
PG_UNROLL
                for (int e = 0; e < n; ++e) r[e] += e == ca ? h : 0.0;
            }
        }
        if (notlast) {
            ld_soa<n>(st.LU, S, s, Um);
            ld_vec<n>(st.mu, S, s + 1, mn);
        }
        if (i > 0) {
            ld_soa<n>(st.LU, S, s - 1, Up);
            ld_vec<n>(st.mu, S, s - 1, mp);
        }
        mvec<n>(Dm, m, acc);
        if (notlast) {
            mvec<n>(Um, mn, t);
PG_UNROLL
            for (int e = 0; e < n; ++e) acc[e] += t[e];
        }
        if (i > 0) {
PG_UNROLL
            for (int e = 0; e < n; ++e) t[e] = 0.0;
            mvec_tn_sub<n>(Up, mp, t);
PG_UNROLL
            for (int e = 0; e < n; ++e) acc[e] -= t[e];
        }
PG_UNROLL
        for (int e = 0; e < n; ++e) {
            st.crb[tidx<n>(q, e)] = r[e];
            st.cmu[tidx<n>(q, e)] = m[e];
            st.cLmu[tidx<n>(q, e)] = acc[e];
        }
        epri += prior_cost_state<n>(st, p, i, nullptr, nullptr, nullptr, lt);
    }
    if constexpr (Coop<n>::value) {
        // n >= 6: right-hand sides per (state, row), collision costs per
        // thread, prior costs one wavefront per state
        for (int w = y * kIterThreads + tid; w < N * n; w += nb * kIterThreads) {
            const int i = w % N;
            prep_rhs_row<n>(st, p, i, w / N, off + i, coff + chain_pos(N, nseg, i), coll_active<n>(p, i));
        }
        for (int i = y * kIterThreads + tid; i < N; i += nb * kIterThreads)
            if (coll_active<n>(p, i)) ecol += st.Ecol[off + i];
        __shared__ double p_lds[(kIterThreads / 64) * Coop<n>::WAVE_LDS];
        const int wave = tid / 64, lane = tid % 64;
        for (int i = y * (kIterThreads / 64) + wave; i < N; i += nb * (kIterThreads / 64)) {
            double o[3];
            coop_prior_cost<n>(st, p, i, p_lds + wave * Coop<n>::WAVE_LDS, lane, o);
            if (lane == 0) epri += o[0] + o[1] + o[2];
        }
    }
    ecol = block_sum(ecol, sh_d);
    epri = block_sum(epri, sh_d);
    // Window 0 of the step sizes (no lookahead): the same width for every
    // plan with an iteration to run, the compute units shared among them;
    // wlist[0] = -width tells the trial kernel to take its items as
    // (plan, slot) = (j / width, j % width).
    int live = 0;
    if (y == 0 && st.lookahead == 0)
        for (int q = tid; q < (int)gridDim.x; q += kIterThreads) live += st.plans[q].active && st.plans[q].iters_left > 0;
    const double nlive = (y == 0 && st.lookahead == 0) ? block_sum((double)live, sh_d) : 0.0;
    if (tid == 0) {
        st.psum[((int64_t)pid * nb + y) * 2 + 0] = ecol;
        st.psum[((int64_t)pid * nb + y) * 2 + 1] = epri;
        if (y == 0) {
            if (st.lookahead == 0) {
                const int w0 = max(st.Wmin, min(st.W, st.wbudget / max((int)nlive, 1)));
                p.wstart = 0;
                p.wwidth = min(w0, p.max_bisect);
                p.wnext = p.wwidth;
                p.firstpass = kNoPass;
                st.wlist[0] = -w0;  // the same value from every plan
            }
            p.phase = 0;
        }
    }
}

// Part 2: one trial step size per workgroup, item j of the window's work
// list (plan, slot), or of the uniform first window set by the prep kernel:
// step size number wstart + slot of the plan's current window.  Workgroup b
// runs on XCD b mod 8.  From a list it takes item (b mod 8) * C + b / 8,
// C = ceil(items / 8): each XCD gets an equal run of the plan-ordered list,
// so a plan's trials share one or two L2s.  In the uniform window, plan q
// runs on XCD q mod 8 (live plans spread over the XCDs even when they hold
// neighbouring slots of a larger context).
// For that step size (Theorem 1):
//   Lambda' = (beta (K^-1 + H) + Lambda_k) / (beta T + 1)  -> marginals, log det, PD
//   (K^-1 + Lambda_k / beta) mu' = eta - g + Lambda_k mu_k / beta
//   KL(q' || q_k) = 1/2 [beta (T dim - tr((K^-1 + H) Sigma')) + dmu^T Lambda_k dmu
//                        + log det Lambda' - log det Lambda_k]
// (the trace term uses Lambda_k = (beta T + 1) Lambda' - beta (K^-1 + H) and
// tr(Lambda' Sigma') = dim).  The natural-gradient step (Sec. 3.1(d)) takes
//   Lambda' = (1 - beta T) Lambda_k + beta (K^-1 + H)
//   (K^-1 + H + (1 / beta - T) Lambda_k) mu' = eta - g + H mu_k + (1 / beta - T) Lambda_k mu_k
// and the trace term beta (T dim - tr((K^-1 + H) Sigma')) / (1 - beta T)
// (Lambda_k = (Lambda' - beta (K^-1 + H)) / (1 - beta T)), or where
// |1 - beta T| < 1/4 the plain tr(Lambda_k Sigma') - dim, Lambda' then
// hardly involving Lambda_k.  Results go to the trial slot (chain order) and
// st.tres (passed, KL, log det, slot).  PAD: see the node scratch below.
template <int n, bool PAD>
__global__ void __launch_bounds__(Coop<n>::value ? Coop<n>::THREADS : kTrialThreads)
    trial_kernel(DevState st, int phw) {
    // work list, or (wlist[0] = -w) the uniform first window of width w
    const int head = st.wlist[0];
    const int kx = (int)blockIdx.x / kNumXcd, x = (int)blockIdx.x % kNumXcd;
    int item;
    if (head < 0) {
        // plan q on XCD q mod 8 with its w slots together, whichever plan
        // slots are live
        const int w = -head, q = x + kNumXcd * (kx / w);
        if (q >= phw) return;
        item = q * 64 + kx % w;
    } else {
        const int items = head;
        const int chunk = (items + kNumXcd - 1) / kNumXcd;
        const int j = x * chunk + kx;
        if (kx >= chunk || j >= items) return;
        item = st.wlist[1 + j];
    }
    constexpr int NN = n * n;
    const int pid = item >> 6, t = item & 63;
    const PlanDev& p = st.plans[pid];
    if (!p.active || p.phase != 0 || t >= p.wwidth) return;
    const int tt = p.wstart + t;
    const int tid = threadIdx.x;
    const int N = p.N, nseg = p.nseg;
    const int64_t coff = p.coff, c0 = (int64_t)t * st.Sc + coff;
    double* res = st.tres + ((int64_t)pid * kMaxBisect + tt) * 4;
    const double beta = ldexp(p.beta_max, -tt);
    const double T = p.temperature;
    const double c = 1.0 / fma(beta, T, 1.0);
    const bool ngd = p.update == PGVIMP_UPDATE_NGD;
    const double omt = fma(-beta, T, 1.0);  // 1 - beta T
    const bool plain = ngd && fabs(omt) < 0.25;
    // views of the plan's inputs and of this trial slot's outputs
    const double *kh = st.cKH + coff * NN, *kd = st.cKD + coff * NN, *lD = st.cLD + coff * NN;
    const double *ku = st.cKU + coff * NN, *lU = st.cLU + coff * NN;
    const double *rb = st.crb + coff * n, *lmu = st.cLmu + coff * n, *cmu = st.cmu + coff * n;
    double *tsd = st.TSD + c0 * NN, *tsu = st.TSU + c0 * NN, *tmu = st.Tmu + c0 * n;
    // the trial precision (its trace term reads the first source: K^-1 + H,
    // or Lambda_k for the plain form) and the mean system
    const BlockSrc MT = plain ? BlockSrc{lD, kh, lU, ku, lD, kh, omt, beta}
                        : ngd ? BlockSrc{kh, lD, ku, lU, kh, lD, beta, omt}
                              : BlockSrc{kh, lD, ku, lU, kh, lD, c * beta, c};
    const BlockSrc MM = ngd ? BlockSrc{kh, lD, ku, lU, rb, lmu, 1.0, 1.0 / beta - T}
                            : BlockSrc{kd, lD, ku, lU, rb, lmu, 1.0, 1.0 / beta};
    bool pd;
    double ld_trial, trKH, quad;
    if constexpr (Coop<n>::value) {
        __shared__ double c_lds[2 * Coop<n>::WAVE_LDS];
        __shared__ double c_sh[Coop<n>::THREADS + 4];
        coop_chain<n>(MT, MM, true, N, sweep_ws<n>(st, 0, c0), sweep_ws<n>(st, 1, c0), tsd, tsu, tmu, cmu, MT.D0,
                      MT.U0, c_lds, c_sh);
        pd = c_sh[1] != 0.0;
        ld_trial = c_sh[0];
        trKH = c_sh[2];
        quad = c_sh[3];
    } else {
        __shared__ double sh_d[kChainThreads + 1];
        __shared__ int sh_i[kChainThreads + 1];
        __shared__ int sh_j[kChainThreads + 1];
        const int half = tid / kChainThreads, lane = tid % kChainThreads;
        // With LDS node scratch a trial workgroup takes just under half a CU's
        // LDS; with PAD, kTrialLdsPad unused bytes keep it to one workgroup per
        // CU.  Two per CU run each other ~1.5x slower, and the dispatcher pairs
        // them up even in windows smaller than the chip; only windows of more
        // workgroups than CUs gain from pairs (1.12x the throughput).
        __shared__ double sg_lds[NodeLds<n>::size + (NodeLds<n>::value && PAD ? kTrialLdsPad / 8 : 0)];
        double* sg = NodeLds<n>::value ? sg_lds + half * kMaxSeg * SegLayout<n, false>::STRIDE
                                       : seg_scratch<n>(st, pid, t, half);
        const Ws ws = sweep_ws<n>(st, half, c0);
        __shared__ double ws_lds[LdsWs<n>::size];
        TS ts = chain_ws<n>(st, ws_lds, pid, t, half, lane, nseg);
        // wave 0: marginals and PD test of the trial precision, with the trace
        // term; wave 1: trial mean, with the quadratic term.  Both helpers pass
        // the same workgroup barriers.
        // per-lane KL partial sums; with LDS node scratch they reuse it (both
        // helpers end with a barrier after their last scratch access)
        __shared__ double sh_t_own[NodeLds<n>::value ? 1 : kTrialThreads];
        double* sh_t = NodeLds<n>::value ? sg_lds : sh_t_own;
        double part = 0.0, ld = 0.0;
        if (half == 0)
            wg_gbp<n, true>(MT, ws, lane, N, nseg, sg, tsd, tsu, &ld, sh_d, sh_i, &part, ts);
        else
            wg_solve<n, true>(MM, ws, lane, N, nseg, sg, tmu, sh_j, cmu, &part, ts);
        sh_t[tid] = part;
        __syncthreads();
        pd = sh_i[kChainThreads] != 0;
        ld_trial = sh_d[kChainThreads];
        // partial sums in lane order: trace from wave 0, quadratic from wave 1
        trKH = 0.0;
        quad = 0.0;
        if (tid == 0) {
            for (int k = 0; k < kChainThreads; ++k) trKH += sh_t[k];
            for (int k = 0; k < kChainThreads; ++k) quad += sh_t[kChainThreads + k];
        }
    }
    if (tid == 0) {
        if (!pd) {
            res[0] = 0.0;
            res[1] = NAN;
            res[2] = NAN;
            res[3] = t;
        } else {
            res[0] = 1.0;
            const double tk = beta * (T * (double)N * n - trKH);
            const double trace = plain ? trKH - (double)N * n : ngd ? tk / omt : tk;
            res[1] = 0.5 * (trace + quad + ld_trial - p.logdet);
            res[2] = ld_trial;
            res[3] = t;
            if (res[1] <= p.kl_bound) atomicMin(&st.plans[pid].firstpass, tt);
        }
    }
}

// Part 3 (after the last window): take the first passing step size in
// halving order and write its trial back, in state order, as the new
// iterate; a plan with no passing step keeps its state (ENOCONV).  The
// windows cover step sizes 0 .. wnext-1 of this iteration without gaps and
// stop after the first passing one, so the scan reads only this
// iteration's results.  Grid (plans,
// iter_blocks): every block finds the same pick and copies its share of the
// states; block 0 does the bookkeeping.
template <int n>
__global__ void __launch_bounds__(kIterThreads) select_kernel(DevState st, int /*unused*/) {
    constexpr int NN = n * n;
    const int pid = blockIdx.x, y = blockIdx.y, nb = gridDim.y;
    PlanDev& p = st.plans[pid];
    if (!p.active || p.phase != 0) return;
    const int tid = threadIdx.x;
    const double* tr = st.tres + (int64_t)pid * kMaxBisect * 4;
    const int evaluated = p.wnext;
    const int pick = p.firstpass != kNoPass ? p.firstpass : -1;
    const double last_kl = evaluated > 0 ? tr[4 * (evaluated - 1) + 1] : NAN;
    // trial slot of step size number pick: its position in its window
    const int slot = pick >= 0 ? (int)tr[4 * pick + 3] : 0;
    const int N = p.N, nseg = p.nseg;
    const int64_t S = st.S, off = p.off, coff = p.coff;
    double beta = 0.0, kl = last_kl, ld = 0.0;
    if (pick >= 0) {
        const double* res = tr + 4 * pick;
        beta = ldexp(p.beta_max, -pick);
        kl = res[1];
        ld = res[2];
        // the trial's precision, with the same operations as the trial kernel
        const bool ngd = p.update == PGVIMP_UPDATE_NGD;
        const double c = 1.0 / fma(beta, p.temperature, 1.0);
        const double omt = fma(-beta, p.temperature, 1.0);
        const bool plain = ngd && fabs(omt) < 0.25;
        const double a0 = plain ? omt : ngd ? beta : c * beta, a1 = plain ? beta : ngd ? omt : c;
        for (int i = y * kIterThreads + tid; i < N; i += nb * kIterThreads) {
            const int64_t s = off + i, qs = coff + chain_pos(N, nseg, i), q = (int64_t)slot * st.Sc + qs;
            const bool notlast = i < N - 1;
            for (int e0 = 0; e0 < NN; e0 += kCopyChunk<NN>) {
                // every load of the chunk before its stores (see prep_kernel)
                constexpr int CH = kCopyChunk<NN>;
                double kh[CH], ld[CH], sd[CH], ku[CH], lu[CH], su[CH];
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const int e = min(e0 + k, NN - 1);
                    kh[k] = st.cKH[tidx<NN>(qs, e)];
                    ld[k] = st.LD[e * S + s];
                    sd[k] = st.TSD[tidx<NN>(q, e)];
                    ku[k] = notlast ? st.KU[e * S + s] : 0.0;
                    lu[k] = notlast ? st.LU[e * S + s] : 0.0;
                    su[k] = notlast ? st.TSU[tidx<NN>(q, e)] : 0.0;
                }
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const int e = e0 + k;
                    if (e >= NN) break;
                    st.LD[e * S + s] = plain ? lin2(a0, ld[k], a1, kh[k]) : lin2(a0, kh[k], a1, ld[k]);
                    st.SD[e * S + s] = sd[k];
                    if (notlast) {
                        st.LU[e * S + s] = plain ? lin2(a0, lu[k], a1, ku[k]) : lin2(a0, ku[k], a1, lu[k]);
                        st.SU[e * S + s] = su[k];
                    }
                }
            }
            double m[n];
#pragma unroll
            for (int e = 0; e < n; ++e) m[e] = st.Tmu[tidx<n>(q, e)];
#pragma unroll
            for (int e = 0; e < n; ++e) st.mu[e * S + s] = m[e];
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
        // J(q_k) = E[psi] - T H(q_k), with H(q_k) from the log det before the update
        const double h_k = 0.5 * (double)N * n * (1.0 + 1.8378770664093453) - 0.5 * p.logdet;
        p.iter_temperature = p.temperature;
        p.entropy_cost = -p.temperature * h_k;
        p.total_cost = epri + ecol + p.entropy_cost;
        p.trials = pick >= 0 ? pick + 1 : p.max_bisect;
        p.trials_total += p.trials;
        // step sizes evaluated: every window up to the one holding the pick
        p.evals_total += evaluated;
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
    }
}

// per-factor prior costs for output: trans at off+i, goal at off+N-1, start at S+plan
template <int n>
__global__ void __launch_bounds__(kChainThreads) prior_cost_kernel(DevState st, int plan) {
    const PlanDev& p = st.plans[plan];
    if constexpr (Coop<n>::value) {
        // n >= 6: one wavefront, state by state
        __shared__ double lds[Coop<n>::WAVE_LDS];
        const int lane = threadIdx.x;
        for (int i = 0; i < p.N; ++i) {
            double o[3];
            coop_prior_cost<n>(st, p, i, lds, lane, o);
            if (lane == 0) {
                if (i < p.N - 1) st.Epri[p.off + i] = o[0];
                if (i == p.N - 1) st.Epri[p.off + i] = o[2];
                if (i == 0) st.Epri[st.S + plan] = o[1];
            }
        }
        return;
    }
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
    const int threads = Coop<n>::value ? Coop<n>::THREADS : mode == CHAIN_INIT ? kTrialThreads : kChainThreads;
    hipLaunchKernelGGL(chain_kernel<n>, dim3(hi - lo), dim3(threads), 0, s, st, mode, lo);
    return hipGetLastError();
}

// part: 0 = prep, 1 = trial (each plan's current window), 2 = select,
// 5 = trial allowing two workgroups per CU (windows larger than the chip)
template <int n>
hipError_t launch_iteration_n(const DevState& st, int phw, int part, int round, hipStream_t s) {
    if (phw <= 0) return hipSuccess;
    const dim3 it(phw, st.iter_blocks);
    if (part == 0) hipLaunchKernelGGL(prep_kernel<n>, it, dim3(kIterThreads), 0, s, st);
    if (part == 1 || part == 5) {
        // covers a list of up to phw * W items and the uniform window
        const int64_t blocks = (int64_t)((phw + kNumXcd - 1) / kNumXcd) * kNumXcd * st.W;
        const int threads = Coop<n>::value ? Coop<n>::THREADS : kTrialThreads;
        if (part == 5 && NodeLds<n>::value)
            hipLaunchKernelGGL((trial_kernel<n, false>), dim3((unsigned)blocks), dim3(threads), 0, s, st, phw);
        else
            hipLaunchKernelGGL((trial_kernel<n, true>), dim3((unsigned)blocks), dim3(threads), 0, s, st, phw);
    }
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
