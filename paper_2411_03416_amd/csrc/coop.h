// Chain factorizations for larger blocks (n >= 6), one wavefront per matrix.
//
// The marginals of a block-tridiagonal precision (Sec. 5.1: GBP on the
// chain, equal to the selected inverse) are computed by a forward
// elimination and a backward recursion:
//   P_0 = D_0,  G_i = P_i^-1 U_i,  P_{i+1} = D_{i+1} - U_i^T G_i,
//   Sigma_{N-1} = P_{N-1}^-1,
//   Sigma_{i,i+1} = -G_i Sigma_{i+1},  Sigma_i = P_i^-1 - Sigma_{i,i+1} G_i^T.
// log det Lambda is the sum of log det P_i, and Lambda is positive definite
// iff every P_i is.  A linear system (D, U) x = r takes the same forward
// elimination with y_0 = r_0, w_i = P_i^-1 y_i, y_{i+1} = r_{i+1} - U_i^T w_i,
// and back substitution x_{N-1} = w_{N-1}, x_i = w_i - G_i x_{i+1}.  The
// backward passes need products only, no inversion.  (GBP's two-sided
// form, Sigma_ii = (P_i + Q_i - D_i)^-1 with the right Schur complements
// Q_i, halves the depth but subtracts blocks far larger than the marginal
// precision on stiff chains; this form does not.)
//
// Within a wavefront the 64 lanes share every block operation.  A block is
// padded to NP x NP (NP = 8 for n = 6, else 16; a spare column carries a
// right-hand side) and held in registers: lane l holds column l % NP of rows
// l / NP + RSTEP t, t < EPL.  Products and factorizations exchange blocks
// through a per-wavefront LDS area; the lanes of one wavefront execute in
// lock step and LDS serves a wavefront's accesses in order, so a
// wavefront-scope fence (no barrier) orders the exchanges.
//
// Included by chain_impl.h after its chain-order helpers (BlockSrc, Ws,
// tiled offsets, lin2).
#pragma once
#include "blockmath.h"
#include "ctx.h"

namespace pg {

template <int n>
struct Coop {
    static constexpr bool value = n >= 6;
    static constexpr int NP = n <= 6 ? 8 : 16;    // padded block (one spare column at least)
    static constexpr int EPL = NP * NP / 64;       // entries per lane
    static constexpr int RSTEP = 64 / NP;          // rows between a lane's entries
    static constexpr int LS = NP + 1;              // LDS row stride in doubles
    static constexpr int BUF = NP * LS;            // one LDS block
    static constexpr int WAVE_LDS = 3 * BUF + 2 * NP;  // three blocks and two vectors per wavefront
    static constexpr int THREADS = 128;                // two wavefronts
};

// A block in registers: entry t of the lane is (row0 + RSTEP t, col).
template <int n>
struct DM {
    double v[Coop<n>::EPL];
};

// Orders the LDS accesses of a wavefront before and after this point.
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int n>
struct Lane {
    int row0, col;
    __device__ __forceinline__ explicit Lane(int lane) : row0(lane / Coop<n>::NP), col(lane % Coop<n>::NP) {}
    __device__ __forceinline__ int row(int t) const { return row0 + Coop<n>::RSTEP * t; }
};

template <int n>
__device__ __forceinline__ void dm_zero(DM<n>& X) {
#pragma unroll
    for (int t = 0; t < Coop<n>::EPL; ++t) X.v[t] = 0.0;
}

// Entry of lane entry t inside the n x n block: padding entries are clamped
// to a real one, so every lane loads (no branch around the loads: those of
// the next state stay in flight behind the current one's arithmetic) and
// padding lanes discard what they read.
template <int n>
__device__ __forceinline__ int dm_e(const Lane<n>& L, int t) {
    const int r = L.row(t) < n ? L.row(t) : n - 1, c = L.col < n ? L.col : n - 1;
    return r * n + c;
}
template <int n>
__device__ __forceinline__ bool dm_in(const Lane<n>& L, int t) {
    return L.row(t) < n && L.col < n;
}

// Block at byte offset off of a tiled chain-order array (entry e = r n + c)
// as loaded: padding entries hold whatever real entry they were clamped to
// (dm_mask zeroes them where the block is used, so a load for the next
// state is not waited for until then).
template <int n>
__device__ __forceinline__ void dm_ld_raw(const double* base, uint32_t off, const Lane<n>& L, DM<n>& X) {
#pragma unroll
    for (int t = 0; t < Coop<n>::EPL; ++t) X.v[t] = ldo(base, off, dm_e<n>(L, t));
}
template <int n>
__device__ __forceinline__ void dm_mask(const Lane<n>& L, DM<n>& X) {
#pragma unroll
    for (int t = 0; t < Coop<n>::EPL; ++t) X.v[t] = dm_in<n>(L, t) ? X.v[t] : 0.0;
}
// The block, zero outside n x n.
template <int n>
__device__ __forceinline__ void dm_ld(const double* base, uint32_t off, const Lane<n>& L, DM<n>& X) {
    dm_ld_raw<n>(base, off, L, X);
    dm_mask<n>(L, X);
}
template <int n>
__device__ __forceinline__ void dm_st(double* base, uint32_t off, const Lane<n>& L, const DM<n>& X) {
#pragma unroll
    for (int t = 0; t < Coop<n>::EPL; ++t) {
        const int r = L.row(t), c = L.col;
        if (r < n && c < n) sto(base, off, r * n + c, X.v[t]);
    }
}
// The two blocks of a source, as loaded (combined by dm_lin2).
template <int n>
struct DM2 {
    DM<n> x0, x1;
};
template <int n>
__device__ __forceinline__ void dm_ld2(const double* X0, const double* X1, uint32_t off, const Lane<n>& L,
                                       DM2<n>& R) {
    dm_ld_raw<n>(X0, off, L, R.x0);
    dm_ld_raw<n>(X1, off, L, R.x1);
}
// a0 X0 + a1 X1 (the same expression as lin2), zero outside the block
template <int n>
__device__ __forceinline__ void dm_lin2(double a0, double a1, const DM2<n>& R, const Lane<n>& L, DM<n>& X) {
#pragma unroll
    for (int t = 0; t < Coop<n>::EPL; ++t) X.v[t] = dm_in<n>(L, t) ? lin2(a0, R.x0.v[t], a1, R.x1.v[t]) : 0.0;
}
// Vector entries r < n of a tiled array with E entries per position, as
// loaded by every lane (lane entry t reads entry min(row, n - 1)); dm_mask_col
// keeps them in the lanes of column `col` only.
template <int n, int E>
__device__ __forceinline__ void dm_ld_vec_raw(const double* base, int64_t q, const Lane<n>& L, DM<n>& X) {
#pragma unroll
    for (int t = 0; t < Coop<n>::EPL; ++t) {
        const int r = L.row(t);
        X.v[t] = base[tidx<E>(q, r < n ? r : n - 1)];
    }
}
template <int n>
__device__ __forceinline__ void dm_mask_col(int col, const Lane<n>& L, DM<n>& X) {
#pragma unroll
    for (int t = 0; t < Coop<n>::EPL; ++t) X.v[t] = (L.col == col && L.row(t) < n) ? X.v[t] : 0.0;
}
// The vector in the lanes of column `col` (the others get 0).
template <int n, int E>
__device__ __forceinline__ void dm_ld_vec(const double* base, int64_t q, int col, const Lane<n>& L, DM<n>& X) {
    dm_ld_vec_raw<n, E>(base, q, L, X);
    dm_mask_col<n>(col, L, X);
}
template <int n, int E>
__device__ __forceinline__ void dm_st_vec(double* base, int64_t q, int col, const Lane<n>& L, const DM<n>& X) {
#pragma unroll
    for (int t = 0; t < Coop<n>::EPL; ++t) {
        const int r = L.row(t);
        if (L.col == col && r < n) base[tidx<E>(q, r)] = X.v[t];
    }
}

template <int n>
__device__ __forceinline__ void dm_put(const DM<n>& X, double* B, const Lane<n>& L) {
#pragma unroll
    for (int t = 0; t < Coop<n>::EPL; ++t) B[L.row(t) * Coop<n>::LS + L.col] = X.v[t];
}
// B = X^T
template <int n>
__device__ __forceinline__ void dm_put_t(const DM<n>& X, double* B, const Lane<n>& L) {
#pragma unroll
    for (int t = 0; t < Coop<n>::EPL; ++t) B[L.col * Coop<n>::LS + L.row(t)] = X.v[t];
}
// V[r] = X[r][col] for r < n
template <int n>
__device__ __forceinline__ void dm_put_col(const DM<n>& X, int col, double* V, const Lane<n>& L) {
#pragma unroll
    for (int t = 0; t < Coop<n>::EPL; ++t)
        if (L.col == col && L.row(t) < n) V[L.row(t)] = X.v[t];
}

// C = op(A) op(B) over the inner index k < n, A and B blocks in LDS (the
// caller fences after writing them).  Column `vcol` of B is read from the
// vector V instead (an augmented right-hand side); vcol = -1: none.
template <int n, bool TA, bool TB>
__device__ __forceinline__ void coop_mul(const double* A, const double* B, const double* V, int vcol,
                                         const Lane<n>& L, DM<n>& C) {
    constexpr int LS = Coop<n>::LS;
    const int c = L.col;
    const bool fromv = c == vcol;
    const double* bp = fromv ? V : (TB ? B + c * LS : B + c);
    const int bs = fromv ? 1 : (TB ? 1 : LS);
#pragma unroll
    for (int t = 0; t < Coop<n>::EPL; ++t) {
        const int r = L.row(t);
        const double* ap = TA ? A + r : A + r * LS;
        const int as = TA ? LS : 1;
        double s = 0.0;
        for (int k = 0; k < n; ++k) s = fma(ap[k * as], bp[k * bs], s);
        C.v[t] = s;
    }
}

// Inverse of the SPD block written to LDS buffer A (read as its lower
// triangle; A and X are overwritten): Cholesky A = L L^T in place, the
// diagonal kept as its reciprocal, X = L^-1, and Ainv = X^T X (bitwise
// symmetric).  Multiplies det by the pivots; returns false if a pivot is
// not positive, not finite or below the smallest normal number (the same
// test as spd_inverse).
//
// For 8 x 8 blocks (one entry per lane) round k also finishes row k of X,
// X[k][c] = (delta_kc - sum_{j<k} L[k][j] X[j][c]) / L[k][k] (row k of L
// and the rows of X above it are final by then): one LDS round per pivot.
// For 16 x 16 blocks that dot product of up to 13 terms would lengthen every
// round, so X follows in a second pass of right-looking substitution on the
// identity, each round one short update (measured faster there).
template <int n>
__device__ __forceinline__ bool coop_spd_inverse(double* A, double* X, const Lane<n>& L, DM<n>& Ainv, DetAcc* det) {
    using C = Coop<n>;
    constexpr int LS = C::LS;
    constexpr bool MERGED = C::NP == 8;
    const int c = L.col;
    bool ok = true;
    wsync();
    // Every round reads all it needs first and then writes every entry of
    // the lane back (unchanged where the round does not touch it): one LDS
    // round trip per round, and no branch around a load.  A lane's entries
    // are written by that lane only, and all reads of a round precede its
    // writes, so the reads see the previous round's values.
    for (int k = 0; k < n; ++k) {
        const double d = A[k * LS + k];
        const double ack = A[(c < n ? c : 0) * LS + k];
        double ark[C::EPL], arc[C::EPL], dot[C::EPL];
#pragma unroll
        for (int t = 0; t < C::EPL; ++t) {
            const int r = L.row(t);
            ark[t] = A[r * LS + k];
            arc[t] = A[r * LS + c];
            dot[t] = 0.0;
            if (MERGED) {
                // row r of X from the final rows above it (used for r = k)
                for (int j = 0; j < k; ++j) dot[t] = fma(A[r * LS + j], X[j * LS + c], dot[t]);
            }
        }
        const bool good = d >= 2.2250738585072014e-308 && d < INFINITY;
        ok = ok && good;
        if (det) det->mul(good ? d : 1.0);
        const double rs = good ? rsqrt_nr(d) : 0.0;
        const double lck = (c > k && c < n) ? ack * rs : 0.0;  // L[c][k]
#pragma unroll
        for (int t = 0; t < C::EPL; ++t) {
            const int r = L.row(t);
            if (MERGED && r == k) X[k * LS + c] = ((c == k ? 1.0 : 0.0) - dot[t]) * rs;
            const double lrk = ark[t] * rs;  // L[r][k]
            double v = arc[t];
            if (r < n && r >= k) {
                if (c == k) v = r == k ? rs : lrk;
                else if (c > k && c <= r) v = fma(-lrk, lck, arc[t]);
            }
            A[r * LS + c] = v;
        }
        wsync();
    }
    if (!MERGED) {
        // X = L^-1: row k of X is finished at step k, then removed from the rows below
#pragma unroll
        for (int t = 0; t < C::EPL; ++t) X[L.row(t) * LS + c] = (L.row(t) == c && c < n) ? 1.0 : 0.0;
        wsync();
        for (int k = 0; k < n; ++k) {
            const double xk = X[k * LS + c] * A[k * LS + k];
            double ark[C::EPL], xrc[C::EPL];
#pragma unroll
            for (int t = 0; t < C::EPL; ++t) {
                const int r = L.row(t);
                ark[t] = A[r * LS + k];
                xrc[t] = X[r * LS + c];
            }
#pragma unroll
            for (int t = 0; t < C::EPL; ++t) {
                const int r = L.row(t);
                const double v = r == k ? xk : (r > k && r < n) ? fma(-ark[t], xk, xrc[t]) : xrc[t];
                X[r * LS + c] = v;
            }
            wsync();
        }
    }
#pragma unroll
    for (int t = 0; t < C::EPL; ++t) {
        const int r = L.row(t);
        double s = 0.0;
        for (int k = 0; k < n; ++k) s = fma(X[k * LS + r], X[k * LS + c], s);
        Ainv.v[t] = (r < n && c < n) ? s : 0.0;
    }
    return ok;
}

// Forward elimination.  Covariance (!RHS): stores P_i^-1 at ws.P and G_i
// at ws.G.  System (RHS): stores G_i at ws.G and w_i at ws.H (n entries of
// an n x n slot).  Positions are plan-local (chain order is state order
// here).  Returns whether every P_i is positive definite; adds log det.
template <int n, bool RHS>
__device__ __forceinline__ bool coop_forward(const BlockSrc& M, int N, const Ws& ws, double* lds, int lane,
                                             double* logdet) {
    using C = Coop<n>;
    constexpr int NN = n * n;
    const Lane<n> L(lane);
    double *bA = lds, *bX = lds + C::BUF, *bB = lds + 2 * C::BUF, *bV = lds + 3 * C::BUF;
    DetAcc det;
    bool ok = true;
    DM<n> P, Y;
    {
        DM2<n> P0;
        dm_ld2<n>(M.D0, M.D1, toff<NN>(0), L, P0);
        dm_lin2<n>(M.a0, M.a1, P0, L, P);
    }
    if (RHS) {
        DM<n> r0, r1;
        dm_ld_vec<n, n>(M.R0, 0, n, L, r0);
        dm_ld_vec<n, n>(M.R1, 0, n, L, r1);
#pragma unroll
        for (int t = 0; t < C::EPL; ++t) Y.v[t] = lin2(M.a0, r0.v[t], M.a1, r1.v[t]);
    }
    for (int i = 0; i < N; ++i) {
        const uint32_t o = toff<NN>(i);
        const bool more = i + 1 < N;
        // the next state's inputs, independent of the recurrence: loaded
        // here and combined after the pivot inversion, so the loads are in
        // flight meanwhile
        // (past the last state they reread it, and are not used)
        const int nx = more ? i + 1 : i;
        DM2<n> Ur, Dr;
        DM<n> r0n, r1n;
        dm_ld2<n>(M.U0, M.U1, o, L, Ur);
        dm_ld2<n>(M.D0, M.D1, toff<NN>(nx), L, Dr);
        if (RHS) {
            dm_ld_vec_raw<n, n>(M.R0, nx, L, r0n);
            dm_ld_vec_raw<n, n>(M.R1, nx, L, r1n);
        }
        wsync();
        dm_put<n>(P, bA, L);
        DM<n> Pinv;
        ok = coop_spd_inverse<n>(bA, bX, L, Pinv, &det) && ok;
        if (!RHS) dm_st<n>(ws.P, o, L, Pinv);
        if (!more && !RHS) break;
        // G = P^-1 [U | y] (U = 0 after the last state), then S = U^T G
        DM<n> U;
        if (more) dm_lin2<n>(M.a0, M.a1, Ur, L, U);
        else dm_zero<n>(U);
        wsync();
        dm_put<n>(Pinv, bA, L);
        dm_put<n>(U, bB, L);
        if (RHS) dm_put_col<n>(Y, n, bV, L);
        wsync();
        DM<n> G;
        coop_mul<n, false, false>(bA, bB, bV, RHS ? n : -1, L, G);
        if (more) dm_st<n>(ws.G, o, L, G);
        if (RHS) dm_st_vec<n, NN>(ws.H, i, n, L, G);
        if (!more) break;
        wsync();
        dm_put<n>(G, bX, L);
        wsync();
        DM<n> S, Dn;
        dm_lin2<n>(M.a0, M.a1, Dr, L, Dn);
        coop_mul<n, true, false>(bB, bX, nullptr, -1, L, S);
#pragma unroll
        for (int t = 0; t < C::EPL; ++t) {
            const int r = L.row(t), c = L.col;
            P.v[t] = (r < n && c < n) ? Dn.v[t] - S.v[t] : 0.0;
            if (RHS) Y.v[t] = (c == n && r < n) ? lin2(M.a0, r0n.v[t], M.a1, r1n.v[t]) - S.v[t] : 0.0;
        }
    }
    *logdet += det.log_value();
    return ok;
}

// Backward recursion of the covariance from the forward elimination's
// P_i^-1 and G_i: Sigma_ii to SDo (bitwise symmetric), Sigma_{i,i+1} to SUo.
// Adds the lane's share of tr(KH_i Sigma_ii) + 2 tr(KU_i^T Sigma_{i,i+1})
// to *part when KH is given.
template <int n>
__device__ __forceinline__ void coop_cov_backward(int N, const Ws& ws, double* SDo, double* SUo, const double* KH,
                                                  const double* KU, double* lds, int lane, double* part) {
    using C = Coop<n>;
    constexpr int NN = n * n;
    const Lane<n> L(lane);
    double *bA = lds, *bX = lds + C::BUF, *bB = lds + 2 * C::BUF;
    DM<n> Sg;
    dm_ld<n>(ws.P, toff<NN>(N - 1), L, Sg);
    dm_st<n>(SDo, toff<NN>(N - 1), L, Sg);
    if (KH) {
        DM<n> K;
        dm_ld<n>(KH, toff<NN>(N - 1), L, K);
#pragma unroll
        for (int t = 0; t < C::EPL; ++t) *part = fma(K.v[t], Sg.v[t], *part);
    }
    // the blocks of state i are loaded during state i + 1 (state 0 rereads
    // its own, unused), masked where used
    DM<n> G, Pinv, Kd, Ku;
    dm_zero<n>(Kd);
    dm_zero<n>(Ku);
    {
        const uint32_t o0 = toff<NN>(N >= 2 ? N - 2 : 0);
        dm_ld_raw<n>(ws.G, o0, L, G);
        dm_ld_raw<n>(ws.P, o0, L, Pinv);
        if (KH) {
            dm_ld_raw<n>(KH, o0, L, Kd);
            dm_ld_raw<n>(KU, o0, L, Ku);
        }
    }
    for (int i = N - 2; i >= 0; --i) {
        const uint32_t o = toff<NN>(i);
        dm_mask<n>(L, G);
        dm_mask<n>(L, Pinv);
        dm_mask<n>(L, Kd);
        dm_mask<n>(L, Ku);
        DM<n> Gn, Pn, Kdn, Kun;
        dm_zero<n>(Kdn);
        dm_zero<n>(Kun);
        {
            const uint32_t on = toff<NN>(i > 0 ? i - 1 : 0);
            dm_ld_raw<n>(ws.G, on, L, Gn);
            dm_ld_raw<n>(ws.P, on, L, Pn);
            if (KH) {
                dm_ld_raw<n>(KH, on, L, Kdn);
                dm_ld_raw<n>(KU, on, L, Kun);
            }
        }
        // Sigma_{i,i+1} = -G Sigma_{i+1}
        wsync();
        dm_put<n>(G, bA, L);
        dm_put<n>(Sg, bB, L);
        wsync();
        DM<n> So;
        coop_mul<n, false, false>(bA, bB, nullptr, -1, L, So);
#pragma unroll
        for (int t = 0; t < C::EPL; ++t) So.v[t] = -So.v[t];
        dm_st<n>(SUo, o, L, So);
        // Sigma_i = P^-1 - Sigma_{i,i+1} G^T, bitwise symmetric: a lane above
        // the diagonal forms the mirrored entry (T[c][r], the same operands
        // in the same order as the lane below; P^-1 is bitwise symmetric), so
        // no second exchange is needed
        wsync();
        dm_put<n>(So, bX, L);
        wsync();
#pragma unroll
        for (int t = 0; t < C::EPL; ++t) {
            const int r = L.row(t), c = L.col;
            const int a = r >= c ? r : c, b = r >= c ? c : r;
            double tv = 0.0;
            for (int k = 0; k < n; ++k) tv = fma(bX[a * C::LS + k], bA[b * C::LS + k], tv);
            Sg.v[t] = Pinv.v[t] - tv;
        }
        dm_st<n>(SDo, o, L, Sg);
        if (KH) {
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < C::EPL; ++t) {
                *part = fma(Kd.v[t], Sg.v[t], *part);
                s = fma(Ku.v[t], So.v[t], s);
            }
            *part = fma(2.0, s, *part);
        }
        G = Gn;
        Pinv = Pn;
        Kd = Kdn;
        Ku = Kun;
    }
}

// Back substitution x_i = w_i - G_i x_{i+1} into xo.  With mu0, adds the
// lane's share of d_i^T LD_i d_i + 2 d_i^T LU_i d_{i+1} (d = x - mu0,
// LD = M.D1, LU = M.U1: the mean step's quadratic KL term) to *part.
template <int n>
__device__ __forceinline__ void coop_rhs_backward(const BlockSrc& M, int N, const Ws& ws, double* xo,
                                                  const double* mu0, double* lds, int lane, double* part) {
    using C = Coop<n>;
    constexpr int NN = n * n;
    const Lane<n> L(lane);
    double *bA = lds, *bV = lds + 3 * C::BUF, *bD = lds + 3 * C::BUF + C::NP;
    // x and d = x - mu0 of the state below, in column 0 of the lanes
    DM<n> x, d;
    dm_zero<n>(d);
    dm_ld_vec<n, NN>(ws.H, N - 1, 0, L, x);
    dm_st_vec<n, n>(xo, N - 1, 0, L, x);
    if (mu0) {
        DM<n> m0;
        dm_ld_vec<n, n>(mu0, N - 1, 0, L, m0);
#pragma unroll
        for (int t = 0; t < C::EPL; ++t) d.v[t] = x.v[t] - m0.v[t];
    }
    // the inputs of state i are loaded during state i + 1 (state 0 rereads
    // its own, unused), masked where used
    DM<n> G, w, m0, LDc, LUc;
    dm_zero<n>(G);
    dm_zero<n>(w);
    dm_zero<n>(m0);
    dm_zero<n>(LDc);
    dm_zero<n>(LUc);
    if (mu0) dm_ld_raw<n>(M.D1, toff<NN>(N - 1), L, LDc);
    for (int i = N - 1; i >= 0; --i) {
        const bool below = i + 1 < N;
        dm_mask<n>(L, G);
        dm_mask_col<n>(0, L, w);
        dm_mask_col<n>(0, L, m0);
        dm_mask<n>(L, LDc);
        dm_mask<n>(L, LUc);
        DM<n> Gn, wn, m0n, LDn, LUn;
        dm_zero<n>(m0n);
        dm_zero<n>(LDn);
        dm_zero<n>(LUn);
        {
            const int iq = i > 0 ? i - 1 : 0;
            const uint32_t on = toff<NN>(iq);
            dm_ld_raw<n>(ws.G, on, L, Gn);
            dm_ld_vec_raw<n, NN>(ws.H, iq, L, wn);
            if (mu0) {
                dm_ld_vec_raw<n, n>(mu0, iq, L, m0n);
                dm_ld_raw<n>(M.D1, on, L, LDn);
                dm_ld_raw<n>(M.U1, on, L, LUn);
            }
        }
        DM<n> xi = x, di = d;
        if (below) {
            wsync();
            dm_put<n>(G, bA, L);
            dm_put_col<n>(x, 0, bV, L);
            wsync();
            DM<n> g;
            coop_mul<n, false, false>(bA, bA, bV, 0, L, g);  // column 0: G x_{i+1}
#pragma unroll
            for (int t = 0; t < C::EPL; ++t) {
                xi.v[t] = w.v[t] - g.v[t];
                di.v[t] = xi.v[t] - m0.v[t];
            }
            dm_st_vec<n, n>(xo, i, 0, L, xi);
        }
        if (mu0) {
            // d_i in bV, d_{i+1} in bD
            wsync();
            dm_put_col<n>(di, 0, bV, L);
            if (below) dm_put_col<n>(d, 0, bD, L);
            wsync();
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < C::EPL; ++t) {
                const int r = L.row(t), c = L.col;
                if (r < n && c < n) {
                    const double ld = LDc.v[t];
                    const double lu = below ? LUc.v[t] : 0.0;
                    const double dn = below ? bD[c] : 0.0;
                    s = fma(bV[r], fma(ld, bV[c], 2.0 * lu * dn), s);
                }
            }
            *part += s;
        }
        x = xi;
        d = di;
        G = Gn;
        w = wn;
        m0 = m0n;
        LDc = LDn;
        LUc = LUn;
    }
}

// Block of state s from a state-major array (entry e of state s at
// X[e S + s]); zero outside n x n.
template <int n>
__device__ __forceinline__ void dm_ld_soa(const double* X, int64_t S, int64_t s, const Lane<n>& L, DM<n>& M) {
#pragma unroll
    for (int t = 0; t < Coop<n>::EPL; ++t) {
        const int r = L.row(t), c = L.col;
        M.v[t] = (r < n && c < n) ? X[(int64_t)(r * n + c) * S + s] : 0.0;
    }
}

// Sum over the 64 lanes of a wavefront in lane order (LDS scratch of 64
// doubles); every lane gets the sum.
__device__ __forceinline__ double wave_sum(double v, double* sh, int lane) {
    wsync();
    sh[lane] = v;
    wsync();
    double s = 0.0;
    for (int k = 0; k < 64; ++k) s += sh[k];
    return s;
}

// Expected prior factor costs touching state i (Sec. 2.2): the transition
// i -> i+1 (i < N-1), 1/2 [tr(W C) + rbar^T W rbar] with W = Q_i^-1,
// C = Cov(x_{i+1} - Phi x_i) = S_{i+1} - Sx^T Phi^T - Phi Sx + Phi S_i Phi^T
// and rbar = mu_{i+1} - Phi mu_i - abar; the start (i = 0) and goal
// (i = N-1) factors 1/2 [tr(W S_i) + r^T W r].  out = (transition, start,
// goal), the same on every lane.  lds: one wavefront's area.
template <int n>
__device__ __forceinline__ void coop_prior_cost(const DevState& st, const PlanDev& p, int i, double* lds, int lane,
                                                double out[3]) {
    using C = Coop<n>;
    constexpr int LS = C::LS;
    const Lane<n> L(lane);
    const int c = L.col;
    double *bA = lds, *bX = lds + C::BUF, *bB = lds + 2 * C::BUF, *bV = lds + 3 * C::BUF,
           *bR = lds + 3 * C::BUF + C::NP;
    const int64_t S = st.S, s = p.off + i;
    double tr_part = 0.0, st_part = 0.0, gl_part = 0.0;
    const bool trans = i < p.N - 1;
    if (trans) {
        DM<n> Phi, Wq, Si, Sn, Sx;
        dm_ld_soa<n>(st.Phi, S, s, L, Phi);
        dm_ld_soa<n>(st.Qinv, S, s, L, Wq);
        dm_ld_soa<n>(st.SD, S, s, L, Si);
        dm_ld_soa<n>(st.SD, S, s + 1, L, Sn);
        dm_ld_soa<n>(st.SU, S, s, L, Sx);
        // rbar = mu_{i+1} - Phi mu_i - abar, in bR
        wsync();
        dm_put<n>(Phi, bA, L);
        if (lane < n) bV[lane] = st.mu[(int64_t)lane * S + s];
        wsync();
        if (lane < n) {
            double pm = 0.0;
            for (int k = 0; k < n; ++k) pm = fma(bA[lane * LS + k], bV[k], pm);
            bR[lane] = st.mu[(int64_t)lane * S + s + 1] - pm - st.abar[(int64_t)lane * S + s];
        }
        // PS = Phi Sx and T = Phi S_i
        dm_put<n>(Sx, bB, L);
        dm_put<n>(Si, bX, L);
        wsync();
        DM<n> PS, T;
        coop_mul<n, false, false>(bA, bB, nullptr, -1, L, PS);
        coop_mul<n, false, false>(bA, bX, nullptr, -1, L, T);
        // C = T Phi^T + Sn - PS - PS^T
        wsync();
        dm_put<n>(T, bX, L);
        dm_put<n>(PS, bB, L);
        wsync();
        DM<n> Cm;
        coop_mul<n, false, true>(bX, bA, nullptr, -1, L, Cm);
#pragma unroll
        for (int t = 0; t < C::EPL; ++t) {
            const int r = L.row(t);
            Cm.v[t] += Sn.v[t] - PS.v[t] - ((r < n && c < n) ? bB[c * LS + r] : 0.0);
        }
        // tr(W C) = sum W[r][c] C[c][r]; rbar^T W rbar
        wsync();
        dm_put<n>(Cm, bX, L);
        wsync();
#pragma unroll
        for (int t = 0; t < C::EPL; ++t) {
            const int r = L.row(t);
            if (r < n && c < n) {
                tr_part = fma(Wq.v[t], bX[c * LS + r], tr_part);
                tr_part = fma(bR[r] * Wq.v[t], bR[c], tr_part);
            }
        }
    }
    for (int endf = 0; endf < 2; ++endf) {
        if ((endf == 0 && i != 0) || (endf == 1 && i != p.N - 1)) continue;
        const double* Wm = endf == 0 ? p.Wstart : p.Wgoal;
        const double* m0 = endf == 0 ? p.mu_start : p.mu_goal;
        double v = 0.0;
#pragma unroll
        for (int t = 0; t < C::EPL; ++t) {
            const int a = L.row(t);
            if (a < n && c < n) {
                const double w = Wm[a * n + c];
                const double ra = st.mu[(int64_t)a * S + s] - m0[a];
                const double rc = st.mu[(int64_t)c * S + s] - m0[c];
                v = fma(w, st.SD[(int64_t)(c * n + a) * S + s], v);
                v = fma(ra * w, rc, v);
            }
        }
        if (endf == 0) st_part = v;
        else gl_part = v;
    }
    // (bX, NP (NP + 1) >= 64 doubles, is the reduction's scratch)
    out[0] = trans ? 0.5 * wave_sum(tr_part, bX, lane) : 0.0;
    out[1] = i == 0 ? 0.5 * wave_sum(st_part, bX, lane) : 0.0;
    out[2] = i == p.N - 1 ? 0.5 * wave_sum(gl_part, bX, lane) : 0.0;
    wsync();
}

// The chain step of one matrix (and optionally a linear system) on two
// wavefronts: wave 0 factors MT and recovers its marginals (SDo, SUo), wave
// 1 solves MM x = r into xo.  Every thread of the workgroup calls this (it
// ends with barriers).  Results in sh (thread 0 reads): sh[0] = log det
// MT, sh[1] = 1 if MT is positive definite, sh[2] = trace term sum (KH, KU
// given), sh[3] = quadratic term sum (mu0 given).  sh holds THREADS + 4
// doubles, lds 2 * WAVE_LDS.
template <int n>
__device__ __forceinline__ void coop_chain(const BlockSrc& MT, const BlockSrc& MM, bool mean, int N, const Ws& w0,
                                           const Ws& w1, double* SDo, double* SUo, double* xo, const double* mu0,
                                           const double* KH, const double* KU, double* lds, double* sh) {
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    double* wl = lds + wave * Coop<n>::WAVE_LDS;
    double* red = sh + 4;
    double part = 0.0;
    if (wave == 0) {
        double ld = 0.0;
        const bool ok = coop_forward<n, false>(MT, N, w0, wl, lane, &ld);
        coop_cov_backward<n>(N, w0, SDo, SUo, KH, KU, wl, lane, &part);
        if (lane == 0) {
            sh[0] = ld;
            sh[1] = ok ? 1.0 : 0.0;
        }
    } else if (mean) {
        double ld = 0.0;
        coop_forward<n, true>(MM, N, w1, wl, lane, &ld);
        coop_rhs_backward<n>(MM, N, w1, xo, mu0, wl, lane, &part);
    }
    red[tid] = part;
    __syncthreads();
    if (tid == 0) {
        double tr = 0.0, qd = 0.0;
        for (int k = 0; k < 64; ++k) tr += red[k];
        for (int k = 64; k < 128; ++k) qd += red[k];
        sh[2] = tr;
        sh[3] = qd;
    }
    __syncthreads();
}

}  // namespace pg
