// Small dense block algebra on register arrays (row-major n x n, FP64).
//
// Used by the chain kernels, where each thread carries a few n x n blocks
// of the block-tridiagonal precision through a sequential elimination.
#pragma once
#include <hip/hip_runtime.h>

namespace pg {

// Block temporaries: for small n they are register arrays; for larger n
// they live in a per-thread workspace in device memory owned by the
// library, so no kernel needs the runtime's private (scratch) segment.
template <int n>
struct RegBlocks {
    static constexpr bool value = (n <= 4);
};

// Bump allocator over a thread's workspace [p, end).  Passed by value: a
// callee's allocations end when it returns.  A request past the end sets
// *flag (the host then fails the call) and reuses the last slots, so no
// access leaves the thread's slice.
struct TS {
    double* p;
    double* end;
    int* flag;
    __device__ __forceinline__ double* take(int cnt) {
        if (p + cnt > end) {
            *flag = 1;
            return end - cnt;
        }
        double* r = p;
        p += cnt;
        return r;
    }
};

// Loop unrolling inside templates on n: full for small blocks, none for
// large ones (unrolled n^3 loops over workspace memory only raise register
// pressure and compile time).
#define PG_UNROLL _Pragma("unroll (n <= 4 ? 64 : 1)")

// Declare an n x n (PG_MAT) or n (PG_VEC) temporary `name`: a register
// array for small n, otherwise a slice taken from the workspace ts (the
// one-element array is dead and removed by the optimiser).
#define PG_MAT(name, ts)                                                   \
    double name##_reg[::pg::RegBlocks<n>::value ? n * n : 1];              \
    double* name = ::pg::RegBlocks<n>::value ? name##_reg : (ts).take(n * n)
#define PG_VEC(name, ts)                                                   \
    double name##_reg[::pg::RegBlocks<n>::value ? n : 1];                  \
    double* name = ::pg::RegBlocks<n>::value ? name##_reg : (ts).take(n)

template <int n>
__device__ __forceinline__ void mzero(double* A) {
PG_UNROLL
    for (int e = 0; e < n * n; ++e) A[e] = 0.0;
}

template <int n>
__device__ __forceinline__ void mcopy(const double* A, double* B) {
PG_UNROLL
    for (int e = 0; e < n * n; ++e) B[e] = A[e];
}

// C = A B
template <int n>
__device__ __forceinline__ void mmul(const double* A, const double* B, double* C) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
PG_UNROLL
            for (int k = 0; k < n; ++k) s = fma(A[i * n + k], B[k * n + j], s);
            C[i * n + j] = s;
        }
}

// C = A^T B
template <int n>
__device__ __forceinline__ void mmul_tn(const double* A, const double* B, double* C) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
PG_UNROLL
            for (int k = 0; k < n; ++k) s = fma(A[k * n + i], B[k * n + j], s);
            C[i * n + j] = s;
        }
}

// C = A B^T
template <int n>
__device__ __forceinline__ void mmul_nt(const double* A, const double* B, double* C) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
PG_UNROLL
            for (int k = 0; k < n; ++k) s = fma(A[i * n + k], B[j * n + k], s);
            C[i * n + j] = s;
        }
}

// C -= A^T B
template <int n>
__device__ __forceinline__ void msub_tn(const double* A, const double* B, double* C) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j < n; ++j) {
            double s = C[i * n + j];
PG_UNROLL
            for (int k = 0; k < n; ++k) s = fma(-A[k * n + i], B[k * n + j], s);
            C[i * n + j] = s;
        }
}

// C -= A B
template <int n>
__device__ __forceinline__ void msub(const double* A, const double* B, double* C) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j < n; ++j) {
            double s = C[i * n + j];
PG_UNROLL
            for (int k = 0; k < n; ++k) s = fma(-A[i * n + k], B[k * n + j], s);
            C[i * n + j] = s;
        }
}

// C -= A B^T
template <int n>
__device__ __forceinline__ void msub_nt(const double* A, const double* B, double* C) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j < n; ++j) {
            double s = C[i * n + j];
PG_UNROLL
            for (int k = 0; k < n; ++k) s = fma(-A[i * n + k], B[j * n + k], s);
            C[i * n + j] = s;
        }
}

// y -= A x
template <int n>
__device__ __forceinline__ void mvec_sub(const double* A, const double* x, double* y) {
PG_UNROLL
    for (int i = 0; i < n; ++i) {
        double s = y[i];
PG_UNROLL
        for (int k = 0; k < n; ++k) s = fma(-A[i * n + k], x[k], s);
        y[i] = s;
    }
}

// y = A x
template <int n>
__device__ __forceinline__ void mvec(const double* A, const double* x, double* y) {
PG_UNROLL
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
PG_UNROLL
        for (int k = 0; k < n; ++k) s = fma(A[i * n + k], x[k], s);
        y[i] = s;
    }
}

// y -= A^T x
template <int n>
__device__ __forceinline__ void mvec_tn_sub(const double* A, const double* x, double* y) {
PG_UNROLL
    for (int i = 0; i < n; ++i) {
        double s = y[i];
PG_UNROLL
        for (int k = 0; k < n; ++k) s = fma(-A[k * n + i], x[k], s);
        y[i] = s;
    }
}

// Inverse of an SPD matrix through its Cholesky factor A = L L^T:
// Ainv = L^-T L^-1.  If logdet is not null, adds log det A (the log of the
// product of the pivots, one logarithm per block).  Returns false (and
// leaves Ainv unspecified) if a pivot is not positive or not finite.
template <int n>
__device__ __forceinline__ bool spd_inverse(const double* A, double* Ainv, double* logdet, TS ts) {
    PG_MAT(L, ts);
PG_UNROLL
    for (int e = 0; e < n * n; ++e) L[e] = 0.0;
    double det = 1.0;
    bool ok = true;
PG_UNROLL
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
PG_UNROLL
        for (int k = 0; k < j; ++k) d = fma(-L[j * n + k], L[j * n + k], d);
        ok = ok && (d > 0.0) && (d < INFINITY);
        d = ok ? d : 1.0;
        const double ljj = sqrt(d);
        const double inv = 1.0 / ljj;
        det *= d;
        L[j * n + j] = ljj;
PG_UNROLL
        for (int i = j + 1; i < n; ++i) {
            double s = A[i * n + j];
PG_UNROLL
            for (int k = 0; k < j; ++k) s = fma(-L[i * n + k], L[j * n + k], s);
            L[i * n + j] = s * inv;
        }
    }
    // W = L^-1 (lower triangular), by forward substitution column by column
    PG_MAT(W, ts);
PG_UNROLL
    for (int e = 0; e < n * n; ++e) W[e] = 0.0;
PG_UNROLL
    for (int i = 0; i < n; ++i) {
        const double inv = 1.0 / L[i * n + i];
        W[i * n + i] = inv;
PG_UNROLL
        for (int j = 0; j < i; ++j) {
            double s = 0.0;
PG_UNROLL
            for (int k = j; k < i; ++k) s = fma(L[i * n + k], W[k * n + j], s);
            W[i * n + j] = -s * inv;
        }
    }
    // Ainv = W^T W, symmetric by construction
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j <= i; ++j) {
            double s = 0.0;
PG_UNROLL
            for (int k = i; k < n; ++k) s = fma(W[k * n + i], W[k * n + j], s);
            Ainv[i * n + j] = s;
            Ainv[j * n + i] = s;
        }
    if (logdet) *logdet += log(det);
    return ok;
}

}  // namespace pg
