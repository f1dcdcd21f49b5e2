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

// 1/sqrt(x) for a positive normal x: the hardware estimate refined by two
// Newton steps for f(y) = y^-2 - x, y <- y (3 - x y^2) / 2 (quadratic
// convergence, a few ulp at the end).
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h, y * y, 1.5);
    y = y * fma(-h, y * y, 1.5);
    return y;
}

// Inverse of an SPD matrix through its Cholesky factor A = L L^T:
// Ainv = L^-T L^-1.  Reads only the lower triangle of A.  If det is not
// null, stores det A (the product of the pivots) there.  Returns false (and
// leaves Ainv unspecified) if a pivot is not positive, not finite or below
// the smallest normal number.  One reciprocal square root per pivot; the
// diagonal of L is kept as its reciprocal, which is what both triangular
// steps use.
template <int n>
__device__ __forceinline__ bool spd_inverse(const double* A, double* Ainv, double* det, TS ts) {
    PG_MAT(L, ts);  // strictly lower part of L; diagonal: 1 / L_jj
    double dt = 1.0;
    bool ok = true;
PG_UNROLL
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
PG_UNROLL
        for (int k = 0; k < j; ++k) d = fma(-L[j * n + k], L[j * n + k], d);
        ok = ok && (d >= 2.2250738585072014e-308) && (d < INFINITY);
        d = ok ? d : 1.0;
        const double inv = rsqrt_nr(d);
        dt *= d;
        L[j * n + j] = inv;
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
    for (int i = 0; i < n; ++i) {
        const double inv = L[i * n + i];
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
    if (det) *det = dt;
    return ok;
}

// Running product of block determinants kept as mantissa * 2^exponent, so
// a sweep takes one logarithm at its end instead of one per block.
struct DetAcc {
    double m = 1.0;
    int e = 0;
    __device__ __forceinline__ void mul(double d) {
        int k;
        m = frexp(m * d, &k);
        e += k;
    }
    __device__ __forceinline__ double log_value() const { return log(m) + e * 0.6931471805599453; }
};

// Lower-triangle (j <= i) variants for symmetric results; the upper
// triangle of C is not touched.
// C -= A^T B
template <int n>
__device__ __forceinline__ void msub_tn_lo(const double* A, const double* B, double* C) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j <= i; ++j) {
            double s = C[i * n + j];
PG_UNROLL
            for (int k = 0; k < n; ++k) s = fma(-A[k * n + i], B[k * n + j], s);
            C[i * n + j] = s;
        }
}
// C -= A B^T
template <int n>
__device__ __forceinline__ void msub_nt_lo(const double* A, const double* B, double* C) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j <= i; ++j) {
            double s = C[i * n + j];
PG_UNROLL
            for (int k = 0; k < n; ++k) s = fma(-A[i * n + k], B[j * n + k], s);
            C[i * n + j] = s;
        }
}
// upper triangle of C from its lower triangle
template <int n>
__device__ __forceinline__ void sym_from_lo(double* C) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j < i; ++j) C[j * n + i] = C[i * n + j];
}
// C = -(A^T B)
template <int n>
__device__ __forceinline__ void mmul_tn_neg(const double* A, const double* B, double* C) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
PG_UNROLL
            for (int k = 0; k < n; ++k) s = fma(-A[k * n + i], B[k * n + j], s);
            C[i * n + j] = s;
        }
}
// C = -(A B)
template <int n>
__device__ __forceinline__ void mmul_neg(const double* A, const double* B, double* C) {
PG_UNROLL
    for (int i = 0; i < n; ++i)
PG_UNROLL
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
PG_UNROLL
            for (int k = 0; k < n; ++k) s = fma(-A[i * n + k], B[k * n + j], s);
            C[i * n + j] = s;
        }
}

}  // namespace pg
