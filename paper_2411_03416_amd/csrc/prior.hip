// GP prior on the device (Sec. 2.2 eq. dynamics_linear, Alg. 1), layout
// conversion between the SoA device arrays and [N][...] caller layouts, and
// statistical linear regression of a nonlinear drift (Sec. 6.2).
//
// Per interval i (A, a, B constant on [t_i, t_{i+1})), with dt:
//   Phi_i, abar_i  from  exp([[A, a], [0, 0]] dt)   (top block row),
//   Q_i            from  exp([[-A, B Qc B^T], [0, A^T]] dt) = [[F11, F12], [0, F22]]
//                  as Q = F22^T F12 (Van Loan 1978).
// The exponentials use scaling and squaring with a degree-18 Taylor
// polynomial (Horner form) once the 1-norm is scaled below 1/2, computed by
// one workgroup per interval with the matrices in LDS.
#include "ctx.h"

namespace pg {

constexpr int kPriorThreads = 64;
constexpr int kMaxAug = 2 * 14;  // largest augmented matrix dimension

__device__ void lds_matmul(const double* A, const double* B, double* C, int dim) {
    for (int e = threadIdx.x; e < dim * dim; e += blockDim.x) {
        const int r = e / dim, c = e % dim;
        double s = 0.0;
        for (int k = 0; k < dim; ++k) s = fma(A[r * dim + k], B[k * dim + c], s);
        C[e] = s;
    }
    __syncthreads();
}

// E = exp(M) for M in LDS (dim <= kMaxAug); T1, T2 are LDS scratch.
__device__ void lds_expm(double* M, double* E, double* T1, double* T2, int dim) {
    __shared__ double sh_norm;
    __shared__ int sh_sq;
    if (threadIdx.x == 0) {
        double nrm = 0.0;
        for (int c = 0; c < dim; ++c) {
            double cs = 0.0;
            for (int r = 0; r < dim; ++r) cs += fabs(M[r * dim + c]);
            nrm = fmax(nrm, cs);
        }
        int sq = 0;
        while (nrm > 0.5 && sq < 60) {
            nrm *= 0.5;
            ++sq;
        }
        sh_norm = nrm;
        sh_sq = sq;
    }
    __syncthreads();
    const int sq = sh_sq;
    const double scale = ldexp(1.0, -sq);
    for (int e = threadIdx.x; e < dim * dim; e += blockDim.x) M[e] *= scale;
    __syncthreads();
    // Horner: E = I + M/1 (I + M/2 (I + ... (I + M/K)))
    const int K = 18;
    for (int e = threadIdx.x; e < dim * dim; e += blockDim.x) E[e] = (e / dim == e % dim) ? 1.0 : 0.0;
    __syncthreads();
    for (int k = K; k >= 1; --k) {
        lds_matmul(M, E, T1, dim);
        const double ik = 1.0 / k;
        for (int e = threadIdx.x; e < dim * dim; e += blockDim.x)
            E[e] = T1[e] * ik + ((e / dim == e % dim) ? 1.0 : 0.0);
        __syncthreads();
    }
    for (int q = 0; q < sq; ++q) {
        lds_matmul(E, E, T2, dim);
        for (int e = threadIdx.x; e < dim * dim; e += blockDim.x) E[e] = T2[e];
        __syncthreads();
    }
}

// Inverse of an SPD matrix by one thread (Cholesky, then L^-T L^-1).
__device__ bool spd_inv_serial(const double* A, double* Ainv, double* L, int n) {
    for (int e = 0; e < n * n; ++e) L[e] = 0.0;
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0.0)) return false;
        const double l = sqrt(d);
        L[j * n + j] = l;
        for (int i = j + 1; i < n; ++i) {
            double s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = s / l;
        }
    }
    // invert L in place (lower triangular)
    for (int i = 0; i < n; ++i) {
        const double inv = 1.0 / L[i * n + i];
        for (int j = 0; j < i; ++j) {
            double s = 0.0;
            for (int k = j; k < i; ++k) s += L[i * n + k] * L[k * n + j];
            L[i * n + j] = -s * inv;
        }
        L[i * n + i] = inv;
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = 0.0;
            for (int k = i; k < n; ++k) s += L[k * n + i] * L[k * n + j];
            Ainv[i * n + j] = s;
            Ainv[j * n + i] = s;
        }
    return true;
}

// Plan plan_lo + blockIdx.y; blockIdx.x < N-1: interval; == N-1: start/goal
// inverses; beyond: nothing.  With time-invariant dynamics every interval
// has the same transition, offset and Grammian: only interval 0 computes
// them and the assembly kernel shares them with the other intervals.
__global__ void __launch_bounds__(kPriorThreads) prior_build_kernel(DevState st, int plan_lo) {
    __shared__ double M[kMaxAug * kMaxAug], E[kMaxAug * kMaxAug], T1[kMaxAug * kMaxAug], T2[kMaxAug * kMaxAug];
    PlanDev& p = st.plans[plan_lo + blockIdx.y];
    if (!p.active) return;
    const int n = st.n, m = p.m;
    const int i = blockIdx.x;
    if (i >= p.N) return;
    const double dt = p.dt;
    const int64_t S = st.S;
    if (!p.ltv && i > 0 && i < p.N - 1) return;
    if (i == p.N - 1) {
        if (threadIdx.x == 0) {
            spd_inv_serial(p.Sig_start, p.Wstart, M, n);
            spd_inv_serial(p.Sig_goal, p.Wgoal, M, n);
        }
        return;
    }
    const double* A = p.A + (int64_t)i * n * n;
    const double* a = p.a + (int64_t)i * n;
    const double* B = p.B + (int64_t)i * n * m;
    // 1) exp([[A, a], [0, 0]] dt)
    const int d1 = n + 1;
    for (int e = threadIdx.x; e < d1 * d1; e += blockDim.x) {
        const int r = e / d1, c = e % d1;
        double v = 0.0;
        if (r < n) v = (c < n) ? A[r * n + c] : a[r];
        M[e] = v * dt;
    }
    __syncthreads();
    lds_expm(M, E, T1, T2, d1);
    const int64_t s = p.off + i;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) st.Phi[e * S + s] = E[(e / n) * d1 + (e % n)];
    for (int r = threadIdx.x; r < n; r += blockDim.x) st.abar[r * S + s] = E[r * d1 + n];
    __syncthreads();
    // 2) Van Loan: exp([[-A, B Qc B^T], [0, A^T]] dt)
    const int d2 = 2 * n;
    for (int e = threadIdx.x; e < d2 * d2; e += blockDim.x) {
        const int r = e / d2, c = e % d2;
        double v = 0.0;
        if (r < n && c < n) {
            v = -A[r * n + c];
        } else if (r < n && c >= n) {
            const int cc = c - n;
            for (int k = 0; k < m; ++k) {
                double bq = 0.0;
                for (int l = 0; l < m; ++l) bq += B[r * m + l] * p.Qc[l * m + k];
                v += bq * B[cc * m + k];
            }
        } else if (r >= n && c >= n) {
            v = A[(c - n) * n + (r - n)];
        }
        M[e] = v * dt;
    }
    __syncthreads();
    lds_expm(M, E, T1, T2, d2);
    // Q = F22^T F12 into T1 (n x n), symmetrised
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int r = e / n, c = e % n;
        double q = 0.0;
        for (int k = 0; k < n; ++k) q += E[(n + k) * d2 + (n + r)] * E[k * d2 + (n + c)];
        T1[e] = q;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int r = e / n, c = e % n;
        T2[e] = 0.5 * (T1[r * n + c] + T1[c * n + r]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (!spd_inv_serial(T2, M, E, n)) {
            for (int e = 0; e < n * n; ++e) M[e] = NAN;
            p.status = PGVIMP_ENOTPD;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) st.Qinv[e * S + s] = M[e];
}

// K^-1 blocks and eta = K^-1 mu_bar from the factor sums (Alg. 1), one
// thread per state.  The block Phi^T Qinv Phi is formed column by column:
// t = Qinv Phi[:, c] (n values in registers), then entry (r, c) = Phi[:, r]^T t,
// n^3 operations per block instead of recomputing t for every entry (the
// sums are the same, in the same order).
constexpr int kAssembleThreads = 64;
template <int n>
__global__ void __launch_bounds__(kAssembleThreads) prior_assemble_kernel(DevState st, int plan_lo) {
    const PlanDev& p = st.plans[plan_lo + blockIdx.y];
    if (!p.active) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = p.N;
    if (i >= N) return;
    const int64_t S = st.S, s = p.off + i;
    // interval blocks of this interval (sI) and of the previous one (sP):
    // interval 0's for time-invariant dynamics, copied to this interval for
    // the later per-state readers
    const int64_t sI = p.ltv ? s : p.off, sP = p.ltv ? s - 1 : p.off;
    if (!p.ltv && i > 0 && i < N - 1) {
        for (int e = 0; e < n * n; ++e) {
            st.Phi[e * S + s] = st.Phi[e * S + sI];
            st.Qinv[e * S + s] = st.Qinv[e * S + sI];
        }
        for (int e = 0; e < n; ++e) st.abar[e * S + s] = st.abar[e * S + sI];
    }
#pragma unroll 1
    for (int c = 0; c < n; ++c) {
        double t[n];
        if (i < N - 1) {
#pragma unroll
            for (int k = 0; k < n; ++k) {
                double v = 0.0;
                for (int l = 0; l < n; ++l) v += st.Qinv[(k * n + l) * S + sI] * st.Phi[(l * n + c) * S + sI];
                t[k] = v;
            }
        }
#pragma unroll 1
        for (int r = 0; r < n; ++r) {
            double v = 0.0;
            if (i == 0) v += p.Wstart[r * n + c];
            if (i == N - 1) v += p.Wgoal[r * n + c];
            if (i < N - 1) {  // Phi^T Qinv Phi
#pragma unroll
                for (int k = 0; k < n; ++k) v += st.Phi[(k * n + r) * S + sI] * t[k];
                double u = 0.0;  // -Phi^T Qinv
                for (int k = 0; k < n; ++k) u -= st.Phi[(k * n + r) * S + sI] * st.Qinv[(k * n + c) * S + sI];
                st.KU[(r * n + c) * S + s] = u;
            }
            if (i > 0) v += st.Qinv[(r * n + c) * S + sP];
            st.KD[(r * n + c) * S + s] = v;
        }
    }
    for (int r = 0; r < n; ++r) {
        double e = 0.0;
        if (i == 0)
            for (int k = 0; k < n; ++k) e += p.Wstart[r * n + k] * p.mu_start[k];
        if (i == N - 1)
            for (int k = 0; k < n; ++k) e += p.Wgoal[r * n + k] * p.mu_goal[k];
        if (i < N - 1) {  // -Phi^T Qinv abar
            for (int k = 0; k < n; ++k) {
                double t = 0.0;
                for (int l = 0; l < n; ++l) t += st.Qinv[(k * n + l) * S + sI] * st.abar[l * S + sI];
                e -= st.Phi[(k * n + r) * S + sI] * t;
            }
        }
        if (i > 0) {
            for (int l = 0; l < n; ++l) e += st.Qinv[(r * n + l) * S + sP] * st.abar[l * S + sP];
        }
        st.eta[r * S + s] = e;
    }
}

hipError_t launch_prior_build(const DevState& st, int plan_lo, int plan_hi, int maxN, hipStream_t s) {
    if (plan_hi <= plan_lo || maxN <= 0) return hipSuccess;
    hipLaunchKernelGGL(prior_build_kernel, dim3(maxN, plan_hi - plan_lo), dim3(kPriorThreads), 0, s, st, plan_lo);
    return hipGetLastError();
}

hipError_t launch_prior_assemble(const DevState& st, int plan_lo, int plan_hi, int maxN, hipStream_t s) {
    if (plan_hi <= plan_lo || maxN <= 0) return hipSuccess;
    const int th = kAssembleThreads;
    const dim3 grid((maxN + th - 1) / th, plan_hi - plan_lo);
    switch (st.n) {
        case 2: hipLaunchKernelGGL(prior_assemble_kernel<2>, grid, dim3(th), 0, s, st, plan_lo); break;
        case 4: hipLaunchKernelGGL(prior_assemble_kernel<4>, grid, dim3(th), 0, s, st, plan_lo); break;
        case 6: hipLaunchKernelGGL(prior_assemble_kernel<6>, grid, dim3(th), 0, s, st, plan_lo); break;
        case 8: hipLaunchKernelGGL(prior_assemble_kernel<8>, grid, dim3(th), 0, s, st, plan_lo); break;
        case 14: hipLaunchKernelGGL(prior_assemble_kernel<14>, grid, dim3(th), 0, s, st, plan_lo); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// SoA <-> [N][...] conversion
// ---------------------------------------------------------------------------
__global__ void gather_kernel(DevState st, int what, int plan, double* out) {
    const PlanDev& p = st.plans[plan];
    const int n = st.n, N = p.N, d = p.d;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t S = st.S, s = p.off + i;
    const int n2 = n * n;
    const bool act = p.coll_kind != PGVIMP_COLL_NONE && !(p.coll_states == 1 && (i == 0 || i == N - 1));
    switch (what) {
        case G_SD:
            if (i < N)
                for (int e = 0; e < n2; ++e) out[(int64_t)i * n2 + e] = st.SD[e * S + s];
            break;
        case G_SU:
            if (i < N - 1)
                for (int e = 0; e < n2; ++e) out[(int64_t)i * n2 + e] = st.SU[e * S + s];
            break;
        case G_MU:
            if (i < N)
                for (int e = 0; e < n; ++e) out[(int64_t)i * n + e] = st.mu[e * S + s];
            break;
        case G_LD:
            if (i < N)
                for (int e = 0; e < n2; ++e) out[(int64_t)i * n2 + e] = st.LD[e * S + s];
            break;
        case G_LU:
            if (i < N - 1)
                for (int e = 0; e < n2; ++e) out[(int64_t)i * n2 + e] = st.LU[e * S + s];
            break;
        case G_ECOL:
            if (i < N) out[i] = act ? st.Ecol[s] : 0.0;
            break;
        case G_GEMB:
            if (i < N) {
                for (int e = 0; e < n; ++e) out[(int64_t)i * n + e] = 0.0;
                if (act)
                    for (int a = 0; a < d; ++a) out[(int64_t)i * n + p.coll_index[a]] = st.gcol[a * S + s];
            }
            break;
        case G_HEMB:
            if (i < N) {
                for (int e = 0; e < n2; ++e) out[(int64_t)i * n2 + e] = 0.0;
                if (act)
                    for (int a = 0; a < d; ++a)
                        for (int b = 0; b < d; ++b)
                            out[(int64_t)i * n2 + p.coll_index[a] * n + p.coll_index[b]] = st.Hcol[(a * d + b) * S + s];
            }
            break;
        case G_EPRI:
            if (i < N) {
                out[1 + i] = st.Epri[s];  // transitions 0..N-2 then goal at N
                if (i == 0) out[0] = st.Epri[S + plan];
            }
            break;
        default:
            break;
    }
}

__global__ void scatter_kernel(DevState st, int what, int plan, const double* in) {
    const PlanDev& p = st.plans[plan];
    const int n = st.n, N = p.N;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t S = st.S, s = p.off + i;
    const int n2 = n * n;
    if (what == G_MU && i < N)
        for (int e = 0; e < n; ++e) st.mu[e * S + s] = in[(int64_t)i * n + e];
    if (what == G_LD && i < N)
        for (int e = 0; e < n2; ++e) st.LD[e * S + s] = in[(int64_t)i * n2 + e];
    if (what == G_LU && i < N - 1)
        for (int e = 0; e < n2; ++e) st.LU[e * S + s] = in[(int64_t)i * n2 + e];
    if (what == G_SD && i < N)
        for (int e = 0; e < n2; ++e) st.SD[e * S + s] = in[(int64_t)i * n2 + e];
}

hipError_t launch_gather(const DevState& st, int what, int plan, int N, double* out, hipStream_t s) {
    const int th = 64;
    hipLaunchKernelGGL(gather_kernel, dim3((N + th - 1) / th), dim3(th), 0, s, st, what, plan, out);
    return hipGetLastError();
}

hipError_t launch_scatter(const DevState& st, int what, int plan, int N, const double* in, hipStream_t s) {
    const int th = 64;
    hipLaunchKernelGGL(scatter_kernel, dim3((N + th - 1) / th), dim3(th), 0, s, st, what, plan, in);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Statistical linear regression (Sec. 6.2): per state, N(mu_i, Sigma_ii),
// tensor GH rule with p points per axis over all n coordinates:
//   fbar = sum W f(x_j),  F = sum W f(x_j) xi_j^T,
//   A = P_yx P_xx^-1 = F L^T (L L^T)^-1 = F L^-1,  a = fbar - A mu
// (sum W xi = 0 removes fbar from P_yx; P_xx = L (sum W xi xi^T) L^T = Sigma).
// One wavefront per state; FP64.
// ---------------------------------------------------------------------------
constexpr int kSlrThreads = 64;
constexpr int kSlrMaxN = 6;

__device__ void quad2d_drift(const double* x, double g, double* f) {
    double sp, cp;
    sincos(x[2], &sp, &cp);
    const double vx = x[3], vz = x[4], w = x[5];
    f[0] = vx * cp - vz * sp;
    f[1] = vx * sp + vz * cp;
    f[2] = w;
    f[3] = vz * w - g * sp;
    f[4] = -vx * w - g * cp;
    f[5] = 0.0;
}

__global__ void __launch_bounds__(kSlrThreads) slr_kernel(DevState st, int plan, double g, int P, double* A_out,
                                                          double* a_out, int write_model) {
    constexpr int n = kSlrMaxN;
    PlanDev& p = st.plans[plan];
    const int i = blockIdx.x;
    const int64_t S = st.S, s = p.off + i;
    const int lane = threadIdx.x;
    double mu[n], Sg[n * n], L[n * n];
    for (int e = 0; e < n; ++e) mu[e] = st.mu[e * S + s];
    for (int e = 0; e < n * n; ++e) Sg[e] = st.SD[e * S + s];
    for (int e = 0; e < n * n; ++e) L[e] = 0.0;
    bool ok = true;
    for (int j = 0; j < n; ++j) {
        double d = Sg[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        ok = ok && d > 0.0;
        const double l = sqrt(ok ? d : 1.0);
        L[j * n + j] = l;
        for (int r = j + 1; r < n; ++r) {
            double v = Sg[r * n + j];
            for (int k = 0; k < j; ++k) v -= L[r * n + k] * L[j * n + k];
            L[r * n + j] = v / l;
        }
    }
    const double* xi1 = st.gh_x64 + P * kMaxGH;
    const double* w1 = st.gh_w64 + P * kMaxGH;
    int nodes = 1;
    for (int k = 0; k < n; ++k) nodes *= P;
    double fb[n], F[n * n];
    for (int e = 0; e < n; ++e) fb[e] = 0.0;
    for (int e = 0; e < n * n; ++e) F[e] = 0.0;
    for (int j = lane; j < nodes; j += kSlrThreads) {
        double xi[n], x[n], f[n], W = 1.0;
        int r = j;
        for (int a = 0; a < n; ++a) {
            const int k = r % P;
            r /= P;
            xi[a] = xi1[k];
            W *= w1[k];
        }
        for (int a = 0; a < n; ++a) {
            double v = mu[a];
            for (int c = 0; c <= a; ++c) v += L[a * n + c] * xi[c];
            x[a] = v;
        }
        quad2d_drift(x, g, f);
        for (int a = 0; a < n; ++a) {
            const double wf = W * f[a];
            fb[a] += wf;
            for (int c = 0; c < n; ++c) F[a * n + c] += wf * xi[c];
        }
    }
    for (int o = kSlrThreads / 2; o >= 1; o >>= 1) {
        for (int e = 0; e < n; ++e) fb[e] += __shfl_xor(fb[e], o, kSlrThreads);
        for (int e = 0; e < n * n; ++e) F[e] += __shfl_xor(F[e], o, kSlrThreads);
    }
    if (lane != 0) return;
    // Li = L^-1; A = F Li; a = fbar - A mu
    double Li[n * n];
    for (int e = 0; e < n * n; ++e) Li[e] = 0.0;
    for (int a = 0; a < n; ++a) {
        const double inv = 1.0 / L[a * n + a];
        Li[a * n + a] = inv;
        for (int c = 0; c < a; ++c) {
            double v = 0.0;
            for (int k = c; k < a; ++k) v += L[a * n + k] * Li[k * n + c];
            Li[a * n + c] = -v * inv;
        }
    }
    double A[n * n], av[n];
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            double v = 0.0;
            for (int k = c; k < n; ++k) v += F[r * n + k] * Li[k * n + c];
            A[r * n + c] = ok ? v : NAN;
        }
    for (int r = 0; r < n; ++r) {
        double v = fb[r];
        for (int c = 0; c < n; ++c) v -= A[r * n + c] * mu[c];
        av[r] = v;
    }
    if (A_out)
        for (int e = 0; e < n * n; ++e) A_out[(int64_t)i * n * n + e] = A[e];
    if (a_out)
        for (int e = 0; e < n; ++e) a_out[(int64_t)i * n + e] = av[e];
    if (write_model && i == 0 && lane == 0) p.ltv = 1;  // the intervals now differ
    if (write_model && i < p.N - 1) {
        for (int e = 0; e < n * n; ++e) p.A[(int64_t)i * n * n + e] = A[e];
        for (int e = 0; e < n; ++e) p.a[(int64_t)i * n + e] = av[e];
    }
}

hipError_t launch_slr_model(const DevState& st, int plan, int N, double gravity, int P, double* A_out,
                            double* a_out, int write_model, hipStream_t s) {
    if (st.n != kSlrMaxN) return hipErrorInvalidValue;
    hipLaunchKernelGGL(slr_kernel, dim3(N), dim3(kSlrThreads), 0, s, st, plan, gravity, P, A_out, a_out,
                       write_model);
    return hipGetLastError();
}

}  // namespace pg
