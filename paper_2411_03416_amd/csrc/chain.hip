// Dispatch of the chain kernels over the supported state dimensions (each
// dimension is compiled in its own translation unit, chain_n<k>.hip).
#include "ctx.h"

namespace pg {

template <int n>
hipError_t launch_chain_n(const DevState& st, int mode, int lo, int hi, hipStream_t s);
template <int n>
hipError_t launch_prior_costs_n(const DevState& st, int plan, int N, hipStream_t s);
template <int n>
hipError_t launch_iteration_n(const DevState& st, int phw, int part, int round, hipStream_t s);

bool chain_supported(int n) { return n == 2 || n == 4 || n == 6 || n == 8 || n == 14; }

hipError_t launch_chain(const DevState& st, int mode, int lo, int hi, hipStream_t s) {
    switch (st.n) {
        case 2: return launch_chain_n<2>(st, mode, lo, hi, s);
        case 4: return launch_chain_n<4>(st, mode, lo, hi, s);
        case 6: return launch_chain_n<6>(st, mode, lo, hi, s);
        case 8: return launch_chain_n<8>(st, mode, lo, hi, s);
        case 14: return launch_chain_n<14>(st, mode, lo, hi, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_iteration(const DevState& st, int phw, int part, int round, hipStream_t s) {
    switch (st.n) {
        case 2: return launch_iteration_n<2>(st, phw, part, round, s);
        case 4: return launch_iteration_n<4>(st, phw, part, round, s);
        case 6: return launch_iteration_n<6>(st, phw, part, round, s);
        case 8: return launch_iteration_n<8>(st, phw, part, round, s);
        case 14: return launch_iteration_n<14>(st, phw, part, round, s);
        default: return hipErrorInvalidValue;
    }
}

// Windows of the step-size halving rule (Alg. 1): every plan evaluates its
// step sizes window by window, each window continuing where the previous
// one ended, until a window holds a passing step.  For window `round`, a
// plan still searching (every plan with an iteration to run, in window 0)
// takes the next clamp(wbudget / searching, Wmin, W) step sizes, never past
// max_bisect: the compute units are shared by the plans that still need
// them, and a few stragglers get wide windows.  With a lookahead, window 0
// is cut to the previous iteration's count plus the lookahead.  The window's
// trials are listed plan by plan in wlist.  Widths change speed, never the
// accepted step.  One block; plans are taken in chunks of 256, thread tid
// owning plan chunk + tid.
constexpr int kWindowThreads = 256;
constexpr int kWindowPlansPerThread = 4;  // plans a thread keeps in registers between the passes
__global__ void __launch_bounds__(kWindowThreads) window_kernel(DevState st, int phw, int round) {
    __shared__ int sh[kWindowThreads];
    __shared__ int total;
    const int tid = threadIdx.x;
    if (tid == 0) total = 0;
    __syncthreads();
    // pass 1: which plans still search; every field a plan needs is loaded
    // at once (no short-circuit chains of dependent loads)
    int next[kWindowPlansPerThread], want[kWindowPlansPerThread];
    int mine = 0;
#pragma unroll
    for (int k = 0; k < kWindowPlansPerThread; ++k) {
        const int pid = tid + k * kWindowThreads;
        next[k] = 0;
        want[k] = 0;
        if (pid >= phw) continue;
        const PlanDev& p = st.plans[pid];
        const int active = p.active, phase = p.phase, fp = p.firstpass, wn = p.wnext, mb = p.max_bisect;
        const int it = p.iters_done, tr = p.trials;
        const int live = active != 0 && phase == 0;
        next[k] = round == 0 ? 0 : wn;
        const int s = live && (round == 0 || fp == kNoPass) && next[k] < mb;
        // a plan's own cap: max_bisect, and in window 0 the lookahead cut
        int cap = mb - next[k];
        if (round == 0 && st.lookahead > 0 && it > 0) cap = min(cap, max(1, tr + st.lookahead));
        want[k] = s ? cap : 0;
        mine += s;
    }
    // plans beyond the register-held ones are visited again in pass 2
    for (int pid = tid + kWindowPlansPerThread * kWindowThreads; pid < phw; pid += kWindowThreads) {
        const PlanDev& p = st.plans[pid];
        const int fp = p.firstpass, wn = round == 0 ? 0 : p.wnext;
        mine += p.active && p.phase == 0 && (round == 0 || fp == kNoPass) && wn < p.max_bisect;
    }
    atomicAdd(&total, mine);
    __syncthreads();
    const int width = max(st.Wmin, min(st.W, st.wbudget / max(total, 1)));
    // pass 2: widths, then the work list in plan order (a block-wide scan per
    // chunk of 256 plans)
    int base = 0;
    for (int c0 = 0, k = 0; c0 < phw; c0 += kWindowThreads, ++k) {
        const int pid = c0 + tid;
        int w = 0;
        if (pid < phw) {
            PlanDev& p = st.plans[pid];
            int nx, cap;
            if (k < kWindowPlansPerThread) {
                nx = next[k];
                cap = want[k];
            } else {
                const int active = p.active, phase = p.phase, fp = p.firstpass, wn = p.wnext, mb = p.max_bisect;
                const int it = p.iters_done, tr = p.trials;
                nx = round == 0 ? 0 : wn;
                const int s = active != 0 && phase == 0 && (round == 0 || fp == kNoPass) && nx < mb;
                cap = mb - nx;
                if (round == 0 && st.lookahead > 0 && it > 0) cap = min(cap, max(1, tr + st.lookahead));
                cap = s ? cap : 0;
            }
            w = min(width, cap);
            if (round == 0 && p.active && p.phase == 0) p.firstpass = kNoPass;
            p.wstart = nx;
            p.wnext = nx + w;
            p.wwidth = w;
        }
        __syncthreads();
        sh[tid] = w;
        __syncthreads();
        for (int o = 1; o < kWindowThreads; o <<= 1) {
            const int v = tid >= o ? sh[tid - o] : 0;
            __syncthreads();
            sh[tid] += v;
            __syncthreads();
        }
        const int first = base + sh[tid] - w;
        for (int t = 0; t < w; ++t) st.wlist[1 + first + t] = pid * 64 + t;
        base += sh[kWindowThreads - 1];
    }
    if (tid == 0) st.wlist[0] = base;
}

hipError_t launch_window(const DevState& st, int phw, int round, hipStream_t s) {
    // without a lookahead, window 0 is uniform and set by the prep kernel
    if (phw <= 0 || (round == 0 && st.lookahead == 0)) return hipSuccess;
    hipLaunchKernelGGL(window_kernel, dim3(1), dim3(kWindowThreads), 0, s, st, phw, round);
    return hipGetLastError();
}

hipError_t launch_prior_costs(const DevState& st, int plan, int N, hipStream_t s) {
    switch (st.n) {
        case 2: return launch_prior_costs_n<2>(st, plan, N, s);
        case 4: return launch_prior_costs_n<4>(st, plan, N, s);
        case 6: return launch_prior_costs_n<6>(st, plan, N, s);
        case 8: return launch_prior_costs_n<8>(st, plan, N, s);
        case 14: return launch_prior_costs_n<14>(st, plan, N, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pg
