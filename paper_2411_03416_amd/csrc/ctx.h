// Device-resident plan table and the context that owns it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "pgvimp.h"

namespace pg {

constexpr int kMaxSeg = 64;      // chain segments per plan (upper bound)
constexpr int kChainThreads = 64; // one wavefront per factorization, one lane per segment
constexpr int kTrialThreads = 128; // trial kernel: marginals and mean solve side by side
constexpr int kIterThreads = 128;  // prep/select kernels (uses the trial kernel's per-thread slots)
constexpr int kIterBlocks = 8;     // prep/select blocks per plan (at most W)
constexpr int kMaxBisect = 64;     // step sizes of the halving sequence per iteration (upper bound)
constexpr int kMaxGH = 10;        // Gauss-Hermite points per dimension
// n x n temporaries a chain-kernel thread may hold at once (n > 4; smaller
// blocks live in registers).  Deepest call paths: segment elimination 15
// live blocks + the first coupling 1 + Cholesky inverse 2 = 18 (8 vectors);
// segment backward sweep 16 blocks; mean-solve backward sweep 10 vectors.
constexpr int kTwsBlocks = 20;
constexpr int kTwsVecs = 16;
// For n = 6, plans of at most this many segments keep the sweeps' block
// temporaries in LDS (one slice per lane of both halves).
constexpr int kLdsWsSegments = 12;
constexpr int32_t kNoPass = 0x7fffffff;
constexpr int kNumXcd = 8;  // XCDs; workgroup b of a launch runs on XCD b mod 8

// Per-plan parameters and statistics, read by every kernel.  One entry per
// plan slot; an empty slot has active = 0.
struct PlanDev {
    int32_t active, N, off, nseg;
    int32_t iters_left, iters_done, max_bisect, coll_kind;
    int32_t d, gh_points, gx, gy;
    int32_t gz, n_spheres, coll_states, status;
    int32_t trials, m, n_iters, trials_total;
    // window of step sizes being evaluated: numbers [wstart, wstart + wwidth);
    // wnext = step sizes evaluated so far in this iteration
    int32_t wstart, wwidth, wnext;
    int32_t firstpass;  // smallest passing step size number so far (kNoPass if none)
    int32_t evals_total;  // step sizes evaluated since the (re)start, speculative ones included
    int32_t ltv;  // 0: every interval has the same dynamics (A, a, B)
    int32_t phase;  // 0 = iteration pending, 1 = no iteration (budget spent)
    int32_t coff;   // start of the plan's chain-order range (capacity Sc)
    int32_t coll_index[PGVIMP_MAX_COLL_DIM];
    int32_t quadrature;  // PGVIMP_QUAD_*
    int32_t update;      // PGVIMP_UPDATE_*
    int32_t rule_n;      // sparse rule: nodes (rows of rule64 / rule32)
    const double* rule64;  // sparse rule rows (xi[0..d-1], W), FP64
    const float* rule32;   // the same rows in FP32
    double temperature, beta_max, kl_bound, cell, dt;
    double inv_cell, hinge_eps, obs_weight, logdet;
    double origin[3];
    double beta, kl, E_coll, E_prior, entropy;
    double iter_temperature, entropy_cost, total_cost;  // cost breakdown of q_k (last iteration)
    const float* sdf;
    const float* sdfq;  // the four corners of every cell of each z-slice (see launch_build_quads)
    // model block (FP64) laid out by the host, see Layout in api.cpp
    double* Wstart;  // Sig_start^-1 [n*n]   (written by the prior kernel)
    double* Wgoal;   // Sig_goal^-1 [n*n]
    const double* mu_start;
    const double* mu_goal;
    const double* Sig_start;
    const double* Sig_goal;
    const double* Qc;    // [m*m]
    double* A;     // [N-1][n*n]  (rewritten by statistical linearisation)
    double* a;     // [N-1][n]
    const double* B;     // [N-1][n*m]
    const double* radius;  // [n_spheres]
    const double* fk;      // base[3], len[7], frac[S], axes[7], link[S] (as doubles)
};

// Device arrays shared by the kernels.  Per-state arrays are SoA:
// X[e * S + s] for entry e of state s, S = capacity in states.
struct DevState {
    int64_t S;       // state capacity
    int32_t n, P;    // state dim, plan capacity
    PlanDev* plans;  // [P]
    int32_t* state_plan;  // [S] plan of each state or -1
    // prior
    double *KD, *KU, *eta;      // K^-1 blocks and K^-1 mu_bar
    double *Phi, *Qinv, *abar;  // per interval (index = state of its start)
    // current iterate
    double *LD, *LU, *mu;  // precision blocks and mean
    double *SD, *SU;       // marginal covariances
    // chain-order copies (capacity Sc) of one iteration's inputs: K^-1 + H
    // (collision Hessians on the diagonal blocks), K^-1, Lambda_k, the mean-
    // solve right-hand side parts rb = eta - g and Lmu = Lambda_k mu_k, mu_k
    int64_t Sc;
    double *cKH, *cKD, *cLD, *cKU, *cLU, *crb, *cLmu, *cmu;
    // trial iterates in chain order: W slots, slot t of position q at t * Sc + q
    // (stride W * Sc)
    double *Tmu, *TSD, *TSU;
    double* tres;  // per (plan, step size number < kMaxBisect): passed, KL, log det, trial slot
    int32_t W;     // trial slots per plan = the widest window of step sizes
    int32_t Wmin;  // the narrowest window (trial_width)
    int32_t wbudget;      // trial workgroups a window may start at once (compute units)
    // work list of the current window: [0] = item count, then one item per
    // trial workgroup, plan * 64 + slot, plan by plan; [0] = -w marks the
    // uniform first window of width w (items decoded from the workgroup)
    int32_t* wlist;
    int32_t iter_blocks;  // blocks per plan of the prep and select kernels
    int32_t lookahead;    // first-window lookahead (0 = full first window)
    double* psum;         // per (plan, prep block): partial E_coll, E_prior
    // collision expectations (d-dim, not embedded): E [S], g [d][S], H [d*d][S]
    double *Ecol, *gcol, *Hcol;
    // prior factor costs [S] (transition starting at state s) and end costs
    double* Epri;
    // chain workspace: sweep temporaries [2][ws_stride][W * Sc] and segment
    // scratch [P][W][2][seg_stride][kMaxSeg]
    double* ws;
    double* seg;
    int32_t ws_stride, seg_stride;
    // per-thread block temporaries of the chain kernels: [P][kChainThreads]
    // slices of tws_stride doubles (kTwsBlocks n x n blocks and kTwsVecs
    // n-vectors each)
    double* tws;
    int64_t tws_stride;
    int* flags;  // [0]: a block workspace request overflowed
    // Gauss-Hermite 1-D tables [kMaxGH+1][kMaxGH] (row p), FP64 and FP32
    const double* gh_x64;
    const double* gh_w64;
    const float* gh_x32;
    const float* gh_w32;
};

// First-fit allocator over [0, capacity) with coalescing free list.
class RangeAlloc {
  public:
    explicit RangeAlloc(int64_t cap = 0) { reset(cap); }
    void reset(int64_t cap) {
        free_.clear();
        if (cap > 0) free_[0] = cap;
        cap_ = cap;
    }
    int64_t alloc(int64_t len, int64_t align = 1) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            int64_t start = (it->first + align - 1) / align * align;
            int64_t end = it->first + it->second;
            if (start + len <= end) {
                int64_t b = it->first;
                free_.erase(it);
                if (start > b) free_[b] = start - b;
                if (start + len < end) free_[start + len] = end - (start + len);
                used_[start] = len;
                return start;
            }
        }
        return -1;
    }
    void release(int64_t start) {
        auto u = used_.find(start);
        if (u == used_.end()) return;
        int64_t len = u->second;
        used_.erase(u);
        auto it = free_.emplace(start, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t high_water() const {
        int64_t hw = 0;
        for (auto& u : used_) hw = std::max(hw, u.first + u.second);
        return hw;
    }

  private:
    std::map<int64_t, int64_t> free_, used_;
    int64_t cap_ = 0;
};

}  // namespace pg

// Kernel launchers (defined in the .hip translation units).
namespace pg {
// prior build for plans [plan_lo, plan_hi) of up to maxN states each
hipError_t launch_prior_build(const DevState& st, int plan_lo, int plan_hi, int maxN, hipStream_t s);
hipError_t launch_prior_assemble(const DevState& st, int plan_lo, int plan_hi, int maxN, hipStream_t s);
hipError_t launch_chain(const DevState& st, int mode, int plan_lo, int plan_hi, hipStream_t s);
// parts of one proximal iteration for plans [0, phw): 0 = prep, 1 = trial
// (each plan's current window), 2 = select
hipError_t launch_iteration(const DevState& st, int phw, int part, int round, hipStream_t s);
// Window `round` of step sizes of the current iteration for plans [0, phw).
hipError_t launch_window(const DevState& st, int phw, int round, hipStream_t s);
// collision expectations of plans [plan_lo, plan_hi) of up to maxN states each
hipError_t launch_expect(const DevState& st, int coll_kind, int d, int p, int quadrature, int precision, int group,
                         int plan_lo,
                         int plan_hi, int maxN, int respect_budget, hipStream_t s);
hipError_t launch_prior_costs(const DevState& st, int plan, int N, hipStream_t s);
hipError_t launch_gather(const DevState& st, int what, int plan, int N, double* out, hipStream_t s);
hipError_t launch_scatter(const DevState& st, int what, int plan, int N, const double* in, hipStream_t s);
hipError_t launch_slr_model(const DevState& st, int plan, int N, double gravity, int p, double* A_out,
                            double* a_out, int write_model, hipStream_t s);
bool chain_supported(int n);
// Writes the corners (v00, v01, v10, v11) of each of the (gx - 1)(gy - 1)
// cells of every z-slice of sdf [gz][gy][gx] to quad, 16 bytes per cell.
hipError_t launch_build_quads(const float* sdf, int gx, int gy, int gz, float* quad, hipStream_t s);
bool expect_supported(int coll_kind, int d, int p, int group, int quadrature);
// factors per expectation workgroup for a launch over `plans` plan slots of
// at most maxN states (group 0 = chosen from the batch)
int expect_group_for(int group, int plans, int maxN, int cus);

// modes of the chain kernel
enum ChainMode { CHAIN_INIT = 0, CHAIN_MARGINALS = 1, CHAIN_REINIT = 3 };
// what to gather/scatter between SoA device arrays and [N][..] host layouts
enum GatherWhat {
    G_SD = 0, G_SU = 1, G_MU = 2, G_LD = 3, G_LU = 4, G_ECOL = 5, G_GEMB = 6, G_HEMB = 7, G_EPRI = 8
};
}  // namespace pg
