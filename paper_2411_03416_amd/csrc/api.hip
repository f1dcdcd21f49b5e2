// Host side of the C ABI declared in include/pgvimp.h: context and arena,
// plan admission/removal, launch sequencing, HIP-graph capture of the
// iteration loop, and kernel timing.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <type_traits>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "ctx.h"

using namespace pg;

namespace {

constexpr int64_t kAlign = 256;
constexpr int kDefaultTrialWidth = 8;
constexpr int kDefaultTrialWidthLarge = 24;  // n >= 6
constexpr int kMaxTrialWidth = 64;
constexpr int kMaxSparseNodes = 65536;  // nodes of a sparse quadrature rule

struct PlanHost {
    bool active = false;
    int N = 0;
    int64_t off = -1;
    int64_t coff = -1;  // chain-order range
    int64_t heap_off = -1;  // model block
    int64_t map_off = -1;   // SDF block (shared by plans with identical maps)
    int coll_kind = 0, d = 0, p = 0, quadrature = 0;
    double dt = 0.0;
    int group = 0;  // factors per expectation workgroup (0 = chosen per launch)
    int max_bisect = 0;
};

// Identity of an SDF grid: its dimensions and two independent 64-bit
// hashes of its values.  Plans whose maps have equal keys share one device
// copy (refcounted); a collision of both hashes between different grids of
// equal dimensions is the only way two maps could be confused.
struct MapKey {
    int32_t gx, gy, gz;
    uint64_t h1, h2;
    bool operator<(const MapKey& o) const {
        if (gx != o.gx) return gx < o.gx;
        if (gy != o.gy) return gy < o.gy;
        if (gz != o.gz) return gz < o.gz;
        if (h1 != o.h1) return h1 < o.h1;
        return h2 < o.h2;
    }
};
struct MapEntry {
    int64_t off;
    int refs;
};

MapKey map_key(const float* sdf, int gx, int gy, int gz) {
    const size_t count = (size_t)gx * gy * gz;
    uint64_t h1 = 0xcbf29ce484222325ull, h2 = 0x9e3779b97f4a7c15ull;
    for (size_t i = 0; i < count; ++i) {
        uint32_t w;
        memcpy(&w, sdf + i, 4);
        h1 = (h1 ^ w) * 0x100000001b3ull;  // FNV-1a over 32-bit words
        h2 += (uint64_t)w * 0xff51afd7ed558ccdull + i;
        h2 = (h2 << 31) | (h2 >> 33);
        h2 *= 0xc4ceb9fe1a85ec53ull;
    }
    return MapKey{gx, gy, gz, h1, h2};
}

struct ClassKey {
    int kind, d, p, group, quadrature;
    bool operator==(const ClassKey& o) const {
        return kind == o.kind && d == o.d && p == o.p && group == o.group && quadrature == o.quadrature;
    }
};

}  // namespace

struct pgvimp_ctx {
    pgvimp_engine_cfg cfg{};
    int n = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* arena = nullptr;
    uint64_t arena_bytes = 0;
    bool own_arena = false;
    char* heap = nullptr;
    int64_t heap_bytes = 0;
    DevState st{};
    RangeAlloc states, cstates, heapalloc;  // states, chain-order ranges, heap
    std::map<MapKey, MapEntry> maps;        // live SDF grids on the heap
    std::vector<double> ghX, ghW;            // 1-D Gauss-Hermite rules [kMaxGH+1][kMaxGH]
    std::vector<PlanHost> plans;
    std::vector<PlanDev> pdev;  // host mirror of the device plan table
    // staging for host I/O
    double* stage = nullptr;
    size_t stage_bytes = 0;
    // graph cache
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int g_iters = -1;
    int64_t g_hw = -1;
    bool g_restart = false;
    int g_rounds = -1;
    int g_maxN = 0;
    std::vector<ClassKey> g_classes;
    bool g_profiled = false;
    // profiling
    bool profile = false;
    std::vector<hipEvent_t> ev;  // pairs per timed launch
    std::vector<int> ev_kind;    // PGVIMP_K_* of each pair
    double t_kind[PGVIMP_NKERNELS] = {};
    int64_t n_kind[PGVIMP_NKERNELS] = {};
    size_t ev_used = 0;
    std::string err;
};

static std::string g_create_err;

#define FAIL(ctx, code, ...)                                                    \
    do {                                                                        \
        char _b[512];                                                           \
        snprintf(_b, sizeof(_b), __VA_ARGS__);                                  \
        if (ctx) (ctx)->err = _b; else g_create_err = _b;                       \
        return code;                                                            \
    } while (0)

#define HCK(ctx, call)                                                              \
    do {                                                                            \
        hipError_t _e = (call);                                                     \
        if (_e != hipSuccess)                                                       \
            FAIL(ctx, PGVIMP_EDEVICE, "%s: %s (%s:%d)", #call, hipGetErrorString(_e), \
                 __FILE__, __LINE__);                                               \
    } while (0)

namespace {

int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Probabilists' Gauss-Hermite rules for p = 1..kMaxGH: nodes are the roots
// of He_p, bracketed by sign changes on a fine grid and refined by Newton
// steps on the three-term recurrence; weights by the Christoffel formula
// w_i = 1 / sum_{k<p} He_k(x_i)^2 / k!, which normalises them to sum to 1.
void hermite_eval(int p, double x, double* hp, double* hpm1) {
    double h0 = 1.0, h1 = x;
    if (p == 0) {
        *hp = 1.0;
        *hpm1 = 0.0;
        return;
    }
    for (int k = 1; k < p; ++k) {
        const double h2 = x * h1 - k * h0;
        h0 = h1;
        h1 = h2;
    }
    *hp = h1;
    *hpm1 = h0;
}

void gh_tables(std::vector<double>& X, std::vector<double>& W) {
    X.assign((kMaxGH + 1) * kMaxGH, 0.0);
    W.assign((kMaxGH + 1) * kMaxGH, 0.0);
    for (int p = 1; p <= kMaxGH; ++p) {
        std::vector<double> roots;
        const double lim = 2.0 * sqrt((double)p) + 2.0, step = 1e-3;
        double hp, hm, prev_x = -lim, prev_v;
        hermite_eval(p, prev_x, &prev_v, &hm);
        for (double x = -lim + step; x <= lim + step; x += step) {
            double v;
            hermite_eval(p, x, &v, &hm);
            if (v == 0.0 || (v > 0) != (prev_v > 0)) {
                double r = (v == 0.0) ? x : prev_x - prev_v * (x - prev_x) / (v - prev_v);
                for (int it = 0; it < 60; ++it) {
                    hermite_eval(p, r, &hp, &hm);
                    const double dr = hp / (p * hm);  // He_p' = p He_{p-1}
                    r -= dr;
                    if (fabs(dr) < 1e-17 * (1.0 + fabs(r))) break;
                }
                roots.push_back(r);
            }
            prev_x = x;
            prev_v = v;
        }
        std::sort(roots.begin(), roots.end());
        for (int i = 0; i < p && i < (int)roots.size(); ++i) {
            const double x = (p % 2 == 1 && i == p / 2) ? 0.0 : roots[i];
            double s = 0.0, h0 = 1.0, h1 = x, fact = 1.0;
            s += 1.0;
            if (p > 1) s += x * x;
            for (int k = 2; k < p; ++k) {
                const double h2 = x * h1 - (k - 1) * h0;
                h0 = h1;
                h1 = h2;
                fact *= k;
                s += h1 * h1 / fact;
            }
            X[p * kMaxGH + i] = x;
            W[p * kMaxGH + i] = 1.0 / s;
        }
    }
}

// Smolyak sparse grid of level k in d dimensions (Sec. 4.3 Lemma 1):
// A(k, d) = sum_{q = max(0, k-d)}^{k-1} (-1)^(k-1-q) C(d-1, k-1-q)
//           sum_{levels l, l_j >= 1, |l| = d + q} U_{l_1} x ... x U_{l_d},
// U_l the l-point Gauss-Hermite rule.  Points shared by several tensor
// rules (coordinates equal to the exact zero of odd rules) are merged by
// adding their weights; rows keep the order of first appearance.  Returns
// rows (xi[0..d-1], W), or an empty vector past max_nodes.
void sparse_rule(int k, int d, const std::vector<double>& X, const std::vector<double>& W, int max_nodes,
                 std::vector<double>& rows) {
    rows.clear();
    std::map<std::vector<double>, size_t> index;
    auto binom = [](int a, int b) {
        double r = 1.0;
        for (int i = 1; i <= b; ++i) r = r * (a - b + i) / i;
        return r;
    };
    std::vector<int> lv(d), at(d);
    for (int q = std::max(0, k - d); q < k; ++q) {
        const double coef = (((k - 1 - q) % 2) ? -1.0 : 1.0) * binom(d - 1, k - 1 - q);
        // every levels vector with entries 1..q+1 summing to d + q
        std::fill(lv.begin(), lv.end(), 1);
        while (true) {
            int sum = 0;
            for (int a = 0; a < d; ++a) sum += lv[a];
            if (sum == d + q) {
                std::fill(at.begin(), at.end(), 0);
                while (true) {
                    std::vector<double> x(d);
                    double w = coef;
                    for (int a = 0; a < d; ++a) {
                        x[a] = X[lv[a] * kMaxGH + at[a]];
                        w *= W[lv[a] * kMaxGH + at[a]];
                    }
                    auto it = index.find(x);
                    if (it == index.end()) {
                        if ((int)index.size() >= max_nodes) {
                            rows.clear();
                            return;
                        }
                        index.emplace(x, rows.size());
                        rows.insert(rows.end(), x.begin(), x.end());
                        rows.push_back(w);
                    } else {
                        rows[it->second + d] += w;
                    }
                    int a = 0;
                    while (a < d && ++at[a] == lv[a]) at[a++] = 0;
                    if (a == d) break;
                }
            }
            int a = 0;
            while (a < d && ++lv[a] > q + 1) lv[a++] = 1;
            if (a == d) break;
        }
    }
}

bool finite_all(const double* v, int64_t cnt) {
    for (int64_t i = 0; i < cnt; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

bool host_spd(const double* A, int n) {
    std::vector<double> L(n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0.0)) return false;
        L[j * n + j] = sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = s / L[j * n + j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (fabs(A[i * n + j] - A[j * n + i]) > 1e-12 * (fabs(A[i * n + j]) + fabs(A[j * n + i]) + 1e-300))
                return false;
    return true;
}

// Segments of the chain for a plan of N states: about sqrt(N), at most
// N/2 (every segment keeps an interior state) and kMaxSeg.
int choose_segments(const pgvimp_ctx* c, int N, int requested = 0) {
    int s = requested > 0 ? requested : c->cfg.segments > 0 ? c->cfg.segments : (int)ceil(sqrt((double)N));
    s = std::min(s, kMaxSeg);
    s = std::min(s, std::max(1, N / 2));
    return std::max(s, 1);
}

int coll_dim_of(int kind) {
    switch (kind) {
        case PGVIMP_COLL_POINT2D: return 2;
        case PGVIMP_COLL_POINT3D: return 3;
        case PGVIMP_COLL_ARM3D: return PGVIMP_ARM_DOF;
        default: return 0;
    }
}

int ensure_stage(pgvimp_ctx* c, size_t bytes) {
    if (bytes <= c->stage_bytes) return PGVIMP_OK;
    if (c->stage) HCK(c, hipFree(c->stage));
    c->stage = nullptr;
    c->stage_bytes = 0;
    HCK(c, hipMalloc(&c->stage, bytes));
    c->stage_bytes = bytes;
    return PGVIMP_OK;
}

// Copy an [N][...] array gathered on the device to the caller.  Host
// output goes through `stage` when given (at least count doubles), else
// through the context's own staging buffer.
int gather_out(pgvimp_ctx* c, int what, int plan, int N, double* out, size_t count, double* stage = nullptr) {
    if (!out) return PGVIMP_OK;
    if (c->cfg.io_on_device) {
        HCK(c, launch_gather(c->st, what, plan, N, out, c->stream));
        return PGVIMP_OK;
    }
    if (!stage) {
        int rc = ensure_stage(c, std::max<size_t>(count, 1) * sizeof(double));
        if (rc) return rc;
        stage = c->stage;
    }
    HCK(c, launch_gather(c->st, what, plan, N, stage, c->stream));
    HCK(c, hipMemcpyAsync(out, stage, count * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HCK(c, hipStreamSynchronize(c->stream));
    return PGVIMP_OK;
}

int upload_plan(pgvimp_ctx* c, int plan) {
    HCK(c, hipMemcpyAsync(c->st.plans + plan, &c->pdev[plan], sizeof(PlanDev), hipMemcpyHostToDevice, c->stream));
    return PGVIMP_OK;
}

int download_plans(pgvimp_ctx* c) {
    int32_t flags[16] = {0};
    HCK(c, hipMemcpyAsync(c->pdev.data(), c->st.plans, sizeof(PlanDev) * c->pdev.size(), hipMemcpyDeviceToHost,
                          c->stream));
    HCK(c, hipMemcpyAsync(flags, c->st.flags, sizeof(flags), hipMemcpyDeviceToHost, c->stream));
    HCK(c, hipStreamSynchronize(c->stream));
    if (flags[0]) FAIL(c, PGVIMP_EDEVICE, "block workspace overflow in a chain kernel (library defect)");
    return PGVIMP_OK;
}

void drop_graph(pgvimp_ctx* c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->g_iters = -1;
}

int validate_problem(pgvimp_ctx* c, const pgvimp_problem* p) {
    const int n = c->n;
    if (!p) FAIL(c, PGVIMP_EINVAL, "null problem");
    if (p->n != n) FAIL(c, PGVIMP_EINVAL, "problem state dim %d != context dim %d", p->n, n);
    if (p->N < 1 || p->m < 1 || p->m > n) FAIL(c, PGVIMP_EINVAL, "bad sizes N=%d m=%d", p->N, p->m);
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) FAIL(c, PGVIMP_EINVAL, "dt must be positive");
    if (!p->A || !p->a || !p->B || !p->Qc || !p->mu_start || !p->Sig_start || !p->mu_goal || !p->Sig_goal)
        FAIL(c, PGVIMP_EINVAL, "null dynamics/boundary pointer");
    const int64_t cnt = p->ltv ? (int64_t)std::max(p->N - 1, 1) : 1;
    if (!finite_all(p->A, cnt * n * n) || !finite_all(p->a, cnt * n) || !finite_all(p->B, cnt * n * p->m) ||
        !finite_all(p->Qc, (int64_t)p->m * p->m) || !finite_all(p->mu_start, n) || !finite_all(p->mu_goal, n) ||
        !finite_all(p->Sig_start, (int64_t)n * n) || !finite_all(p->Sig_goal, (int64_t)n * n))
        FAIL(c, PGVIMP_EINVAL, "non-finite dynamics or boundary input");
    if (!host_spd(p->Sig_start, n) || !host_spd(p->Sig_goal, n) || !host_spd(p->Qc, p->m))
        FAIL(c, PGVIMP_EINVAL, "start/goal covariance or Qc not symmetric positive definite");
    if (!(p->temperature > 0.0) || !(p->beta_max > 0.0) || !(p->kl_bound > 0.0) || p->max_bisect < 1 ||
        p->max_bisect > kMaxBisect || p->n_iters < 0)
        FAIL(c, PGVIMP_EINVAL, "bad iteration parameters");
    if (p->mu_init && !finite_all(p->mu_init, (int64_t)p->N * n)) FAIL(c, PGVIMP_EINVAL, "non-finite mu_init");
    if (p->coll_kind == PGVIMP_COLL_NONE) return PGVIMP_OK;
    const int d = coll_dim_of(p->coll_kind);
    if (d == 0 || p->coll_dim != d || d > n) FAIL(c, PGVIMP_EINVAL, "collision kind/dim mismatch");
    for (int k = 0; k < d; ++k)
        if (p->coll_index[k] < 0 || p->coll_index[k] >= n) FAIL(c, PGVIMP_EINVAL, "coll_index out of range");
    const int group = p->expect_group > 0 ? p->expect_group : c->cfg.expect_group;
    if (p->update != PGVIMP_UPDATE_PROX && p->update != PGVIMP_UPDATE_NGD)
        FAIL(c, PGVIMP_EINVAL, "unknown update rule %d", p->update);
    if (p->quadrature != PGVIMP_QUAD_TENSOR && p->quadrature != PGVIMP_QUAD_SPARSE)
        FAIL(c, PGVIMP_EINVAL, "unknown quadrature %d", p->quadrature);
    if (!expect_supported(p->coll_kind, d, p->gh_points, group, p->quadrature))
        FAIL(c, PGVIMP_EINVAL, "unsupported quadrature shape kind=%d d=%d p=%d group=%d", p->coll_kind, d,
             p->gh_points, group);
    const bool is3 = p->coll_kind != PGVIMP_COLL_POINT2D;
    if (!p->sdf || p->gx < 2 || p->gy < 2 || (is3 ? p->gz < 2 : p->gz != 1))
        FAIL(c, PGVIMP_EINVAL, "bad SDF grid");
    // lookups address the table of cell corners (16 bytes a cell, about four
    // times the grid) with 32-bit byte offsets
    if ((int64_t)(p->gx - 1) * (p->gy - 1) * p->gz * 16 > INT32_MAX)
        FAIL(c, PGVIMP_EINVAL, "SDF grid too large: its table of cell corners is over 2 GiB");
    if (!(p->cell > 0.0) || !std::isfinite(p->hinge_eps) || !(p->obs_weight >= 0.0))
        FAIL(c, PGVIMP_EINVAL, "bad grid cell or hinge parameters");
    if (p->n_spheres < 1 || p->n_spheres > PGVIMP_MAX_SPHERES || !p->sphere_radius)
        FAIL(c, PGVIMP_EINVAL, "bad sphere count");
    if (p->coll_kind != PGVIMP_COLL_ARM3D && p->n_spheres != 1) FAIL(c, PGVIMP_EINVAL, "point robots take one sphere");
    if (p->coll_kind == PGVIMP_COLL_ARM3D) {
        if (!p->fk_base || !p->fk_link_len || !p->fk_sphere_frac || !p->fk_axes || !p->fk_sphere_link)
            FAIL(c, PGVIMP_EINVAL, "missing kinematic parameters");
        for (int k = 0; k < PGVIMP_ARM_DOF; ++k)
            if (p->fk_axes[k] < 0 || p->fk_axes[k] > 2) FAIL(c, PGVIMP_EINVAL, "bad joint axis");
        for (int s = 0; s < p->n_spheres; ++s) {
            if (p->fk_sphere_link[s] < 0 || p->fk_sphere_link[s] >= PGVIMP_ARM_DOF)
                FAIL(c, PGVIMP_EINVAL, "bad sphere link");
            if (s > 0 && p->fk_sphere_link[s] < p->fk_sphere_link[s - 1])
                FAIL(c, PGVIMP_EINVAL, "spheres must be sorted by link");
        }
    }
    return PGVIMP_OK;
}

}  // namespace

// Staging area of the allocation-free entry point (host output of
// pgvimp_factor_expectations_noalloc).  Each device holds its own copy for
// the life of the process; host code must use the per-device address from
// hipGetSymbolAddress, never the array's name.
constexpr int64_t kNoAllocDoubles = int64_t(1) << 19;  // 4 MiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current), looked
// up once per device.
hipError_t scratch_address(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = (double*)ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

extern "C" {

const char* pgvimp_last_error(const pgvimp_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

int64_t pgvimp_device_bytes(const pgvimp_ctx* ctx) { return ctx ? (int64_t)ctx->arena_bytes : 0; }

static int64_t layout_bytes(const pgvimp_engine_cfg* cfg);

// Narrowest window of trial step sizes per plan (1..kMaxTrialWidth).  For
// n >= 6 a trial is a long chain of latency-bound block steps, so the
// default evaluates more step sizes at once (several trials share a compute
// unit) rather than in windows one after another.
static int64_t trial_width(const pgvimp_engine_cfg* cfg) {
    if (cfg->trial_width > 0) return std::min<int64_t>(cfg->trial_width, kMaxTrialWidth);
    return cfg->n >= 6 ? kDefaultTrialWidthLarge : kDefaultTrialWidth;
}
// Trial slots per plan = the widest window (trial_width..kMaxTrialWidth,
// default twice trial_width, or trial_width for n >= 6).
static int64_t trial_slots(const pgvimp_engine_cfg* cfg) {
    const int64_t w = trial_width(cfg);
    const int64_t s = cfg->trial_slots > 0 ? cfg->trial_slots : (cfg->n >= 6 ? w : 2 * w);
    return std::min<int64_t>(kMaxTrialWidth, std::max(w, s));
}

int64_t pgvimp_arena_bytes(const pgvimp_engine_cfg* cfg) {
    if (!cfg || !chain_supported(cfg->n) || cfg->max_plans < 1 || cfg->max_states < 1 || cfg->heap_bytes < 0)
        return PGVIMP_EINVAL;
    return layout_bytes(cfg);
}

// Carves the arena into the per-state, per-plan and per-segment arrays; with
// c == nullptr only the total size is computed.
static int64_t carve(pgvimp_ctx* c, const pgvimp_engine_cfg* cfg, DevState& st, char* base) {
    const int n = cfg->n;
    const int64_t S = cfg->max_states, P = cfg->max_plans;
    const int dmax = std::min(n, PGVIMP_MAX_COLL_DIM);
    const int ws_stride = 3 * n * n + n;
    const int seg_stride = std::max(5 * n * n, 4 * n * n + 3 * n);  // larger scratch layout per slot
    int64_t off = 0;
    auto take = [&](auto** ptr, int64_t bytes) {
        if (base) *ptr = (std::remove_reference_t<decltype(**ptr)>*)(base + off);
        off += align_up(bytes);
    };
    take(&st.plans, P * (int64_t)sizeof(PlanDev));
    take(&st.state_plan, S * 4);
    const int64_t W = trial_slots(cfg);
    // chain-order capacity: each plan's range is rounded up to whole rows of
    // its segments and to whole tiles of 32 positions, and starts on a tile
    // (fewer than kMaxSeg + 2 * 32 extra positions per plan)
    const int64_t Sc = (S + (kMaxSeg + 64) * P + 31) / 32 * 32;
    double** sq[] = {&st.KD, &st.KU, &st.Phi, &st.Qinv, &st.LD, &st.LU, &st.SD, &st.SU};
    for (auto p : sq) take(p, S * n * n * 8);
    double** vec[] = {&st.eta, &st.abar, &st.mu};
    for (auto p : vec) take(p, S * n * 8);
    double** csq[] = {&st.cKH, &st.cKD, &st.cLD, &st.cKU, &st.cLU};
    for (auto p : csq) take(p, Sc * n * n * 8);
    double** cvec[] = {&st.crb, &st.cLmu, &st.cmu};
    for (auto p : cvec) take(p, Sc * n * 8);
    take(&st.TSD, W * Sc * n * n * 8);
    take(&st.TSU, W * Sc * n * n * 8);
    take(&st.Tmu, W * Sc * n * 8);
    take(&st.tres, P * kMaxBisect * 4 * 8);
    take(&st.wlist, (P * kMaxTrialWidth + 1) * 4);
    take(&st.psum, P * kIterBlocks * 2 * 8);
    take(&st.Ecol, S * 8);
    take(&st.gcol, S * dmax * 8);
    take(&st.Hcol, S * dmax * dmax * 8);
    take(&st.Epri, (S + P) * 8);
    take(&st.ws, 2 * W * Sc * ws_stride * 8);
    // reduced-chain node scratch and per-thread block workspace of the
    // segmented sweeps: in LDS or registers for n <= 4; n >= 6 takes the
    // wavefront-per-matrix path, which needs neither
    const bool seg_ws = n > 4 && n < 6;
    take(&st.seg, seg_ws ? P * W * 2 * kMaxSeg * (int64_t)seg_stride * 8 : 0);
    const int64_t tws_stride = seg_ws ? (int64_t)kTwsBlocks * n * n + (int64_t)kTwsVecs * n : 0;
    take(&st.tws, P * W * kTrialThreads * tws_stride * 8);
    take(&st.flags, 16 * 4);
    take(&st.gh_x64, (kMaxGH + 1) * kMaxGH * 8);
    take(&st.gh_w64, (kMaxGH + 1) * kMaxGH * 8);
    take(&st.gh_x32, (kMaxGH + 1) * kMaxGH * 4);
    take(&st.gh_w32, (kMaxGH + 1) * kMaxGH * 4);
    if (c) {
        c->heap = base + off;
        c->heap_bytes = align_up(cfg->heap_bytes);
    }
    off += align_up(cfg->heap_bytes);
    st.S = S;
    st.Sc = Sc;
    st.n = n;
    st.P = (int32_t)P;
    st.ws_stride = ws_stride;
    st.seg_stride = seg_stride;
    st.tws_stride = tws_stride;
    st.W = (int32_t)W;
    st.Wmin = (int32_t)trial_width(cfg);
    st.iter_blocks = (int32_t)std::min<int64_t>(kIterBlocks, W);
    st.lookahead = std::max(0, cfg->trial_lookahead);
    return off;
}

static int64_t layout_bytes(const pgvimp_engine_cfg* cfg) {
    DevState tmp{};
    return carve(nullptr, cfg, tmp, nullptr);
}

static int ctx_alloc(pgvimp_ctx* c) {
    const int n = c->n;
    const int64_t S = c->cfg.max_states, P = c->cfg.max_plans;
    (void)n;
    DevState& st = c->st;
    const int64_t total = layout_bytes(&c->cfg);
    if (c->cfg.dev_arena) {
        if ((uint64_t)total > c->cfg.arena_bytes)
            FAIL(c, PGVIMP_ENOMEM, "arena of %llu bytes too small, need %lld", (unsigned long long)c->cfg.arena_bytes,
                 (long long)total);
        if (((uintptr_t)c->cfg.dev_arena) % kAlign) FAIL(c, PGVIMP_EINVAL, "arena must be 256-byte aligned");
        c->arena = (char*)c->cfg.dev_arena;
        c->own_arena = false;
    } else {
        hipError_t e = hipMalloc(&c->arena, total);
        if (e != hipSuccess) FAIL(c, PGVIMP_ENOMEM, "hipMalloc(%lld): %s", (long long)total, hipGetErrorString(e));
        c->own_arena = true;
    }
    c->arena_bytes = total;
    carve(c, &c->cfg, st, c->arena);
    int cus = 0;
    HCK(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->cfg.device));
    st.wbudget = std::max(1, cus);
    c->states.reset(S);
    c->cstates.reset(c->st.Sc);
    c->heapalloc.reset(c->heap_bytes);
    c->plans.assign(P, PlanHost{});
    c->pdev.assign(P, PlanDev{});
    // tables and empty plan slots
    std::vector<double> X, W;
    gh_tables(X, W);
    c->ghX = X;
    c->ghW = W;
    std::vector<float> Xf(X.begin(), X.end()), Wf(W.begin(), W.end());
    HCK(c, hipMemcpy((void*)st.gh_x64, X.data(), X.size() * 8, hipMemcpyHostToDevice));
    HCK(c, hipMemset(st.flags, 0, 16 * 4));
    HCK(c, hipMemcpy((void*)st.gh_w64, W.data(), W.size() * 8, hipMemcpyHostToDevice));
    HCK(c, hipMemcpy((void*)st.gh_x32, Xf.data(), Xf.size() * 4, hipMemcpyHostToDevice));
    HCK(c, hipMemcpy((void*)st.gh_w32, Wf.data(), Wf.size() * 4, hipMemcpyHostToDevice));
    HCK(c, hipMemcpy(st.plans, c->pdev.data(), P * sizeof(PlanDev), hipMemcpyHostToDevice));
    std::vector<int32_t> neg(S, -1);
    HCK(c, hipMemcpy(st.state_plan, neg.data(), S * 4, hipMemcpyHostToDevice));
    return PGVIMP_OK;
}

int pgvimp_create(const pgvimp_problem* probs, int32_t n_probs, const pgvimp_engine_cfg* cfg, pgvimp_ctx** out) {
    if (!out) FAIL((pgvimp_ctx*)nullptr, PGVIMP_EINVAL, "null output pointer");
    *out = nullptr;
    if (!cfg) FAIL((pgvimp_ctx*)nullptr, PGVIMP_EINVAL, "null config");
    if (!chain_supported(cfg->n)) FAIL((pgvimp_ctx*)nullptr, PGVIMP_EINVAL, "state dim %d not supported", cfg->n);
    if (cfg->max_plans < 1 || cfg->max_states < 1 || cfg->heap_bytes < 0 || n_probs < 0 || n_probs > cfg->max_plans ||
        cfg->use_graph < 0 || cfg->use_graph > 2 || cfg->trial_width < 0 || cfg->trial_lookahead < 0 || cfg->trial_slots < 0 ||
        (n_probs > 0 && !probs) || (cfg->precision != PGVIMP_FP64 && cfg->precision != PGVIMP_MIXED) ||
        cfg->segments < 0 || cfg->segments > kMaxSeg)
        FAIL((pgvimp_ctx*)nullptr, PGVIMP_EINVAL, "invalid engine configuration");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        FAIL((pgvimp_ctx*)nullptr, PGVIMP_EDEVICE, "no HIP device available");
    if (cfg->device < 0 || cfg->device >= ndev) FAIL((pgvimp_ctx*)nullptr, PGVIMP_EINVAL, "bad device index");
    pgvimp_ctx* c = new pgvimp_ctx();
    c->cfg = *cfg;
    c->n = cfg->n;
    int rc = PGVIMP_OK;
    if (hipSetDevice(cfg->device) != hipSuccess) {
        g_create_err = "hipSetDevice failed";
        delete c;
        return PGVIMP_EDEVICE;
    }
    double* scr = nullptr;
    if (scratch_address(cfg->device, &scr) != hipSuccess) {
        g_create_err = "hipGetSymbolAddress of the staging scratch failed";
        delete c;
        return PGVIMP_EDEVICE;
    }
    if (cfg->stream) {
        c->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            g_create_err = "stream creation failed";
            delete c;
            return PGVIMP_EDEVICE;
        }
        c->own_stream = true;
    }
    rc = ctx_alloc(c);
    if (rc == PGVIMP_OK) {
        for (int i = 0; i < n_probs && rc == PGVIMP_OK; ++i) {
            int32_t id;
            rc = pgvimp_add_plan(c, &probs[i], &id);
        }
    }
    if (rc != PGVIMP_OK) {
        g_create_err = c->err;
        pgvimp_destroy(c);
        return rc;
    }
    *out = c;
    return PGVIMP_OK;
}

int pgvimp_destroy(pgvimp_ctx* c) {
    if (!c) return PGVIMP_EINVAL;
    (void)hipSetDevice(c->cfg.device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    for (auto e : c->ev) (void)hipEventDestroy(e);
    if (c->stage) (void)hipFree(c->stage);
    if (c->own_arena && c->arena) (void)hipFree(c->arena);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return PGVIMP_OK;
}

int pgvimp_set_stream(pgvimp_ctx* c, void* stream) {
    if (!c) return PGVIMP_EINVAL;
    HCK(c, hipStreamSynchronize(c->stream));
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    c->own_stream = false;
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        HCK(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    drop_graph(c);
    return PGVIMP_OK;
}

int pgvimp_sync(pgvimp_ctx* c) {
    if (!c) return PGVIMP_EINVAL;
    HCK(c, hipStreamSynchronize(c->stream));
    return PGVIMP_OK;
}

// FP64 values of a plan's model block: start/goal factors, Qc, per-interval
// dynamics, sphere radii, forward-kinematics data and the sparse rule
// (FP64 rows, then FP32 rows two per slot).
static int64_t model_count_of(int n, int m, int N, int ns, int64_t rule_vals) {
    const int64_t nI = std::max(N - 1, 1);
    const int64_t fk_count = 3 + PGVIMP_ARM_DOF + ns + PGVIMP_ARM_DOF + ns;
    return 4 * (int64_t)n * n + 2 * n + (int64_t)m * m + nI * n * n + nI * n + nI * n * m + ns + fk_count +
           rule_vals + (rule_vals + 1) / 2;
}

// Device bytes of a plan's map: the FP32 grid and the four corners of every
// cell of each z-slice (one 16-byte load per bilinear lookup, two per
// trilinear one).
static int64_t map_bytes(const pgvimp_problem* p) {
    if (p->coll_kind == PGVIMP_COLL_NONE) return 0;
    return align_up((int64_t)p->gx * p->gy * p->gz * 4) + align_up((int64_t)(p->gx - 1) * (p->gy - 1) * p->gz * 16);
}

int64_t pgvimp_plan_heap_bytes(const pgvimp_problem* p) {
    if (!p || p->n < 1 || p->m < 1 || p->N < 1) return PGVIMP_EINVAL;
    const bool coll = p->coll_kind != PGVIMP_COLL_NONE;
    const int ns = coll ? std::max(p->n_spheres, 1) : 1;
    int64_t rule_vals = 0;
    if (coll && p->quadrature == PGVIMP_QUAD_SPARSE) {
        std::vector<double> X, W, rule;
        gh_tables(X, W);
        if (p->gh_points < 1 || p->gh_points > kMaxGH) return PGVIMP_EINVAL;
        sparse_rule(p->gh_points, coll_dim_of(p->coll_kind), X, W, kMaxSparseNodes, rule);
        if (rule.empty()) return PGVIMP_EINVAL;
        rule_vals = (int64_t)rule.size();
    }
    return map_bytes(p) + align_up(model_count_of(p->n, p->m, p->N, ns, rule_vals) * 8);
}

int pgvimp_add_plan(pgvimp_ctx* c, const pgvimp_problem* p, int32_t* plan_out) {
    if (!c || !plan_out) return PGVIMP_EINVAL;
    int rc = validate_problem(c, p);
    if (rc) return rc;
    HCK(c, hipSetDevice(c->cfg.device));
    int slot = -1;
    for (int i = 0; i < (int)c->plans.size(); ++i)
        if (!c->plans[i].active) {
            slot = i;
            break;
        }
    if (slot < 0) FAIL(c, PGVIMP_EBUSY, "no free plan slot (max_plans=%d)", c->cfg.max_plans);
    const int n = c->n, m = p->m, N = p->N;
    const int nI = std::max(N - 1, 1);
    const bool coll = p->coll_kind != PGVIMP_COLL_NONE;
    const int ns = coll ? p->n_spheres : 1;
    // heap blocks: the SDF grid (shared with live plans of the same map),
    // and the plan's FP64 model data
    const int64_t sdf_bytes = map_bytes(p);
    const int64_t fk_count = 3 + PGVIMP_ARM_DOF + ns + PGVIMP_ARM_DOF + ns;
    // sparse quadrature rule of the collision expectations (rows xi, W), FP64
    // then FP32 (packed two per double slot)
    std::vector<double> rule;
    const int dcol = coll ? coll_dim_of(p->coll_kind) : 0;
    if (coll && p->quadrature == PGVIMP_QUAD_SPARSE) {
        sparse_rule(p->gh_points, dcol, c->ghX, c->ghW, kMaxSparseNodes, rule);
        if (rule.empty()) FAIL(c, PGVIMP_EINVAL, "sparse rule of level %d in %d dimensions exceeds %d nodes",
                               p->gh_points, dcol, kMaxSparseNodes);
    }
    const int64_t rule_vals = (int64_t)rule.size();
    const int64_t model_count = model_count_of(n, m, N, ns, rule_vals);
    const int64_t bytes = align_up(model_count * 8);
    MapKey mkey{};
    bool map_new = false;
    if (coll) {
        mkey = map_key(p->sdf, p->gx, p->gy, p->gz);
        map_new = c->maps.find(mkey) == c->maps.end();
    }
    const int64_t soff = c->states.alloc(N);
    if (soff < 0) FAIL(c, PGVIMP_ENOMEM, "no room for %d states", N);
    // n >= 6: the chain kernels sweep the whole plan from both ends (one
    // wavefront per sweep), state order is chain order
    const int nseg = c->n >= 6 ? 1 : choose_segments(c, N, p->segments);
    const int64_t clen = ((int64_t)((N + nseg - 1) / nseg) * nseg + 31) / 32 * 32;
    const int64_t coff = c->cstates.alloc(clen, 32);
    if (coff < 0) {
        c->states.release(soff);
        FAIL(c, PGVIMP_ENOMEM, "no room for %lld chain positions", (long long)clen);
    }
    const int64_t hoff = c->heapalloc.alloc(bytes, kAlign);
    const int64_t moff = map_new ? c->heapalloc.alloc(sdf_bytes, kAlign) : coll ? c->maps[mkey].off : -1;
    if (hoff < 0 || (map_new && moff < 0)) {
        c->states.release(soff);
        c->cstates.release(coff);
        if (hoff >= 0) c->heapalloc.release(hoff);
        if (moff >= 0 && map_new) c->heapalloc.release(moff);
        FAIL(c, PGVIMP_ENOMEM, "no heap room for %lld bytes of map/model data",
             (long long)(bytes + (map_new ? sdf_bytes : 0)));
    }
    char* base = coll ? c->heap + moff : nullptr;  // the SDF grid
    double* model = (double*)(c->heap + hoff);
    std::vector<double> h(model_count, 0.0);
    int64_t o = 0;
    PlanDev pd{};
    auto take = [&](int64_t cnt) {
        double* dptr = model + o;
        o += cnt;
        return dptr;
    };
    double* Wstart = take(n * n);
    double* Wgoal = take(n * n);
    double* mus = take(n);
    double* mug = take(n);
    double* Ss = take(n * n);
    double* Sgl = take(n * n);
    double* Qc = take(m * m);
    double* A = take((int64_t)nI * n * n);
    double* a = take((int64_t)nI * n);
    double* B = take((int64_t)nI * n * m);
    double* rad = take(ns);
    double* fk = take(fk_count);
    double* rule64 = take(rule_vals);
    float* rule32 = (float*)take((rule_vals + 1) / 2);
    auto hput = [&](double* dst, const double* src, int64_t cnt) { memcpy(&h[dst - model], src, cnt * 8); };
    hput(mus, p->mu_start, n);
    hput(mug, p->mu_goal, n);
    hput(Ss, p->Sig_start, n * n);
    hput(Sgl, p->Sig_goal, n * n);
    hput(Qc, p->Qc, m * m);
    for (int i = 0; i < nI; ++i) {
        const int src = p->ltv ? i : 0;
        hput(A + (int64_t)i * n * n, p->A + (int64_t)src * n * n, n * n);
        hput(a + (int64_t)i * n, p->a + (int64_t)src * n, n);
        hput(B + (int64_t)i * n * m, p->B + (int64_t)src * n * m, n * m);
    }
    if (rule_vals > 0) {
        hput(rule64, rule.data(), rule_vals);
        float* r32 = (float*)&h[(double*)rule32 - model];
        for (int64_t e = 0; e < rule_vals; ++e) r32[e] = (float)rule[e];
    }
    if (coll) {
        hput(rad, p->sphere_radius, ns);
        if (p->coll_kind == PGVIMP_COLL_ARM3D) {
            double* f = &h[fk - model];
            memcpy(f, p->fk_base, 3 * 8);
            memcpy(f + 3, p->fk_link_len, PGVIMP_ARM_DOF * 8);
            memcpy(f + 3 + PGVIMP_ARM_DOF, p->fk_sphere_frac, ns * 8);
            for (int k = 0; k < PGVIMP_ARM_DOF; ++k) f[3 + PGVIMP_ARM_DOF + ns + k] = p->fk_axes[k];
            for (int s = 0; s < ns; ++s) f[3 + 2 * PGVIMP_ARM_DOF + ns + s] = p->fk_sphere_link[s];
        }
        if (map_new) {
            HCK(c, hipMemcpyAsync(base, p->sdf, (size_t)p->gx * p->gy * p->gz * 4, hipMemcpyHostToDevice,
                                  c->stream));
            HCK(c, launch_build_quads((const float*)base, p->gx, p->gy, p->gz,
                                      (float*)(base + align_up((int64_t)p->gx * p->gy * p->gz * 4)), c->stream));
        }
    }
    HCK(c, hipMemcpyAsync(model, h.data(), model_count * 8, hipMemcpyHostToDevice, c->stream));
    pd.active = 1;
    pd.N = N;
    pd.off = (int32_t)soff;
    pd.nseg = nseg;
    pd.coff = (int32_t)coff;
    pd.iters_left = p->n_iters;
    pd.n_iters = p->n_iters;
    pd.dt = p->dt;
    pd.max_bisect = p->max_bisect;
    pd.ltv = p->ltv ? 1 : 0;
    pd.coll_kind = p->coll_kind;
    pd.d = coll ? coll_dim_of(p->coll_kind) : 0;
    pd.gh_points = p->gh_points;
    pd.quadrature = coll ? p->quadrature : PGVIMP_QUAD_TENSOR;
    pd.update = p->update;
    pd.rule_n = dcol > 0 ? (int32_t)(rule_vals / (dcol + 1)) : 0;
    pd.rule64 = rule_vals > 0 ? rule64 : nullptr;
    pd.rule32 = rule_vals > 0 ? rule32 : nullptr;
    pd.gx = p->gx;
    pd.gy = p->gy;
    pd.gz = p->gz;
    pd.n_spheres = ns;
    pd.coll_states = p->coll_states;
    pd.m = m;
    for (int k = 0; k < PGVIMP_MAX_COLL_DIM; ++k) pd.coll_index[k] = p->coll_index[k];
    pd.temperature = p->temperature;
    pd.beta_max = p->beta_max;
    pd.kl_bound = p->kl_bound;
    pd.cell = p->cell;
    pd.inv_cell = 1.0 / p->cell;
    pd.hinge_eps = p->hinge_eps;
    pd.obs_weight = p->obs_weight;
    for (int k = 0; k < 3; ++k) pd.origin[k] = p->origin[k];
    pd.sdf = coll ? (const float*)base : nullptr;
    pd.sdfq = coll ? (const float*)(base + align_up((int64_t)p->gx * p->gy * p->gz * 4)) : nullptr;
    pd.Wstart = Wstart;
    pd.Wgoal = Wgoal;
    pd.mu_start = mus;
    pd.mu_goal = mug;
    pd.Sig_start = Ss;
    pd.Sig_goal = Sgl;
    pd.Qc = Qc;
    pd.A = A;
    pd.a = a;
    pd.B = B;
    pd.radius = rad;
    pd.fk = fk;
    c->pdev[slot] = pd;
    rc = upload_plan(c, slot);
    if (rc) return rc;
    std::vector<int32_t> own(N, slot);
    HCK(c, hipMemcpyAsync(c->st.state_plan + soff, own.data(), N * 4, hipMemcpyHostToDevice, c->stream));
    PlanHost& ph = c->plans[slot];
    ph.active = true;
    ph.N = N;
    ph.off = soff;
    ph.coff = coff;
    ph.heap_off = hoff;
    ph.map_off = moff;
    if (coll) {
        if (map_new) c->maps[mkey] = MapEntry{moff, 0};
        c->maps[mkey].refs += 1;
    }
    ph.coll_kind = p->coll_kind;
    ph.d = pd.d;
    ph.p = p->gh_points;
    ph.quadrature = pd.quadrature;
    ph.dt = p->dt;
    ph.max_bisect = p->max_bisect;
    ph.group = !coll ? 0 : p->expect_group > 0 ? p->expect_group : c->cfg.expect_group;
    // prior (Alg. 1) and initial state
    HCK(c, launch_prior_build(c->st, slot, slot + 1, N, c->stream));
    HCK(c, launch_prior_assemble(c->st, slot, slot + 1, N, c->stream));
    HCK(c, launch_chain(c->st, CHAIN_INIT, slot, slot + 1, c->stream));
    if (p->mu_init) {
        rc = ensure_stage(c, (size_t)N * n * 8);
        if (rc) return rc;
        HCK(c, hipMemcpyAsync(c->stage, p->mu_init, (size_t)N * n * 8, hipMemcpyHostToDevice, c->stream));
        HCK(c, launch_scatter(c->st, G_MU, slot, N, c->stage, c->stream));
    }
    rc = download_plans(c);
    if (rc) return rc;
    if (c->pdev[slot].status != 0) {
        pgvimp_remove_plan(c, slot);
        FAIL(c, PGVIMP_ENOTPD, "prior precision of the new plan is not positive definite");
    }
    *plan_out = slot;
    return PGVIMP_OK;
}

int pgvimp_remove_plan(pgvimp_ctx* c, int32_t plan) {
    if (!c || plan < 0 || plan >= (int)c->plans.size() || !c->plans[plan].active) return PGVIMP_EINVAL;
    HCK(c, hipSetDevice(c->cfg.device));
    PlanHost& ph = c->plans[plan];
    std::vector<int32_t> neg(ph.N, -1);
    HCK(c, hipMemcpyAsync(c->st.state_plan + ph.off, neg.data(), ph.N * 4, hipMemcpyHostToDevice, c->stream));
    c->pdev[plan] = PlanDev{};
    int rc = upload_plan(c, plan);
    if (rc) return rc;
    HCK(c, hipStreamSynchronize(c->stream));
    c->states.release(ph.off);
    c->cstates.release(ph.coff);
    c->heapalloc.release(ph.heap_off);
    if (ph.map_off >= 0)
        for (auto it = c->maps.begin(); it != c->maps.end(); ++it)
            if (it->second.off == ph.map_off) {
                if (--it->second.refs == 0) {
                    c->heapalloc.release(it->second.off);
                    c->maps.erase(it);
                }
                break;
            }
    ph = PlanHost{};
    return PGVIMP_OK;
}

static bool plan_ok(pgvimp_ctx* c, int plan) {
    return c && plan >= 0 && plan < (int)c->plans.size() && c->plans[plan].active;
}

int pgvimp_set_budget(pgvimp_ctx* c, int32_t plan, int32_t iters_left) {
    if (!plan_ok(c, plan) || iters_left < 0) return PGVIMP_EINVAL;
    int rc = download_plans(c);
    if (rc) return rc;
    c->pdev[plan].iters_left = iters_left;
    rc = upload_plan(c, plan);
    if (rc) return rc;
    HCK(c, hipStreamSynchronize(c->stream));
    return PGVIMP_OK;
}

int pgvimp_set_temperature(pgvimp_ctx* c, int32_t plan, double temperature) {
    if (!plan_ok(c, plan)) return PGVIMP_EINVAL;
    if (!(temperature > 0.0) || !std::isfinite(temperature))
        FAIL(c, PGVIMP_EINVAL, "temperature must be positive and finite");
    HCK(c, hipSetDevice(c->cfg.device));
    int rc = download_plans(c);
    if (rc) return rc;
    c->pdev[plan].temperature = temperature;
    if ((rc = upload_plan(c, plan))) return rc;
    HCK(c, hipStreamSynchronize(c->stream));
    return PGVIMP_OK;
}

int pgvimp_marginals(pgvimp_ctx* c, int32_t plan, double* cov_diag, double* cov_off, double* logdet) {
    if (!plan_ok(c, plan)) return PGVIMP_EINVAL;
    HCK(c, hipSetDevice(c->cfg.device));
    const int N = c->plans[plan].N, n = c->n;
    HCK(c, launch_chain(c->st, CHAIN_MARGINALS, plan, plan + 1, c->stream));
    int rc = download_plans(c);
    if (rc) return rc;
    if (c->pdev[plan].status == PGVIMP_ENOTPD) FAIL(c, PGVIMP_ENOTPD, "precision of plan %d not positive definite", plan);
    if ((rc = gather_out(c, G_SD, plan, N, cov_diag, (size_t)N * n * n))) return rc;
    if ((rc = gather_out(c, G_SU, plan, N, cov_off, (size_t)std::max(N - 1, 0) * n * n))) return rc;
    if (logdet) *logdet = c->pdev[plan].logdet;
    return PGVIMP_OK;
}

int pgvimp_factor_expectations(pgvimp_ctx* c, int32_t plan, double* E_coll, double* grad, double* hess,
                               double* E_prior) {
    if (!plan_ok(c, plan)) return PGVIMP_EINVAL;
    HCK(c, hipSetDevice(c->cfg.device));
    const PlanHost& ph = c->plans[plan];
    const int N = ph.N, n = c->n;
    if (ph.coll_kind != PGVIMP_COLL_NONE)
        HCK(c, launch_expect(c->st, ph.coll_kind, ph.d, ph.p, ph.quadrature, c->cfg.precision, ph.group, plan, plan + 1, N, 0,
                             c->stream));
    HCK(c, launch_prior_costs(c->st, plan, N, c->stream));
    int rc;
    if ((rc = gather_out(c, G_ECOL, plan, N, E_coll, N))) return rc;
    if ((rc = gather_out(c, G_GEMB, plan, N, grad, (size_t)N * n))) return rc;
    if ((rc = gather_out(c, G_HEMB, plan, N, hess, (size_t)N * n * n))) return rc;
    if ((rc = gather_out(c, G_EPRI, plan, N, E_prior, (size_t)N + 1))) return rc;
    HCK(c, hipStreamSynchronize(c->stream));
    return PGVIMP_OK;
}

int pgvimp_factor_expectations_noalloc(pgvimp_ctx* c, int32_t plan, double* E_coll, double* grad, double* hess,
                                       double* E_prior) {
    if (!plan_ok(c, plan)) return PGVIMP_EINVAL;
    HCK(c, hipSetDevice(c->cfg.device));
    const PlanHost& ph = c->plans[plan];
    const int N = ph.N, n = c->n;
    const int64_t need = std::max<int64_t>((int64_t)N * n * n, (int64_t)N + 1);
    if (!c->cfg.io_on_device && need > kNoAllocDoubles)
        FAIL(c, PGVIMP_ENOMEM, "plan %d needs %lld doubles of staging, the allocation-free limit is %lld", plan,
             (long long)need, (long long)kNoAllocDoubles);
    double* stage = nullptr;
    HCK(c, scratch_address(c->cfg.device, &stage));
    if (ph.coll_kind != PGVIMP_COLL_NONE)
        HCK(c, launch_expect(c->st, ph.coll_kind, ph.d, ph.p, ph.quadrature, c->cfg.precision, ph.group, plan, plan + 1, N, 0,
                             c->stream));
    HCK(c, launch_prior_costs(c->st, plan, N, c->stream));
    int rc;
    if ((rc = gather_out(c, G_ECOL, plan, N, E_coll, N, stage))) return rc;
    if ((rc = gather_out(c, G_GEMB, plan, N, grad, (size_t)N * n, stage))) return rc;
    if ((rc = gather_out(c, G_HEMB, plan, N, hess, (size_t)N * n * n, stage))) return rc;
    if ((rc = gather_out(c, G_EPRI, plan, N, E_prior, (size_t)N + 1, stage))) return rc;
    HCK(c, hipStreamSynchronize(c->stream));
    return PGVIMP_OK;
}

// Distinct quadrature classes among live plans.
static std::vector<ClassKey> live_classes(pgvimp_ctx* c) {
    std::vector<ClassKey> v;
    for (auto& ph : c->plans) {
        if (!ph.active || ph.coll_kind == PGVIMP_COLL_NONE) continue;
        // sparse plans of every level share one launch: each reads its own rule
        ClassKey k{ph.coll_kind, ph.d, ph.quadrature == PGVIMP_QUAD_SPARSE ? 0 : ph.p, ph.group, ph.quadrature};
        if (std::find(v.begin(), v.end(), k) == v.end()) v.push_back(k);
    }
    return v;
}

static int plan_high_water(pgvimp_ctx* c) {
    int hw = 0;
    for (int i = 0; i < (int)c->plans.size(); ++i)
        if (c->plans[i].active) hw = i + 1;
    return hw;
}

static int active_plans(pgvimp_ctx* c) {
    int a = 0;
    for (auto& ph : c->plans) a += ph.active ? 1 : 0;
    return a;
}

static int max_live_N(pgvimp_ctx* c) {
    int m = 0;
    for (auto& ph : c->plans)
        if (ph.active) m = std::max(m, ph.N);
    return m;
}

// Windows of trial step sizes that cover max_bisect for every live plan
// when every window is as narrow as allowed: a first window of at least one
// step size (trial_width without lookahead), then windows of trial_width.
static int trial_rounds(pgvimp_ctx* c) {
    int mb = 1;
    for (auto& ph : c->plans)
        if (ph.active) mb = std::max(mb, ph.max_bisect);
    const int W = c->st.Wmin;
    return c->st.lookahead > 0 ? 1 + (mb - 1 + W - 1) / W : (mb + W - 1) / W;
}

// Enqueue n_iters iterations; with timing, bracket each launch by events.
// phw: plan slots covered; maxN: bound on the live plans' lengths that
// sizes the grids (kernels stride over longer plans).
static int enqueue_iters(pgvimp_ctx* c, int n_iters, const std::vector<ClassKey>& cls, int64_t shw, int phw,
                         int maxN, bool timed, bool restart) {
    const int rounds = trial_rounds(c);
    c->ev_used = 0;
    // record an event pair around each launch when timing (kind = PGVIMP_K_*)
    auto begin = [&](int kind) -> int {
        if (!timed) return PGVIMP_OK;
        while (c->ev.size() < c->ev_used + 2) {
            hipEvent_t e;
            HCK(c, hipEventCreate(&e));
            c->ev.push_back(e);
            c->ev_kind.push_back(0);
        }
        c->ev_kind[c->ev_used] = kind;
        HCK(c, hipEventRecord(c->ev[c->ev_used], c->stream));
        return PGVIMP_OK;
    };
    auto end = [&]() -> int {
        if (!timed) return PGVIMP_OK;
        HCK(c, hipEventRecord(c->ev[c->ev_used + 1], c->stream));
        c->ev_used += 2;
        return PGVIMP_OK;
    };
    int rc;
    if (restart) {
        // every live plan: prior from its stored dynamics, mu_0 = prior mean,
        // Lambda_0 = K^-1, marginals, budget reset (Alg. 1 set-up)
        if ((rc = begin(PGVIMP_K_RESTART))) return rc;
        HCK(c, launch_prior_build(c->st, 0, phw, maxN, c->stream));
        HCK(c, launch_prior_assemble(c->st, 0, phw, maxN, c->stream));
        HCK(c, launch_chain(c->st, CHAIN_INIT, 0, phw, c->stream));
        if ((rc = end())) return rc;
    }
    for (int it = 0; it < n_iters; ++it) {
        for (auto& k : cls) {
            if ((rc = begin(PGVIMP_K_EXPECT))) return rc;
            HCK(c, launch_expect(c->st, k.kind, k.d, k.p, k.quadrature, c->cfg.precision, k.group, 0, phw, maxN, 1, c->stream));
            if ((rc = end())) return rc;
        }
        if ((rc = begin(PGVIMP_K_PREP))) return rc;
        HCK(c, launch_iteration(c->st, phw, 0, 0, c->stream));
        if ((rc = end())) return rc;
        for (int r = 0; r < rounds; ++r) {
            HCK(c, launch_window(c->st, phw, r, c->stream));
            if ((rc = begin(PGVIMP_K_TRIAL))) return rc;
            // the first window of a batch larger than the chip may pair
            // workgroups on a CU (not for capacity-sized serving graphs,
            // where the live plans are unknown when the graph is captured)
            const bool pair = r == 0 && c->cfg.use_graph != 2 && c->st.lookahead == 0 &&
                              (int64_t)active_plans(c) * c->st.Wmin > c->st.wbudget;
            HCK(c, launch_iteration(c->st, phw, pair ? 5 : 1, r, c->stream));
            if ((rc = end())) return rc;
        }
        if ((rc = begin(PGVIMP_K_SELECT))) return rc;
        HCK(c, launch_iteration(c->st, phw, 2, 0, c->stream));
        if ((rc = end())) return rc;
    }
    return PGVIMP_OK;
}

static int collect_times(pgvimp_ctx* c) {
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.f;
        HCK(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
        c->t_kind[c->ev_kind[i]] += ms;
        c->n_kind[c->ev_kind[i]] += 1;
    }
    c->ev_used = 0;
    return PGVIMP_OK;
}

static int run_iters(pgvimp_ctx* c, int32_t n_iters, pgvimp_stats* per_plan, bool restart);

int pgvimp_expect_all(pgvimp_ctx* c, int32_t reps) {
    if (!c || reps < 1) return PGVIMP_EINVAL;
    HCK(c, hipSetDevice(c->cfg.device));
    const std::vector<ClassKey> cls = live_classes(c);
    const int64_t shw = c->states.high_water();
    c->ev_used = 0;
    for (int r = 0; r < reps; ++r)
        for (auto& k : cls) {
            if (c->profile) {
                while (c->ev.size() < c->ev_used + 2) {
                    hipEvent_t e;
                    HCK(c, hipEventCreate(&e));
                    c->ev.push_back(e);
                    c->ev_kind.push_back(0);
                }
                c->ev_kind[c->ev_used] = PGVIMP_K_EXPECT;
                HCK(c, hipEventRecord(c->ev[c->ev_used], c->stream));
            }
            HCK(c, launch_expect(c->st, k.kind, k.d, k.p, k.quadrature, c->cfg.precision, k.group, 0, (int)c->plans.size(),
                                 max_live_N(c), 1, c->stream));
            if (c->profile) {
                HCK(c, hipEventRecord(c->ev[c->ev_used + 1], c->stream));
                c->ev_used += 2;
            }
        }
    HCK(c, hipStreamSynchronize(c->stream));
    if (c->profile) return collect_times(c);
    return PGVIMP_OK;
}

int pgvimp_prox_step(pgvimp_ctx* c, int32_t n_iters, pgvimp_stats* per_plan) {
    return run_iters(c, n_iters, per_plan, false);
}

int pgvimp_solve(pgvimp_ctx* c, int32_t n_iters, pgvimp_stats* per_plan) {
    return run_iters(c, n_iters, per_plan, true);
}

static int run_iters(pgvimp_ctx* c, int32_t n_iters, pgvimp_stats* per_plan, bool restart) {
    if (!c || n_iters < 0) return PGVIMP_EINVAL;
    HCK(c, hipSetDevice(c->cfg.device));
    const std::vector<ClassKey> cls = live_classes(c);
    const int64_t shw = c->cfg.use_graph == 2 ? c->cfg.max_states : c->states.high_water();
    const int phw = plan_high_water(c);
    const bool timed = c->profile;
    int rc;
    if ((n_iters > 0 || restart) && phw > 0) {
        // Timed runs launch eagerly: events recorded during graph capture
        // cannot be queried for elapsed time.
        if (c->cfg.use_graph && !timed) {
            // grid-size bound, rounded up so that a captured graph serves
            // plans of growing length without re-capture
            int gN = 64;
            while (gN < max_live_N(c)) gN *= 2;
            if (!c->gexec || c->g_iters != n_iters || c->g_hw != shw || !(c->g_classes == cls) ||
                c->g_profiled != timed || c->g_restart != restart || c->g_rounds != trial_rounds(c) ||
                c->g_maxN < max_live_N(c)) {
                drop_graph(c);
                HCK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
                rc = enqueue_iters(c, n_iters, cls, shw, (int)c->plans.size(), gN, timed, restart);
                hipGraph_t g = nullptr;
                hipError_t e2 = hipStreamEndCapture(c->stream, &g);
                if (rc) {
                    if (g) (void)hipGraphDestroy(g);
                    return rc;
                }
                HCK(c, e2);
                c->graph = g;
                HCK(c, hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
                c->g_iters = n_iters;
                c->g_hw = shw;
                c->g_restart = restart;
                c->g_rounds = trial_rounds(c);
                c->g_maxN = gN;
                c->g_classes = cls;
                c->g_profiled = timed;
            }
            HCK(c, hipGraphLaunch(c->gexec, c->stream));
        } else {
            rc = enqueue_iters(c, n_iters, cls, shw, phw, max_live_N(c), timed, restart);
            if (rc) return rc;
        }
    }
    HCK(c, hipStreamSynchronize(c->stream));
    if (timed && phw > 0) {
        rc = collect_times(c);
        if (rc) return rc;
    }
    rc = download_plans(c);
    if (rc) return rc;
    if (per_plan) {
        for (int i = 0; i < (int)c->plans.size(); ++i) {
            pgvimp_stats& s = per_plan[i];
            memset(&s, 0, sizeof(s));
            if (!c->plans[i].active) continue;
            const PlanDev& p = c->pdev[i];
            s.beta = p.beta;
            s.kl = p.kl;
            s.E_coll = p.E_coll;
            s.E_prior = p.E_prior;
            s.logdet = p.logdet;
            s.entropy = p.entropy;
            s.temperature = p.iter_temperature;
            s.entropy_cost = p.entropy_cost;
            s.total_cost = p.total_cost;
            s.status = p.status;
            s.trials = p.trials;
            s.iters_done = p.iters_done;
            s.iters_left = p.iters_left;
            s.trials_total = p.trials_total;
            s.evals_total = p.evals_total;
        }
    }
    return PGVIMP_OK;
}

int pgvimp_get_state(pgvimp_ctx* c, int32_t plan, double* mu, double* prec_diag, double* prec_off) {
    if (!plan_ok(c, plan)) return PGVIMP_EINVAL;
    HCK(c, hipSetDevice(c->cfg.device));
    const int N = c->plans[plan].N, n = c->n;
    int rc;
    if ((rc = gather_out(c, G_MU, plan, N, mu, (size_t)N * n))) return rc;
    if ((rc = gather_out(c, G_LD, plan, N, prec_diag, (size_t)N * n * n))) return rc;
    if ((rc = gather_out(c, G_LU, plan, N, prec_off, (size_t)std::max(N - 1, 0) * n * n))) return rc;
    HCK(c, hipStreamSynchronize(c->stream));
    return PGVIMP_OK;
}

int pgvimp_set_state(pgvimp_ctx* c, int32_t plan, const double* mu, const double* prec_diag, const double* prec_off) {
    if (!plan_ok(c, plan)) return PGVIMP_EINVAL;
    HCK(c, hipSetDevice(c->cfg.device));
    const int N = c->plans[plan].N, n = c->n;
    const size_t nd = (size_t)N * n * n, no = (size_t)std::max(N - 1, 0) * n * n, nm = (size_t)N * n;
    if ((mu && !finite_all(mu, nm)) || (prec_diag && !finite_all(prec_diag, nd)) || (prec_off && !finite_all(prec_off, no)))
        FAIL(c, PGVIMP_EINVAL, "non-finite state");
    // back up the current state in the staging buffer: [mu | D | U | new]
    const size_t tot = nm + nd + no;
    int rc = ensure_stage(c, 2 * tot * 8 + 64);
    if (rc) return rc;
    double* bk = c->stage;
    double* nw = c->stage + tot;
    HCK(c, launch_gather(c->st, G_MU, plan, N, bk, c->stream));
    HCK(c, launch_gather(c->st, G_LD, plan, N, bk + nm, c->stream));
    HCK(c, launch_gather(c->st, G_LU, plan, N, bk + nm + nd, c->stream));
    if (mu) {
        HCK(c, hipMemcpyAsync(nw, mu, nm * 8, hipMemcpyHostToDevice, c->stream));
        HCK(c, launch_scatter(c->st, G_MU, plan, N, nw, c->stream));
    }
    if (prec_diag) {
        HCK(c, hipMemcpyAsync(nw + nm, prec_diag, nd * 8, hipMemcpyHostToDevice, c->stream));
        HCK(c, launch_scatter(c->st, G_LD, plan, N, nw + nm, c->stream));
    }
    if (prec_off && no) {
        HCK(c, hipMemcpyAsync(nw + nm + nd, prec_off, no * 8, hipMemcpyHostToDevice, c->stream));
        HCK(c, launch_scatter(c->st, G_LU, plan, N, nw + nm + nd, c->stream));
    }
    HCK(c, launch_chain(c->st, CHAIN_MARGINALS, plan, plan + 1, c->stream));
    rc = download_plans(c);
    if (rc) return rc;
    if (c->pdev[plan].status == PGVIMP_ENOTPD) {
        HCK(c, launch_scatter(c->st, G_MU, plan, N, bk, c->stream));
        HCK(c, launch_scatter(c->st, G_LD, plan, N, bk + nm, c->stream));
        HCK(c, launch_scatter(c->st, G_LU, plan, N, bk + nm + nd, c->stream));
        HCK(c, launch_chain(c->st, CHAIN_MARGINALS, plan, plan + 1, c->stream));
        rc = download_plans(c);
        if (rc) return rc;
        FAIL(c, PGVIMP_ENOTPD, "new precision of plan %d not positive definite; state unchanged", plan);
    }
    return PGVIMP_OK;
}

int pgvimp_slr_linearize(pgvimp_ctx* c, int32_t plan, int32_t model, const double* model_params, int32_t gh_points,
                         int32_t rebuild_prior, double* A_out, double* a_out) {
    if (!plan_ok(c, plan)) return PGVIMP_EINVAL;
    if (model != PGVIMP_MODEL_QUAD2D || c->n != 6) FAIL(c, PGVIMP_EINVAL, "model %d needs a 6-dim state", model);
    if (gh_points < 1 || gh_points > kMaxGH) FAIL(c, PGVIMP_EINVAL, "gh_points out of range");
    const double g = model_params ? model_params[0] : 9.81;
    if (!std::isfinite(g)) FAIL(c, PGVIMP_EINVAL, "non-finite model parameter");
    HCK(c, hipSetDevice(c->cfg.device));
    const int N = c->plans[plan].N, n = c->n;
    const size_t nA = (size_t)N * n * n, na = (size_t)N * n;
    double* dA = nullptr;
    double* da = nullptr;
    int rc;
    if (c->cfg.io_on_device) {
        dA = A_out;
        da = a_out;
    } else if (A_out || a_out) {
        rc = ensure_stage(c, (nA + na) * 8);
        if (rc) return rc;
        dA = A_out ? c->stage : nullptr;
        da = a_out ? c->stage + nA : nullptr;
    }
    HCK(c, launch_slr_model(c->st, plan, N, g, gh_points, dA, da, rebuild_prior ? 1 : 0, c->stream));
    if (rebuild_prior) {
        HCK(c, launch_prior_build(c->st, plan, plan + 1, N, c->stream));
        HCK(c, launch_prior_assemble(c->st, plan, plan + 1, N, c->stream));
        HCK(c, launch_chain(c->st, CHAIN_REINIT, plan, plan + 1, c->stream));
    }
    if (!c->cfg.io_on_device) {
        if (A_out) HCK(c, hipMemcpyAsync(A_out, dA, nA * 8, hipMemcpyDeviceToHost, c->stream));
        if (a_out) HCK(c, hipMemcpyAsync(a_out, da, na * 8, hipMemcpyDeviceToHost, c->stream));
    }
    rc = download_plans(c);
    if (rc) return rc;
    if (c->pdev[plan].status == PGVIMP_ENOTPD) FAIL(c, PGVIMP_ENOTPD, "linearised prior of plan %d not positive definite", plan);
    return PGVIMP_OK;
}

int pgvimp_slr_round(pgvimp_ctx* c, int32_t plan, int32_t model, const double* model_params, int32_t gh_points,
                     const double* nominal_mean, const double* nominal_cov, int32_t n_iters, double* A_out,
                     double* a_out) {
    if (!plan_ok(c, plan)) return PGVIMP_EINVAL;
    if (n_iters < 0) FAIL(c, PGVIMP_EINVAL, "negative iteration budget");
    if ((nominal_mean == nullptr) != (nominal_cov == nullptr))
        FAIL(c, PGVIMP_EINVAL, "the nominal mean and covariance are given together");
    HCK(c, hipSetDevice(c->cfg.device));
    const int N = c->plans[plan].N, n = c->n;
    if (nominal_mean) {
        // the first round linearises about the nominal N(xbar_i, Sigbar_i):
        // it becomes the plan's mean and marginals before the regression
        const size_t nm = (size_t)N * n, nd = (size_t)N * n * n;
        if (!finite_all(nominal_mean, nm) || !finite_all(nominal_cov, nd))
            FAIL(c, PGVIMP_EINVAL, "non-finite nominal trajectory");
        for (int i = 0; i < N; ++i)
            if (!host_spd(nominal_cov + (size_t)i * n * n, n))
                FAIL(c, PGVIMP_EINVAL, "nominal covariance of state %d is not symmetric positive definite", i);
        int rc = ensure_stage(c, (nm + nd) * 8);
        if (rc) return rc;
        HCK(c, hipMemcpyAsync(c->stage, nominal_mean, nm * 8, hipMemcpyHostToDevice, c->stream));
        HCK(c, hipMemcpyAsync(c->stage + nm, nominal_cov, nd * 8, hipMemcpyHostToDevice, c->stream));
        HCK(c, launch_scatter(c->st, G_MU, plan, N, c->stage, c->stream));
        HCK(c, launch_scatter(c->st, G_SD, plan, N, c->stage + nm, c->stream));
        HCK(c, hipStreamSynchronize(c->stream));
    }
    int rc = pgvimp_slr_linearize(c, plan, model, model_params, gh_points, 1, A_out, a_out);
    if (rc) return rc;
    c->pdev[plan].iters_left = n_iters;
    if ((rc = upload_plan(c, plan))) return rc;
    HCK(c, hipStreamSynchronize(c->stream));
    return PGVIMP_OK;
}

int pgvimp_slr_round_many(pgvimp_ctx* c, int32_t n_plans, const int32_t* plans, int32_t model,
                          const double* model_params, int32_t gh_points, int32_t n_iters, int32_t* status) {
    if (!c || n_plans < 1 || !plans) return PGVIMP_EINVAL;
    if (n_iters < 0) FAIL(c, PGVIMP_EINVAL, "negative iteration budget");
    if (model != PGVIMP_MODEL_QUAD2D || c->n != 6) FAIL(c, PGVIMP_EINVAL, "model %d needs a 6-dim state", model);
    if (gh_points < 1 || gh_points > kMaxGH) FAIL(c, PGVIMP_EINVAL, "gh_points out of range");
    const double g = model_params ? model_params[0] : 9.81;
    if (!std::isfinite(g)) FAIL(c, PGVIMP_EINVAL, "non-finite model parameter");
    std::vector<char> listed(c->plans.size(), 0);
    int lo = (int)c->plans.size(), hi = 0, maxN = 1;
    for (int k = 0; k < n_plans; ++k) {
        const int pl = plans[k];
        if (!plan_ok(c, pl) || listed[pl]) FAIL(c, PGVIMP_EINVAL, "plan %d is not live or listed twice", pl);
        listed[pl] = 1;
        lo = std::min(lo, pl);
        hi = std::max(hi, pl + 1);
        maxN = std::max(maxN, c->plans[pl].N);
    }
    HCK(c, hipSetDevice(c->cfg.device));
    for (int k = 0; k < n_plans; ++k)
        HCK(c, launch_slr_model(c->st, plans[k], c->plans[plans[k]].N, g, gh_points, nullptr, nullptr, 1, c->stream));
    // the rebuild runs over [lo, hi) with the unlisted live plans hidden
    int rc = download_plans(c);
    if (rc) return rc;
    std::vector<int> hidden;
    for (int i = lo; i < hi; ++i)
        if (c->pdev[i].active && !listed[i]) {
            c->pdev[i].active = 0;
            hidden.push_back(i);
        }
    for (int i : hidden)
        if ((rc = upload_plan(c, i))) return rc;
    HCK(c, launch_prior_build(c->st, lo, hi, maxN, c->stream));
    HCK(c, launch_prior_assemble(c->st, lo, hi, maxN, c->stream));
    HCK(c, launch_chain(c->st, CHAIN_REINIT, lo, hi, c->stream));
    if ((rc = download_plans(c))) return rc;
    for (int i : hidden) {
        c->pdev[i].active = 1;
        if ((rc = upload_plan(c, i))) return rc;
    }
    for (int k = 0; k < n_plans; ++k) {
        PlanDev& pd = c->pdev[plans[k]];
        const bool bad = pd.status == PGVIMP_ENOTPD;
        if (status) status[k] = bad ? PGVIMP_ENOTPD : PGVIMP_OK;
        pd.iters_left = bad ? 0 : n_iters;
        if ((rc = upload_plan(c, plans[k]))) return rc;
    }
    HCK(c, hipStreamSynchronize(c->stream));
    return PGVIMP_OK;
}

int pgvimp_launch_shape(pgvimp_ctx* c, int32_t N, int32_t* segments, int32_t* group) {
    if (!c || N < 1) return PGVIMP_EINVAL;
    if (segments) {
        // the segments of the first live plan of N states, else the default
        *segments = choose_segments(c, N);
        for (size_t i = 0; i < c->plans.size(); ++i)
            if (c->plans[i].active && c->plans[i].N == N) {
                *segments = c->pdev[i].nseg;
                break;
            }
    }
    if (group) {
        // the group the expectation kernel takes for the live plans' class
        // of the first live plan (the default when none is live)
        int req = c->cfg.expect_group;
        for (auto& ph : c->plans)
            if (ph.active && ph.coll_kind != PGVIMP_COLL_NONE) {
                req = ph.group;
                break;
            }
        *group = expect_group_for(req, plan_high_water(c), std::max(max_live_N(c), 1), c->st.wbudget);
    }
    return PGVIMP_OK;
}

int pgvimp_profile(pgvimp_ctx* c, int32_t enable) {
    if (!c) return PGVIMP_EINVAL;
    c->profile = enable != 0;
    return PGVIMP_OK;
}

int pgvimp_kernel_times(pgvimp_ctx* c, int32_t reset, double* mean_ms, int64_t* launches) {
    if (!c) return PGVIMP_EINVAL;
    for (int k = 0; k < PGVIMP_NKERNELS; ++k) {
        if (mean_ms) mean_ms[k] = c->n_kind[k] ? c->t_kind[k] / c->n_kind[k] : 0.0;
        if (launches) launches[k] = c->n_kind[k];
        if (reset) {
            c->t_kind[k] = 0.0;
            c->n_kind[k] = 0;
        }
    }
    return PGVIMP_OK;
}

}  // extern "C"
