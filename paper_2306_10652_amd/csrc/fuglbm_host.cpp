// Host side of the C ABI declared in include/fuglbm.h: lattice-unit
// constants, buffer carving, launch tables, hipGraph replay, sticky errors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/fuglbm.h"
#include "kernels.h"

// A roctx range over one library call (visible with rocprofv3
// --marker-trace beside the kernels the call launches).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

namespace {

thread_local std::string g_err;

fuglbm_status fail(fuglbm_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

fuglbm_status hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return FUGLBM_EDEVICE;
}

#define HIP_TRY(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

// Cubic equations of state p = RT/(v - b) - a alpha/((v + d1 b)(v + d2 b)):
// a = omega_a R^2 Tc^2 / pc, b = omega_b R Tc / pc put the critical point at
// (Tc, pc); u = d1 + d2 and w = d1 d2 are kept exact.
struct CubicEos {
    double omega_a, omega_b, d1, d2, u, w;
};

CubicEos cubic_eos(int eos) {
    const double s2 = std::sqrt(2.0);
    const double c2 = std::pow(2.0, 1.0 / 3.0);
    switch (eos) {
        case FUGLBM_EOS_SRK:   // Soave-Redlich-Kwong
            return {1.0 / (9.0 * (c2 - 1.0)), (c2 - 1.0) / 3.0, 1.0, 0.0, 1.0, 0.0};
        case FUGLBM_EOS_VDW:   // van der Waals
            return {27.0 / 64.0, 1.0 / 8.0, 0.0, 0.0, 0.0, 0.0};
        default:               // Peng-Robinson, the paper's (Section II.C)
            return {0.457235529, 0.077796074, 1.0 + s2, 1.0 - s2, 2.0, -1.0};
    }
}

// alpha_i(T): PR as in Section II.C (two branches split at omega = 0.49);
// SRK with Soave's m(omega); 1 for vdW.
double cubic_alpha(int eos, double w, double Tr) {
    if (eos == FUGLBM_EOS_VDW) return 1.0;
    double m;
    if (eos == FUGLBM_EOS_SRK)
        m = 0.480 + 1.574 * w - 0.176 * w * w;
    else
        m = w <= 0.49 ? 0.374640 + 1.54226 * w - 0.26992 * w * w
                      : 0.379642 + 1.48503 * w - 0.164423 * w * w + 0.016666 * w * w * w;
    const double sa = 1.0 + m * (1.0 - std::sqrt(Tr));
    return sa * sa;
}

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int lattice_Q(int lat) { return lat == 0 ? 9 : 19; }
int lattice_D(int lat) { return lat == 0 ? 2 : 3; }

// Fused-kernel rows per work item.  A work item re-reads 4 warm-up rows, so
// longer items waste less; items run in rounds of (CUs x resident
// workgroups per CU).  Pick rows (>= 8, <= ny) minimising
// rounds * (rows + 4).
int compute_units() {
    static int cus = 0;
    if (!cus) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            v > 0)
            cus = v;
        else
            cus = 256;
    }
    return cus;
}

// Fused variants: 2 = register-ring kernel, 3 = store-wave kernel.
bool ws_usable(int ncomp, bool fp32) {
    return ncomp <= fused_ws_max_comp() && fused_ws_fits(ncomp, fp32) &&
           fused_ws_blocks_per_cu(ncomp, fp32) > 0;
}

int blocks_per_cu(int kernel, int ncomp, bool fp32) {
    return kernel == 3 ? fused_ws_blocks_per_cu(ncomp, fp32) : fused_blocks_per_cu(ncomp, fp32);
}

hipError_t launch_fused(int kernel, int ncomp, bool fp32, const FusedItem *items, int nitems,
                        const FusedSim *sims, int flip, hipStream_t st) {
    return kernel == 3 ? launch_fused_d2q9_ws(ncomp, fp32, items, nitems, sims, flip, st)
                       : launch_fused_d2q9(ncomp, fp32, items, nitems, sims, flip, st);
}

// The fused variant used before (or without) timing: the store-wave kernel
// where it is built and fits, else the register-ring kernel.
int default_fused(int ncomp, bool fp32) { return ws_usable(ncomp, fp32) ? 3 : 2; }

int auto_rows(int nx, int ny, int ncomp, bool fp32, int kernel = 2) {
    const int strips = (nx + FUSED_OUT - 1) / FUSED_OUT;
    const int64_t slots = (int64_t)compute_units() * blocks_per_cu(kernel, ncomp, fp32);
    if (ny <= 8) return ny;
    int best = 8;
    int64_t best_cost = INT64_MAX;
    for (int rows = 8; rows <= ny; ++rows) {
        const int64_t items = (int64_t)strips * ((ny + rows - 1) / rows);
        const int64_t rounds = (items + slots - 1) / slots;
        const int64_t cost = rounds * (rows + 4);
        if (cost < best_cost) {
            best_cost = cost;
            best = rows;
        }
    }
    return best;
}

}  // namespace

struct fuglbm_mixture {
    int N;
    int eos;
    double RT;
    double b[FUG_MAXC], aa[FUG_MAXC], sqk[FUG_MAXC], M[FUG_MAXC];
    double aij[FUG_MAXC * FUG_MAXC];
    double tau;
};

// Layout of one simulation's device memory (offsets from base, 256-aligned).
struct Carve {
    size_t buf0, buf1, cst, status, rho, psi, s, j, u, snap, part, fsim, items, total;
    int max_items;
};

static Carve carve(int N, int lat, bool fp32, int nx, int ny, int nz) {
    Carve c{};
    const int64_t ns = (int64_t)nx * ny * nz;
    const int Q = lattice_Q(lat), D = lattice_D(lat);
    const size_t pop = align256((size_t)(fp32 ? PopLayout<float>(N, Q, nx, (int64_t)ny * nz).bytes((int64_t)ny * nz)
                                              : PopLayout<double>(N, Q, nx, (int64_t)ny * nz).bytes((int64_t)ny * nz)));
    size_t o = 0;
    c.buf0 = o; o += pop;
    c.buf1 = o; o += pop;
    c.cst = o; o += align256(sizeof(SimConst));
    c.status = o; o += 256;
    c.rho = o; o += align256((size_t)N * ns * 8);
    c.psi = o; o += align256((size_t)N * ns * 8);
    c.s = o; o += align256((size_t)ns * 8);
    c.j = o; o += align256((size_t)D * ns * 8);
    c.u = o; o += align256((size_t)D * ns * 8);
    c.snap = o; o += align256((size_t)N * ns * 8);
    c.part = o; o += align256(((size_t)1024 + 1) * (N + 1) * DIAG_QUANT * 8);
    c.fsim = o; o += align256(sizeof(FusedSim));
    c.max_items = 0;
    if (lat == 0) {
        const int strips = (nx + FUSED_OUT - 1) / FUSED_OUT;
        c.max_items = strips * ny + 8;   // rows >= 1 per item
    }
    c.items = o; o += align256((size_t)c.max_items * sizeof(FusedItem));
    c.total = o;
    return c;
}

struct GraphCache {
    hipGraphExec_t exec = nullptr;
    int steps = 0;
    int kernel = 0;
    int rows = 0;
};

struct fuglbm_sim {
    const fuglbm_mixture *mix;
    int lattice;
    bool fp32;
    int nx, ny, nz, N, Q, D;
    int64_t ns;
    char *base;
    bool owned;
    Carve cv;
    void *buf[2];
    int parity;            // buffer holding the current state
    SimConst hc;           // host copy of the constant block
    SimConst *dc;
    uint32_t *status;
    double *rho_f, *psi_f, *s_f, *j_f, *u_f, *snap, *part;
    FusedSim *fsim;
    FusedItem *items;
    int nitems;
    int kernel;            // 1 generic, 2 fused (register ring), 3 fused (store waves)
    int rows;
    bool auto_kernel;      // fused variant chosen by timing (not fixed by the caller)
    bool autotune;         // rows chosen by timing (not fixed by the caller)
    bool tuned;            // autotune done (or answered from the cache)
    int64_t step;
    int64_t snap_step;
    bool have_snap;
    uint32_t sticky;
    hipStream_t last_stream;
    // recorded on last_stream after each enqueuing call: a call on another
    // stream waits for it on the device (done_valid: the record is current)
    hipEvent_t done;
    bool done_valid;
    GraphCache graph;
    uint64_t uid;          // never reused; batch tables key on it, not on the address
};

// Work about to be enqueued on st waits (on the device) for the
// simulation's earlier work on another stream: its own event, so no
// reference to that stream is kept.
static fuglbm_status order_after(fuglbm_sim *s, hipStream_t st) {
    if (s->done_valid && s->last_stream != st) HIP_TRY(hipStreamWaitEvent(st, s->done, 0));
    s->last_stream = st;
    return FUGLBM_OK;
}

static fuglbm_status mark_done(fuglbm_sim *s, hipStream_t st) {
    HIP_TRY(hipEventRecord(s->done, st));
    s->done_valid = true;
    s->last_stream = st;
    return FUGLBM_OK;
}

static int64_t pop_bytes(const fuglbm_sim *s) {
    const int64_t rows = (int64_t)s->ny * s->nz;
    return s->fp32 ? PopLayout<float>(s->N, s->Q, s->nx, rows).bytes(rows)
                   : PopLayout<double>(s->N, s->Q, s->nx, rows).bytes(rows);
}

// The fused kernel indexes a buffer with 32-bit element offsets.
static bool fused_fits(const fuglbm_sim *s) {
    const int64_t elems = pop_bytes(s) / (s->fp32 ? 4 : 8);
    return s->lattice == FUGLBM_D2Q9 && elems < ((int64_t)1 << 32);
}

// Launch variants: 1 = four-pass generic kernels, 2 / 3 = fused one-pass
// D2Q9 kernels (register ring / store wavefronts).
static bool is_fused(int kernel) { return kernel == 2 || kernel == 3; }

// The variant a simulation starts with (and kernel 0 of set_tuning picks).
static int default_kernel(const fuglbm_sim *s) {
    return fused_fits(s) ? default_fused(s->N, s->fp32) : 1;
}

static uint64_t next_sim_uid() {
    static uint64_t n = 0;
    return ++n;
}

namespace {

hipStream_t capture_stream() {
    static hipStream_t s = nullptr;
    if (!s) {
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    }
    return s;
}

// Work items of one simulation for `rows` rows per item, in launch order.
// Logical order: chunk-major (a band of rows across the full width).
// Workgroups are handed to the 8 XCDs round-robin; XCD k gets the k-th
// contiguous slice of the logical order, so neighbouring items (which
// re-read each other's halo) share that XCD's L2.
std::vector<FusedItem> item_list(const fuglbm_sim *s, int rows) {
    const int strips = (s->nx + FUSED_OUT - 1) / FUSED_OUT;
    const int chunks = (s->ny + rows - 1) / rows;
    std::vector<FusedItem> logical;
    for (int c = 0; c < chunks; ++c)
        for (int t = 0; t < strips; ++t)
            logical.push_back({0, t * FUSED_OUT, c * rows, std::min(rows, s->ny - c * rows)});
    const int n = (int)logical.size();
    const int per = (n + 7) / 8;
    std::vector<FusedItem> it((size_t)per * 8, FusedItem{-1, 0, 0, 0});
    for (int b = 0; b < per * 8; ++b) {
        const int k = b % 8, q = b / 8;
        const int li = k * per + q;
        if (li < n) it[b] = logical[li];
    }
    return it;
}

fuglbm_status build_items(fuglbm_sim *s) {
    const std::vector<FusedItem> it = item_list(s, s->rows);
    if ((int)it.size() > s->cv.max_items) return fail(FUGLBM_EINVAL, "too many work items");
    s->nitems = (int)it.size();
    HIP_TRY(hipMemcpy(s->items, it.data(), it.size() * sizeof(FusedItem), hipMemcpyHostToDevice));
    return FUGLBM_OK;
}

void drop_graph(fuglbm_sim *s) {
    if (s->graph.exec) (void)hipGraphExecDestroy(s->graph.exec);
    s->graph = GraphCache{};
}

hipError_t launch_one_step(fuglbm_sim *s, int flip_parity, hipStream_t st) {
    if (is_fused(s->kernel))
        return launch_fused(s->kernel, s->N, s->fp32, s->items, s->nitems, s->fsim, flip_parity,
                            st);
    return launch_step_generic(s->lattice, s->fp32, s->dc, s->N, s->nx, s->ny, s->nz, s->buf[flip_parity],
                               s->buf[flip_parity ^ 1], s->rho_f, s->psi_f, s->s_f, s->j_f,
                               s->u_f, s->status, s->hc.omega != 1.0, st);
}

constexpr int GRAPH_STEPS = 32;  // even: a replay returns to the same parity

fuglbm_status ensure_graph(fuglbm_sim *s) {
    if (s->graph.exec && s->graph.kernel == s->kernel && s->graph.rows == s->rows)
        return FUGLBM_OK;
    drop_graph(s);
    hipStream_t cs = capture_stream();
    if (!cs) return fail(FUGLBM_EDEVICE, "cannot create capture stream");
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < GRAPH_STEPS; ++k) {
        hipError_t e = launch_one_step(s, k & 1, cs);
        if (e != hipSuccess) {
            hipGraph_t g = nullptr;
            if (hipStreamEndCapture(cs, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
            return hip_fail(e, "capture");
        }
    }
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamEndCapture(cs, &g));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    s->graph.exec = ex;
    s->graph.steps = GRAPH_STEPS;
    s->graph.kernel = s->kernel;
    s->graph.rows = s->rows;
    return FUGLBM_OK;
}

// ---- rows-per-item autotuner ---------------------------------------------
// Candidates are timed on trial launches that read the current state and
// write the other buffer without swapping them: the state does not move,
// and the next real step overwrites what the trials wrote.  (Every rows
// value gives bitwise the same new state, since each site's arithmetic does
// not depend on which work item computes it.)  The winner is cached per
// (nx, ny, N, precision) for the process, and per batch shape for batched
// launches.
constexpr int TUNE_ROWS[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256};
constexpr int TUNE_LAUNCHES = 4;

std::vector<int> tune_candidates(int ny, int model) {
    std::vector<int> c;
    for (int r : TUNE_ROWS)
        if (r < ny) c.push_back(r);
    c.push_back(ny);
    if (model > 0 && model < ny) c.push_back(model);
    std::sort(c.begin(), c.end());
    c.erase(std::unique(c.begin(), c.end()), c.end());
    return c;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer() {
        if (hipEventCreate(&a) != hipSuccess) a = nullptr;
        if (hipEventCreate(&b) != hipSuccess) b = nullptr;
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    Timer(const Timer &) = delete;
    Timer &operator=(const Timer &) = delete;
    bool ok() const { return a && b; }
};

// Times `launch` (TUNE_LAUNCHES back-to-back launches) after `prepare(r)`
// for every candidate r; returns the fastest.
template <class Prep, class Launch>
// Candidates are timed in two passes, in order and then in reverse order,
// and ranked by the sum: the GPU's clocks still rise during the first
// hundreds of milliseconds of sustained work, so a single pass would favour
// the candidates timed last.
fuglbm_status time_candidates(const std::vector<int> &cand, hipStream_t st, Prep prepare,
                              Launch launch, int &best, float *best_time = nullptr) {
    Timer tm;
    if (!tm.ok()) return fail(FUGLBM_EDEVICE, "hipEventCreate");
    std::vector<float> sum(cand.size(), 0.f);
    bool warm = false;
    for (int pass = 0; pass < 2; ++pass) {
        for (size_t q = 0; q < cand.size(); ++q) {
            const size_t k = pass == 0 ? q : cand.size() - 1 - q;
            fuglbm_status rc = prepare(cand[k]);
            if (rc != FUGLBM_OK) return rc;
            if (!warm) {   // first launch of the kernel: not timed
                HIP_TRY(launch());
                warm = true;
            }
            HIP_TRY(hipEventRecord(tm.a, st));
            for (int j = 0; j < TUNE_LAUNCHES; ++j) HIP_TRY(launch());
            HIP_TRY(hipEventRecord(tm.b, st));
            HIP_TRY(hipEventSynchronize(tm.b));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, tm.a, tm.b));
            sum[k] += ms;
        }
    }
    float best_ms = 1e30f;
    best = cand.empty() ? 0 : cand[0];
    for (size_t k = 0; k < cand.size(); ++k)
        if (sum[k] < best_ms) {
            best_ms = sum[k];
            best = cand[k];
        }
    if (best_time) *best_time = best_ms;
    return FUGLBM_OK;
}

std::map<std::tuple<int, int, int, int>, int> &tune_cache() {
    static std::map<std::tuple<int, int, int, int>, int> m;
    return m;
}

fuglbm_status set_rows(fuglbm_sim *s, int rows, hipStream_t st) {
    if (rows == s->rows) return FUGLBM_OK;
    HIP_TRY(hipStreamSynchronize(st));   // queued launches still read the item table
    s->rows = rows;
    return build_items(s);
}

// With the variant left to the tuner, both fused variants are timed (each
// at its own rows candidates) and the faster (variant, rows) is kept; the
// cache entry holds kernel * 65536 + rows.  Every candidate's work table
// is uploaded once, before any timing, and the candidates run back to back
// with an event pair each and one synchronisation at the end: the GPU
// stays busy through the whole trial, so the candidates are timed under
// the same sustained load (with a host wait between candidates the clocks
// fall back and the early candidates run slower).
fuglbm_status autotune_rows(fuglbm_sim *s, hipStream_t st) {
    const TraceRange trace_range("fuglbm autotune rows");
    const bool both = s->auto_kernel && ws_usable(s->N, s->fp32);
    const int tag = both ? 0 : s->kernel;
    const auto key = std::make_tuple(s->nx, s->ny, s->N, (s->fp32 ? 1 : 0) + 2 * tag);
    auto hit = tune_cache().find(key);
    int best_k = s->kernel, best = 0;
    if (hit != tune_cache().end()) {
        best_k = hit->second >> 16;
        best = hit->second & 0xffff;
    } else {
        struct Cand {
            int kernel, rows;
            size_t off, n;
        };
        std::vector<Cand> cand;
        std::vector<FusedItem> all;
        for (int k : {2, 3}) {
            if (both ? false : k != s->kernel) continue;
            if (k == 3 && !ws_usable(s->N, s->fp32)) continue;
            for (int r : tune_candidates(s->ny, auto_rows(s->nx, s->ny, s->N, s->fp32, k))) {
                const std::vector<FusedItem> it = item_list(s, r);
                cand.push_back({k, r, all.size(), it.size()});
                all.insert(all.end(), it.begin(), it.end());
            }
        }
        // the candidates' tables; freed once the stream has drained (also on
        // an early error return, while trial launches may still read them)
        struct DevTables {
            FusedItem *p = nullptr;
            hipStream_t st;
            ~DevTables() {
                if (p) {
                    (void)hipStreamSynchronize(st);
                    (void)hipFree(p);
                }
            }
        } tables{nullptr, st};
        HIP_TRY(hipMalloc(&tables.p, all.size() * sizeof(FusedItem)));
        FusedItem *dev = tables.p;
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(hipMemcpy(dev, all.data(), all.size() * sizeof(FusedItem), hipMemcpyHostToDevice));
        // two passes, in order and in reverse order, ranked by the sum (see
        // time_candidates), queued back to back with one wait at the end
        std::vector<Timer> tm(2 * cand.size());
        for (auto &t : tm)
            if (!t.ok()) return fail(FUGLBM_EDEVICE, "hipEventCreate");
        // the trial launches read the current state and write the spare
        // buffer (parity unchanged): the state does not move
        auto launch = [&](const Cand &c) {
            return launch_fused(c.kernel, s->N, s->fp32, dev + c.off, (int)c.n, s->fsim, s->parity,
                                st);
        };
        for (size_t i = 0; i < cand.size(); ++i)   // first launch of each variant: not timed
            if (i == 0 || cand[i].kernel != cand[i - 1].kernel) HIP_TRY(launch(cand[i]));
        const size_t nc = cand.size();
        for (size_t q = 0; q < 2 * nc; ++q) {
            const size_t i = q < nc ? q : 2 * nc - 1 - q;
            HIP_TRY(hipEventRecord(tm[q].a, st));
            for (int j = 0; j < TUNE_LAUNCHES; ++j) HIP_TRY(launch(cand[i]));
            HIP_TRY(hipEventRecord(tm[q].b, st));
        }
        HIP_TRY(hipEventSynchronize(tm.back().b));
        float best_ms = 1e30f;
        for (size_t i = 0; i < nc; ++i) {
            float m1 = 0.f, m2 = 0.f;
            HIP_TRY(hipEventElapsedTime(&m1, tm[i].a, tm[i].b));
            HIP_TRY(hipEventElapsedTime(&m2, tm[2 * nc - 1 - i].a, tm[2 * nc - 1 - i].b));
            const float ms = m1 + m2;
            if (ms < best_ms) {
                best_ms = ms;
                best_k = cand[i].kernel;
                best = cand[i].rows;
            }
        }
        tune_cache()[key] = best_k * 65536 + best;
    }
    HIP_TRY(hipStreamSynchronize(st));
    s->kernel = best_k;
    s->tuned = true;
    return set_rows(s, best, st);
}

fuglbm_status sync_status(fuglbm_sim *s) {
    HIP_TRY(hipStreamSynchronize(s->last_stream));
    uint32_t st = 0;
    HIP_TRY(hipMemcpy(&st, s->status, sizeof(uint32_t), hipMemcpyDeviceToHost));
    s->sticky |= st;
    return FUGLBM_OK;
}

}  // namespace

extern "C" {

const char *fuglbm_last_error(void) { return g_err.c_str(); }

fuglbm_status fuglbm_init_mixture(const fuglbm_mixture_desc *d, fuglbm_mixture **out) {
    if (!d || !out) return fail(FUGLBM_EINVAL, "null argument");
    *out = nullptr;
    const int N = d->ncomp;
    if (N < 1 || N > FUGLBM_MAX_COMP) return fail(FUGLBM_EINVAL, "ncomp out of range");
    if (!d->Tc_K || !d->pc_bar || !d->omega || !d->M_gmol)
        return fail(FUGLBM_EINVAL, "null component array");
    if (d->ref_comp < 0 || d->ref_comp >= N) return fail(FUGLBM_EINVAL, "ref_comp out of range");
    if (d->eos < FUGLBM_EOS_PR || d->eos > FUGLBM_EOS_VDW) return fail(FUGLBM_EINVAL, "unknown eos");
    if (!(d->T_K > 0) || !std::isfinite(d->T_K)) return fail(FUGLBM_EINVAL, "T_K must be > 0");
    if (!(d->tau > 0.5) || !std::isfinite(d->tau)) return fail(FUGLBM_EINVAL, "tau must be > 1/2");
    if (!(d->kappa_ref_lu >= 0) || !std::isfinite(d->kappa_ref_lu))
        return fail(FUGLBM_EINVAL, "kappa_ref_lu must be >= 0");
    for (int i = 0; i < N; ++i) {
        if (!(d->Tc_K[i] > 0) || !(d->pc_bar[i] > 0) || !(d->M_gmol[i] > 0) ||
            !std::isfinite(d->omega[i]) || !std::isfinite(d->Tc_K[i]) ||
            !std::isfinite(d->pc_bar[i]) || !std::isfinite(d->M_gmol[i]))
            return fail(FUGLBM_EINVAL, "component constants must be positive and finite");
    }
    if (d->kij) {
        for (int i = 0; i < N; ++i) {
            if (d->kij[i * N + i] != 0.0) return fail(FUGLBM_EINVAL, "kij diagonal must be 0");
            for (int j = 0; j < N; ++j) {
                if (!std::isfinite(d->kij[i * N + j]) || d->kij[i * N + j] != d->kij[j * N + i])
                    return fail(FUGLBM_EINVAL, "kij must be finite and symmetric");
                if (!(d->kij[i * N + j] < 1.0)) return fail(FUGLBM_EINVAL, "kij must be < 1");
            }
        }
    }
    auto *m = new (std::nothrow) fuglbm_mixture();
    if (!m) return fail(FUGLBM_ENOMEM, "host allocation");
    const double a_ref = d->a_ref_lu > 0 ? d->a_ref_lu : 2.0 / 49.0;
    const double b_ref = d->b_ref_lu > 0 ? d->b_ref_lu : 2.0 / 21.0;
    const double R = d->R_lu > 0 ? d->R_lu : 1.0;
    const int c = d->ref_comp;
    const CubicEos E = cubic_eos(d->eos);
    // reference component's critical point in lattice units from a and b
    const double Tc_ref = (a_ref / b_ref) * (E.omega_b / E.omega_a) / R;
    const double pc_ref = E.omega_b * R * Tc_ref / b_ref;
    const double Tsc = Tc_ref / d->Tc_K[c];     // lattice units per K
    const double psc = pc_ref / d->pc_bar[c];   // lattice units per bar
    m->N = N;
    m->eos = d->eos;
    m->tau = d->tau;
    m->RT = R * d->T_K * Tsc;
    double a_lu[FUG_MAXC];
    for (int i = 0; i < N; ++i) {
        const double Tc = d->Tc_K[i] * Tsc, pc = d->pc_bar[i] * psc;
        a_lu[i] = E.omega_a * R * R * Tc * Tc / pc;
        m->b[i] = E.omega_b * R * Tc / pc;
        m->aa[i] = a_lu[i] * cubic_alpha(d->eos, d->omega[i], d->T_K / d->Tc_K[i]);
        m->M[i] = d->M_gmol[i] / d->M_gmol[c];
    }
    for (int i = 0; i < N; ++i) {
        m->sqk[i] = std::sqrt(d->kappa_ref_lu * a_lu[i] / a_lu[c]);
        for (int j = 0; j < N; ++j) {
            const double k = d->kij ? d->kij[i * N + j] : 0.0;
            m->aij[i * FUG_MAXC + j] = std::sqrt(m->aa[i] * m->aa[j]) * (1.0 - k);
        }
    }
    *out = m;
    return FUGLBM_OK;
}

fuglbm_status fuglbm_lattice_constants(const fuglbm_mixture *m, double *out, size_t n) {
    if (!m || !out) return fail(FUGLBM_EINVAL, "null argument");
    const int N = m->N;
    if (n < (size_t)(1 + 4 * N + N * N)) return fail(FUGLBM_EINVAL, "output too small");
    size_t k = 0;
    out[k++] = m->RT;
    for (int i = 0; i < N; ++i) {
        out[k++] = m->b[i];
        out[k++] = m->aa[i];
        out[k++] = m->sqk[i];
        out[k++] = m->M[i];
    }
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) out[k++] = m->aij[i * FUG_MAXC + j];
    return FUGLBM_OK;
}

void fuglbm_destroy_mixture(fuglbm_mixture *m) { delete m; }

size_t fuglbm_fields_bytes(int32_t ncomp, fuglbm_lattice lattice, fuglbm_precision prec,
                           int32_t nx, int32_t ny, int32_t nz) {
    if (ncomp < 1 || ncomp > FUGLBM_MAX_COMP || nx < 1 || ny < 1 || nz < 1) return 0;
    if (lattice != FUGLBM_D2Q9 && lattice != FUGLBM_D3Q19) return 0;
    return carve(ncomp, lattice, prec == FUGLBM_FP32_STORAGE, nx, ny, nz).total;
}

fuglbm_status fuglbm_init_fields(const fuglbm_mixture *mix, fuglbm_lattice lattice,
                                 fuglbm_precision prec, int32_t nx, int32_t ny, int32_t nz,
                                 const double *rho, void *dev_buf, void *hip_stream,
                                 fuglbm_sim **out) {
    const TraceRange trace_range("fuglbm_init_fields");
    if (!mix || !rho || !out) return fail(FUGLBM_EINVAL, "null argument");
    *out = nullptr;
    if (lattice != FUGLBM_D2Q9 && lattice != FUGLBM_D3Q19) return fail(FUGLBM_EINVAL, "lattice");
    if (prec != FUGLBM_FP64 && prec != FUGLBM_FP32_STORAGE) return fail(FUGLBM_EINVAL, "precision");
    if (nx < 1 || ny < 1 || nz < 1) return fail(FUGLBM_EINVAL, "grid sizes must be >= 1");
    if (lattice == FUGLBM_D2Q9 && nz != 1) return fail(FUGLBM_EINVAL, "D2Q9 needs nz == 1");
    const int64_t ns = (int64_t)nx * ny * nz;
    if (ns > (int64_t)1 << 31) return fail(FUGLBM_EINVAL, "grid too large");
    const int N = mix->N;
    // physical admissibility of the initial field (rho_i > 0, finite, b_m rt < 1)
    for (int64_t s = 0; s < ns; ++s) {
        double eta = 0.0;
        for (int i = 0; i < N; ++i) {
            const double r = rho[(int64_t)i * ns + s];
            if (!std::isfinite(r) || !(r > 0.0))
                return fail(FUGLBM_EUNPHYSICAL, "rho_i must be finite and > 0");
            eta += mix->b[i] * r / mix->M[i];
        }
        if (!(eta < 1.0)) return fail(FUGLBM_EUNPHYSICAL, "b_m * rt >= 1 (outside the EOS domain)");
    }
    auto *s = new (std::nothrow) fuglbm_sim();
    if (!s) return fail(FUGLBM_ENOMEM, "host allocation");
    s->mix = mix;
    s->lattice = lattice;
    s->fp32 = prec == FUGLBM_FP32_STORAGE;
    s->nx = nx; s->ny = ny; s->nz = nz;
    s->N = N;
    s->Q = lattice_Q(lattice);
    s->D = lattice_D(lattice);
    s->ns = ns;
    s->cv = carve(N, lattice, s->fp32, nx, ny, nz);
    hipStream_t st = (hipStream_t)hip_stream;
    s->last_stream = st;
    if (dev_buf) {
        if (((uintptr_t)dev_buf & 255) != 0) {
            delete s;
            return fail(FUGLBM_EINVAL, "dev_buf must be 256-byte aligned");
        }
        s->base = (char *)dev_buf;
        s->owned = false;
    } else {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, s->cv.total);
        if (e != hipSuccess) {
            delete s;
            return fail(FUGLBM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        s->base = (char *)p;
        s->owned = true;
    }
    s->buf[0] = s->base + s->cv.buf0;
    s->buf[1] = s->base + s->cv.buf1;
    s->dc = (SimConst *)(s->base + s->cv.cst);
    s->status = (uint32_t *)(s->base + s->cv.status);
    s->rho_f = (double *)(s->base + s->cv.rho);
    s->psi_f = (double *)(s->base + s->cv.psi);
    s->s_f = (double *)(s->base + s->cv.s);
    s->j_f = (double *)(s->base + s->cv.j);
    s->u_f = (double *)(s->base + s->cv.u);
    s->snap = (double *)(s->base + s->cv.snap);
    s->part = (double *)(s->base + s->cv.part);
    s->fsim = (FusedSim *)(s->base + s->cv.fsim);
    s->items = (FusedItem *)(s->base + s->cv.items);
    s->parity = 0;
    if (hipEventCreateWithFlags(&s->done, hipEventDisableTiming) != hipSuccess) {
        if (s->owned) (void)hipFree(s->base);
        delete s;
        return fail(FUGLBM_EDEVICE, "hipEventCreate");
    }
    s->done_valid = false;
    // constant block
    SimConst &c = s->hc;
    std::memset(&c, 0, sizeof(c));
    c.N = N;
    c.lattice = lattice;
    c.nx = nx; c.ny = ny; c.nz = nz;
    c.nsites = ns;
    c.omega = 1.0 / mix->tau;
    c.fcoef = 1.0 - 1.0 / (2.0 * mix->tau);
    c.RT = mix->RT;
    {
        const CubicEos E = cubic_eos(mix->eos);
        c.eos = mix->eos;
        c.d1 = E.d1;
        c.d2 = E.d2;
        c.eu = E.u;
        c.ew = E.w;
        c.dk = mix->eos == FUGLBM_EOS_VDW ? 0.0 : 1.0 / (E.d1 - E.d2);
    }
    for (int i = 0; i < N; ++i) {
        c.b[i] = mix->b[i];
        c.M[i] = mix->M[i];
        c.invM[i] = 1.0 / mix->M[i];
        c.sqk[i] = mix->sqk[i];
        for (int j = 0; j < N; ++j) c.aij[i * FUG_MAXC + j] = mix->aij[i * FUG_MAXC + j];
    }
    fuglbm_status rc = FUGLBM_OK;
    auto bail = [&](fuglbm_status r) {
        (void)hipEventDestroy(s->done);
        if (s->owned) (void)hipFree(s->base);
        delete s;
        return r;
    };
    hipError_t e = hipMemcpy(s->dc, &c, sizeof(SimConst), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(hip_fail(e, "upload constants"));
    // stage rho in the second population buffer, then g = geq(rho, u = 0)
    e = hipMemcpy(s->buf[1], rho, (size_t)N * ns * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(hip_fail(e, "upload rho"));
    e = hipMemset(s->status, 0, 256);
    if (e != hipSuccess) return bail(hip_fail(e, "clear status"));
    e = launch_init(lattice, s->fp32, s->dc, ns, (const double *)s->buf[1], s->buf[0], st);
    if (e != hipSuccess) return bail(hip_fail(e, "init kernel"));
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bail(hip_fail(e, "init sync"));
    // fused-kernel tables (D2Q9)
    FusedSim fs{};
    fs.c = s->dc;
    fs.buf[0] = s->buf[0];
    fs.buf[1] = s->buf[1];
    fs.status = s->status;
    fs.parity = 0;
    e = hipMemcpy(s->fsim, &fs, sizeof(FusedSim), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(hip_fail(e, "upload fused sim"));
    const bool fused = fused_fits(s);
    s->kernel = default_kernel(s);
    s->rows = fused ? auto_rows(nx, ny, N, s->fp32, s->kernel) : 0;
    s->auto_kernel = fused;
    if (fused) {
        rc = build_items(s);
        if (rc != FUGLBM_OK) return bail(rc);
    }
    s->step = 0;
    s->snap_step = 0;
    s->have_snap = false;
    s->sticky = 0;
    s->autotune = fused;
    s->tuned = false;
    s->uid = next_sim_uid();
    *out = s;
    return FUGLBM_OK;
}

fuglbm_status fuglbm_get_tuning(const fuglbm_sim *s, int32_t *kernel, int32_t *rows) {
    if (!s) return fail(FUGLBM_EINVAL, "null sim");
    if (kernel) *kernel = s->kernel;
    if (rows) *rows = is_fused(s->kernel) ? s->rows : 0;
    return FUGLBM_OK;
}

fuglbm_status fuglbm_set_tuning(fuglbm_sim *s, int32_t kernel, int32_t rows) {
    if (!s) return fail(FUGLBM_EINVAL, "null sim");
    if (kernel < 0 || kernel > 3) return fail(FUGLBM_EINVAL, "kernel must be 0, 1, 2 or 3");
    if (is_fused(kernel) && !fused_fits(s))
        return fail(FUGLBM_EINVAL, "the fused kernel is D2Q9 only, with < 2^32 elements per buffer");
    if (kernel == 3 && !ws_usable(s->N, s->fp32))
        return fail(FUGLBM_EINVAL, "the store-wave fused kernel is built for at most 10 components");
    if (rows < 0) return fail(FUGLBM_EINVAL, "rows must be >= 0");
    const int k = kernel == 0 ? default_kernel(s) : kernel;
    s->auto_kernel = kernel == 0 && is_fused(k);
    int r = s->rows;
    if (is_fused(k)) {
        r = rows == 0 ? auto_rows(s->nx, s->ny, s->N, s->fp32, k) : std::min<int>(rows, s->ny);
        s->autotune = rows == 0;
        s->tuned = false;
    }
    HIP_TRY(hipStreamSynchronize(s->last_stream));
    s->kernel = k;
    if (r != s->rows) {
        s->rows = r;
        fuglbm_status rc = build_items(s);
        if (rc != FUGLBM_OK) return rc;
    }
    drop_graph(s);
    return FUGLBM_OK;
}

fuglbm_status fuglbm_sim_info(const fuglbm_sim *s, int32_t *Q, int32_t *D, int64_t *sites,
                              int64_t *alg_bytes, int32_t *kernel) {
    if (!s) return fail(FUGLBM_EINVAL, "null sim");
    if (Q) *Q = s->Q;
    if (D) *D = s->D;
    if (sites) *sites = s->ns;
    // algorithmic bytes: every population read and written once (no padding)
    if (alg_bytes) *alg_bytes = 2 * (int64_t)s->N * s->ns * (8 + (s->Q - 1) * (s->fp32 ? 4 : 8));
    if (kernel) *kernel = s->kernel;
    return FUGLBM_OK;
}

fuglbm_status fuglbm_step_n(fuglbm_sim *s, int64_t nsteps, void *hip_stream) {
    const TraceRange trace_range("fuglbm_step_n");
    if (!s) return fail(FUGLBM_EINVAL, "null sim");
    if (nsteps < 0) return fail(FUGLBM_EINVAL, "nsteps must be >= 0");
    if (s->sticky) return fail(FUGLBM_ENONFINITE, "simulation has a sticky device error");
    hipStream_t st = (hipStream_t)hip_stream;
    {
        fuglbm_status rc = order_after(s, st);
        if (rc != FUGLBM_OK) return rc;
    }
    int64_t left = nsteps;
    if (left > 0 && is_fused(s->kernel) && s->autotune && !s->tuned) {
        fuglbm_status rc = autotune_rows(s, st);
        if (rc != FUGLBM_OK) return rc;
    }
    // odd parity first so that graph replays start from buffer 0
    if (left > 0 && s->parity == 1 && left >= 2 * GRAPH_STEPS) {
        hipError_t e = launch_one_step(s, s->parity, st);
        if (e != hipSuccess) return hip_fail(e, "step launch");
        s->parity ^= 1;
        --left;
        ++s->step;
    }
    if (left >= 2 * GRAPH_STEPS && s->parity == 0) {
        fuglbm_status rc = ensure_graph(s);
        if (rc != FUGLBM_OK) return rc;
        while (left >= GRAPH_STEPS) {
            HIP_TRY(hipGraphLaunch(s->graph.exec, st));
            left -= GRAPH_STEPS;
            s->step += GRAPH_STEPS;
        }
    }
    for (; left > 0; --left) {
        hipError_t e = launch_one_step(s, s->parity, st);
        if (e != hipSuccess) return hip_fail(e, "step launch");
        s->parity ^= 1;
        ++s->step;
    }
    return mark_done(s, st);
}

fuglbm_status fuglbm_read_moments(fuglbm_sim *s, double *rho_out, double *u_out,
                                  fuglbm_diag *diag) {
    const TraceRange trace_range("fuglbm_read_moments");
    if (!s) return fail(FUGLBM_EINVAL, "null sim");
    hipStream_t st = s->last_stream;
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(launch_fields(s->lattice, s->fp32, s->dc, s->nx, s->ny, s->nz, s->buf[s->parity],
                          s->rho_f, s->psi_f, s->s_f, s->j_f, u_out ? s->u_f : nullptr, s->status,
                          st));
    HIP_TRY(hipStreamSynchronize(st));
    if (rho_out)
        HIP_TRY(hipMemcpy(rho_out, s->rho_f, (size_t)s->N * s->ns * 8, hipMemcpyDeviceToHost));
    if (u_out)
        HIP_TRY(hipMemcpy(u_out, s->u_f, (size_t)s->D * s->ns * 8, hipMemcpyDeviceToHost));
    fuglbm_status rc = sync_status(s);
    if (rc != FUGLBM_OK) return rc;
    if (diag) {
        rc = fuglbm_diagnostics(s, diag);
        if (rc != FUGLBM_OK && rc != FUGLBM_ENONFINITE) return rc;
    }
    if (s->sticky) return fail(FUGLBM_ENONFINITE, "device status bits set");
    return FUGLBM_OK;
}

// Diagnostics: the fields pass (rho_i, j, force-corrected u of the current
// state), then per-block partial sums and one fixed-order final sum per
// quantity on the device; the host reads the (N + 1) x DIAG_QUANT totals.
fuglbm_status fuglbm_diagnostics(fuglbm_sim *s, fuglbm_diag *diag) {
    const TraceRange trace_range("fuglbm_diagnostics");
    if (!s || !diag) return fail(FUGLBM_EINVAL, "null argument");
    hipStream_t st = s->last_stream;
    const int nblk = diag_blocks(s->ns);
    const int N = s->N;
    double *fin = s->part + (size_t)1024 * (N + 1) * DIAG_QUANT;
    HIP_TRY(launch_fields(s->lattice, s->fp32, s->dc, s->nx, s->ny, s->nz, s->buf[s->parity],
                          s->rho_f, s->psi_f, s->s_f, s->j_f, s->u_f, s->status, st));
    HIP_TRY(launch_diag(s->D, N, s->ns, s->rho_f, s->j_f, s->u_f, s->snap, s->part, nblk, fin,
                        s->have_snap ? 1 : 0, st));
    double tot[(FUGLBM_MAX_COMP + 1) * DIAG_QUANT];
    HIP_TRY(hipMemcpyAsync(tot, fin, sizeof(double) * (N + 1) * DIAG_QUANT, hipMemcpyDeviceToHost,
                           st));
    HIP_TRY(hipStreamSynchronize(st));
    std::memset(diag, 0, sizeof(*diag));
    diag->step = s->step;
    for (int i = 0; i < N; ++i) diag->mass[i] = tot[i * DIAG_QUANT];
    for (int d = 0; d < s->D; ++d) {
        diag->momentum_pop[d] = tot[N * DIAG_QUANT + d];
        diag->momentum[d] = tot[N * DIAG_QUANT + 3 + d];
    }
    double res = 0.0;
    const int64_t K = s->step - s->snap_step;
    if (s->have_snap && K > 0)
        for (int i = 0; i < N; ++i)
            res = std::max(res, tot[i * DIAG_QUANT + 1] / ((double)K * tot[i * DIAG_QUANT]));
    diag->residual = res;
    s->have_snap = true;
    s->snap_step = s->step;
    fuglbm_status rc = sync_status(s);
    if (rc != FUGLBM_OK) return rc;
    diag->status = s->sticky;
    if (s->sticky) return fail(FUGLBM_ENONFINITE, "device status bits set");
    return FUGLBM_OK;
}

extern "C++" {
// Column of the stored moving population a of column x (pop_col).
static int host_pop_col(const fuglbm_sim *s, int a, int x) {
    return s->lattice == FUGLBM_D3Q19 ? pop_col<D3Q19>(a, x, s->nx) : pop_col<D2Q9>(a, x, s->nx);
}

// Host copy of one buffer <-> [N][Q][sites] FP64 (the layout is PopLayout,
// the moving populations' columns pop_col).
template <typename ST>
void unpack_pops(const fuglbm_sim *s, const char *buf, double *g) {
    const PopLayout<ST> P(s->N, s->Q, s->nx, (int64_t)s->ny * s->nz);
    const int64_t rows = (int64_t)s->ny * s->nz;
    for (int i = 0; i < s->N; ++i)
        for (int a = 0; a < s->Q; ++a)
            for (int64_t r = 0; r < rows; ++r) {
                double *o = g + ((size_t)i * s->Q + a) * s->ns + (size_t)r * s->nx;
                if (a == 0) {
                    const double *src = (const double *)(buf + P.rest(r, i, 0));
                    for (int x = 0; x < s->nx; ++x) o[x] = src[x];
                } else {
                    const ST *src = (const ST *)(buf + P.move(r, i, a, 0));
                    for (int x = 0; x < s->nx; ++x) o[x] = (double)src[host_pop_col(s, a, x)];
                }
            }
}

template <typename ST>
void pack_pops(const fuglbm_sim *s, const double *g, char *buf) {
    const PopLayout<ST> P(s->N, s->Q, s->nx, (int64_t)s->ny * s->nz);
    const int64_t rows = (int64_t)s->ny * s->nz;
    for (int i = 0; i < s->N; ++i)
        for (int a = 0; a < s->Q; ++a)
            for (int64_t r = 0; r < rows; ++r) {
                const double *in = g + ((size_t)i * s->Q + a) * s->ns + (size_t)r * s->nx;
                if (a == 0) {
                    double *dst = (double *)(buf + P.rest(r, i, 0));
                    for (int x = 0; x < s->nx; ++x) dst[x] = in[x];
                } else {
                    ST *dst = (ST *)(buf + P.move(r, i, a, 0));
                    for (int x = 0; x < s->nx; ++x) dst[host_pop_col(s, a, x)] = (ST)in[x];
                }
            }
}
}  // extern "C++"

fuglbm_status fuglbm_read_populations(fuglbm_sim *s, double *g_out) {
    if (!s || !g_out) return fail(FUGLBM_EINVAL, "null argument");
    HIP_TRY(hipStreamSynchronize(s->last_stream));
    std::vector<char> tmp((size_t)pop_bytes(s));
    HIP_TRY(hipMemcpy(tmp.data(), s->buf[s->parity], tmp.size(), hipMemcpyDeviceToHost));
    if (s->fp32)
        unpack_pops<float>(s, tmp.data(), g_out);
    else
        unpack_pops<double>(s, tmp.data(), g_out);
    return FUGLBM_OK;
}

fuglbm_status fuglbm_write_populations(fuglbm_sim *s, const double *g_in, int64_t step) {
    if (!s || !g_in) return fail(FUGLBM_EINVAL, "null argument");
    if (step < 0) return fail(FUGLBM_EINVAL, "step must be >= 0");
    HIP_TRY(hipStreamSynchronize(s->last_stream));
    std::vector<char> tmp((size_t)pop_bytes(s));
    if (s->fp32)
        pack_pops<float>(s, g_in, tmp.data());
    else
        pack_pops<double>(s, g_in, tmp.data());
    HIP_TRY(hipMemcpy(s->buf[0], tmp.data(), tmp.size(), hipMemcpyHostToDevice));
    s->parity = 0;
    s->step = step;
    s->have_snap = false;
    return FUGLBM_OK;
}

fuglbm_status fuglbm_poke_population(fuglbm_sim *s, int32_t comp, int32_t a, int64_t site,
                                     double value) {
    if (!s) return fail(FUGLBM_EINVAL, "null sim");
    if (comp < 0 || comp >= s->N || a < 0 || a >= s->Q || site < 0 || site >= s->ns)
        return fail(FUGLBM_EINVAL, "index out of range");
    HIP_TRY(hipStreamSynchronize(s->last_stream));
    const int64_t row = site / s->nx;
    const int x = (int)(site - row * s->nx);
    char *b = (char *)s->buf[s->parity];
    if (a == 0) {
        const int64_t off = s->fp32 ? PopLayout<float>(s->N, s->Q, s->nx, (int64_t)s->ny * s->nz).rest(row, comp, x)
                                    : PopLayout<double>(s->N, s->Q, s->nx, (int64_t)s->ny * s->nz).rest(row, comp, x);
        HIP_TRY(hipMemcpy(b + off, &value, 8, hipMemcpyHostToDevice));
    } else if (s->fp32) {
        const float f = (float)value;
        const int64_t off = PopLayout<float>(s->N, s->Q, s->nx, (int64_t)s->ny * s->nz).move(row, comp, a, host_pop_col(s, a, x));
        HIP_TRY(hipMemcpy(b + off, &f, 4, hipMemcpyHostToDevice));
    } else {
        const int64_t off = PopLayout<double>(s->N, s->Q, s->nx, (int64_t)s->ny * s->nz).move(row, comp, a, host_pop_col(s, a, x));
        HIP_TRY(hipMemcpy(b + off, &value, 8, hipMemcpyHostToDevice));
    }
    return FUGLBM_OK;
}

void forget_sim_in_batches(const fuglbm_sim *s);

void fuglbm_destroy_sim(fuglbm_sim *s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->last_stream);
    forget_sim_in_batches(s);
    drop_graph(s);
    if (s->done) (void)hipEventDestroy(s->done);
    if (s->owned) (void)hipFree(s->base);
    delete s;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched stepping: D2Q9 simulations on the fused kernel that share the
// component count and precision run as ONE launch per step over a combined
// work-item table; the table is rebuilt only when the set of simulations
// (or their buffer parities) changes.
// ---------------------------------------------------------------------------
namespace {

struct BatchTable {
    std::vector<fuglbm_sim *> sims;
    std::vector<uint64_t> uids;
    std::vector<int> parity0;
    FusedSim *dsims = nullptr;
    FusedItem *ditems = nullptr;
    size_t cap_sims = 0, cap_items = 0;
    int nitems = 0;
    int kernel = 2;                   // fused variant of the launches
    hipGraphExec_t graph = nullptr;   // GRAPH_STEPS launches starting at flip 0
    hipStream_t last_stream = nullptr;
    bool used = false;                // last_stream is meaningful
};

fuglbm_status batch_graph(BatchTable &bt, int ncomp, bool fp32) {
    if (bt.graph) return FUGLBM_OK;
    hipStream_t cs = capture_stream();
    if (!cs) return fail(FUGLBM_EDEVICE, "cannot create capture stream");
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < GRAPH_STEPS; ++k) {
        hipError_t e =
            launch_fused(bt.kernel, ncomp, fp32, bt.ditems, bt.nitems, bt.dsims, k & 1, cs);
        if (e != hipSuccess) {
            hipGraph_t g = nullptr;
            if (hipStreamEndCapture(cs, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
            return hip_fail(e, "batch capture");
        }
    }
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamEndCapture(cs, &g));
    hipError_t e = hipGraphInstantiate(&bt.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        bt.graph = nullptr;
        return hip_fail(e, "hipGraphInstantiate (batch)");
    }
    return FUGLBM_OK;
}

std::map<std::pair<int, int>, BatchTable> &batch_tables() {
    static std::map<std::pair<int, int>, BatchTable> t;
    return t;
}

// rows > 0: every member uses min(rows, ny) rows per item; 0: its own.
// kernel: the fused variant (0: that of the first member).
fuglbm_status build_batch(BatchTable &bt, const std::vector<fuglbm_sim *> &group, hipStream_t st,
                          int rows = 0, int kernel = 0) {
    HIP_TRY(hipStreamSynchronize(st));  // the old table may still be read by queued launches
    if (bt.graph) {
        (void)hipGraphExecDestroy(bt.graph);
        bt.graph = nullptr;
    }
    bt.kernel = kernel ? kernel : group[0]->kernel;
    std::vector<FusedSim> hs;
    std::vector<FusedItem> logical;
    for (size_t k = 0; k < group.size(); ++k) {
        fuglbm_sim *s = group[k];
        FusedSim fs{};
        fs.c = s->dc;
        fs.buf[0] = s->buf[0];
        fs.buf[1] = s->buf[1];
        fs.status = s->status;
        fs.parity = s->parity;
        hs.push_back(fs);
        const int strips = (s->nx + FUSED_OUT - 1) / FUSED_OUT;
        const int rw = rows > 0 ? std::min(rows, s->ny) : s->rows;
        const int chunks = (s->ny + rw - 1) / rw;
        for (int c = 0; c < chunks; ++c)
            for (int t = 0; t < strips; ++t)
                logical.push_back({(int32_t)k, t * FUSED_OUT, c * rw, std::min(rw, s->ny - c * rw)});
    }
    const int n = (int)logical.size();
    const int per = (n + 7) / 8;
    std::vector<FusedItem> items((size_t)per * 8, FusedItem{-1, 0, 0, 0});
    for (int b = 0; b < per * 8; ++b) {
        const int li = (b % 8) * per + b / 8;
        if (li < n) items[b] = logical[li];
    }
    if (hs.size() > bt.cap_sims) {
        if (bt.dsims) (void)hipFree(bt.dsims);
        bt.cap_sims = hs.size() * 2;
        HIP_TRY(hipMalloc(&bt.dsims, bt.cap_sims * sizeof(FusedSim)));
    }
    if (items.size() > bt.cap_items) {
        if (bt.ditems) (void)hipFree(bt.ditems);
        bt.cap_items = items.size() * 2;
        HIP_TRY(hipMalloc(&bt.ditems, bt.cap_items * sizeof(FusedItem)));
    }
    HIP_TRY(hipMemcpy(bt.dsims, hs.data(), hs.size() * sizeof(FusedSim), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(bt.ditems, items.data(), items.size() * sizeof(FusedItem),
                      hipMemcpyHostToDevice));
    bt.nitems = (int)items.size();
    bt.sims = group;
    bt.uids.clear();
    for (auto *sp : group) bt.uids.push_back(sp->uid);
    bt.parity0.clear();
    for (auto *s : group) bt.parity0.push_back(s->parity);
    return FUGLBM_OK;
}

// Batched launches: the rows-per-item autotuner over one uniform rows value
// for all members, cached per batch class: component count, precision, and
// the power-of-two classes of the total strip-rows (strips x ny summed over
// members, which sets the item count against the resident slots) and of the
// tallest member.  Batches of a serving loop change members often; a class
// key lets them reuse one tuning.  Leaves bt built with the chosen rows.
static int log2_class(int64_t v) {
    int k = 0;
    while (v > 1) {
        v >>= 1;
        ++k;
    }
    return k;
}

fuglbm_status tune_batch(BatchTable &bt, const std::vector<fuglbm_sim *> &group, int nc, bool f32,
                         hipStream_t st) {
    static std::map<std::tuple<int, int, int, int>, int> cache;   // kernel * 65536 + rows
    for (auto *s : group)
        if (!s->autotune) return build_batch(bt, group, st);   // rows fixed by the caller
    bool auto_k = true;
    for (auto *s : group) auto_k = auto_k && s->auto_kernel;
    const bool both = auto_k && ws_usable(nc, f32);
    int64_t strip_rows = 0;
    int ny_max = 1;
    for (auto *s : group) {
        strip_rows += (int64_t)((s->nx + FUSED_OUT - 1) / FUSED_OUT) * s->ny;
        ny_max = std::max(ny_max, s->ny);
    }
    const int tag = both ? 0 : group[0]->kernel;
    const auto key = std::make_tuple(nc, (f32 ? 1 : 0) + 2 * tag, log2_class(strip_rows),
                                     log2_class(ny_max));
    auto hit = cache.find(key);
    if (hit != cache.end())
        return build_batch(bt, group, st, hit->second & 0xffff, hit->second >> 16);
    int best_k = group[0]->kernel, best = 0;
    float best_ms = 1e30f;
    for (int k : {2, 3}) {
        if (both ? false : k != group[0]->kernel) continue;
        if (k == 3 && !ws_usable(nc, f32)) continue;
        int r = 0;
        float ms = 0.f;
        fuglbm_status rc = time_candidates(
            tune_candidates(ny_max, 0), st, [&](int rr) { return build_batch(bt, group, st, rr, k); },
            [&]() { return launch_fused(k, nc, f32, bt.ditems, bt.nitems, bt.dsims, 0, st); }, r,
            &ms);
        if (rc != FUGLBM_OK) return rc;
        if (ms < best_ms) {
            best_ms = ms;
            best_k = k;
            best = r;
        }
    }
    cache[key] = best_k * 65536 + best;
    return build_batch(bt, group, st, best, best_k);
}

}  // namespace

// Batched multi-pass step (D3Q19, and D2Q9 simulations on the multi-pass
// kernels): one member table per (lattice, storage precision, tau != 1),
// cached while the member set is the same; four launches per step over all
// members (no tuning: the multi-pass kernels have no variants), runs of
// GRAPH_STEPS steps replayed from a captured graph as for the fused tables.
struct GenBatch {
    std::vector<fuglbm_sim *> sims;
    std::vector<uint64_t> uids;
    std::vector<int> parity0;
    GenMember *dm = nullptr;
    size_t cap = 0;
    int64_t total[3] = {0, 0, 0};
    int lattice = 0, fp32 = 0, keep = 0;
    hipGraphExec_t graph = nullptr;   // GRAPH_STEPS steps starting at flip 0
    hipStream_t last_stream = nullptr;
    bool used = false;   // last_stream is meaningful
};

hipError_t gen_batch_step(const GenBatch &gb, int flip, hipStream_t st) {
    return launch_step_generic_batch(gb.lattice, gb.fp32 != 0, gb.keep != 0, gb.dm,
                                     (int)gb.sims.size(), gb.total, flip, st);
}

void drop_gen_graph(GenBatch &gb) {
    if (gb.graph) (void)hipGraphExecDestroy(gb.graph);
    gb.graph = nullptr;
}

fuglbm_status gen_batch_graph(GenBatch &gb) {
    if (gb.graph) return FUGLBM_OK;
    hipStream_t cs = capture_stream();
    if (!cs) return fail(FUGLBM_EDEVICE, "cannot create capture stream");
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < GRAPH_STEPS; ++k) {
        hipError_t e = gen_batch_step(gb, k & 1, cs);
        if (e != hipSuccess) {
            hipGraph_t g = nullptr;
            if (hipStreamEndCapture(cs, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
            return hip_fail(e, "multi-pass batch capture");
        }
    }
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamEndCapture(cs, &g));
    hipError_t e = hipGraphInstantiate(&gb.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        gb.graph = nullptr;
        return hip_fail(e, "hipGraphInstantiate (multi-pass batch)");
    }
    return FUGLBM_OK;
}

std::map<std::tuple<int, int, int>, GenBatch> &gen_batches() {
    static std::map<std::tuple<int, int, int>, GenBatch> t;
    return t;
}

fuglbm_status build_gen_batch(GenBatch &gb, const std::vector<fuglbm_sim *> &group) {
    std::vector<GenMember> m(group.size());
    int64_t acc[3] = {0, 0, 0};
    for (size_t k = 0; k < group.size(); ++k) {
        const fuglbm_sim *s = group[k];
        int64_t u[3];
        generic_units(s->lattice == FUGLBM_D2Q9 ? 0 : 1, s->N, s->nx, s->ny, s->nz, u);
        GenMember &g = m[k];
        g.c = s->dc;
        g.buf[0] = s->buf[0];
        g.buf[1] = s->buf[1];
        g.rho_f = s->rho_f;
        g.psi_f = s->psi_f;
        g.s_f = s->s_f;
        g.j_f = s->j_f;
        g.u_f = s->u_f;
        g.status = s->status;
        for (int p = 0; p < 3; ++p) g.end[p] = (acc[p] += u[p]);
        g.parity = s->parity;
        g.pad = 0;
    }
    if (acc[0] > INT32_MAX - 8 || acc[1] > INT32_MAX - 8 || acc[2] > INT32_MAX - 8)
        return fail(FUGLBM_EINVAL, "batch too large for one launch");
    if (gb.cap < m.size()) {
        if (gb.dm) HIP_TRY(hipFree(gb.dm));
        gb.dm = nullptr;
        gb.cap = 0;
        HIP_TRY(hipMalloc(&gb.dm, m.size() * sizeof(GenMember)));
        gb.cap = m.size();
    }
    HIP_TRY(hipMemcpy(gb.dm, m.data(), m.size() * sizeof(GenMember), hipMemcpyHostToDevice));
    gb.sims = group;
    gb.uids.clear();
    gb.parity0.clear();
    for (auto *s : group) {
        gb.uids.push_back(s->uid);
        gb.parity0.push_back(s->parity);
    }
    for (int p = 0; p < 3; ++p) gb.total[p] = acc[p];
    gb.lattice = group[0]->lattice == FUGLBM_D2Q9 ? 0 : 1;
    gb.fp32 = group[0]->fp32 ? 1 : 0;
    gb.keep = group[0]->hc.omega != 1.0 ? 1 : 0;
    drop_gen_graph(gb);   // captured with the old table's size
    return FUGLBM_OK;
}

// A destroyed simulation's buffers may be handed to someone else: drop every
// cached table (and its captured graph) that still refers to it.
void forget_sim_in_batches(const fuglbm_sim *s) {
    for (auto &kv : gen_batches()) {
        GenBatch &gb = kv.second;
        for (size_t k = 0; k < gb.sims.size(); ++k) {
            if (gb.sims[k] == s && gb.uids[k] == s->uid) {
                drop_gen_graph(gb);
                gb.sims.clear();
                gb.uids.clear();
                gb.parity0.clear();
                break;
            }
        }
    }
    for (auto &kv : batch_tables()) {
        BatchTable &bt = kv.second;
        for (size_t k = 0; k < bt.sims.size(); ++k) {
            if (bt.sims[k] == s && bt.uids[k] == s->uid) {
                if (bt.graph) {
                    (void)hipGraphExecDestroy(bt.graph);
                    bt.graph = nullptr;
                }
                bt.sims.clear();
                bt.uids.clear();
                bt.parity0.clear();
                break;
            }
        }
    }
}

extern "C" fuglbm_status fuglbm_step_many(fuglbm_sim *const *sims, int32_t count, int64_t nsteps,
                                          void *hip_stream) {
    const TraceRange trace_range("fuglbm_step_many");
    if (count < 0 || (count > 0 && !sims)) return fail(FUGLBM_EINVAL, "bad sims array");
    if (nsteps < 0) return fail(FUGLBM_EINVAL, "nsteps must be >= 0");
    hipStream_t st = (hipStream_t)hip_stream;
    std::map<std::pair<int, int>, std::vector<fuglbm_sim *>> groups;
    std::vector<fuglbm_sim *> others;
    bool skipped = false;
    for (int k = 0; k < count; ++k) {
        fuglbm_sim *s = sims[k];
        if (!s) return fail(FUGLBM_EINVAL, "null sim in batch");
        for (int q = 0; q < k; ++q)
            if (sims[q] == s) return fail(FUGLBM_EINVAL, "duplicate sim in batch");
        if (s->sticky) {
            skipped = true;
            continue;
        }
        if (s->lattice == FUGLBM_D2Q9 && is_fused(s->kernel))
            groups[{s->N, s->fp32 ? 1 : 0}].push_back(s);
        else
            others.push_back(s);
    }
    for (int k = 0; k < count; ++k) {
        if (sims[k]->sticky) continue;
        fuglbm_status rc = order_after(sims[k], st);
        if (rc != FUGLBM_OK) return rc;
    }
    for (auto &kv : groups) {
        auto &group = kv.second;
        BatchTable &bt = batch_tables()[kv.first];
        // the table (and its graph) is shared state: launches queued on
        // another stream must finish before this call rebuilds or reuses it
        if (bt.used && bt.last_stream != st) HIP_TRY(hipStreamSynchronize(bt.last_stream));
        bt.last_stream = st;
        bt.used = true;
        bool same = bt.sims.size() == group.size();
        for (size_t k = 0; same && k < group.size(); ++k)
            same = bt.sims[k] == group[k] && bt.uids[k] == group[k]->uid;
        int flip = 0;
        if (same) {
            flip = group[0]->parity ^ bt.parity0[0];
            for (size_t k = 0; k < group.size(); ++k)
                if ((group[k]->parity ^ bt.parity0[k]) != flip) same = false;
        }
        const int nc = kv.first.first;
        const bool f32 = kv.first.second != 0;
        int64_t left = nsteps;
        if (!same) {
            fuglbm_status rc = left > 0 ? tune_batch(bt, group, nc, f32, st)
                                        : build_batch(bt, group, st);
            if (rc != FUGLBM_OK) return rc;
            flip = 0;
        }
        if (left >= 2 * GRAPH_STEPS && flip == 1) {
            hipError_t e =
                launch_fused(bt.kernel, nc, f32, bt.ditems, bt.nitems, bt.dsims, flip, st);
            if (e != hipSuccess) return hip_fail(e, "batched step launch");
            flip = 0;
            --left;
        }
        if (left >= GRAPH_STEPS && flip == 0) {
            // replay a captured run of GRAPH_STEPS launches (even: parity returns)
            fuglbm_status rc = batch_graph(bt, nc, f32);
            if (rc != FUGLBM_OK) return rc;
            while (left >= GRAPH_STEPS) {
                HIP_TRY(hipGraphLaunch(bt.graph, st));
                left -= GRAPH_STEPS;
            }
        }
        for (; left > 0; --left) {
            hipError_t e =
                launch_fused(bt.kernel, nc, f32, bt.ditems, bt.nitems, bt.dsims, flip, st);
            if (e != hipSuccess) return hip_fail(e, "batched step launch");
            flip ^= 1;
        }
        for (auto *s : group) {
            s->parity ^= (int)(nsteps & 1);
            s->step += nsteps;
            s->last_stream = st;
        }
    }
    // multi-pass members: one table per (lattice, precision, tau != 1)
    std::map<std::tuple<int, int, int>, std::vector<fuglbm_sim *>> ggroups;
    for (auto *s : others)
        ggroups[{s->lattice, s->fp32 ? 1 : 0, s->hc.omega != 1.0 ? 1 : 0}].push_back(s);
    for (auto &kv : ggroups) {
        auto &group = kv.second;
        GenBatch &gb = gen_batches()[kv.first];
        // the table is shared state: launches queued on another stream must
        // finish before this call rebuilds or reuses it
        if (gb.used && gb.last_stream != st) HIP_TRY(hipStreamSynchronize(gb.last_stream));
        gb.last_stream = st;
        gb.used = true;
        bool same = gb.sims.size() == group.size();
        for (size_t k = 0; same && k < group.size(); ++k)
            same = gb.sims[k] == group[k] && gb.uids[k] == group[k]->uid;
        int flip = 0;
        if (same) {
            flip = group[0]->parity ^ gb.parity0[0];
            for (size_t k = 0; k < group.size(); ++k)
                if ((group[k]->parity ^ gb.parity0[k]) != flip) same = false;
        }
        if (!same) {
            // launches queued on st may still read the table that the
            // rebuild overwrites (the upload is not ordered after them)
            HIP_TRY(hipStreamSynchronize(st));
            fuglbm_status rc = build_gen_batch(gb, group);
            if (rc != FUGLBM_OK) return rc;
            flip = 0;
        }
        int64_t left = nsteps;
        if (left >= 2 * GRAPH_STEPS && flip == 1) {
            hipError_t e = gen_batch_step(gb, flip, st);
            if (e != hipSuccess) return hip_fail(e, "batched multi-pass step launch");
            flip = 0;
            --left;
        }
        if (left >= GRAPH_STEPS && flip == 0) {
            // replay a captured run of GRAPH_STEPS steps (even: parity returns)
            fuglbm_status rc = gen_batch_graph(gb);
            if (rc != FUGLBM_OK) return rc;
            while (left >= GRAPH_STEPS) {
                HIP_TRY(hipGraphLaunch(gb.graph, st));
                left -= GRAPH_STEPS;
            }
        }
        for (; left > 0; --left) {
            hipError_t e = gen_batch_step(gb, flip, st);
            if (e != hipSuccess) return hip_fail(e, "batched multi-pass step launch");
            flip ^= 1;
        }
        for (auto *s : group) {
            s->parity ^= (int)(nsteps & 1);
            s->step += nsteps;
            s->last_stream = st;
        }
    }
    for (int k = 0; k < count; ++k) {
        if (sims[k]->sticky) continue;
        fuglbm_status rc = mark_done(sims[k], st);
        if (rc != FUGLBM_OK) return rc;
    }
    if (skipped) return fail(FUGLBM_ENONFINITE, "some simulations have a sticky device error");
    return FUGLBM_OK;
}

// ---------------------------------------------------------------------------
// Batched stepping without allocation (fuglbm_step_many_noalloc).
//
// The batch's work tables (per-member pointers and geometry, then the work
// items in the same XCD-dealt order as fuglbm_step_many) live in `scratch`,
// a file-scope device array of fixed size that every call on a device
// shares.  They are written on the device by a table kernel whose member
// data arrive as kernel arguments, so a call needs no device allocation,
// no graph instantiation and no copy from host memory; the steps are plain
// launches of the fused kernel.  `scratch` is a host-side stand-in in host
// code: its device address is looked up once per device
// (hipGetSymbolAddress) and only that address is ever passed on.
// ---------------------------------------------------------------------------
namespace {

constexpr int NA_MAX_MEMBERS = 256;                // simulations per call
constexpr int NA_MAX_ITEMS = 65536;                // fused work items per call
constexpr int NA_CHUNK = 32;                       // members per table-kernel launch
constexpr size_t NA_GEOM_OFF = 0;                  // int4 {nx, ny, rows, first item}
constexpr size_t NA_SIMS_OFF = NA_GEOM_OFF + 16 * NA_MAX_MEMBERS;
constexpr size_t NA_ITEMS_OFF = NA_SIMS_OFF + sizeof(FusedSim) * NA_MAX_MEMBERS;
constexpr size_t NA_SCRATCH_BYTES = NA_ITEMS_OFF + sizeof(FusedItem) * NA_MAX_ITEMS;

static __device__ __align__(256) unsigned char scratch[NA_SCRATCH_BYTES];

struct NaMember {
    const SimConst *c;
    void *buf0, *buf1;
    uint32_t *status;
    int32_t parity, nx, ny, rows;
};

struct NaChunk {
    int32_t base;                 // index of m[0] among the group's members
    int32_t count;                // members in this chunk
    int32_t first[NA_CHUNK];      // each member's first logical item in the group
    NaMember m[NA_CHUNK];
};

// Members [base, base + count) of one group: pointers and geometry.
__global__ void k_na_members(NaChunk a, FusedSim *sims, int4 *geom) {
    const int t = threadIdx.x;
    if (t >= a.count) return;
    const NaMember &m = a.m[t];
    FusedSim fs;
    fs.c = m.c;
    fs.buf[0] = m.buf0;
    fs.buf[1] = m.buf1;
    fs.status = m.status;
    fs.parity = m.parity;
    fs.pad = 0;
    sims[a.base + t] = fs;
    geom[a.base + t] = make_int4(m.nx, m.ny, m.rows, a.first[t]);
}

// Work items of one group: logical item li (member-major, then chunk of
// rows, then strip) goes to slot (li % per) * 8 + li / per, so XCD k
// (workgroups are dealt round-robin) runs the k-th contiguous slice.
__global__ void k_na_items(const int4 *geom, int nmem, int nlogical, int per, FusedItem *items) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= per * 8) return;
    const int li = (b % 8) * per + b / 8;
    FusedItem it{-1, 0, 0, 0};
    if (li < nlogical) {
        int k = 0;
        while (k + 1 < nmem && geom[k + 1].w <= li) ++k;
        const int4 g = geom[k];
        const int strips = (g.x + FUSED_OUT - 1) / FUSED_OUT;
        const int local = li - g.w;
        const int c = local / strips, t = local % strips;
        it.sim = k;
        it.x0 = t * FUSED_OUT;
        it.y0 = c * g.z;
        it.rows = min(g.z, g.y - c * g.z);
    }
    items[b] = it;
}

std::mutex na_mutex;
void *na_ptr[64];

// Device address of `scratch` on the current device (looked up once).
fuglbm_status na_scratch(char **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(FUGLBM_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(na_mutex);
    if (!na_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        na_ptr[dev] = p;
    }
    *out = (char *)na_ptr[dev];
    return FUGLBM_OK;
}

}  // namespace

extern "C" fuglbm_status fuglbm_step_many_noalloc(fuglbm_sim *const *sims, int32_t count,
                                                  int64_t nsteps, void *hip_stream) {
    const TraceRange trace_range("fuglbm_step_many_noalloc");
    if (count < 0 || (count > 0 && !sims)) return fail(FUGLBM_EINVAL, "bad sims array");
    if (nsteps < 0) return fail(FUGLBM_EINVAL, "nsteps must be >= 0");
    if (count > NA_MAX_MEMBERS)
        return fail(FUGLBM_EINVAL, "at most 256 simulations per call");
    hipStream_t st = (hipStream_t)hip_stream;
    // members by (ncomp, precision) class, in call order; sticky ones skipped
    int cls[NA_MAX_MEMBERS];
    int key[NA_MAX_MEMBERS], nkeys = 0;
    bool skipped = false;
    int64_t total_items = 0;
    for (int k = 0; k < count; ++k) {
        fuglbm_sim *s = sims[k];
        if (!s) return fail(FUGLBM_EINVAL, "null sim in batch");
        for (int q = 0; q < k; ++q)
            if (sims[q] == s) return fail(FUGLBM_EINVAL, "duplicate sim in batch");
        if (s->lattice != FUGLBM_D2Q9 || !is_fused(s->kernel))
            return fail(FUGLBM_EINVAL, "only D2Q9 simulations on a fused kernel");
        if (s->rows < 1) return fail(FUGLBM_EINVAL, "simulation without fused rows");
        cls[k] = -1;
        if (s->sticky) {
            skipped = true;
            continue;
        }
        const int kk = s->N * 2 + (s->fp32 ? 1 : 0);
        int g = 0;
        while (g < nkeys && key[g] != kk) ++g;
        if (g == nkeys) key[nkeys++] = kk;
        cls[k] = g;
        const int64_t strips = (s->nx + FUSED_OUT - 1) / FUSED_OUT;
        total_items += strips * ((s->ny + s->rows - 1) / s->rows) + 7;   // + XCD padding
    }
    if (total_items > NA_MAX_ITEMS)
        return fail(FUGLBM_EINVAL, "batch needs more than 65536 work items");
    if (nkeys == 0 || nsteps == 0) {
        if (skipped) return fail(FUGLBM_ENONFINITE, "some simulations have a sticky device error");
        return FUGLBM_OK;
    }
    char *base = nullptr;
    fuglbm_status rc = na_scratch(&base);
    if (rc != FUGLBM_OK) return rc;
    int4 *geom = (int4 *)(base + NA_GEOM_OFF);
    FusedSim *dsims = (FusedSim *)(base + NA_SIMS_OFF);
    FusedItem *ditems = (FusedItem *)(base + NA_ITEMS_OFF);
    int mem_off = 0, item_off = 0;
    for (int g = 0; g < nkeys; ++g) {
        // this group's members, their first logical items
        NaChunk ch;
        int nmem = 0, nlogical = 0;
        fuglbm_sim *first = nullptr;
        ch.base = 0;
        ch.count = 0;
        for (int k = 0; k < count; ++k) {
            if (cls[k] != g) continue;
            fuglbm_sim *s = sims[k];
            if (!first) first = s;
            NaMember &m = ch.m[ch.count];
            m.c = s->dc;
            m.buf0 = s->buf[0];
            m.buf1 = s->buf[1];
            m.status = s->status;
            m.parity = s->parity;
            m.nx = s->nx;
            m.ny = s->ny;
            m.rows = s->rows;
            ch.first[ch.count] = nlogical;
            nlogical += ((s->nx + FUSED_OUT - 1) / FUSED_OUT) * ((s->ny + s->rows - 1) / s->rows);
            ++ch.count;
            ++nmem;
            if (ch.count == NA_CHUNK) {
                hipLaunchKernelGGL(k_na_members, dim3(1), dim3(NA_CHUNK), 0, st, ch,
                                   dsims + mem_off, geom + mem_off);
                ch.base += NA_CHUNK;
                ch.count = 0;
            }
        }
        if (ch.count > 0)
            hipLaunchKernelGGL(k_na_members, dim3(1), dim3(NA_CHUNK), 0, st, ch, dsims + mem_off,
                               geom + mem_off);
        const int per = (nlogical + 7) / 8;
        const int nitems = per * 8;
        hipLaunchKernelGGL(k_na_items, dim3((nitems + 255) / 256), dim3(256), 0, st,
                           geom + mem_off, nmem, nlogical, per, ditems + item_off);
        HIP_TRY(hipGetLastError());
        const int ncomp = first->N;
        const bool f32 = first->fp32;
        const int kern = first->kernel == 3 && ws_usable(ncomp, f32) ? 3 : 2;
        for (int64_t t = 0; t < nsteps; ++t) {
            hipError_t e = launch_fused(kern, ncomp, f32, ditems + item_off, nitems,
                                        dsims + mem_off, (int)(t & 1), st);
            if (e != hipSuccess) return hip_fail(e, "batched step launch");
        }
        mem_off += nmem;
        item_off += nitems;
    }
    for (int k = 0; k < count; ++k) {
        if (cls[k] < 0) continue;
        fuglbm_sim *s = sims[k];
        s->parity ^= (int)(nsteps & 1);
        s->step += nsteps;
        s->last_stream = st;
        s->done_valid = false;   // not recorded here (the caller orders streams)
    }
    if (skipped) return fail(FUGLBM_ENONFINITE, "some simulations have a sticky device error");
    return FUGLBM_OK;
}
