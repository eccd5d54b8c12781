// Batched solves of many independent instances.
//
// All instances advance together, one batch stage per step: stage tau runs one
// expectation launch over the contraction tiles of every instance and one sweep launch
// per tile class over the (instance, price state, SoC tile) blocks of that class.
// Instance i is at its own stage T_i - tau + 1: every instance starts at tau = 1 with
// its last stage, and shorter horizons finish earlier (inactive once T_i - tau + 1 < 1).
// The whole sequence (an init launch and the per-stage
// launches) is captured once into a HIP graph and replayed; new input/output pointers
// are written into the device descriptor table before each replay, so the graph never
// needs re-capture.
//
// Tile classes: instances are grouped by the move span (w_up + w_down + 1); each group
// gets a sweep tile shape, either the built-in choice or the fastest of the candidate
// shapes timed on the group's own work list (autotuning), remembered in a text cache.
// The shape never changes results (every shape is bitwise equal), only speed.
#include "dp_host.h"

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

using namespace dpgpu;

namespace {

// (tile outputs, waves per block).  A scan pass covers 512 next states per wave, and a
// tile of TS outputs with w moves per side scans TS + w - 1 of them: tiles of 448 (960)
// keep windows up to 64 in one (two) passes.
const dpk::SweepShape kCandidates[] = {
    {512, 8}, {960, 8}, {448, 8}, {512, 4}, {448, 4}, {256, 4}, {448, 2},
    {256, 2}, {192, 2}, {448, 1}, {256, 1}, {192, 1}, {128, 1}, {64, 1},
};

// Instances fall into independent groups, one branch of the graph each.  Panel class c
// (K <= 32, <= 64, <= 128) is dealt round-robin into SPLIT[c] groups, so that one group's
// sweeps can run beside another's expectation; the last group holds the strips (K > 128).
// Splitting the costliest class in two gives four panel branches, one per hardware queue
// of a process; more branches than queues measured slower.
constexpr int SPLIT[3] = {1, 1, 2};
constexpr int STRIP_GROUP = SPLIT[0] + SPLIT[1] + SPLIT[2];
constexpr int NGROUPS = STRIP_GROUP + 1;

struct TileClass {
    dpk::SweepShape sh;
    int span_lo, span_hi;
    std::vector<int> inst;
    std::vector<dpk::SweepItem> items;      // ordered by group, then heavier instances first
    int goff[NGROUPS] = {}, gn[NGROUPS] = {};
    dpk::SweepItem *d_items = nullptr;
    size_t lds = 0;
    double tuned_us = -1.0;
};

int span_bucket(int span)
{
    int b = 0;
    while ((32 << b) < span && b < 10) ++b;
    return b;   // spans (16 << b, 32 << b]; bucket 0 also takes every span <= 16
}

bool shape_fits(const dpk::SweepShape &sh, int w_up, int w_down)
{
    const size_t tile = (dpk::sweep_lds_bytes(sh, w_up, w_down) + 15) & ~(size_t)15;
    return tile * dpk::batched_tiles_per_block(sh) <= 160 * 1024;
}

std::string shape_str(const dpk::SweepShape &sh)
{
    char b[64];
    snprintf(b, sizeof b, "%d %d", sh.TS, sh.NW);
    return b;
}

}  // namespace

struct dp_batch_plan {
    int n = 0;
    int Tmax = 0;
    std::vector<dp_problem> probs;
    std::vector<int> group;                // branch of each instance
    std::vector<dpk::BatchDesc> hdesc;
    std::vector<size_t> region;            // per-instance workspace offsets
    dpk::BatchDesc *ddesc = nullptr;
    dpk::BatchDesc *hstage = nullptr;      // pinned staging for descriptor updates
    std::vector<TileClass> classes;
    dpk::ContractItem *d_citems = nullptr;     // strip items (instances with K > 128)
    int n_citems = 0;
    dpk::ContractItem *d_pitems = nullptr;     // panel items (instances with K <= 128),
    int n_pitems = 0;                          // contiguous per group
    int pan_off[NGROUPS] = {}, pan_n[NGROUPS] = {}, pan_kmax[NGROUPS] = {};
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t cap = nullptr;
    hipStream_t branch[NGROUPS] = {};      // capture streams of the graph's group branches
    hipEvent_t fork = nullptr, join[NGROUPS] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
    std::string text;
};

static void destroy_plan(dp_batch_plan *p)
{
    if (!p) return;
    if (p->staged_pending) (void)hipEventSynchronize(p->staged);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (auto &c : p->classes)
        if (c.d_items) (void)hipFree(c.d_items);
    if (p->d_citems) (void)hipFree(p->d_citems);
    if (p->d_pitems) (void)hipFree(p->d_pitems);
    if (p->ddesc) (void)hipFree(p->ddesc);
    if (p->hstage) (void)hipHostFree(p->hstage);
    if (p->ws) (void)hipFree(p->ws);
    if (p->staged) (void)hipEventDestroy(p->staged);
    if (p->fork) (void)hipEventDestroy(p->fork);
    for (int g = 0; g < NGROUPS; ++g) {
        if (p->join[g]) (void)hipEventDestroy(p->join[g]);
        if (p->branch[g]) (void)hipStreamDestroy(p->branch[g]);
    }
    if (p->cap) (void)hipStreamDestroy(p->cap);
    delete p;
}

// The stages of one instance group on stream s: per batch stage its expectation launch,
// then its share of every sweep class.
static int enqueue_group(dp_batch_plan *p, int g, hipStream_t s)
{
    hipError_t e = hipSuccess;
    for (int tau = 1; tau <= p->Tmax; ++tau) {
        if (g != STRIP_GROUP && p->pan_n[g]) {
            e = dpk::launch_batched_panel(p->ddesc, p->d_pitems + p->pan_off[g], p->pan_n[g], tau,
                                          p->pan_kmax[g], s);
            if (e != hipSuccess) return hip_fail(e, "batched expectation (panels)");
        }
        if (g == STRIP_GROUP && p->n_citems) {
            e = dpk::launch_batched_contract(p->ddesc, p->d_citems, p->n_citems, tau, s);
            if (e != hipSuccess) return hip_fail(e, "batched expectation (strips)");
        }
        for (auto &c : p->classes) {
            if (!c.gn[g]) continue;
            e = dpk::launch_batched_sweep(p->ddesc, c.d_items + c.goff[g], c.gn[g], tau, c.sh,
                                          c.lds, s);
            if (e != hipSuccess) return hip_fail(e, "batched sweep");
        }
    }
    return DP_OK;
}

static bool group_used(const dp_batch_plan *p, int g)
{
    if (g != STRIP_GROUP ? p->pan_n[g] > 0 : p->n_citems > 0) return true;
    for (auto &c : p->classes)
        if (c.gn[g]) return true;
    return false;
}

// Launch one whole batched solve on `s` (the capture stream): the init kernel, then one
// branch per instance group on its own stream (groups share no data, so the branches run
// concurrently and fill each other's launch tails), joined back into `s`.
static int enqueue_all(dp_batch_plan *p, hipStream_t s)
{
    hipError_t e = dpk::launch_batched_init(p->ddesc, p->n, s);
    if (e != hipSuccess) return hip_fail(e, "batched init");
    e = hipEventRecord(p->fork, s);
    if (e != hipSuccess) return hip_fail(e, "fork");
    bool first = true;
    for (int g = 0; g < NGROUPS; ++g) {
        if (!group_used(p, g)) continue;
        hipStream_t sg = first ? s : p->branch[g];
        if (!first && (e = hipStreamWaitEvent(sg, p->fork, 0)) != hipSuccess) return hip_fail(e, "fork");
        int rc = enqueue_group(p, g, sg);
        if (rc != DP_OK) return rc;
        if (!first) {
            if ((e = hipEventRecord(p->join[g], sg)) != hipSuccess) return hip_fail(e, "join");
            if ((e = hipStreamWaitEvent(s, p->join[g], 0)) != hipSuccess) return hip_fail(e, "join");
        }
        first = false;
    }
    return DP_OK;
}

// Built-in sweep shape of a span class when no tuning is asked for: short windows take
// small blocks (many instances' rows in flight per CU), long ones the single solve's tile.
static dpk::SweepShape batch_default_shape(const dp_problem *pb, int span_hi)
{
    dpk::SweepShape sh = span_hi <= 128   ? dpk::SweepShape{448, 1}
                         : span_hi <= 256 ? dpk::SweepShape{448, 2}
                         : span_hi <= 512 ? dpk::SweepShape{512, 4}
                                          : pick_shape(pb);
    return sh;
}

static int build_items(dp_batch_plan *p, TileClass &c, hipStream_t s)
{
    c.items.clear();
    c.lds = 0;
    const int TS = dpk::sweep_tile(c.sh);
    // by instance group (a contiguous range per group), then heavier instances (wider
    // spans, more outputs) first, for a short tail
    std::vector<int> order = c.inst;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        const int ga = p->group[a], gb = p->group[b];
        if (ga != gb) return ga < gb;
        const auto &x = p->probs[a].st, &y = p->probs[b].st;
        return (long)(x.w_up + x.w_down) * p->probs[a].K > (long)(y.w_up + y.w_down) * p->probs[b].K;
    });
    for (int g = 0; g < NGROUPS; ++g) c.gn[g] = 0;
    for (int i : order) {
        const dp_problem &pb = p->probs[i];
        const int g = p->group[i];
        if (c.gn[g] == 0) c.goff[g] = (int)c.items.size();
        const int tiles = (pb.st.S + TS - 1) / TS;
        for (int k = 0; k < pb.K; ++k)
            for (int tl = 0; tl < tiles; ++tl) c.items.push_back({i, k, tl});
        c.gn[g] = (int)c.items.size() - c.goff[g];
        c.lds = std::max(c.lds, dpk::sweep_lds_bytes(c.sh, pb.st.w_up, pb.st.w_down));
    }
    if (c.d_items) {
        (void)hipFree(c.d_items);
        c.d_items = nullptr;
    }
    if (c.items.empty()) return DP_OK;
    hipError_t e = hipMalloc(&c.d_items, sizeof(dpk::SweepItem) * c.items.size());
    if (e == hipSuccess)
        e = hipMemcpyAsync(c.d_items, c.items.data(), sizeof(dpk::SweepItem) * c.items.size(),
                           hipMemcpyHostToDevice, s);
    // the host table is reused or freed after this call returns
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "batch item table");
    return DP_OK;
}

// Time the class's sweep over a few stages with each candidate shape on the plan's own
// workspace (values are irrelevant to the cost), on stream s; keep the fastest.
static int autotune_class(dp_batch_plan *p, TileClass &c, const float *zeros_lam, hipStream_t s)
{
    double best_us = 1e30;
    dpk::SweepShape best = c.sh;
    // every descriptor: the plan's workspace, zero prices (a [Tmax][Kmax] zero block), no
    // inputs or outputs of the caller
    for (int i = 0; i < p->n; ++i) {
        p->hstage[i] = p->hdesc[i];
        p->hstage[i].lam = zeros_lam;
        p->hstage[i].P = nullptr;
        p->hstage[i].pol = nullptr;
        p->hstage[i].V1 = nullptr;
    }
    hipError_t e = hipMemcpyAsync(p->ddesc, p->hstage, sizeof(dpk::BatchDesc) * p->n,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "tune descriptors");
    e = dpk::launch_batched_init(p->ddesc, p->n, s);
    if (e != hipSuccess) return hip_fail(e, "tune init");
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "tune event");
    if ((e = hipEventCreate(&e1)) != hipSuccess) return hip_fail(e, "tune event");
    int rc = DP_OK;
    for (const auto &cand : kCandidates) {
        bool fits = true;
        for (int i : c.inst) fits &= shape_fits(cand, p->probs[i].st.w_up, p->probs[i].st.w_down);
        if (!fits) continue;
        TileClass trial;
        trial.sh = cand;
        trial.inst = c.inst;
        if ((rc = build_items(p, trial, s)) != DP_OK) break;
        // tau = 1 keeps every instance active (stage T_i); the W buffer holds zeros
        double t_min = 1e30;
        // the minimum over 5 timed repeats of 6 stages (after one warm-up): single launches
        // of the smaller classes last tens of microseconds, where one repeat is noisy
        for (int rep = 0; rep < 6 && rc == DP_OK; ++rep) {
            e = hipEventRecord(e0, s);
            for (int st = 0; st < 6 && e == hipSuccess; ++st)
                e = dpk::launch_batched_sweep(p->ddesc, trial.d_items, (int)trial.items.size(), 1,
                                              trial.sh, trial.lds, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) rc = hip_fail(e, "tune timing");
            if (rep > 0) t_min = std::min(t_min, ms * 1e3 / 6.0);
        }
        if (trial.d_items) {
            (void)hipStreamSynchronize(s);    // the timed launches read the table
            (void)hipFree(trial.d_items);
        }
        if (rc != DP_OK) break;
        if (t_min < best_us) {
            best_us = t_min;
            best = cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != DP_OK) return rc;
    c.sh = best;
    c.tuned_us = best_us;
    return DP_OK;
}

static std::map<int, dpk::SweepShape> read_cache(const char *path)
{
    std::map<int, dpk::SweepShape> m;
    if (!path) return m;
    FILE *f = fopen(path, "r");
    if (!f) return m;
    char line[256];
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        // "bucket tile waves  # comment"; lines of any other form are skipped
        int b, ts, nw, extra;
        if (sscanf(line, "%d %d %d %d", &b, &ts, &nw, &extra) == 3) {
            dpk::SweepShape sh = {ts, nw};
            if (dpk::sweep_shape_supported(sh)) m[b] = sh;
        }
    }
    fclose(f);
    return m;
}

static void append_cache(const char *path, int bucket, const dpk::SweepShape &sh, double us)
{
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%d %s  # span (%d, %d], %.2f us per stage sweep of the tuning batch\n", bucket,
            shape_str(sh).c_str(), 16 << bucket, 32 << bucket, us);
    fclose(f);
}

extern "C" {

int dp_batch_plan_create(dp_batch_plan **out, int n, const dp_problem *probs,
                         const char *tune_cache, void *stream_)
{
    if (!out) return fail(DP_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !probs) return fail(DP_EINVAL, "need n >= 1 problems");
    hipStream_t s = static_cast<hipStream_t>(stream_);
    dp_batch_plan *p = new (std::nothrow) dp_batch_plan;
    if (!p) return fail(DP_ENOMEM, "plan allocation");
    p->n = n;
    p->probs.assign(probs, probs + n);
    p->group.resize(n);
    int dealt[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
        const int K = probs[i].K;
        if (K > 128) {
            p->group[i] = STRIP_GROUP;
            continue;
        }
        const int c = dpk::panel_class(K);
        int g0 = 0;
        for (int q = 0; q < c; ++q) g0 += SPLIT[q];
        p->group[i] = g0 + (dealt[c]++) % SPLIT[c];
    }
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        int rc = validate_problem(&p->probs[i]);
        if (rc != DP_OK) {
            destroy_plan(p);
            return fail(rc, "problem %d: %s", i, dp_last_error());
        }
        if (p->probs[i].flags != 0 || p->probs[i].ckpt_every != 0) {
            destroy_plan(p);
            return fail(DP_EINVAL, "problem %d: batched solves take no flags or checkpoints", i);
        }
        // the single solve's state plus the expectation plane W (the batch forms W_t in
        // its own launches)
        p->region.push_back(total);
        const SolveLayout Li = solve_layout(&p->probs[i]);
        total += Li.total + ((sizeof(float) * (size_t)p->probs[i].K * Li.Spad + 255) & ~(size_t)255);
        p->Tmax = std::max(p->Tmax, p->probs[i].T);
    }
    int Kmax = 1;
    for (auto &pb : p->probs) Kmax = std::max(Kmax, pb.K);
    const size_t zoff = total;
    total += 256 + sizeof(float) * (size_t)Kmax * (size_t)p->Tmax;   // zero prices for tuning
    hipError_t e = hipMalloc(&p->ws, total);
    if (e == hipSuccess) e = hipMemsetAsync(p->ws, 0, total, s);
    if (e == hipSuccess) e = hipMalloc(&p->ddesc, sizeof(dpk::BatchDesc) * n);
    if (e == hipSuccess) e = hipHostMalloc(&p->hstage, sizeof(dpk::BatchDesc) * n);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->staged, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
    for (int g = 0; g < NGROUPS && e == hipSuccess; ++g) {
        e = hipStreamCreateWithFlags(&p->branch[g], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join[g], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        destroy_plan(p);
        return hip_fail(e, "plan allocation");
    }
    p->ws_bytes = total;
    const float *zeros_lam = reinterpret_cast<const float *>(p->ws + zoff);
    p->hdesc.resize(n);
    std::vector<dpk::ContractItem> citems, pgroup[NGROUPS];
    for (int i = 0; i < n; ++i) {
        const dp_problem &pb = p->probs[i];
        const SolveLayout L = solve_layout(&pb);
        char *base = p->ws + p->region[i];
        dpk::BatchDesc &d = p->hdesc[i];
        d.T = pb.T;
        d.K = pb.K;
        d.S = pb.st.S;
        d.w_up = pb.st.w_up;
        d.w_down = pb.st.w_down;
        d.ld = L.Spad;
        d.pay = {pb.st.delta, pb.st.eta_c, pb.st.eta_d, pb.st.c_deg, pb.st.c_start};
        d.lam = nullptr;
        d.P = nullptr;
        d.V1 = nullptr;
        d.pol = nullptr;
        d.vbuf0 = reinterpret_cast<float *>(base + L.vA);
        d.vbuf1 = reinterpret_cast<float *>(base + L.vB);
        d.W = reinterpret_cast<float *>(base + L.total);
        d.off = reinterpret_cast<double *>(base + L.off);
        // K <= 128: one item = up to four 64-column panels over every row tile (P_t in
        // LDS); otherwise one item = a strip of four adjacent 16 x 16 tiles of one row tile
        const int ntm = (pb.K + 15) / 16, ntn = (pb.st.S + 15) / 16;
        if (pb.K <= 128) {
            // items of up to four panels (P_t staged once per item); two for K > 64, whose
            // items are long enough that finer ones balance the CUs better
            const int c = dpk::panel_class(pb.K), g = p->group[i];
            const int ppi = c == 2 ? 2 : 4;
            for (int tn = 0; tn < ntn; tn += 4 * ppi)
                pgroup[g].push_back({i, std::min(ppi, (ntn - tn + 3) / 4), tn});
            p->pan_kmax[g] = std::max(p->pan_kmax[g], pb.K);
        } else {
            for (int tn = 0; tn < ntn; tn += 4)
                for (int tm = 0; tm < ntm; ++tm) citems.push_back({i, tm, tn});
        }
    }
    p->n_citems = (int)citems.size();
    std::vector<dpk::ContractItem> pitems;
    for (int g = 0; g < NGROUPS; ++g) {
        p->pan_off[g] = (int)pitems.size();
        p->pan_n[g] = (int)pgroup[g].size();
        pitems.insert(pitems.end(), pgroup[g].begin(), pgroup[g].end());
    }
    p->n_pitems = (int)pitems.size();
    e = hipSuccess;
    if (!citems.empty()) {
        e = hipMalloc(&p->d_citems, sizeof(dpk::ContractItem) * citems.size());
        if (e == hipSuccess)
            e = hipMemcpyAsync(p->d_citems, citems.data(), sizeof(dpk::ContractItem) * citems.size(),
                               hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess && !pitems.empty()) {
        e = hipMalloc(&p->d_pitems, sizeof(dpk::ContractItem) * pitems.size());
        if (e == hipSuccess)
            e = hipMemcpyAsync(p->d_pitems, pitems.data(), sizeof(dpk::ContractItem) * pitems.size(),
                               hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);     // host tables are freed on return
    if (e != hipSuccess) {
        destroy_plan(p);
        return hip_fail(e, "expectation item table");
    }

    // Tile classes by span bucket.
    std::map<int, std::vector<int>> buckets;
    for (int i = 0; i < n; ++i)
        buckets[span_bucket(p->probs[i].st.w_up + p->probs[i].st.w_down + 1)].push_back(i);
    std::map<int, dpk::SweepShape> cached = read_cache(tune_cache);
    int rc = DP_OK;
    for (auto &kv : buckets) {
        TileClass c;
        c.inst = kv.second;
        c.span_lo = kv.first == 0 ? 1 : (16 << kv.first) + 1;
        c.span_hi = 32 << kv.first;
        c.sh = batch_default_shape(&p->probs[c.inst[0]], c.span_hi);
        auto it = cached.find(kv.first);
        bool fits_all = true;
        if (it != cached.end()) {
            for (int i : c.inst) fits_all &= shape_fits(it->second, p->probs[i].st.w_up, p->probs[i].st.w_down);
            if (fits_all) c.sh = it->second;
        }
        if (tune_cache && (it == cached.end() || !fits_all)) {
            rc = autotune_class(p, c, zeros_lam, s);
            if (rc != DP_OK) break;
            append_cache(tune_cache, kv.first, c.sh, c.tuned_us);
        }
        for (int i : c.inst)
            if (!shape_fits(c.sh, p->probs[i].st.w_up, p->probs[i].st.w_down)) {
                rc = fail(DP_ENOTSUP, "problem %d: move window needs more LDS than a CU holds", i);
                break;
            }
        if (rc != DP_OK) break;
        p->classes.push_back(c);
    }
    if (rc == DP_OK) {
        // merge classes that ended with the same shape (fewer launches per stage)
        std::vector<TileClass> merged;
        for (auto &c : p->classes) {
            bool done = false;
            for (auto &m : merged)
                if (memcmp(&m.sh, &c.sh, sizeof c.sh) == 0) {
                    m.inst.insert(m.inst.end(), c.inst.begin(), c.inst.end());
                    m.span_lo = std::min(m.span_lo, c.span_lo);
                    m.span_hi = std::max(m.span_hi, c.span_hi);
                    done = true;
                    break;
                }
            if (!done) merged.push_back(c);
        }
        p->classes = merged;
        for (auto &c : p->classes) {
            c.d_items = nullptr;
            if ((rc = build_items(p, c, s)) != DP_OK) break;
        }
    }
    if (rc == DP_OK) {
        // capture the whole solve into a graph on the plan's stream
        e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) rc = hip_fail(e, "begin capture");
        if (rc == DP_OK) {
            rc = enqueue_all(p, p->cap);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(p->cap, &g);
            if (rc == DP_OK && e != hipSuccess) rc = hip_fail(e, "end capture");
            p->graph = g;
        }
        if (rc == DP_OK) {
            e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) rc = hip_fail(e, "graph instantiate");
        }
    }
    if (rc != DP_OK) {
        destroy_plan(p);
        return rc;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) {
        destroy_plan(p);
        return hip_fail(e, "plan set-up");
    }
    // description
    char buf[512];
    snprintf(buf, sizeof buf, "dp_batch_plan: %d instances, %d batch stages, %d expectation panels + %d strips, %zu bytes workspace\n",
             n, p->Tmax, p->n_pitems, p->n_citems, p->ws_bytes);
    p->text = buf;
    for (auto &c : p->classes) {
        snprintf(buf, sizeof buf, "  class span %d..%d: tile %d on %d waves, %zu instances, %zu blocks/stage, %zu B LDS%s\n",
                 c.span_lo, c.span_hi, c.sh.TS, c.sh.NW, c.inst.size(),
                 c.items.size(), c.lds, c.tuned_us >= 0 ? " (autotuned)" : "");
        p->text += buf;
    }
    *out = p;
    return DP_OK;
}

static int check_ptrs(dp_batch_plan *p, const float *const *lam, const float *const *P,
                      float *const *V1, int16_t *const *policy)
{
    if (!p) return fail(DP_EINVAL, "plan is NULL");
    if (!lam || !P || !V1) return fail(DP_EINVAL, "lam, P and V1 arrays must be non-NULL");
    for (int i = 0; i < p->n; ++i) {
        if (!lam[i] || !P[i] || !V1[i]) return fail(DP_EINVAL, "instance %d: NULL pointer", i);
        if (policy && !policy[i]) return fail(DP_EINVAL, "instance %d: NULL policy pointer", i);
    }
    return DP_OK;
}

// Copy the call's pointers into the device descriptor table (pinned staging, async on s).
static int upload_descriptors(dp_batch_plan *p, const float *const *lam, const float *const *P,
                              float *const *V1, int16_t *const *policy, hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (p->staged_pending) e = hipEventSynchronize(p->staged);   // staging buffer free again
    if (e != hipSuccess) return hip_fail(e, "staging wait");
    for (int i = 0; i < p->n; ++i) {
        p->hstage[i] = p->hdesc[i];
        p->hstage[i].lam = lam[i];
        p->hstage[i].P = P[i];
        p->hstage[i].V1 = V1[i];
        p->hstage[i].pol = policy ? policy[i] : nullptr;
    }
    e = hipMemcpyAsync(p->ddesc, p->hstage, sizeof(dpk::BatchDesc) * p->n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(p->staged, s);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    p->staged_pending = true;
    return DP_OK;
}

int dp_batch_solve(dp_batch_plan *p, const float *const *lam, const float *const *P,
                   float *const *V1, int16_t *const *policy, void *stream_)
{
    int rc = check_ptrs(p, lam, P, V1, policy);
    if (rc != DP_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream_);
    rc = upload_descriptors(p, lam, P, V1, policy, s);
    if (rc != DP_OK) return rc;
    hipError_t e = hipGraphLaunch(p->exec, s);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return DP_OK;
}

int dp_batch_solve_eager(dp_batch_plan *p, const float *const *lam, const float *const *P,
                         float *const *V1, int16_t *const *policy, void *stream_)
{
    int rc = check_ptrs(p, lam, P, V1, policy);
    if (rc != DP_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream_);
    rc = upload_descriptors(p, lam, P, V1, policy, s);
    if (rc != DP_OK) return rc;
    return enqueue_all(p, s);
}

int dp_batch_solve_looped(dp_batch_plan *p, const float *const *lam, const float *const *P,
                          float *const *V1, int16_t *const *policy, void *stream_)
{
    int rc = check_ptrs(p, lam, P, V1, policy);
    if (rc != DP_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream_);
    for (int i = 0; i < p->n; ++i) {
        StageOutputs o = {};
        o.v1 = V1[i];
        o.pol = policy ? policy[i] : nullptr;
        rc = run_stages(&p->probs[i], 1, p->probs[i].T, lam[i], P[i], nullptr, nullptr, o,
                        p->ws + p->region[i], s);
        if (rc != DP_OK) return rc;
    }
    return DP_OK;
}

int dp_batch_plan_describe(const dp_batch_plan *p, char *buf, size_t len)
{
    if (!p || !buf || len == 0) return fail(DP_EINVAL, "plan and buffer must be non-NULL");
    snprintf(buf, len, "%s", p->text.c_str());
    return DP_OK;
}

void dp_batch_plan_destroy(dp_batch_plan *p) { destroy_plan(p); }

}  // extern "C"
