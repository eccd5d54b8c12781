// Host side of libdpgpu: argument validation, workspace layout, the stage loop of the
// backward induction and the forward-in-time adjoint driver.  See include/dpgpu.h.
#include "dp_host.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

namespace {

thread_local std::string g_last_error;

}  // namespace

namespace dpgpu {

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(DP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace dpgpu

namespace {

using dpgpu::fail;
using dpgpu::hip_fail;

dpk::SweepShape g_shape_override = {0, 0};

// Optional per-kernel timing (dp_set_timing): HIP events recorded on the caller's stream
// around every sweep and expectation launch of dp_solve.
struct KernelTimer {
    bool on = false;
    unsigned flags = hipEventDefault;
    std::vector<hipEvent_t> ev;      // pairs (start, stop)
    std::vector<int> kind;           // 0 = sweep, 1 = expectation
    size_t used = 0;
} g_timer;

hipError_t timer_mark(hipStream_t s, int kind, bool start)
{
    if (!g_timer.on) return hipSuccess;
    if (start) {
        if (g_timer.used + 2 > g_timer.ev.size()) {
            for (int i = 0; i < 256; ++i) {
                hipEvent_t e;
                hipError_t r = hipEventCreateWithFlags(&e, g_timer.flags);
                if (r != hipSuccess) return r;
                g_timer.ev.push_back(e);
            }
        }
        g_timer.kind.push_back(kind);
    }
    return hipEventRecord(g_timer.ev[g_timer.used++], s);
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int pad64(int x) { return (x + 63) & ~63; }

}  // namespace

namespace dpgpu {

int validate_problem(const dp_problem *pb)
{
    if (!pb) return fail(DP_EINVAL, "problem pointer is NULL");
    const dp_storage &st = pb->st;
    if (pb->T < 1) return fail(DP_EINVAL, "T must be >= 1 (got %d)", pb->T);
    if (pb->K < 1 || pb->K > DP_MAX_K) return fail(DP_EINVAL, "K must be in [1, %d] (got %d)", DP_MAX_K, pb->K);
    if (st.S < 2 || st.S > DP_MAX_S) return fail(DP_EINVAL, "S must be in [2, %d] (got %d)", DP_MAX_S, st.S);
    if (st.w_up < 0 || st.w_down < 0) return fail(DP_EINVAL, "move windows must be >= 0");
    if (st.reserved != 0) return fail(DP_EINVAL, "dp_storage.reserved must be 0");
    if (!(st.delta > 0.0f) || !isfinite(st.delta)) return fail(DP_EINVAL, "delta must be finite and > 0");
    if (!(st.eta_c > 0.0f && st.eta_c <= 1.0f)) return fail(DP_EINVAL, "eta_c must be in (0, 1]");
    if (!(st.eta_d > 0.0f && st.eta_d <= 1.0f)) return fail(DP_EINVAL, "eta_d must be in (0, 1]");
    if (!(st.c_deg >= 0.0f) || !isfinite(st.c_deg)) return fail(DP_EINVAL, "c_deg must be finite and >= 0");
    if (!(st.c_start >= 0.0f) || !isfinite(st.c_start)) return fail(DP_EINVAL, "c_start must be finite and >= 0");
    if (pb->flags & ~(uint32_t)(DP_STORE_V_ALL | DP_VALIDATE)) return fail(DP_EINVAL, "unknown flag bits 0x%x", pb->flags);
    if (pb->ckpt_every < 0) return fail(DP_EINVAL, "ckpt_every must be >= 0");
    if (pick_shape(pb).TS == 0)
        return fail(DP_ENOTSUP, "move window %d..%d needs more LDS than a CU holds",
                    -st.w_down, st.w_up);
    return DP_OK;
}

static bool fits(const dpk::SweepShape &sh, const dp_problem *pb)
{
    return dpk::sweep_lds_bytes(sh, pb->st.w_up, pb->st.w_down, pb->K) <= 160 * 1024;
}

dpk::SweepShape pick_shape(const dp_problem *pb)
{
    const dpk::SweepShape none{0, 0};
    if (g_shape_override.TS) return fits(g_shape_override, pb) ? g_shape_override : none;
    // Tiles of 512 SoC indices on eight waves: one block per CU for the 50 x 2001 and
    // 100 x 1001 grids, whose blocks are bound by staging the expectation row (the halo of
    // a tile is its move window, so a wider tile re-reads less of it per output).  Windows
    // too wide for that LDS fall back to 64 outputs on one wave (the least LDS per span).
    dpk::SweepShape sh = dpk::SweepShape{512, 8};
    if (fits(sh, pb)) return sh;
    sh = dpk::SweepShape{64, 1};
    return fits(sh, pb) ? sh : none;
}

SolveLayout solve_layout(const dp_problem *pb, size_t cap)
{
    SolveLayout L = solve_layout(pb);
    // a smaller ring of row sums only launches their computation more often
    while (L.total > cap && L.npk > 1) {
        L.npk >>= 1;
        L.total = L.rho + align256(sizeof(double) * (size_t)L.npk * pb->K);
    }
    return L;
}

SolveLayout solve_layout(const dp_problem *pb)
{
    SolveLayout L;
    L.Spad = pad64(pb->st.S);
    const size_t plane = align256(sizeof(float) * (size_t)pb->K * L.Spad);
    size_t o = 0;
    L.vA = o; o += plane;
    L.vB = o; o += plane;
    L.off = o; o += align256(sizeof(double) * ((size_t)pb->T + 2));
    L.flag = o; o += 256;
    // rho_k - 1 of P_t for every stage, formed by one launch before the first stage (a launch
    // between two stages adds its duration and a launch gap to the chain); for very long
    // horizons the ring is halved until it takes at most 64 MiB
    L.npk = pb->T;
    while (L.npk > 32 && sizeof(double) * (size_t)L.npk * pb->K > ((size_t)64 << 20))
        L.npk = (L.npk + 1) / 2;
    L.rho = o; o += align256(sizeof(double) * (size_t)L.npk * pb->K);
    L.total = o;
    return L;
}

int n_ckpt_slots(const dp_problem *pb)
{
    const int E = pb->ckpt_every > 0 ? pb->ckpt_every : 16;
    // slots m = 1 .. M-1 hold stage 1 + m E (<= T)
    return (pb->T - 1) / E;
}

size_t ckpt_bytes(const dp_problem *pb)
{
    const int M = n_ckpt_slots(pb);
    return align256(sizeof(float) * (size_t)M * pb->K * pb->st.S) + align256(sizeof(double) * (size_t)(M > 0 ? M : 1));
}

// Backward induction over stages [t_lo, t_hi] (1-based) of the problem.  The terminal
// state (stage t_hi + 1) is v_src (absolute v_term or a normalised checkpoint) with
// offset *off_src (device pointer or NULL = 0).  Absolute values of stage t go to
// out.vall slice t - t_lo (or out.v1 for t = t_lo), policies to out.pol slice t - t_lo.
int run_stages(const dp_problem *pb, int t_lo, int t_hi, const float *lam, const float *P,
               const float *v_src, const double *off_src, const StageOutputs &out, void *ws,
               hipStream_t stream, size_t ws_cap, bool timing)
{
    const int K = pb->K, S = pb->st.S;
    const SolveLayout L = solve_layout(pb, ws_cap);
    auto timer_mark = [timing](hipStream_t st, int kind, bool start) {
        return timing ? ::timer_mark(st, kind, start) : hipSuccess;
    };
    char *base = static_cast<char *>(ws);
    float *vbuf[2] = {reinterpret_cast<float *>(base + L.vA), reinterpret_cast<float *>(base + L.vB)};
    double *off = reinterpret_cast<double *>(base + L.off);   // off[t] = C_t, t = t_lo..t_hi+1
    const size_t KS = (size_t)K * S;
    const int nst = t_hi - t_lo + 1;

    float *vabs_term = out.vall ? out.vall + (size_t)nst * KS : nullptr;
    hipError_t e = dpk::launch_init_terminal(v_src, off_src, K, S, vbuf[0], L.Spad,
                                             off + (t_hi + 1), vabs_term, stream);
    if (e != hipSuccess) return hip_fail(e, "init_terminal");

    const int E = out.ckpt_every > 0 ? out.ckpt_every : 16;
    const dpk::SweepShape sh = pick_shape(pb);
    if (sh.TS == 0)
        return fail(DP_ENOTSUP, "move window %d..%d needs more LDS than a CU holds",
                    -pb->st.w_down, pb->st.w_up);
    if (!dpk::sweep_shape_supported(sh)) return fail(DP_EINVAL, "unsupported sweep shape");
    // One launch per stage: each sweep block forms its own row of the expectation
    // W_t = P_t V_{t+1} from the normalised V_{t+1} (fused; bitwise the tile chain).
    dpk::SweepArgs a;
    a.W = nullptr;
    a.ldw = 0;
    a.ldvn = L.Spad;
    a.K = K;
    a.S = S;
    a.w_up = pb->st.w_up;
    a.w_down = pb->st.w_down;
    a.pay = {pb->st.delta, pb->st.eta_c, pb->st.eta_d, pb->st.c_deg, pb->st.c_start};
    a.ldv = L.Spad;
    int cur = 0;
    double *rho = reinterpret_cast<double *>(base + L.rho);   // rho_k - 1 of stages pk_lo..
    int pk_lo = t_hi + 1;          // the row sums held are of stages pk_lo .. pk_lo + npk - 1
    for (int t = t_hi; t >= t_lo; --t) {
        const float *vin = vbuf[cur];
        float *vout = vbuf[cur ^ 1];
        if (t < pk_lo) {           // row sums of the next chunk of stages (downwards from t)
            pk_lo = t - L.npk + 1 > t_lo ? t - L.npk + 1 : t_lo;
            e = dpk::launch_row_sums(P + (size_t)(pk_lo - 1) * K * K, K, t - pk_lo + 1, rho,
                                     stream);
            if (e != hipSuccess) return hip_fail(e, "row sums");
        }
        a.Vn = vin;
        a.Vn0 = vin;
        a.lam = lam + (size_t)(t - 1) * K;
        a.P = P + (size_t)(t - 1) * K * K;
        a.rho1 = rho + (size_t)(t - pk_lo) * K;
        a.off_next = off + (t + 1);
        a.off_cur = off + t;
        a.vnorm = vout;
        a.vabs = out.vall ? out.vall + (size_t)(t - t_lo) * KS : (t == t_lo ? out.v1 : nullptr);
        a.pol = out.pol ? out.pol + (size_t)(t - t_lo) * KS : nullptr;
        a.ckpt_v = nullptr;
        a.ckpt_off = nullptr;
        if (out.ckpt_v && t >= 2 && (t - 1) % E == 0) {
            const int m = (t - 1) / E;   // slot m holds stage 1 + m E
            a.ckpt_v = out.ckpt_v + (size_t)(m - 1) * KS;
            a.ckpt_off = out.ckpt_off + (m - 1);
        }
        if ((e = timer_mark(stream, 0, true)) != hipSuccess) return hip_fail(e, "timer");
        e = dpk::launch_sweep(a, sh, stream);
        if (e != hipSuccess) return hip_fail(e, "sweep");
        if ((e = timer_mark(stream, 0, false)) != hipSuccess) return hip_fail(e, "timer");
        cur ^= 1;
    }
    return DP_OK;
}

// DP_VALIDATE: rows of P (entries >= 0, |row sum - 1| <= 1e-6) and, if given, every
// policy entry a feasible next state.  Synchronises the stream (the flag is read back).
int validate_device_inputs(const dp_problem *pb, const float *P, const int16_t *policy,
                           int *flag, hipStream_t stream)
{
    int host[2] = {0, 0};
    hipError_t e = hipSuccess;
    for (int c = 0; c < 2 && e == hipSuccess; ++c) {
        if (c == 1 && !policy) break;
        e = hipMemcpyAsync(flag, &host[c], sizeof(int), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = c == 0 ? dpk::launch_validate_P(P, pb->T, pb->K, flag, stream)
                       : dpk::launch_validate_policy(policy, (size_t)pb->T * pb->K * pb->st.S,
                                                     pb->st.S, pb->st.w_up, pb->st.w_down, flag,
                                                     stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&host[c], flag, sizeof(int), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
    }
    if (e != hipSuccess) return hip_fail(e, "validate inputs");
    if (host[0]) return fail(DP_EBADPROB, "a row of P has a negative entry or does not sum to 1");
    if (host[1]) return fail(DP_EINVAL, "a policy entry is not a feasible next state");
    return DP_OK;
}

void ckpt_pointers(const dp_problem *pb, void *ckpt, float **cv, double **co)
{
    const int M = n_ckpt_slots(pb);
    char *b = static_cast<char *>(ckpt);
    *cv = reinterpret_cast<float *>(b);
    *co = reinterpret_cast<double *>(b + align256(sizeof(float) * (size_t)M * pb->K * pb->st.S));
}

}  // namespace dpgpu

using namespace dpgpu;

extern "C" {

int dp_abi_version(void) { return DPGPU_ABI_VERSION; }

const char *dp_strerror(int code)
{
    switch (code) {
    case DP_OK: return "success";
    case DP_EINVAL: return "invalid argument";
    case DP_EBADPROB: return "transition rows are not stochastic";
    case DP_ENOWS: return "workspace missing or too small";
    case DP_EHIP: return "HIP runtime error";
    case DP_ETIMEOUT: return "reserved error code";
    case DP_ENOMEM: return "host allocation failed";
    case DP_ENOTSUP: return "not supported by this library";
    default: return "unknown error";
    }
}

const char *dp_last_error(void) { return g_last_error.c_str(); }

// Tuning hook: force the sweep tile shape (tile outputs per block, waves per block);
// tile = 0 restores the built-in choice.
int dp_set_sweep_shape(int tile, int waves)
{
    dpk::SweepShape sh = {tile, waves};
    if (tile == 0) {
        g_shape_override = dpk::SweepShape{0, 0};
        return DP_OK;
    }
    if (!dpk::sweep_shape_supported(sh))
        return fail(DP_EINVAL, "unsupported sweep shape: tile %d, %d waves", tile, waves);
    g_shape_override = sh;
    return DP_OK;
}

int dp_set_timing(int on)
{
    // 1: default events; 2: events without the system-scope fence (lighter packets)
    const unsigned flags = on == 2 ? hipEventDisableSystemFence : hipEventDefault;
    if (flags != g_timer.flags) {
        for (hipEvent_t e : g_timer.ev) (void)hipEventDestroy(e);
        g_timer.ev.clear();
        g_timer.flags = flags;
    }
    g_timer.on = on != 0;
    g_timer.used = 0;
    g_timer.kind.clear();
    return DP_OK;
}

int dp_get_timing(double *sweep_ms, int *n_sweep, double *expect_ms, int *n_expect)
{
    double t[2] = {0.0, 0.0};
    int n[2] = {0, 0};
    for (size_t i = 0; 2 * i + 1 < g_timer.used; ++i) {
        hipError_t e = hipEventSynchronize(g_timer.ev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "timing sync");
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, g_timer.ev[2 * i], g_timer.ev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "timing elapsed");
        const int k = g_timer.kind[i];
        t[k] += ms;
        n[k] += 1;
    }
    if (sweep_ms) *sweep_ms = t[0];
    if (n_sweep) *n_sweep = n[0];
    if (expect_ms) *expect_ms = t[1];
    if (n_expect) *n_expect = n[1];
    g_timer.used = 0;
    g_timer.kind.clear();
    return DP_OK;
}

size_t dp_workspace_bytes(const dp_problem *pb)
{
    if (validate_problem(pb) != DP_OK) return 0;
    return solve_layout(pb).total;
}

size_t dp_ckpt_bytes(const dp_problem *pb)
{
    if (validate_problem(pb) != DP_OK) return 0;
    if (pb->ckpt_every < 1) return 0;
    return ckpt_bytes(pb);
}

int dp_solve(const dp_problem *pb, const float *lam, const float *P, const float *v_term,
             float *V, int16_t *policy, void *ckpt, void *ws, size_t ws_bytes, void *stream_)
{
    int rc = validate_problem(pb);
    if (rc != DP_OK) return rc;
    if (!lam || !P || !V) return fail(DP_EINVAL, "lam, P and V must be non-NULL");
    if (ckpt && pb->ckpt_every < 1) return fail(DP_EINVAL, "ckpt given but ckpt_every < 1");
    const SolveLayout L = solve_layout(pb);
    if (!ws || ws_bytes < L.total) return fail(DP_ENOWS, "workspace needs %zu bytes (got %zu)", L.total, ws_bytes);
    if (((uintptr_t)ws & 255) != 0) return fail(DP_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if (pb->flags & DP_VALIDATE) {
        rc = validate_device_inputs(pb, P, nullptr, reinterpret_cast<int *>(static_cast<char *>(ws) + L.flag), stream);
        if (rc != DP_OK) return rc;
    }
    StageOutputs out = {};
    const size_t KS = (size_t)pb->K * pb->st.S;
    if (pb->flags & DP_STORE_V_ALL) out.vall = V;
    else out.v1 = V;
    out.pol = policy;
    out.ckpt_every = pb->ckpt_every;
    if (ckpt) ckpt_pointers(pb, ckpt, &out.ckpt_v, &out.ckpt_off);
    (void)KS;
    return run_stages(pb, 1, pb->T, lam, P, v_term, nullptr, out, ws, stream);
}

// ------------------------------------------------------------------------------------
// Allocation-free solve: the solver state lives in a file-scope device array of this
// translation unit.  Its address on each device comes from hipGetSymbolAddress, taken once
// per device with that device current; only that address is ever handed to kernels or
// copies.
// ------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[DP_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64];

static int scratch_for_current_device(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(DP_ENOTSUP, "device index %d beyond 63", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(DP_EHIP, "no device address for the solver scratch");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return DP_OK;
}

// ------------------------------------------------------------------------------------
// Adjoint.
// ------------------------------------------------------------------------------------
struct AdjLayout {
    int Spad, G;            // G: stages per grad_P launch (nu_t planes kept for a group)
    int npk;                // stages of P_t^T held repacked for the transport
    size_t mu, nu, scale, flag, PpT, vseg, polseg, solve_ws, total;
};

static AdjLayout adj_layout(const dp_problem *pb, bool ckpt_mode)
{
    AdjLayout L = {};
    L.Spad = pad64(pb->st.S);
    const size_t plane = align256(sizeof(float) * (size_t)pb->K * L.Spad);
    size_t o = 0;
    // grad_P_t needs nu_t only, off the stage-to-stage path: nu_t of G consecutive stages
    // are kept and their grad_P computed in one launch (G <= 16, <= 256 MB of planes)
    L.G = 16;
    while (L.G > 1 && (size_t)L.G * plane > ((size_t)256 << 20)) L.G >>= 1;
    if (L.G > pb->T) L.G = pb->T;
    L.mu = o; o += plane;
    L.nu = o; o += (size_t)L.G * plane;
    L.scale = o; o += 256;
    L.flag = o; o += 256;
    // P_t^T repacked for the transport, up to 32 stages per pack launch (<= 64 MB)
    const size_t pk = sizeof(float) * dpk::packed_P_floats(pb->K);
    L.npk = 32;
    while (L.npk > 1 && (size_t)L.npk * pk > ((size_t)64 << 20)) L.npk >>= 1;
    if (L.npk > pb->T) L.npk = pb->T;
    L.PpT = o; o += align256((size_t)L.npk * pk);
    if (ckpt_mode) {
        // two segment buffers: segment m + 1 is re-solved into one while the adjoint of
        // segment m reads the other
        const int E = pb->ckpt_every > 0 ? pb->ckpt_every : 16;
        const size_t KS = (size_t)pb->K * pb->st.S;
        L.vseg = o; o += 2 * align256(sizeof(float) * (size_t)(E + 1) * KS);
        L.polseg = o; o += 2 * align256(sizeof(int16_t) * (size_t)E * KS);
        L.solve_ws = o; o += solve_layout(pb).total;
    }
    L.total = o;
    return L;
}

// A stream per device for the checkpointed adjoint's segment re-solves, created on first
// use and kept until the process ends (default priority).  Calls that share it are ordered
// on it; every use is forked from and joined back into the caller's stream with events.
static hipError_t side_stream(hipStream_t *out)
{
    static std::mutex mu;
    static std::vector<hipStream_t> streams;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)streams.size() <= dev) streams.resize(dev + 1, nullptr);
    if (!streams[dev]) {
        e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
        if (e != hipSuccess) {
            streams[dev] = nullptr;
            return e;
        }
    }
    *out = streams[dev];
    return hipSuccess;
}

// Events of one checkpointed dp_adjoint call, destroyed on every return path (the runtime
// releases an event destroyed before its recorded work completes once that work is done).
struct AdjEvents {
    hipEvent_t fork = nullptr, solved[2] = {nullptr, nullptr}, used[2] = {nullptr, nullptr};
    ~AdjEvents()
    {
        if (fork) (void)hipEventDestroy(fork);
        for (int i = 0; i < 2; ++i) {
            if (solved[i]) (void)hipEventDestroy(solved[i]);
            if (used[i]) (void)hipEventDestroy(used[i]);
        }
    }
    hipError_t create()
    {
        hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        for (int i = 0; i < 2 && e == hipSuccess; ++i) {
            e = hipEventCreateWithFlags(&solved[i], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&used[i], hipEventDisableTiming);
        }
        return e;
    }
};

int dp_solve_noalloc(const dp_problem *pb, const float *lam, const float *P,
                     const float *v_term, float *V, int16_t *policy, void *ckpt, void *stream_)
{
    int rc = validate_problem(pb);
    if (rc != DP_OK) return rc;
    if (!lam || !P || !V) return fail(DP_EINVAL, "lam, P and V must be non-NULL");
    if (ckpt && pb->ckpt_every < 1) return fail(DP_EINVAL, "ckpt given but ckpt_every < 1");
    if (pb->flags & DP_VALIDATE)
        return fail(DP_EINVAL, "DP_VALIDATE reads a flag back to the host; use dp_solve");
    const SolveLayout L = solve_layout(pb, DP_NOALLOC_SCRATCH_BYTES);
    if (L.total > DP_NOALLOC_SCRATCH_BYTES)
        return fail(DP_ENOTSUP, "the solver state needs %zu bytes; dp_solve_noalloc holds %zu "
                    "(use dp_solve with a workspace)", L.total, (size_t)DP_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    if ((rc = scratch_for_current_device(&ws)) != DP_OK) return rc;
    StageOutputs out = {};
    if (pb->flags & DP_STORE_V_ALL) out.vall = V;
    else out.v1 = V;
    out.pol = policy;
    out.ckpt_every = pb->ckpt_every;
    if (ckpt) ckpt_pointers(pb, ckpt, &out.ckpt_v, &out.ckpt_off);
    return run_stages(pb, 1, pb->T, lam, P, v_term, nullptr, out, ws,
                      static_cast<hipStream_t>(stream_), DP_NOALLOC_SCRATCH_BYTES, false);
}

size_t dp_adjoint_workspace_bytes(const dp_problem *pb)
{
    if (validate_problem(pb) != DP_OK) return 0;
    return adj_layout(pb, pb->ckpt_every >= 1).total;
}

int dp_adjoint(const dp_problem *pb, const float *lam, const float *P, const float *v_term,
               const float *V_all, const int16_t *policy, const void *ckpt, const float *seed,
               float *grad_lam, float *grad_P, float *grad_vterm, void *ws, size_t ws_bytes,
               void *stream_)
{
    int rc = validate_problem(pb);
    if (rc != DP_OK) return rc;
    const int K = pb->K, S = pb->st.S, T = pb->T;
    if (!lam || !P || !seed || !grad_lam || !grad_P) return fail(DP_EINVAL, "lam, P, seed, grad_lam, grad_P must be non-NULL");
    const bool ckpt_mode = (ckpt != nullptr);
    if (ckpt_mode) {
        if (V_all || policy) return fail(DP_EINVAL, "give either (V_all, policy) or ckpt, not both");
        if (pb->ckpt_every < 1) return fail(DP_EINVAL, "ckpt mode needs ckpt_every >= 1");
    } else if (!V_all || !policy) {
        return fail(DP_EINVAL, "full-storage mode needs V_all and policy");
    }
    const AdjLayout L = adj_layout(pb, ckpt_mode);
    if (!ws || ws_bytes < L.total) return fail(DP_ENOWS, "adjoint workspace needs %zu bytes (got %zu)", L.total, ws_bytes);
    if (((uintptr_t)ws & 255) != 0) return fail(DP_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    char *base = static_cast<char *>(ws);
    if (pb->flags & DP_VALIDATE) {
        rc = validate_device_inputs(pb, P, ckpt_mode ? nullptr : policy,
                                    reinterpret_cast<int *>(base + L.flag), stream);
        if (rc != DP_OK) return rc;
    }
    float *mu = reinterpret_cast<float *>(base + L.mu);
    float *nu = reinterpret_cast<float *>(base + L.nu);
    const size_t plane = align256(sizeof(float) * (size_t)K * L.Spad) / sizeof(float);
    const size_t KS = (size_t)K * S;
    const dpk::Payoff pay = {pb->st.delta, pb->st.eta_c, pb->st.eta_d, pb->st.c_deg, pb->st.c_start};
    double *scale = reinterpret_cast<double *>(base + L.scale);
    hipError_t e = dpk::launch_copy_rows(seed, S, mu, L.Spad, K, S, stream);
    if (e != hipSuccess) return hip_fail(e, "seed copy");
    e = dpk::launch_adjoint_scale(seed, KS, scale, stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint scale");

    const int E = ckpt_mode ? pb->ckpt_every : T;
    const int nseg = (T + E - 1) / E;
    float *cv = nullptr;
    double *co = nullptr;
    if (ckpt_mode) ckpt_pointers(pb, const_cast<void *>(ckpt), &cv, &co);
    const size_t vseg_bytes = align256(sizeof(float) * (size_t)(E + 1) * KS);
    const size_t pseg_bytes = align256(sizeof(int16_t) * (size_t)E * KS);

    // Checkpoint mode: segment m is re-solved backward from its checkpoint on a side stream
    // into segment buffer m % 2, while this stream runs the adjoint of segment m - 1 from
    // the other buffer.  solved[b] orders a re-solve before its adjoint; used[b] orders the
    // adjoint of segment m before the re-solve of segment m + 2 rewrites its buffer.
    hipStream_t side = nullptr;
    AdjEvents ev;
    hipEvent_t side_last = nullptr;     // the side stream's last recorded event (for the join)
    if (ckpt_mode) {
        e = side_stream(&side);
        if (e == hipSuccess) e = ev.create();
        if (e == hipSuccess) e = hipEventRecord(ev.fork, stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(side, ev.fork, 0);
        if (e != hipSuccess) return hip_fail(e, "adjoint side stream");
    }
    auto resolve = [&](int m) -> int {
        const int t_lo = 1 + m * E, t_hi = t_lo + E - 1 < T ? t_lo + E - 1 : T;
        const int b = m & 1;
        if (m >= 2) {
            const hipError_t ew = hipStreamWaitEvent(side, ev.used[b], 0);
            if (ew != hipSuccess) return hip_fail(ew, "segment buffer wait");
        }
        const float *src;
        const double *src_off;
        if (t_hi == T) {
            src = v_term;
            src_off = nullptr;
        } else {
            const int mc = t_hi / E;         // stage t_hi + 1 = 1 + mc E
            src = cv + (size_t)(mc - 1) * KS;
            src_off = co + (mc - 1);
        }
        StageOutputs out = {};
        out.vall = reinterpret_cast<float *>(base + L.vseg + b * vseg_bytes);
        out.pol = reinterpret_cast<int16_t *>(base + L.polseg + b * pseg_bytes);
        out.ckpt_every = E;
        const int rs = run_stages(pb, t_lo, t_hi, lam, P, src, src_off, out, base + L.solve_ws, side);
        if (rs != DP_OK) return rs;
        const hipError_t er = hipEventRecord(ev.solved[b], side);
        if (er != hipSuccess) return hip_fail(er, "segment event");
        side_last = ev.solved[b];
        return DP_OK;
    };
    float *PpT = reinterpret_cast<float *>(base + L.PpT);
    const size_t pk = dpk::packed_P_floats(K);
    int pk_lo = 1, pk_hi = 0;      // the packed stages are pk_lo .. pk_hi
    auto stages = [&]() -> int {
        if (ckpt_mode && (rc = resolve(0)) != DP_OK) return rc;
        for (int m = 0; m < nseg; ++m) {
            const int t_lo = 1 + m * E, t_hi = t_lo + E - 1 < T ? t_lo + E - 1 : T;
            const float *Vseg;   // slice (t - t_lo) holds V_t, slice t_hi + 1 - t_lo holds V_{t_hi+1}
            const int16_t *pseg;
            if (ckpt_mode) {
                if (m + 1 < nseg && (rc = resolve(m + 1)) != DP_OK) return rc;
                e = hipStreamWaitEvent(stream, ev.solved[m & 1], 0);
                if (e != hipSuccess) return hip_fail(e, "segment wait");
                Vseg = reinterpret_cast<const float *>(base + L.vseg + (m & 1) * vseg_bytes);
                pseg = reinterpret_cast<const int16_t *>(base + L.polseg + (m & 1) * pseg_bytes);
            } else {
                Vseg = V_all + (size_t)(t_lo - 1) * KS;
                pseg = policy + (size_t)(t_lo - 1) * KS;
            }
            for (int g0 = t_lo; g0 <= t_hi; g0 += L.G) {
                const int g1 = g0 + L.G - 1 < t_hi ? g0 + L.G - 1 : t_hi;
                for (int t = g0; t <= g1; ++t) {
                    const int16_t *pol_t = pseg + (size_t)(t - t_lo) * KS;
                    float *nu_t = nu + (size_t)(t - g0) * plane;
                    e = dpk::launch_pushforward(mu, L.Spad, pol_t, K, S, pay, scale, nu_t,
                                                L.Spad, grad_lam + (size_t)(t - 1) * K, stream);
                    if (e != hipSuccess) return hip_fail(e, "pushforward");
                    // mu_{t+1} = P_t^T nu_t, A = P_t^T from the repacked ring
                    if (t > pk_hi) {       // repack the next chunk of stages (upwards from t)
                        pk_lo = t;
                        pk_hi = t + L.npk - 1 < T ? t + L.npk - 1 : T;
                        e = dpk::launch_pack_P(P + (size_t)(t - 1) * K * K, true, K,
                                               pk_hi - pk_lo + 1, PpT, stream);
                        if (e != hipSuccess) return hip_fail(e, "pack P^T");
                    }
                    e = dpk::launch_contract_packed(PpT + (size_t)(t - pk_lo) * pk, nu_t, L.Spad,
                                                    mu, L.Spad, K, S, stream);
                    if (e != hipSuccess) return hip_fail(e, "transport");
                }
                e = dpk::launch_gradP(nu, plane, L.Spad, Vseg + (size_t)(g0 + 1 - t_lo) * KS,
                                      KS, K, S, g1 - g0 + 1, grad_P + (size_t)(g0 - 1) * K * K,
                                      stream);
                if (e != hipSuccess) return hip_fail(e, "grad_P");
            }
            if (ckpt_mode) {
                e = hipEventRecord(ev.used[m & 1], stream);
                if (e != hipSuccess) return hip_fail(e, "segment event");
            }
        }
        return DP_OK;
    };
    rc = stages();
    if (side_last) {
        // join: whatever the side stream was given is done before this call's later work
        const hipError_t ej = hipStreamWaitEvent(stream, side_last, 0);
        if (rc == DP_OK && ej != hipSuccess) rc = hip_fail(ej, "join");
    }
    if (rc != DP_OK) return rc;
    if (grad_vterm) {
        e = dpk::launch_copy_rows(mu, L.Spad, grad_vterm, S, K, S, stream);
        if (e != hipSuccess) return hip_fail(e, "grad_vterm copy");
    }
    return DP_OK;
}

}  // extern "C"
