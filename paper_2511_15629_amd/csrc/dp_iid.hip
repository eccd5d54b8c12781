// Stagewise-independent prices on the paper's power-action grid (Sec. II-B, III;
// Algorithm 1 with its interpolated endpoint columns).  See include/dpgpu.h.
#include "dp_host.h"

#include <math.h>

using namespace dpgpu;

namespace {

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct IidGrid {
    int n_c, n_d, P;
};

// n_c = ceil(p_bar eta / delta), n_d = ceil(p_bar / (delta eta)) (Sec. III-A), in FP64 on
// the FP32 parameters, with a 1e-12 guard so exact quotients do not round up.
IidGrid iid_grid(const dp_iid_problem *pb)
{
    const double d = pb->delta, e = pb->eta, p = pb->p_bar;
    IidGrid g;
    g.n_c = (int)ceil(p * e / d - 1e-12);
    g.n_d = (int)ceil(p / (d * e) - 1e-12);
    if (g.n_c < 1) g.n_c = 1;
    if (g.n_d < 1) g.n_d = 1;
    g.P = g.n_c + g.n_d + 1;
    return g;
}

int validate_iid(const dp_iid_problem *pb)
{
    if (!pb) return fail(DP_EINVAL, "problem pointer is NULL");
    if (pb->T < 1) return fail(DP_EINVAL, "T must be >= 1");
    if (pb->R < 1 || pb->R > 4096) return fail(DP_EINVAL, "R must be in [1, 4096]");
    if (pb->S < 2 || pb->S > DP_MAX_S) return fail(DP_EINVAL, "S must be in [2, %d]", DP_MAX_S);
    if (!(pb->delta > 0.0f) || !isfinite(pb->delta)) return fail(DP_EINVAL, "delta must be finite and > 0");
    if (!(pb->eta > 0.0f && pb->eta <= 1.0f)) return fail(DP_EINVAL, "eta must be in (0, 1]");
    if (!(pb->p_bar > 0.0f) || !isfinite(pb->p_bar)) return fail(DP_EINVAL, "p_bar must be finite and > 0");
    if (pb->flags & ~(uint32_t)DP_STORE_V_ALL) return fail(DP_EINVAL, "unknown flag bits");
    if (pb->reserved != 0) return fail(DP_EINVAL, "reserved must be 0");
    const IidGrid g = iid_grid(pb);
    if (g.P > 32767) return fail(DP_EINVAL, "power grid has %d actions (int16 policy limit)", g.P);
    if (dpk::iid_lds_bytes(pb->R, pb->S, g.n_c - 1, g.n_d - 1) > 160 * 1024)
        return fail(DP_ENOTSUP, "R = %d samples with %d actions need more LDS than a CU holds", pb->R, g.P);
    return DP_OK;
}

struct IidLayout {
    size_t v0, v1, endc, endd, off, total;
};

IidLayout iid_layout(const dp_iid_problem *pb)
{
    IidLayout L;
    size_t o = 0;
    L.v0 = o; o += a256(sizeof(float) * pb->S);
    L.v1 = o; o += a256(sizeof(float) * pb->S);
    L.endc = o; o += a256(sizeof(dpk::IidEnd) * pb->S);
    L.endd = o; o += a256(sizeof(dpk::IidEnd) * pb->S);
    L.off = o; o += a256(sizeof(double) * ((size_t)pb->T + 2));
    L.total = o;
    return L;
}

}  // namespace

extern "C" {

int dp_iid_action_grid(const dp_iid_problem *pb, int *P, int *n_c, int *n_d)
{
    int rc = validate_iid(pb);
    if (rc != DP_OK) return rc;
    const IidGrid g = iid_grid(pb);
    if (P) *P = g.P;
    if (n_c) *n_c = g.n_c;
    if (n_d) *n_d = g.n_d;
    return DP_OK;
}

size_t dp_iid_workspace_bytes(const dp_iid_problem *pb)
{
    if (validate_iid(pb) != DP_OK) return 0;
    return iid_layout(pb).total;
}

int dp_solve_iid(const dp_iid_problem *pb, const float *lam, const float *prob, float *V,
                 int16_t *policy, void *ws, size_t ws_bytes, void *stream_)
{
    int rc = validate_iid(pb);
    if (rc != DP_OK) return rc;
    if (!lam || !prob || !V) return fail(DP_EINVAL, "lam, prob and V must be non-NULL");
    const IidLayout L = iid_layout(pb);
    if (!ws || ws_bytes < L.total) return fail(DP_ENOWS, "workspace needs %zu bytes (got %zu)", L.total, ws_bytes);
    if (((uintptr_t)ws & 255) != 0) return fail(DP_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const IidGrid g = iid_grid(pb);
    const int T = pb->T, R = pb->R, S = pb->S;
    char *base = static_cast<char *>(ws);
    float *vp[2] = {reinterpret_cast<float *>(base + L.v0), reinterpret_cast<float *>(base + L.v1)};
    dpk::IidEnd *endc = reinterpret_cast<dpk::IidEnd *>(base + L.endc);
    dpk::IidEnd *endd = reinterpret_cast<dpk::IidEnd *>(base + L.endd);
    double *off = reinterpret_cast<double *>(base + L.off);   // off[t] = offset of V_t, t = 0..T
    const bool all = (pb->flags & DP_STORE_V_ALL) != 0;
    hipError_t e = dpk::launch_iid_tables(S, (double)pb->delta, (double)pb->eta, (double)pb->p_bar,
                                          endc, endd, stream);
    if (e != hipSuccess) return hip_fail(e, "endpoint tables");
    e = dpk::launch_iid_init(vp[0], S, off + T, all ? V + (size_t)T * S : nullptr, stream);
    if (e != hipSuccess) return hip_fail(e, "init");
    dpk::IidArgs a;
    a.endc = endc;
    a.endd = endd;
    a.R = R;
    a.S = S;
    a.w_up = g.n_c - 1;
    a.w_down = g.n_d - 1;
    a.P = g.P;
    a.pay = {pb->delta, pb->eta, pb->eta, 0.0f, 0.0f};
    a.p_bar = pb->p_bar;
    int cur = 0;
    for (int t = T; t >= 1; --t) {
        a.Vin = vp[cur];
        a.Vout = vp[cur ^ 1];
        a.lam = lam + (size_t)(t - 1) * R;
        a.prob = prob + (size_t)(t - 1) * R;
        a.off_next = off + t;
        a.off_cur = off + (t - 1);
        a.vabs = all ? V + (size_t)(t - 1) * S : (t == 1 ? V : nullptr);
        a.pol = policy ? policy + (size_t)(t - 1) * R * S : nullptr;
        e = dpk::launch_iid_stage(a, stream);
        if (e != hipSuccess) return hip_fail(e, "independent-price stage");
        cur ^= 1;
    }
    return DP_OK;
}

}  // extern "C"
