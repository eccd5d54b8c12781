// Host-only paths of libdpgpu (argument validation, workspace and checkpoint sizes,
// error reporting, the paper-mode grid sizes, plan creation's checks), for a build whose
// host code carries the address and undefined-behaviour sanitizers.  Nothing here reaches
// the device: every call below returns before its first HIP runtime call.  Exit status 0
// when every call returned what the header documents.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "dpgpu.h"

static int bad = 0;
#define EXPECT(c)                                                  \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "line %d: %s failed\n", __LINE__, #c); \
            bad = 1;                                               \
        }                                                          \
    } while (0)

static dp_problem good()
{
    dp_problem pb;
    memset(&pb, 0, sizeof pb);
    pb.T = 12;
    pb.K = 7;
    pb.st.S = 300;
    pb.st.w_up = 30;
    pb.st.w_down = 45;
    pb.st.delta = 0.25f;
    pb.st.eta_c = 0.9f;
    pb.st.eta_d = 0.95f;
    pb.st.c_deg = 1.0f;
    pb.st.c_start = 0.5f;
    return pb;
}

int main()
{
    EXPECT(dp_abi_version() == DPGPU_ABI_VERSION);
    for (int c = 0; c >= -8; --c) EXPECT(dp_strerror(c) != NULL && strlen(dp_strerror(c)) > 0);
    dp_problem pb = good();
    const size_t ws = dp_workspace_bytes(&pb);
    EXPECT(ws > 0 && ws % 256 == 0);
    EXPECT(dp_adjoint_workspace_bytes(&pb) > 0);
    EXPECT(dp_ckpt_bytes(&pb) == 0);          // ckpt_every = 0
    pb.ckpt_every = 5;
    EXPECT(dp_ckpt_bytes(&pb) > 0);
    EXPECT(dp_adjoint_workspace_bytes(&pb) > ws);
    // every invalid field is rejected on the host, with a message
    for (int f = 0; f < 14; ++f) {
        dp_problem q = good();
        switch (f) {
        case 0: q.T = 0; break;
        case 1: q.K = 0; break;
        case 2: q.K = DP_MAX_K + 1; break;
        case 3: q.st.S = 1; break;
        case 4: q.st.S = DP_MAX_S + 1; break;
        case 5: q.st.w_up = -1; break;
        case 6: q.st.reserved = 3; break;
        case 7: q.st.delta = 0.0f; break;
        case 8: q.st.eta_c = 1.5f; break;
        case 9: q.st.eta_d = NAN; break;
        case 10: q.st.c_deg = -1.0f; break;
        case 11: q.st.c_start = INFINITY; break;
        case 12: q.flags = 0x80; break;
        case 13: q.ckpt_every = -1; break;
        }
        EXPECT(dp_workspace_bytes(&q) == 0);
        EXPECT(strlen(dp_last_error()) > 0);
        EXPECT(dp_solve(&q, (float *)256, (float *)256, NULL, (float *)256, NULL, NULL,
                        (void *)256, 1 << 20, NULL) == DP_EINVAL);
    }
    EXPECT(dp_workspace_bytes(NULL) == 0);
    // a window too wide for any tile's LDS
    dp_problem w = good();
    w.st.S = DP_MAX_S;
    w.st.w_up = w.st.w_down = 12000;
    EXPECT(dp_workspace_bytes(&w) == 0);
    // missing pointers, small or misaligned workspace: rejected before device work
    EXPECT(dp_solve(&pb, NULL, (float *)256, NULL, (float *)256, NULL, NULL, (void *)256, ws, NULL) == DP_EINVAL);
    pb.ckpt_every = 0;
    EXPECT(dp_solve(&pb, (float *)256, (float *)256, NULL, (float *)256, NULL, NULL, (void *)256, ws - 1, NULL) == DP_ENOWS);
    EXPECT(dp_solve(&pb, (float *)256, (float *)256, NULL, (float *)256, NULL, NULL, (void *)4097, ws, NULL) == DP_EINVAL);
    EXPECT(dp_solve(&pb, (float *)256, (float *)256, NULL, (float *)256, NULL, (void *)256, (void *)256, ws, NULL) == DP_EINVAL);
    const size_t aws = dp_adjoint_workspace_bytes(&pb);
    EXPECT(dp_adjoint(&pb, (float *)256, (float *)256, NULL, (float *)256, NULL, NULL, (float *)256,
                      (float *)256, (float *)256, NULL, (void *)256, aws, NULL) == DP_EINVAL);
    EXPECT(dp_adjoint(&pb, (float *)256, (float *)256, NULL, (float *)256, (int16_t *)256, NULL,
                      (float *)256, (float *)256, (float *)256, NULL, (void *)256, aws - 1, NULL) == DP_ENOWS);
    // paper-mode grid sizes (Table 3: eta = sqrt(0.85), delta = 0.1 gives P = 22, 0.01 gives 203)
    dp_iid_problem ip;
    memset(&ip, 0, sizeof ip);
    ip.T = 10; ip.R = 20; ip.S = 41; ip.delta = 0.1f; ip.eta = sqrtf(0.85f); ip.p_bar = 1.0f;
    int P = 0, nc = 0, nd = 0;
    EXPECT(dp_iid_action_grid(&ip, &P, &nc, &nd) == DP_OK && P == 22 && P == nc + nd + 1);
    ip.delta = 0.01f; ip.S = 401;
    EXPECT(dp_iid_action_grid(&ip, &P, &nc, &nd) == DP_OK && P == 203);
    EXPECT(dp_iid_workspace_bytes(&ip) > 0);
    ip.R = 0;
    EXPECT(dp_iid_workspace_bytes(&ip) == 0);
    // plans: bad problems and flags are rejected before any allocation
    dp_batch_plan *plan = (dp_batch_plan *)1;
    dp_problem probs[2] = {good(), good()};
    probs[1].K = 0;
    EXPECT(dp_batch_plan_create(&plan, 2, probs, NULL, NULL) == DP_EINVAL && plan == NULL);
    probs[1] = good();
    probs[1].flags = DP_STORE_V_ALL;
    EXPECT(dp_batch_plan_create(&plan, 2, probs, NULL, NULL) == DP_EINVAL && plan == NULL);
    EXPECT(dp_batch_plan_create(&plan, 0, probs, NULL, NULL) == DP_EINVAL);
    EXPECT(dp_batch_plan_create(NULL, 2, probs, NULL, NULL) == DP_EINVAL);
    char buf[64];
    EXPECT(dp_batch_plan_describe(NULL, buf, sizeof buf) == DP_EINVAL);
    dp_batch_plan_destroy(NULL);
    // tuning hooks (host state only)
    EXPECT(dp_set_sweep_shape(96, 4) == DP_EINVAL);
    EXPECT(dp_set_sweep_shape(512, 3) == DP_EINVAL);
    EXPECT(dp_set_sweep_shape(2048, 8) == DP_EINVAL);
    EXPECT(dp_set_sweep_shape(512, 8) == DP_OK);
    EXPECT(dp_set_sweep_shape(0, 0) == DP_OK);
    printf(bad ? "FAILED\n" : "ok\n");
    return bad;
}
