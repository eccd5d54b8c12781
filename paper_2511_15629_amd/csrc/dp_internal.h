// Internal declarations shared by the kernel and host translation units of libdpgpu.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpk {

// Payoff parameters of one instance (FP32 on the device).
struct Payoff {
    float delta, eta_c, eta_d, c_deg, c_start;
};

// One stage of the Bellman sweep (Eq. (5)): inputs W_t (expectation) and lam_t,
// outputs the normalised values, optional absolute values, policies, checkpoint.
struct SweepArgs {
    const float *W;          // [K][ldw] expectation W_t (when Vn is null)
    int ldw;
    const float *Vn;         // [K][ldvn] normalised V_{t+1}: the block forms its W_t row
    int ldvn;                //   itself (fused expectation; W unused); nullptr: read W
    const float *Vn0;        // V_{t+1}[0][0] (normalised): the stage's normalisation constant
    const float *lam;        // [K]
    const float *P;          // [K][K] P_t: the fused expectation's rows, and the row sums
                             // rho_k when rho1 is null (nullable then: rows sum to 1)
    const double *rho1;      // [K] rho_k - 1, precomputed (nullable: use P, or 0)
    int K, S, w_up, w_down;
    Payoff pay;
    const double *off_next;  // C_{t+1}
    double *off_cur;         // C_t (written by block (0,0))
    float *vnorm;            // out [K][ldv] normalised V_t = U - shift
    int ldv;
    float *vabs;             // out [K][S] absolute V_t (nullable)
    int16_t *pol;            // out [K][S] (nullable)
    float *ckpt_v;           // out [K][S] normalised copy (nullable)
    double *ckpt_off;        // out C_t (nullable)
};

struct SweepShape {
    int TS, NW;              // outputs per block (SoC tile), waves per block
};

// rho1[t][k] = (sum of row k of P_t, FP64, the sweep's fixed order) - 1 for nstage stages
hipError_t launch_row_sums(const float *P, int K, int nstage, double *rho1, hipStream_t stream);

// Batched solves: one descriptor per instance, flattened work lists.
struct BatchDesc {
    int T, K, S, w_up, w_down, ld;
    Payoff pay;
    const float *lam;        // [T][K]
    const float *P;          // [T][K][K]
    float *V1;               // [K][S] absolute values of stage 1
    int16_t *pol;            // [T][K][S] or null
    float *vbuf0, *vbuf1;    // normalised values ping-pong [K][ld]
    float *W;                // expectation [K][ld]
    double *off;             // offsets C_t, t = 1..T+1
};
struct SweepItem {
    int inst, k, tile;
};
struct ContractItem {
    int inst, tm, tn;      // strips: row tile, first column tile; panels: panel count, first column tile
};

hipError_t launch_batched_init(const BatchDesc *desc, int n, hipStream_t stream);
hipError_t launch_batched_contract(const BatchDesc *desc, const ContractItem *items, int n,
                                   int tau, hipStream_t stream);
// Column-panel expectation for K <= 128 (one block per item of up to four 64-column
// panels; ContractItem.tm = panel count, .tn = first 16-column tile).  One launch covers
// the items of one class panel_class(K) (K <= 32, <= 64, <= 128); kmax = the largest K
// among them.
int panel_class(int K);
hipError_t launch_batched_panel(const BatchDesc *desc, const ContractItem *items, int n, int tau,
                                int kmax, hipStream_t stream);
// Sweep tiles per block in batched launches (four for one-wave shapes, else one); the
// block's LDS is that many 16-byte aligned copies of sweep_lds_bytes.
int batched_tiles_per_block(const SweepShape &sh);
hipError_t launch_batched_sweep(const BatchDesc *desc, const SweepItem *items, int n, int tau,
                                const SweepShape &sh, size_t lds, hipStream_t stream);

// Stagewise-independent prices on the paper's power grid (Algorithm 1 as printed):
// R price samples per stage, interior actions = whole SoC steps [-w_down, w_up], plus the
// two endpoint actions -p_bar (charge) and +p_bar (discharge) whose next states are
// interpolated between two grid points.
struct IidEnd {              // per SoC index s, one endpoint action
    int lo, hi;              // next-state indices (lo = -1: infeasible)
    float b;                 // interpolation factor
};
struct IidArgs {
    const float *Vin;        // normalised V_t [S]
    float *Vout;             // normalised V_{t-1} [S]
    const float *lam;        // lam_t [R]
    const float *prob;       // pi_t [R]
    const IidEnd *endc;      // charge endpoint table [S]
    const IidEnd *endd;      // discharge endpoint table [S]
    int R, S, w_up, w_down, P;
    int TS, NP;              // outputs per block, partial sums per output (set by the launcher)
    Payoff pay;              // interior payoff (delta, eta_c = eta_d = eta, costs)
    float p_bar;
    const double *off_next;  // C_t (offset of Vin)
    double *off_cur;         // C_{t-1}
    float *vabs;             // [S] absolute V_{t-1} (nullable)
    int16_t *pol;            // [R][S] action index into the ascending power grid (nullable)
};
struct IidShape {
    int TS, threads, NP, RB;   // outputs per block, threads, partial sums, samples per unit
};
IidShape iid_shape(int R, int S);
hipError_t launch_iid_stage(const IidArgs &a, hipStream_t stream);
size_t iid_lds_bytes(int R, int S, int w_up, int w_down);
hipError_t launch_iid_tables(int S, double delta, double eta, double p_bar, IidEnd *endc,
                             IidEnd *endd, hipStream_t stream);
hipError_t launch_iid_init(float *V, int S, double *off, float *vabs, hipStream_t stream);

// Stage kernels (launchers; all asynchronous on `stream`).
// P_t (or P_t^T with transA) of nstage consecutive stages repacked into the MFMA lane
// order (packed_P_floats(K) floats per stage), and the contraction reading it; bitwise the
// same as every other expectation kernel (the tile chain).
size_t packed_P_floats(int K);
hipError_t launch_pack_P(const float *P, bool transA, int K, int nstage, float *Pp,
                         hipStream_t stream);
hipError_t launch_contract_packed(const float *Ap, const float *B, int ldb, float *C, int ldc,
                                  int K, int N, hipStream_t stream);
hipError_t launch_sweep(const SweepArgs &a, const SweepShape &sh, hipStream_t stream);
int sweep_tile(const SweepShape &sh);       // outputs per block along s
size_t sweep_lds_bytes(const SweepShape &sh, int w_up, int w_down, int K_fused = 0);
bool sweep_shape_supported(const SweepShape &sh);

// Initialise the normalised terminal state: vnorm = v_term (or 0, or a checkpoint),
// off[0] = offset, optional absolute copy into vabs.
hipError_t launch_init_terminal(const float *src, const double *src_off, int K, int S,
                                float *vnorm, int ldv, double *off, float *vabs,
                                hipStream_t stream);

// Adjoint stage kernels.
hipError_t launch_pushforward(const float *mu, int ldm, const int16_t *pol, int K, int S,
                              Payoff pay, const double *scale, float *nu, int ldn,
                              float *grad_lam, hipStream_t stream);
hipError_t launch_adjoint_scale(const float *seed, size_t n, double *scale, hipStream_t stream);
// grad_P of G consecutive stages: stage g of the group reads nu + g nu_stride ([K][ldn])
// and V + g v_stride ([K][S]) and writes gP + g K K.
hipError_t launch_gradP(const float *nu, size_t nu_stride, int ldn, const float *V,
                        size_t v_stride, int K, int S, int G, float *gP, hipStream_t stream);
hipError_t launch_copy_rows(const float *src, int lds, float *dst, int ldd, int K, int S,
                            hipStream_t stream);
hipError_t launch_fill(float *dst, size_t n, float v, hipStream_t stream);
hipError_t launch_validate_P(const float *P, int T, int K, int *flag, hipStream_t stream);
hipError_t launch_validate_policy(const int16_t *pol, size_t n, int S, int w_up, int w_down,
                                  int *flag, hipStream_t stream);

}  // namespace dpk
