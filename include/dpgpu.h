/*
 * dpgpu -- MI355X (gfx950) backward induction for multistage stochastic storage
 * arbitrage on a Markov price chain.  C ABI of libdpgpu.so.
 *
 * The method (T. Lee, A. Sun, "GPU-Accelerated Dynamic Programming for Multistage
 * Stochastic Energy Storage Arbitrage"):
 *   - storage model: Sec. II-A, Eq. (1) objective sum_t lambda_t p_t, Eq. (2) state
 *     transition F (charging raises the state of charge by eta |p|, discharging lowers it
 *     by p / eta);
 *   - feasible actions: Eq. (4), discretised on the recombining grid of Sec. III-A, where
 *     every interior power action moves the state of charge by a whole number of steps;
 *   - Bellman recursion: Eq. (5)-(6) with the terminal value of Eq. (6) (zero unless given);
 *   - tensor backward induction: Algorithm 1 (next-state gather, -inf mask of infeasible
 *     pairs, payoff tensor, max over actions, expectation).
 * This library generalises the expectation of Algorithm 1 from independent price samples
 * to a Markov chain with per-stage transition matrices P_t (the independent case is the
 * special case where every row of P_t is the next stage's probability vector).
 *
 * Indexing (0-based): stage t = 1..T is array slice t-1; price state k in [0, K);
 * state-of-charge index s in [0, S) meaning energy s * delta.  A move to next index j
 * is feasible iff max(0, s - w_down) <= j <= min(S - 1, s + w_up).  It sells
 *   g(d) = -d * delta / eta_c   (d = j - s > 0, charging),
 *   g(d) = -d * delta * eta_d   (d < 0, discharging),   g(0) = 0    [MWh]
 * and earns r(lambda, d) = lambda * g(d) - c_deg * |g(d)| - c_start * [d != 0]  [$].
 * For every stage, price state k and index s the library computes
 *   W_t[k][j] = sum_{k'} P_t[k][k'] * V_{t+1}[k'][j]                  (expectation),
 *   V_t[k][s] = max_{feasible j} r(lam_t[k], j - s) + W_t[k][j]        (Bellman max),
 *   policy_t[k][s] = smallest j attaining the max                    (argmax),
 * in FP32 arithmetic with FP32 accumulation.
 *
 * Memory: every array argument is DEVICE memory owned by the caller unless stated
 * otherwise; arrays are dense, row-major, with the shapes given below.  The library
 * never frees caller memory.  Calls are asynchronous on the given HIP stream (a
 * hipStream_t passed as void*, NULL = the null stream); device faults surface at the
 * next synchronisation.  Return value: DP_OK or a negative DP_E* code; dp_last_error()
 * gives a thread-local description of the last failure.  No exception or abort crosses
 * this interface.
 */
#ifndef DPGPU_H
#define DPGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPGPU_ABI_VERSION 1

/* Error codes. */
#define DP_OK        0
#define DP_EINVAL   -1   /* bad dimension, pointer or parameter (checked on the host)   */
#define DP_EBADPROB -2   /* transition rows not stochastic (only with DP_VALIDATE)       */
#define DP_ENOWS    -3   /* workspace missing or smaller than the *_workspace_bytes()    */
#define DP_EHIP     -4   /* a HIP runtime call failed                                    */
#define DP_ETIMEOUT -5   /* reserved (no call of this version returns it)                 */
#define DP_ENOMEM   -6   /* host allocation failed (plans only)                          */
#define DP_ENOTSUP  -7   /* valid request outside what this library supports             */

/* Limits. */
#define DP_MAX_S 32767   /* next-state indices are stored as int16                       */
#define DP_MAX_K 1024

/* Flags of dp_problem.flags. */
#define DP_STORE_V_ALL 0x1u  /* V output holds all stages [T+1][K][S] (else V_1 [K][S])   */
#define DP_VALIDATE    0x2u  /* check P >= 0 and |row sum - 1| <= 1e-6 (and, in dp_adjoint,
                                that every given policy entry is a feasible next state)
                                before any other device work; synchronises the stream   */

/* Battery on the state-of-charge grid (Sec. III-A): S points 0, delta, ..., (S-1) delta;
 * per-stage move limits w_up (charging) and w_down (discharging) in grid steps. */
typedef struct dp_storage {
    int32_t S;        /* 2 .. DP_MAX_S                                              */
    int32_t w_up;     /* >= 0                                                       */
    int32_t w_down;   /* >= 0                                                       */
    int32_t reserved; /* must be 0                                                  */
    float delta;      /* MWh per grid step, > 0                                     */
    float eta_c;      /* charging efficiency, (0, 1]                                */
    float eta_d;      /* discharging efficiency, (0, 1]                             */
    float c_deg;      /* $ per MWh of grid-side throughput |g|, >= 0                */
    float c_start;    /* $ per stage with a non-zero move, >= 0                     */
} dp_storage;

typedef struct dp_problem {
    int32_t T;           /* stages, >= 1                                           */
    int32_t K;           /* price states, 1 .. DP_MAX_K                            */
    dp_storage st;
    uint32_t flags;      /* DP_STORE_V_ALL | DP_VALIDATE                           */
    int32_t ckpt_every;  /* stages between value checkpoints (>= 1); used by
                            dp_ckpt_bytes / dp_solve(ckpt != NULL) / dp_adjoint     */
} dp_problem;

int dp_abi_version(void);
const char *dp_strerror(int code);
const char *dp_last_error(void);

/* Tuning hook: force the Bellman-sweep tile shape for later solves in this process --
 * `tile` SoC indices per block (a multiple of 64, 64..1024) on `waves` waves (1, 2, 4 or
 * 8).  tile = 0 restores the built-in choice.  The shape never changes results: every
 * shape yields bitwise the same values and policies.  DP_EINVAL for a shape this library
 * has no kernel for; a later solve whose move window does not fit the forced shape's LDS
 * returns DP_ENOTSUP.  Not thread-safe with concurrent solves. */
int dp_set_sweep_shape(int tile, int waves);

/* Measurement hook: while on (1, or 2 for events created without the system-scope
 * fence), dp_solve records a pair of HIP events on its stream around
 * every stage launch (the Bellman sweep with its fused expectation; the expectation count
 * stays 0).  dp_get_timing waits for the
 * recorded events, returns the summed elapsed milliseconds and launch counts of each
 * kind since the last call (or since dp_set_timing), and resets the record.  Host-side
 * state of this process; not thread-safe with concurrent solves. */
int dp_set_timing(int on);
int dp_get_timing(double *sweep_ms, int *n_sweep, double *expect_ms, int *n_expect);

/* Bytes of device workspace dp_solve needs (0 on invalid input). */
size_t dp_workspace_bytes(const dp_problem *pb);

/* Bytes of the checkpoint buffer: the solver's internal value state (FP32 values
 * relative to an FP64 per-stage offset) at stages 1 + m * ckpt_every, m >= 1, that
 * lie in [2, T].  Opaque layout; only dp_adjoint reads it. */
size_t dp_ckpt_bytes(const dp_problem *pb);

/* Backward induction t = T..1 (Eq. (5)-(6), Algorithm 1 with a Markov expectation).
 *   lam     [T][K]     price level of state k at stage t ($/MWh)
 *   P       [T][K][K]  P_t[k][k'] = Pr(state k' at t+1 | state k at t); rows are used as
 *                      given (a row summing to 1 + e weights the continuation by 1 + e);
 *                      entries >= 0 and row sums within 1e-5 of 1 are assumed by
 *                      dp_adjoint's fixed-point accumulator, and checked with DP_VALIDATE
 *   v_term  [K][S]     value of ending in (k, s) after stage T; NULL means 0
 *   V       out: [T+1][K][S] (DP_STORE_V_ALL; slice T is v_term) or [K][S] (V_1 only)
 *   policy  out: [T][K][S] int16 next-state index j, or NULL
 *   ckpt    out: dp_ckpt_bytes(pb) bytes for a later dp_adjoint, or NULL
 *   ws      workspace of at least dp_workspace_bytes(pb) bytes, 256-byte aligned
 * Errors (all checked on the host before any device work, except DP_EBADPROB and DP_EHIP):
 * DP_EINVAL (bad dimension, parameter or pointer), DP_ENOWS, DP_ENOTSUP (a move window
 * w_up + w_down + 1 wider than the LDS of any sweep tile holds, about 19,800 moves),
 * DP_EBADPROB (DP_VALIDATE found a bad row of P), DP_EHIP. */
int dp_solve(const dp_problem *pb, const float *lam, const float *P, const float *v_term,
             float *V, int16_t *policy, void *ckpt, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): dp_solve without the workspace argument.  The
 * solver state lives in a device array inside the library, DP_NOALLOC_SCRATCH_BYTES per GPU,
 * held from the library's first use on that GPU until the process ends; the call allocates
 * nothing.  Arguments and results as dp_solve (bitwise the same values and policies).
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU (concurrent
 * streams, threads, processes sharing a device context) race and must be ordered by the
 * caller; the array needs no clearing between calls.
 * Errors: as dp_solve, plus DP_ENOTSUP when the problem's solver state exceeds the array
 * (about 3 K S_pad 4 bytes + 8 (T + 2) bytes + repacked rows of P; S_pad = S rounded up to
 * 64), and DP_EINVAL with DP_VALIDATE (validation reads a flag back to the host). */
#define DP_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int dp_solve_noalloc(const dp_problem *pb, const float *lam, const float *P,
                     const float *v_term, float *V, int16_t *policy, void *ckpt, void *stream);

/* Bytes of device workspace dp_adjoint needs. */
size_t dp_adjoint_workspace_bytes(const dp_problem *pb);

/* Adjoint of J = sum_{k,s} seed[k][s] V_1[k][s] for the policies of the forward solve
 * (exact wherever the argmax is unique).  Runs forward in time: the occupation measure
 * mu_1 = seed is pushed through the stored policy of each stage, then through P_t:
 *   grad_lam[t][k]   = sum_s mu_t[k][s] g(policy_t[k][s] - s)
 *   nu_t[k][j]       = sum_{s: policy_t[k][s] = j} mu_t[k][s]
 *   grad_P[t][k][k'] = sum_j nu_t[k][j] V_{t+1}[k'][j]
 *   mu_{t+1}         = P_t^T nu_t ;   grad_vterm = mu_{T+1}.
 * Inputs: either (V_all [T+1][K][S] and policy [T][K][S]) from dp_solve with
 * DP_STORE_V_ALL, or ckpt from dp_solve(ckpt != NULL) with V_all = policy = NULL, in
 * which case every segment of ckpt_every stages is recomputed from its checkpoint
 * (bitwise the same values and policies as the forward solve).
 *   seed [K][S]; outputs grad_lam [T][K], grad_P [T][K][K], grad_vterm [K][S] (or NULL).
 * With ckpt, the re-solve of each segment runs on a library-owned stream of the current
 * device (one per device, created on first use), overlapping the adjoint of the previous
 * segment; it is forked from and joined back into `stream` with events, and calls from
 * several threads are ordered on it.
 * Errors: as dp_solve; with DP_VALIDATE in pb->flags also DP_EBADPROB (a bad row of P)
 * and DP_EINVAL (a caller-given policy entry outside the feasible move window).  Without
 * DP_VALIDATE a policy entry outside [0, S) moves no mass (it is never used as an
 * address); other infeasible entries give the gradient of that (infeasible) policy. */
int dp_adjoint(const dp_problem *pb, const float *lam, const float *P, const float *v_term,
               const float *V_all, const int16_t *policy, const void *ckpt,
               const float *seed, float *grad_lam, float *grad_P, float *grad_vterm,
               void *ws, size_t ws_bytes, void *stream);

/* ---- Stagewise-independent prices on the paper's power-action grid ------------------
 * The model of Sec. II-B solved exactly as Algorithm 1 prints it: at each stage t the price
 * takes R sampled levels lam[t][r] with probabilities prob[t][r] (sum 1), independent of
 * the past; the actions are the recombining power grid of Sec. III-A,
 *   p_hat = [-p_bar, -(n_c-1) delta/eta, ..., -delta/eta, 0, delta eta, ..., (n_d-1) delta eta, p_bar],
 *   n_c = ceil(p_bar eta / delta), n_d = ceil(p_bar / (delta eta)), P = n_c + n_d + 1,
 * whose interior entries move the state of charge by whole grid steps and whose two
 * endpoints are interpolated between the neighbouring grid values (Algorithm 1's next-state
 * proxies, floor/ceil indices and interpolation factors, computed in FP64); pairs leaving
 * [0, s_bar] are infeasible.  Payoff lam p (no costs).  For t = T..1:
 *   Q_{t-1}(s, r) = max_p lam[t][r] p + V_t(s + F(p)),  V_{t-1}(s) = sum_r prob[t][r] Q_{t-1}(s, r),
 * with V_T = 0.  FP32 arithmetic, same device-memory and stream conventions as above. */
typedef struct dp_iid_problem {
    int32_t T;           /* stages, >= 1                                                 */
    int32_t R;           /* price samples per stage, 1 .. 4096                           */
    int32_t S;           /* SoC grid points 0, delta, ..., (S-1) delta; 2 .. DP_MAX_S   */
    int32_t reserved;    /* must be 0                                                    */
    float delta;         /* MWh per grid step, > 0                                       */
    float eta;           /* one-way efficiency, (0, 1]                                   */
    float p_bar;         /* power capacity (MWh per stage), > 0                          */
    uint32_t flags;      /* DP_STORE_V_ALL                                               */
} dp_iid_problem;

/* Action-grid sizes of the problem (host only, no GPU use). */
int dp_iid_action_grid(const dp_iid_problem *pb, int *P, int *n_c, int *n_d);
size_t dp_iid_workspace_bytes(const dp_iid_problem *pb);
/*   lam, prob [T][R]; V out: [T+1][S] (DP_STORE_V_ALL; slice t is V_t, slice T is 0) or
 *   [S] (V_0 only); policy [T][R][S] int16 index into p_hat (ascending power) of the
 *   chosen action at stage t (slice t-1), ties to the smallest next state, or NULL. */
int dp_solve_iid(const dp_iid_problem *pb, const float *lam, const float *prob, float *V,
                 int16_t *policy, void *ws, size_t ws_bytes, void *stream);

/* Batched solves of many independent instances (not in the paper; Sec. V's duration sweeps
 * are such batches).  All instances advance stage-synchronously: batch stage tau puts
 * instance i at its own stage T_i - tau + 1.  Instances are grouped by expectation kernel
 * (K <= 32, <= 64, two alternating halves of K <= 128, and K > 128); each group is one
 * stream of launches (per tau, one expectation launch, then one sweep launch per tile
 * class that has instances in the group), and the groups run concurrently.
 * A plan owns the device descriptor table, the work tables, its device workspace (one
 * solver region per instance) and a HIP graph of the whole launch sequence, captured once
 * at creation; it is created for a fixed list of problems (host array probs[n], flags must
 * be 0, ckpt_every ignored) and replayed with new data.
 * tune_cache: path of a text cache of autotuned sweep tile shapes (created or extended;
 * the fastest shape per move-span class, timed at creation), or NULL to use the built-in
 * shapes without tuning (one- and two-wave tiles for move spans up to 256, four waves up
 * to 512, the single solve's choice beyond).
 * stream: the set-up's device work (zeroing the workspace, uploading the work tables,
 * timing the candidate shapes) is issued on this stream, after its pending work; the call
 * synchronises it before returning, so the plan is ready when the call returns.
 * Errors: DP_EINVAL (bad problem or pointer), DP_ENOTSUP (a move window wider than the LDS
 * of any sweep tile holds), DP_ENOMEM, DP_EHIP.  The plan must be destroyed with
 * dp_batch_plan_destroy. */
typedef struct dp_batch_plan dp_batch_plan;

int dp_batch_plan_create(dp_batch_plan **out, int n, const dp_problem *probs,
                         const char *tune_cache, void *stream);

/* Solve every instance i: lam[i] [T_i][K_i], P[i] [T_i][K_i][K_i] (device pointers held
 * in HOST arrays of length n), outputs V1[i] [K_i][S_i] and policy[i] [T_i][K_i][S_i]
 * (policy may be NULL, or an array with a pointer for every instance).  Terminal values
 * are zero.  Each call copies the pointers into the device descriptor table (from a pinned
 * staging buffer, asynchronously on `stream`) and replays the graph on `stream`, so new
 * pointers need no re-capture.  Results are bitwise those of dp_batch_solve_looped.
 * Calls on one plan must be ordered: issue them on one stream, or synchronise between
 * them, since every call rewrites the same descriptor table and workspace. */
int dp_batch_solve(dp_batch_plan *plan, const float *const *lam, const float *const *P,
                   float *const *V1, int16_t *const *policy, void *stream);

/* The same launches as dp_batch_solve, issued directly instead of replaying the graph:
 * the group streams are forked from `stream` with events and joined back into it.  For
 * measuring what the graph saves; results are bitwise those of dp_batch_solve.  The same
 * ordering rule holds. */
int dp_batch_solve_eager(dp_batch_plan *plan, const float *const *lam, const float *const *P,
                         float *const *V1, int16_t *const *policy, void *stream);

/* Same batch, one ordinary dp_solve per instance on the stream (for comparison). */
int dp_batch_solve_looped(dp_batch_plan *plan, const float *const *lam,
                          const float *const *P, float *const *V1,
                          int16_t *const *policy, void *stream);

/* Description of the plan's tile choices: writes a NUL-terminated text into buf. */
int dp_batch_plan_describe(const dp_batch_plan *plan, char *buf, size_t len);

void dp_batch_plan_destroy(dp_batch_plan *plan);

#ifdef __cplusplus
}
#endif
#endif /* DPGPU_H */
