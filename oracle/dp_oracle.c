/*
 * FP64 reference for the Markov-chain storage-arbitrage DP.  TEST INFRASTRUCTURE ONLY:
 * only the test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load this library.  It shares no code, header or table with the HIP path.
 *
 * What it computes (the plain definition, written out with loops):
 *
 *   Payoff (Sec. II-A, Eq. (1a) objective lambda_t p_t and Eq. (2) state transition F):
 *     a move of d = j - s grid steps sells g(d) MWh to the grid,
 *       g(d) = -d delta / eta_c  (d > 0, charging: the grid supplies d delta / eta_c),
 *       g(d) = -d delta eta_d    (d < 0, discharging: the grid receives |d| delta eta_d),
 *       g(0) = 0,
 *     and earns r(lambda, d) = lambda g(d) - c_deg |g(d)| - c_start [d != 0].
 *   Feasible moves (Eq. (4), on the recombining grid of Sec. III-A):
 *     j in J(s) = [max(0, s - W_d), min(S - 1, s + W_c)].
 *   Bellman recursion (Eq. (5)-(6), generalised from stagewise independence to a
 *   Markov price chain whose state k is observed before acting):
 *     V_{T+1} = terminal value (0 by default, the base case of Eq. (6)),
 *     W_t[k][j]  = sum_{k'} P_t[k][k'] V_{t+1}[k'][j]        (conditional expectation),
 *     V_t[k][s]  = max_{j in J(s)} r(lambda_t[k], j - s) + W_t[k][j],
 *     pi_t[k][s] = the smallest j attaining that maximum.
 *   With every row of P_t equal to the next stage's probability vector this reduces
 *   to Algorithm 1 (Markov state = the sampled price), which the tests check.
 *
 *   Adjoint of J = sum_{k,s} Omega[k][s] V_1[k][s] for fixed policies (exact wherever
 *   the argmax is unique):  mu_1 = Omega;  for t = 1..T
 *     grad_lam_t[k]   = sum_s mu_t[k][s] g(pi_t[k][s] - s),
 *     nu_t[k][j]      = sum_{s : pi_t[k][s] = j} mu_t[k][s],
 *     grad_P_t[k][k'] = sum_j nu_t[k][j] V_{t+1}[k'][j],
 *     mu_{t+1}[k'][j] = sum_k P_t[k][k'] nu_t[k][j];
 *   grad of the terminal value = mu_{T+1}.
 *
 * Layout: lam [T][K], P [T][K][K] (row = from-state), values [K][S] per stage,
 * policies int16 [T][K][S] holding the next SoC index j.  All inputs arrive as FP32
 * (the values the GPU also consumes) and are widened exactly to FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int S, w_up, w_down;
    double delta, eta_c, eta_d, c_deg, c_start;
} ostore;

static double g_move(const ostore *st, int d)
{
    if (d > 0) return -(double)d * st->delta / st->eta_c;
    if (d < 0) return -(double)d * st->delta * st->eta_d;
    return 0.0;
}

static double reward(const ostore *st, double lam, int d)
{
    double g = g_move(st, d);
    return lam * g - st->c_deg * fabs(g) - (d != 0 ? st->c_start : 0.0);
}

static ostore mk(int S, int w_up, int w_down, double delta, double eta_c, double eta_d,
                 double c_deg, double c_start)
{
    ostore st = {S, w_up, w_down, delta, eta_c, eta_d, c_deg, c_start};
    return st;
}

static void set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* One Bellman stage.  Vnext [K][S] -> W [K][S] (may be NULL), Vt [K][S], pol [K][S]
 * (may be NULL).  lam_t [K] and P_t [K][K] are FP32 inputs. */
int oracle_stage(int K, int S, int w_up, int w_down, double delta, double eta_c,
                 double eta_d, double c_deg, double c_start, const float *lam_t,
                 const float *P_t, const double *Vnext, double *W, double *Vt,
                 int16_t *pol, int nthreads)
{
    ostore st = mk(S, w_up, w_down, delta, eta_c, eta_d, c_deg, c_start);
    set_threads(nthreads);
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < K; ++k) {
        double *w = (double *)malloc(sizeof(double) * (size_t)S);
        for (int j = 0; j < S; ++j) {
            double acc = 0.0;
            for (int kp = 0; kp < K; ++kp)
                acc += (double)P_t[(size_t)k * K + kp] * Vnext[(size_t)kp * S + j];
            w[j] = acc;
        }
        double lam = (double)lam_t[k];
        for (int s = 0; s < S; ++s) {
            int jlo = s - w_down < 0 ? 0 : s - w_down;
            int jhi = s + w_up > S - 1 ? S - 1 : s + w_up;
            double best = -INFINITY;
            int arg = -1;
            for (int j = jlo; j <= jhi; ++j) {
                double q = reward(&st, lam, j - s) + w[j];
                if (q > best) { best = q; arg = j; }
            }
            Vt[(size_t)k * S + s] = best;
            if (pol) pol[(size_t)k * S + s] = (int16_t)arg;
        }
        if (W) memcpy(W + (size_t)k * S, w, sizeof(double) * (size_t)S);
        free(w);
    }
    return 0;
}

/* Whole backward induction.  V_all [(T+1)][K][S] (may be NULL: then only two rolling
 * buffers are held), V1 [K][S] (always written), pol [T][K][S] (may be NULL),
 * v_term [K][S] (NULL means zero). */
int oracle_solve(int T, int K, int S, int w_up, int w_down, double delta, double eta_c,
                 double eta_d, double c_deg, double c_start, const float *lam,
                 const float *P, const double *v_term, double *V_all, double *V1,
                 int16_t *pol, int nthreads)
{
    size_t KS = (size_t)K * S;
    double *a = (double *)calloc(KS, sizeof(double));
    double *b = (double *)calloc(KS, sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    if (v_term) memcpy(a, v_term, KS * sizeof(double));
    if (V_all) memcpy(V_all + (size_t)T * KS, a, KS * sizeof(double));
    for (int t = T; t >= 1; --t) {          /* stage t uses lam_t, P_t (0-based t-1) */
        const float *lam_t = lam + (size_t)(t - 1) * K;
        const float *P_t = P + (size_t)(t - 1) * K * K;
        int16_t *pol_t = pol ? pol + (size_t)(t - 1) * KS : NULL;
        oracle_stage(K, S, w_up, w_down, delta, eta_c, eta_d, c_deg, c_start, lam_t, P_t,
                     a, NULL, b, pol_t, nthreads);
        if (V_all) memcpy(V_all + (size_t)(t - 1) * KS, b, KS * sizeof(double));
        double *tmp = a; a = b; b = tmp;
    }
    memcpy(V1, a, KS * sizeof(double));
    free(a);
    free(b);
    return 0;
}

/* Adjoint for fixed policies.  V_all [(T+1)][K][S] FP64 values (V_{t+1} is used at
 * stage t), pol [T][K][S], seed [K][S].  Outputs grad_lam [T][K], grad_P [T][K][K],
 * grad_vterm [K][S] (may be NULL). */
int oracle_adjoint(int T, int K, int S, int w_up, int w_down, double delta, double eta_c,
                   double eta_d, double c_deg, double c_start, const float *lam,
                   const float *P, const double *V_all, const int16_t *pol,
                   const double *seed, double *grad_lam, double *grad_P,
                   double *grad_vterm, int nthreads)
{
    (void)lam;
    ostore st = mk(S, w_up, w_down, delta, eta_c, eta_d, c_deg, c_start);
    size_t KS = (size_t)K * S;
    double *mu = (double *)malloc(KS * sizeof(double));
    double *nu = (double *)malloc(KS * sizeof(double));
    if (!mu || !nu) { free(mu); free(nu); return -1; }
    memcpy(mu, seed, KS * sizeof(double));
    set_threads(nthreads);
    for (int t = 1; t <= T; ++t) {
        const int16_t *pt = pol + (size_t)(t - 1) * KS;
        const float *Pt = P + (size_t)(t - 1) * K * K;
        const double *Vn = V_all + (size_t)t * KS;     /* V_{t+1} */
        int k;
#pragma omp parallel for schedule(static)
        for (k = 0; k < K; ++k) {
            double gl = 0.0;
            for (int j = 0; j < S; ++j) nu[(size_t)k * S + j] = 0.0;
            for (int s = 0; s < S; ++s) {              /* ascending s: fixed order */
                int j = pt[(size_t)k * S + s];
                double m = mu[(size_t)k * S + s];
                gl += m * g_move(&st, j - s);
                nu[(size_t)k * S + j] += m;
            }
            grad_lam[(size_t)(t - 1) * K + k] = gl;
        }
#pragma omp parallel for schedule(static)
        for (k = 0; k < K; ++k) {
            for (int kp = 0; kp < K; ++kp) {
                double acc = 0.0;
                for (int j = 0; j < S; ++j) acc += nu[(size_t)k * S + j] * Vn[(size_t)kp * S + j];
                grad_P[((size_t)(t - 1) * K + k) * K + kp] = acc;
            }
        }
        int kp;
#pragma omp parallel for schedule(static)
        for (kp = 0; kp < K; ++kp) {
            for (int j = 0; j < S; ++j) {
                double acc = 0.0;
                for (int kk = 0; kk < K; ++kk)
                    acc += (double)Pt[(size_t)kk * K + kp] * nu[(size_t)kk * S + j];
                mu[(size_t)kp * S + j] = acc;
            }
        }
    }
    if (grad_vterm) memcpy(grad_vterm, mu, KS * sizeof(double));
    free(mu);
    free(nu);
    return 0;
}

/* Objective of a fixed policy set: J = sum Omega V^pi_1 where V^pi is evaluated by
 * backward policy evaluation (no maximisation).  Used to check that the adjoint is
 * the derivative of the value of the *policy*. */
int oracle_policy_value(int T, int K, int S, int w_up, int w_down, double delta,
                        double eta_c, double eta_d, double c_deg, double c_start,
                        const float *lam, const float *P, const double *v_term,
                        const int16_t *pol, double *V1)
{
    ostore st = mk(S, w_up, w_down, delta, eta_c, eta_d, c_deg, c_start);
    size_t KS = (size_t)K * S;
    double *a = (double *)calloc(KS, sizeof(double));
    double *b = (double *)calloc(KS, sizeof(double));
    double *w = (double *)malloc((size_t)S * sizeof(double));
    if (!a || !b || !w) { free(a); free(b); free(w); return -1; }
    if (v_term) memcpy(a, v_term, KS * sizeof(double));
    for (int t = T; t >= 1; --t) {
        const float *Pt = P + (size_t)(t - 1) * K * K;
        const int16_t *pt = pol + (size_t)(t - 1) * KS;
        for (int k = 0; k < K; ++k) {
            for (int j = 0; j < S; ++j) {
                double acc = 0.0;
                for (int kp = 0; kp < K; ++kp) acc += (double)Pt[(size_t)k * K + kp] * a[(size_t)kp * S + j];
                w[j] = acc;
            }
            double l = (double)lam[(size_t)(t - 1) * K + k];
            for (int s = 0; s < S; ++s) {
                int j = pt[(size_t)k * S + s];
                b[(size_t)k * S + s] = reward(&st, l, j - s) + w[j];
            }
        }
        double *tmp = a; a = b; b = tmp;
    }
    memcpy(V1, a, KS * sizeof(double));
    free(a); free(b); free(w);
    return 0;
}
