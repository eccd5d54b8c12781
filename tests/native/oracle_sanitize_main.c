/*
 * Runs the FP64 oracle's entry points on small random problems, for a build with the
 * address and undefined-behaviour sanitizers (the sanitizers report any out-of-bounds
 * access, use after free or undefined arithmetic).  Also checks a few properties that
 * hold for any input: finite values, policies inside the feasible move window, the
 * adjoint's mass conservation under row-stochastic transitions, and the value of the
 * returned policies equal to the solve's values.  Exit status 0 when all hold.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_solve(int T, int K, int S, int w_up, int w_down, double delta, double eta_c,
                 double eta_d, double c_deg, double c_start, const float *lam, const float *P,
                 const double *v_term, double *V_all, double *V1, int16_t *pol, int nthreads);
int oracle_adjoint(int T, int K, int S, int w_up, int w_down, double delta, double eta_c,
                   double eta_d, double c_deg, double c_start, const float *lam,
                   const float *P, const double *V_all, const int16_t *pol,
                   const double *seed, double *grad_lam, double *grad_P,
                   double *grad_vterm, int nthreads);
int oracle_policy_value(int T, int K, int S, int w_up, int w_down, double delta,
                        double eta_c, double eta_d, double c_deg, double c_start,
                        const float *lam, const float *P, const double *v_term,
                        const int16_t *pol, double *V1);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double urand(void)   /* xorshift64*, uniform in [0, 1) */
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (double)((rng_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static int run_case(int T, int K, int S, int wu, int wd, double c_start)
{
    size_t KS = (size_t)K * S;
    float *lam = malloc(sizeof(float) * T * K);
    float *P = malloc(sizeof(float) * T * K * K);
    double *V = malloc(sizeof(double) * (T + 1) * KS), *V1 = malloc(sizeof(double) * KS);
    double *Vp = malloc(sizeof(double) * KS), *seed = malloc(sizeof(double) * KS);
    int16_t *pol = malloc(sizeof(int16_t) * T * KS);
    double *gl = malloc(sizeof(double) * T * K), *gP = malloc(sizeof(double) * T * K * K);
    double *gv = malloc(sizeof(double) * KS);
    for (int i = 0; i < T * K; ++i) lam[i] = (float)(urand() * 100.0 - 20.0);
    /* rows on the 2^-24 grid summing to exactly 1: K - 1 random numerators, the last row
       entry takes the rest */
    for (int r = 0; r < T * K; ++r) {
        long left = 1L << 24;
        for (int c = 0; c < K; ++c) {
            long n = c + 1 < K ? (long)(urand() * (double)left / (K - c)) : left;
            left -= n;
            P[(size_t)r * K + c] = (float)((double)n / 16777216.0);
        }
    }
    double mass = 0.0;
    for (size_t i = 0; i < KS; ++i) mass += (seed[i] = urand());
    int bad = 0;
    bad |= oracle_solve(T, K, S, wu, wd, 0.25, 0.9, 0.92, 1.0, c_start, lam, P, NULL, V, V1, pol, 2);
    for (size_t i = 0; i < (size_t)(T + 1) * KS; ++i) bad |= !isfinite(V[i]);
    for (int t = 0; t < T; ++t)
        for (int k = 0; k < K; ++k)
            for (int s = 0; s < S; ++s) {
                int j = pol[((size_t)t * K + k) * S + s];
                bad |= j < (s - wd < 0 ? 0 : s - wd) || j > (s + wu > S - 1 ? S - 1 : s + wu);
            }
    bad |= oracle_policy_value(T, K, S, wu, wd, 0.25, 0.9, 0.92, 1.0, c_start, lam, P, NULL, pol, Vp);
    for (size_t i = 0; i < KS; ++i) bad |= fabs(Vp[i] - V1[i]) > 1e-9 * (1.0 + fabs(V1[i]));
    bad |= oracle_adjoint(T, K, S, wu, wd, 0.25, 0.9, 0.92, 1.0, c_start, lam, P, V, pol, seed, gl, gP, gv, 2);
    double m2 = 0.0;
    for (size_t i = 0; i < KS; ++i) m2 += gv[i];
    bad |= fabs(m2 - mass) > 1e-9 * mass;
    free(lam); free(P); free(V); free(V1); free(Vp); free(seed); free(pol); free(gl); free(gP); free(gv);
    if (bad) fprintf(stderr, "case T=%d K=%d S=%d w=%d/%d failed\n", T, K, S, wu, wd);
    return bad;
}

int main(void)
{
    int bad = 0;
    bad |= run_case(3, 2, 2, 1, 1, 0.0);
    bad |= run_case(5, 3, 7, 2, 3, 1.0);
    bad |= run_case(4, 5, 40, 0, 0, 0.0);
    bad |= run_case(6, 7, 129, 128, 128, 0.5);
    bad |= run_case(2, 1, 300, 20, 35, 2.0);
    printf(bad ? "FAILED\n" : "ok\n");
    return bad;
}
