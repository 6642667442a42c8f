/* Sanitizer driver for the oracle's brute-force ray march (test
 * infrastructure): compiled together with oracle/bruteforce.c under
 * AddressSanitizer and UndefinedBehaviorSanitizer, it marches a seeded random
 * scene (with and without an environment map, whole grid and a crop, and the
 * argument checks) and prints every fluence so that the test can compare them
 * with the regular build's. */
#include <stdio.h>
#include <stdlib.h>

int bf_fluence_env(int S, const double *eps, const double *sig, int M, int r0, int r1, int c0,
                   int c1, const double *env, int K, double *out);
int bf_fluence(int S, const double *eps, const double *sig, int M, int r0, int r1, int c0,
               int c1, double *out);
double bf_radiance(int S, const double *eps, const double *sig, double px, double py,
                   double dx, double dy);

/* 64-bit linear congruential generator (Knuth's MMIX constants), top 53 bits. */
static unsigned long long lcg_state = 12345u;
static double uniform(void) {
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) / 9007199254740992.0;
}

int main(void) {
    enum { S = 12, M = 96 };
    double *eps = malloc(sizeof(double) * S * S), *sig = malloc(sizeof(double) * S * S);
    double *out = malloc(sizeof(double) * S * S);
    for (int i = 0; i < S * S; ++i) {
        eps[i] = uniform() < 0.3 ? 3.0 * uniform() : 0.0;
        sig[i] = 1.5 * uniform();
    }
    for (int i = 0; i < S * S; ++i) printf("in %d %.17g %.17g\n", i, eps[i], sig[i]);
    const double env[5] = {0.5, 1.0, 1.5, 0.25, 2.0};
    if (bf_fluence(S, eps, sig, M, 0, S, 0, S, out) != 0) return 2;
    for (int i = 0; i < S * S; ++i) printf("plain %d %.17g\n", i, out[i]);
    if (bf_fluence_env(S, eps, sig, M, 2, 7, 3, 11, env, 5, out) != 0) return 3;
    for (int i = 0; i < 5 * 8; ++i) printf("env %d %.17g\n", i, out[i]);
    printf("ray %.17g\n", bf_radiance(S, eps, sig, 0.5, 0.5, 0.6, 0.8));
    /* rejected arguments return -1 and touch nothing */
    if (bf_fluence(S, eps, sig, M, 0, S + 1, 0, S, out) != -1) return 4;
    if (bf_fluence(S, eps, sig, 0, 0, S, 0, S, out) != -1) return 5;
    if (bf_fluence_env(S, eps, sig, M, 0, S, 0, S, NULL, 3, out) != -1) return 6;
    free(eps);
    free(sig);
    free(out);
    return 0;
}
