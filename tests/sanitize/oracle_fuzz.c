/* Drives the oracle (oracle/pic_oracle.c) over small runs of every scheme and every entry
 * point the tests use -- tiny particle counts, the smallest grids, fast particles crossing
 * several cells, imposed magnetic fields -- built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitizers.py. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nv, scheme, order, n_cells;
    int64_t n_particles;
    double length, dt, c, b_ext[3];
    int32_t cc, pad;
} ocfg;

typedef struct {
    double kinetic, field_e, field_b, total, max_gamma_dev;
    int64_t fallbacks;
    int32_t nonfinite, pad;
} odiag;

int oracle_run_gamma(const ocfg *, double *, double *, const double *, double *, double *,
                     int64_t, int, odiag *, double *);
int oracle_std_run(const ocfg *, double *, double *, const double *, double *, int64_t, int,
                   int, odiag *);
int oracle_tlm_run(const ocfg *, double *, double *, const double *, double *, int64_t, int,
                   double, int, double *, double *, double *, double *, double *, odiag *);
void oracle_cn_solve(int, double, double, const double *, double *);
void oracle_binomial(int, const double *, double *);

static double urand(uint64_t *s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return ((*s >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

int main(void)
{
    uint64_t seed = 7;
    int runs = 0;
    const int64_t nps[] = {1, 2, 5, 64, 301};
    const int ngs[] = {3, 4, 5, 8, 17};
    for (int ip = 0; ip < 5; ++ip)
        for (int ig = 0; ig < 5; ++ig)
            for (int order = 1; order <= 2; ++order)
                for (int scheme = 0; scheme <= 5; ++scheme) {
                    const int64_t np = nps[ip];
                    const int ng = ngs[ig];
                    if (ng < 2 * order + 1)
                        continue;
                    const int em = scheme == 2 || scheme >= 4;
                    const int nv = (em || (ip + ig) % 2) ? 3 : 1;
                    ocfg c = {nv, scheme == 3 ? 0 : scheme, order, ng, np, 5.0, 0.3, 1.0,
                              {0.0, 0.0, 0.0}};
                    if (nv == 3) {
                        c.b_ext[0] = 0.3;
                        c.b_ext[2] = -0.7;
                    }
                    /* exact charge conservation on the electrostatic tent runs */
                    c.cc = (scheme <= 1 && order == 1 && (ip + ig) % 3 == 0) ? 1 : 0;
                    double *x = malloc(sizeof(double) * np), *v = malloc(sizeof(double) * 3 * np);
                    double *w = malloc(sizeof(double) * np);
                    double E[3 * 17] = {0}, B[2 * 17] = {0}, g[301];
                    for (int64_t p = 0; p < np; ++p) {
                        x[p] = 15.0 * urand(&seed) - 5.0;         /* outside [0, L) too */
                        for (int k = 0; k < nv; ++k)
                            v[k * np + p] = 8.0 * (urand(&seed) - 0.5);
                        w[p] = 5.0 / np * (0.5 + urand(&seed));
                    }
                    for (int i = 0; i < ng; ++i)
                        B[ng + i] = 0.1 * sin(i);
                    odiag rec[7];
                    int rc;
                    if (scheme == 3)
                        rc = oracle_std_run(&c, x, v, w, E, 6, ip % 2, 1, rec);
                    else
                        rc = oracle_run_gamma(&c, x, v, (ip % 2) ? w : NULL, E, B, 6,
                                              !em, rec, np <= 301 ? g : NULL);
                    if (rc != 0) {
                        printf("FAILED: oracle rejected scheme %d np %lld ng %d\n", scheme,
                               (long long)np, ng);
                        return 1;
                    }
                    if (scheme == 0 && nv == 1 && !c.cc) {
                        double dx[2 * 301], dv[2 * 301], dE[2 * 17], J, dJ[2];
                        for (int64_t p = 0; p < 2 * np; ++p) {
                            dx[p] = urand(&seed);
                            dv[p] = urand(&seed);
                        }
                        rc = oracle_tlm_run(&c, x, v, NULL, E, 4, 1, 0.3, 2, dx, dv, dE, &J, dJ, rec);
                        if (rc != 0)
                            return 1;
                    }
                    free(x); free(v); free(w);
                    ++runs;
                }
    double r[17], y[17];
    for (int i = 0; i < 17; ++i)
        r[i] = urand(&seed);
    oracle_cn_solve(17, 0.3, 0.01, r, y);
    oracle_binomial(17, r, y);
    printf("ok: %d oracle runs\n", runs);
    return 0;
}
