/*
 * ORACLE -- test infrastructure, not product code.
 *
 * Exercises every entry of the C oracle on small problems so that a build with the address and
 * undefined-behaviour sanitizers (tests/test_oracle_sanitize.py) checks its memory accesses and
 * arithmetic: couplings of the three geometries, Philox draws, the three ansaetze in Monte Carlo
 * and enumeration mode, the parameter-space, sample-space and SNR solves (real and Hermitian),
 * the eigen-decompositions, and threaded trajectory runs with both schemes and both
 * unravellings.  Exits 0 when every call returned its expected status.
 */
#include "otvmc_oracle.c"

#include <stdio.h>

static int fails = 0;
#define EXPECT(cond)                                                                   \
    do {                                                                               \
        if (!(cond)) {                                                                 \
            fprintf(stderr, "sanitize_driver: %s failed at line %d\n", #cond, __LINE__); \
            ++fails;                                                                   \
        }                                                                              \
    } while (0)

static void one_problem(int n, int kind, int nh_or_d, int ns, int enumerate, int want_solve, int reg)
{
    double *J = calloc((size_t)n * n, sizeof(double));
    EXPECT(orc_couplings(n >= 4 && n % 2 == 0 ? 1 : 0, n, 1, 1.5, 1.0, J) == ORC_OK);
    int32_t kinds[3] = {ORC_SIGMA_MINUS, ORC_SIGMA_PLUS, ORC_SIGMA_Z};
    int32_t sites[3] = {0, n - 1, n / 2};
    double rates[3] = {0.1, 0.05, 0.02};
    orc_problem pb = {n, J, 0.7, 3, kinds, sites, rates};
    orc_ansatz an = {kind, kind == ORC_RBM ? nh_or_d : 0, kind == ORC_LJPH ? nh_or_d : 0};
    int m = orc_n_params(&an, n);
    orc_config cf = {ns, 4, 2, 1, 3, enumerate, 0.01, 1e-3, ORC_HEUN, 2, 1, 5, 0, reg, 4.0};
    double *theta = calloc(2 * (size_t)m, sizeof(double));
    for (int k = 0; k < 2 * m; ++k) theta[k] = 0.03 * ((k * 37 % 11) - 5);
    int8_t *chains = malloc((size_t)4 * n);
    orc_init_chains(5, 0, n, 4, chains);
    double dw[3];
    orc_draw_dw(5, 0, 0, 3, 0.01, dw);
    int nss = enumerate ? (1 << n) : ns;
    int8_t *samples = malloc((size_t)nss * n);
    double *eloc = malloc(sizeof(double) * 2 * nss), *G = malloc(sizeof(double) * 2 * nss);
    size_t sdim = want_solve == 3 ? (size_t)ns : (size_t)m;
    double *S = malloc(sizeof(double) * 2 * sdim * sdim), *F = malloc(sizeof(double) * 2 * m);
    double *Nn = malloc(sizeof(double) * 2 * 3 * m), *D = malloc(sizeof(double) * 2 * m);
    double *bm = malloc(sizeof(double) * 6), *ob = malloc(sizeof(double) * 2 * m);
    double *delta = malloc(sizeof(double) * 2 * m), *eig = malloc(sizeof(double) * 2 * m);
    int64_t acc[4];
    double obs[9], sec[3], dq;
    orc_eval_out out = {samples, eloc, S, F, Nn, D, bm, ob, delta, acc, obs, sec, &dq, eig, G};
    EXPECT(orc_eval(&pb, &an, &cf, theta, chains, 0, 0, 0, 1, dw, want_solve, &out) == ORC_OK);
    cf.n_steps = 2;
    cf.obs_every = 1;
    double *th_out = malloc(sizeof(double) * 2 * (size_t)m * 2), *obs_out = malloc(sizeof(double) * 2 * 3 * 9);
    double lq[2 * 3];
    int32_t st[2];
    if (!enumerate && want_solve == 1) {
        EXPECT(orc_run(&pb, &an, &cf, theta, 2, 0, 2, th_out, obs_out, st, lq) == ORC_OK);
        cf.linear = 1;
        cf.scheme = ORC_MIDPOINT;
        EXPECT(orc_run(&pb, &an, &cf, theta, 2, 0, 2, th_out, obs_out, st, lq) == ORC_OK);
    }
    free(J); free(theta); free(chains); free(samples); free(eloc); free(G); free(S); free(F); free(Nn);
    free(D); free(bm); free(ob); free(delta); free(eig); free(th_out); free(obs_out);
}

int main(void)
{
    uint32_t ctr[4] = {0, 0, 0, 0}, key[2] = {0, 0}, r[4];
    orc_philox(ctr, key, r);
    double J2[16 * 16];
    EXPECT(orc_couplings(2, 4, 4, 3.0, 1.0, J2) == ORC_OK);
    one_problem(6, ORC_JASTROW, 0, 64, 0, 1, ORC_REG_SHIFT);
    one_problem(6, ORC_JASTROW, 0, 64, 1, 1, ORC_REG_SHIFT);
    one_problem(6, ORC_JASTROW, 0, 16, 0, 3, ORC_REG_SHIFT);
    one_problem(6, ORC_JASTROW, 0, 64, 0, 1, ORC_REG_SNR);
    one_problem(5, ORC_RBM, 3, 64, 0, 1, ORC_REG_SHIFT);
    one_problem(5, ORC_RBM, 3, 64, 0, 1, ORC_REG_SNR);
    one_problem(5, ORC_RBM, 4, 16, 0, 3, ORC_REG_SHIFT);
    one_problem(8, ORC_LJPH, 1, 64, 0, 1, ORC_REG_SHIFT);
    one_problem(8, ORC_LJPH, 2, 64, 0, 1, ORC_REG_SNR);
    one_problem(70, ORC_LJPH, 1, 32, 0, 1, ORC_REG_SHIFT);
    double A[9] = {2, 1, 0, 1, 3, 1, 0, 1, 4}, V[9], lam[3];
    EXPECT(orc_eigh_sym(3, A, V, lam) == ORC_OK);
    if (fails) return 1;
    printf("sanitize_driver: ok\n");
    return 0;
}
