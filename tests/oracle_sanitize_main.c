/*
 * Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * oracle (test infrastructure only; built and run by
 * tests/test_oracle_sanitizers.py with gcc on the host).  It calls every
 * oracle function on small lattices, including the boundary sizes (L = 1, 2,
 * odd L, all images), so that an out-of-bounds access, a use of freed memory
 * or undefined arithmetic in the oracle aborts the run.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

static void fill(int L, uint64_t seed, double *s) { orc_init_spins(L, seed, 0, s); }

int main(void)
{
    const int sizes[] = {1, 2, 3, 4, 6, 8};
    for (unsigned k = 0; k < sizeof sizes / sizeof sizes[0]; ++k) {
        const int L = sizes[k];
        const long N = (long)L * L;
        double *W = calloc(4 * N, sizeof(double)), *We = calloc(4 * N, sizeof(double));
        double *s = calloc(3 * N, sizeof(double)), *h = calloc(3 * N, sizeof(double));
        double *h2 = calloc(3 * N, sizeof(double)), *acc = calloc(N, sizeof(double));
        double *dE = calloc(N, sizeof(double)), *u2 = calloc(N, sizeof(double)), *S = calloc(3 * N, sizeof(double));
        double out[ORC_NOBS], parts[4], hs[3], var[3];
        orc_params p = {0.7, 1.0, 1.5, -0.5, 0.2, 11u, 3u, 0u};
        orc_lattice_sum_kernel(L, 2, W);
        orc_lattice_sum_ewald(L, L / 4.0 > 0.5 ? L / 4.0 : 0.5, We);
        fill(L, 5, s);
        orc_field(L, W, s, h);
        orc_field_images(L, 2, s, h2);
        orc_field_site(L, W, s, N - 1, hs);
        orc_energy(L, W, &p, s, parts);
        const double T3[3] = {0.0, 0.0, 1.0};
        (void)orc_delta_e(L, W, &p, s, h, 0, T3);
        uint64_t a = 0;
        orc_sweep_sequential(L, W, &p, s, h, 7, 2, &a);
        if (L % 2 == 0) {
            orc_sweep_checkerboard(L, W, &p, s, 9, 2, &a);
            orc_trial_energies(L, W, &p, s, h, 9, 1, dE, u2, S);
        }
        if (L >= 2 && L % 2 == 0) {
            orc_sweep_coset(L, W, &p, s, 2, 3, 1, &a);
            (void)orc_coset_error(L, 2, 0);
            (void)orc_coset_error(L, 2, 1);
        }
        orc_observables(L, W, &p, s, out, acc);
        orc_observables(L, NULL, &p, s, out, NULL);
        double rows[4 * ORC_NOBS];
        for (int t = 0; t < 4; ++t) orc_observables(L, NULL, &p, s, rows + t * ORC_NOBS, NULL);
        orc_variances(4, rows, var);
        (void)orc_staggered_susceptibility(L, 1.0, 4, rows);
        orc_params pi = p;
        pi.model = 1;
        orc_init_ising(L, 4, 1, s);
        orc_sweep_sequential(L, W, &pi, s, h, 1, 1, &a);
        double *obs = calloc(3 * ORC_NOBS, sizeof(double)), *eacc = calloc(2 * N, sizeof(double));
        fill(L, 6, s);
        orc_run(L, 1, &p, s, 0, 1, 3, 0, 1, obs, 2, eacc, &a);
        if (L % 2 == 0) orc_run(L, 1, &p, s, 0, 1, 3, 1, 0, obs, 0, NULL, &a);
        if (L >= 2) {
            orc_params lad[2] = {p, p};
            lad[1].T = 1.1;
            double *sl = calloc(2 * 3 * N, sizeof(double));
            double E[2] = {-1.0, -2.0};
            uint32_t rounds[2] = {1, 2};
            uint64_t swaps[2] = {0, 0};
            fill(L, 7, sl);
            fill(L, 8, sl + 3 * N);
            orc_pt_swap(L, 2, lad, sl, E, rounds, 0, swaps);
            free(sl);
        }
        free(obs); free(eacc);
        free(W); free(We); free(s); free(h); free(h2); free(acc); free(dE); free(u2); free(S);
    }
    printf("sanitized oracle run complete\n");
    return 0;
}
