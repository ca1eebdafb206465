/*
 * oracle.h -- FP64 CPU reference of the dipolar Heisenberg Monte Carlo hot
 * path (Stamps & Ambrose, arXiv:1211.6234).  TEST INFRASTRUCTURE ONLY: see
 * oracle.c.  Not shared with, and not included by, the HIP library.
 */
#ifndef ORC_ORACLE_H
#define ORC_ORACLE_H

#include <stdint.h>

typedef struct {
    double T;            /* temperature, k_B = 1, exchange units          */
    double J;            /* nearest-neighbour exchange (ferromagnetic > 0) */
    double K2, K4;       /* anisotropy: -K2 sz^2 - K4 sz^4 per site        */
    double g;            /* dipole strength C_D / J                        */
    uint64_t seed;       /* Philox key                                     */
    uint32_t replica_id; /* Philox counter word 2                          */
    uint32_t model;      /* 0: Heisenberg, trial uniform on the sphere;
                            1: Ising, s = (0, 0, +-1), trial = reversal   */
} orc_params;

/* observable slots of one sample (one state of one replica) */
enum {
    ORC_OBS_E = 0,        /* total energy per site (NaN without a field)  */
    ORC_OBS_EEX = 1,
    ORC_OBS_EDIP = 2,
    ORC_OBS_EANI = 3,
    ORC_OBS_MX = 4,
    ORC_OBS_MY = 5,
    ORC_OBS_MZ = 6,
    ORC_OBS_MABS = 7,     /* |M|, M = (1/N) sum s                           */
    ORC_OBS_MPAR = 8,     /* sqrt(Mx^2 + My^2), eq. (16) before averaging   */
    ORC_OBS_MZABS = 9,
    ORC_OBS_NH = 10,      /* 10,11,12: n_h^x, n_h^y, n_h^z, eq. (14)         */
    ORC_OBS_NV = 13,      /* 13,14,15: n_v^x, n_v^y, n_v^z                   */
    ORC_OBS_ORIENT = 16,  /* 16,17,18: |n_h - n_v| / (n_h + n_v), eq. (15)   */
    ORC_OBS_WALLDENS = 19,/* (n_v^z + n_h^z) / (4N)                         */
    ORC_OBS_Q = 20,       /* (1/N) sum (arccos sz - pi/2)^2                 */
    ORC_OBS_ETASUM = 21,  /* (1/N) sum_i sqrt(acc_i) after accumulating      */
    ORC_OBS_MSTH = 22,    /* (1/N) sum_i s_iz (-1)^y: horizontal stripes, width 1 */
    ORC_OBS_MSTV = 23,    /* (1/N) sum_i s_iz (-1)^x: vertical stripes, width 1   */
    ORC_OBS_ETAS = 24,    /* (2/pi)(1/N) sum_i |theta_i - pi/2|: eq. (17) over this state */
    ORC_OBS_NONFINITE = 25, /* sites whose spin has a NaN or infinite component (a health count) */
    ORC_NOBS = 26
};

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01(uint32_t x);
void orc_draw(uint64_t seed, uint32_t replica, uint32_t sweep, uint32_t site,
              uint32_t purpose, double u[4]);
void orc_direction(double u0, double u1, double S[3]);

void orc_lattice_sum_kernel(int L, int M, double *W);
void orc_lattice_sum_ewald(int L, double eta, double *W);
void orc_field_site(int L, const double *W, const double *s, long i, double h[3]);
void orc_field(int L, const double *W, const double *s, double *h);
void orc_field_images(int L, int M, const double *s, double *h);

void orc_energy(int L, const double *W, const orc_params *p, const double *s, double parts[4]);
double orc_delta_e(int L, const double *W, const orc_params *p, const double *s,
                   const double *h, long k, const double S[3]);
int orc_metropolis_accept(double dE, double T, double u);

void orc_init_spins(int L, uint64_t seed, uint32_t replica, double *s);
void orc_init_ising(int L, uint64_t seed, uint32_t replica, double *s);
void orc_sweep_sequential(int L, const double *W, const orc_params *p, double *s, double *h,
                          uint32_t sweep0, int nsweeps, uint64_t *accepted);
void orc_trial_energies(int L, const double *W, const orc_params *p, const double *s,
                        const double *h, uint32_t sweep, int color, double *dE, double *u2,
                        double *S_out);
void orc_sweep_coset(int L, const double *W, const orc_params *p, double *s, int l,
                     uint32_t sweep0, int nsweeps, uint64_t *accepted);
double orc_coset_error(int L, int l, int all_images);
void orc_pt_swap(int L, int R, const orc_params *p, double *s, const double *E, const uint32_t *round,
                 int parity, uint64_t *swaps);
void orc_sweep_checkerboard(int L, const double *W, const orc_params *p, double *s,
                            uint32_t sweep0, int nsweeps, uint64_t *accepted);
void orc_observables(int L, const double *W, const orc_params *p, const double *s,
                     double *out, double *eta_acc);
void orc_variances(int nsamp, const double *obs, double var[3]);
double orc_staggered_susceptibility(int L, double T, int nsamp, const double *obs);
void orc_run(int L, int M, const orc_params *p, double *s, uint32_t sweep0, int nburn, int nsamp,
             int mode, int with_energy, double *obs, int nbatch, double *eta_acc,
             uint64_t *accepted);

#endif
