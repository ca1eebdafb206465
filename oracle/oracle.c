/*
 * oracle.c -- plain, slow, FP64 CPU reference of the dipolar Heisenberg
 * Monte Carlo hot path (Stamps & Ambrose, arXiv:1211.6234).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header, table or
 * constant generator with the HIP library: every formula below is written
 * out again from the paper.
 *
 * Model (Sec. 2.1 eq. (1); Sec. 4 eqs. (11)-(12)), in exchange units J = 1
 * with g = C_D / J:
 *   E = -J sum_i s_i.(s_{i+x} + s_{i+y})            exchange, each bond once
 *     + (g/2) sum_i s_i . h_i,  h = W (*) s          dipole incl. self images
 *     - sum_i (K2 s_iz^2 + K4 s_iz^4)                anisotropy
 * W(rho) is the periodic-image sum of the dipole tensor (Sec. 2.1, eq. (1)
 * and the image construction leading to eq. (2)), truncated to a centred box
 * of half-width (M + 1/2) L with weight 1/2 on box edges (1/4 on corners).
 *
 * Conventions (readings of the paper where it is silent or garbled):
 *  - lattice site i = y*L + x, x fastest; colour c(i) = (x + y) mod 2.
 *  - spins are stored component-major: s[3][N] (x, y, z planes).
 *  - W is stored as W[4][L][L]: planes xx, yy, xy, zz (xz = yz = 0 because
 *    every image vector lies in the plane).
 *  - random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *    key = (seed low word, seed high word), counter = (site, sweep, replica,
 *    purpose); purpose 0 draws initial spins, purpose 1 draws Metropolis
 *    moves.  u_k = (x_k + 1/2) * 2^-32 lies in (0, 1).
 *  - trial move (Appendix A draws a uniform direction): z = 1 - 2 u0,
 *    phi = 2 pi u1, S = (sqrt(1 - z^2) cos phi, sqrt(1 - z^2) sin phi, z),
 *    with sqrt(1 - z^2) evaluated as 2 sqrt(u0 (1 - u0)) (the same number).
 *  - Metropolis (Sec. 2.2, eq. (7)): accept iff dE <= 0 or u2 < exp(-dE/T).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define PI 3.14159265358979323846264338327950288

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of a multiply/xor   */
/* bijection keyed by a Weyl sequence.                                 */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {            /* key schedule: add the Weyl constants */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

double orc_u01(uint32_t x)
{
    return ((double)x + 0.5) * (1.0 / 4294967296.0);
}

void orc_draw(uint64_t seed, uint32_t replica, uint32_t sweep, uint32_t site,
              uint32_t purpose, double u[4])
{
    uint32_t ctr[4] = {site, sweep, replica, purpose};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    for (int k = 0; k < 4; ++k) u[k] = orc_u01(x[k]);
}

void orc_direction(double u0, double u1, double S[3])
{
    double z = 1.0 - 2.0 * u0;
    double rxy = 2.0 * sqrt(u0 * (1.0 - u0));
    double phi = 2.0 * PI * u1;
    S[0] = rxy * cos(phi);
    S[1] = rxy * sin(phi);
    S[2] = z;
}

/* ------------------------------------------------------------------ */
/* Lattice-summed dipole tensor (Sec. 2.1).                            */
/* ------------------------------------------------------------------ */
static long imod(long a, long n)
{
    long r = a % n;
    return r < 0 ? r + n : r;
}

/* Weight of one image coordinate c (integer) in the box |c| <= (M+1/2)L:
 * 1 strictly inside, 1/2 on the edge, 0 outside. */
static double edge_weight(long c, int L, int M)
{
    long twice = 2 * labs(c);
    long edge = (long)(2 * M + 1) * L;
    if (twice < edge) return 1.0;
    if (twice == edge) return 0.5;
    return 0.0;
}

/* Dipole tensor of one separation r (eq. (1) with C_D = 1):
 * D_ab(r) = (delta_ab - 3 r_a r_b / r^2) / r^3, r in the plane. */
static void dipole_tensor(double rx, double ry, double D[4])
{
    double r2 = rx * rx + ry * ry;
    double r = sqrt(r2);
    double r3 = r2 * r;
    D[0] = (1.0 - 3.0 * rx * rx / r2) / r3;   /* xx */
    D[1] = (1.0 - 3.0 * ry * ry / r2) / r3;   /* yy */
    D[2] = (-3.0 * rx * ry / r2) / r3;        /* xy */
    D[3] = 1.0 / r3;                          /* zz */
}

void orc_lattice_sum_kernel(int L, int M, double *W)
{
    const long N = (long)L * L;
    for (int py = 0; py < L; ++py) {
        for (int px = 0; px < L; ++px) {
            double acc[4] = {0, 0, 0, 0};
            for (int b = -M - 1; b <= M + 1; ++b) {
                long ry = py + (long)b * L;
                double wy = edge_weight(ry, L, M);
                if (wy == 0.0) continue;
                for (int a = -M - 1; a <= M + 1; ++a) {
                    long rx = px + (long)a * L;
                    double wx = edge_weight(rx, L, M);
                    if (wx == 0.0) continue;
                    if (rx == 0 && ry == 0) continue;
                    double D[4];
                    dipole_tensor((double)rx, (double)ry, D);
                    for (int c = 0; c < 4; ++c) acc[c] += wx * wy * D[c];
                }
            }
            for (int c = 0; c < 4; ++c) W[c * N + (long)py * L + px] = acc[c];
        }
    }
}

/*
 * All periodic images (Sec. 2.1, eqs. (3)-(5)): W_inf(rho) = sum over every
 * lattice vector G = (aL, bL) of D(rho + G), the G = 0 term omitted at
 * rho = 0.  The image sum converges slowly, so it is split as in the
 * Ewald-Harris construction the paper cites, specialised to dipoles in the
 * plane z = 0:
 *   1/r = erfc(r / 2eta) / r  +  erf(r / 2eta) / r.
 * The first part decays fast and is summed over images in real space; the
 * second is smooth and is summed over the reciprocal lattice k = 2 pi (m, n) / L
 * with its in-plane Fourier transform (2 pi / |k|) erfc(|k| eta) (the z = 0
 * form of eq. (5)).  D = -grad grad (1/r), so each part contributes minus
 * its second derivatives; the k = 0 term is a constant and drops out.  At
 * rho = 0 the smooth part of the omitted G = 0 term, -d_a d_b [erf(r/2eta)/r]
 * at r = 0 = (4 / (3 sqrt(pi))) (1/2eta)^3 delta_ab, is removed.  The
 * in-plane components come from the sums; W_zz = -(W_xx + W_yy) because every
 * image term is trace-free.  The result does not depend on eta; the image and
 * wave-vector ranges are chosen so the neglected terms are below 1e-17 of
 * the largest.
 */
void orc_lattice_sum_ewald(int L, double eta, double *W)
{
    const long N = (long)L * L;
    const double a = 1.0 / (2.0 * eta);
    const double two_over_sqrtpi = 2.0 / sqrt(PI);
    const int nreal = (int)ceil(13.0 * eta / L) + 1;            /* a r >= 6.5 beyond */
    const int nrecip = (int)ceil(6.5 * L / (2.0 * PI * eta)) + 1;   /* |k| eta >= 6.5 beyond */
    for (int py = 0; py < L; ++py) {
        for (int px = 0; px < L; ++px) {
            double xx = 0.0, yy = 0.0, xy = 0.0;
            /* real-space part: -d_a d_b of erfc(a r) / r at r = rho + G */
            for (int bb = -nreal; bb <= nreal; ++bb) {
                for (int aa = -nreal; aa <= nreal; ++aa) {
                    const double rx = px + (double)aa * L, ry = py + (double)bb * L;
                    const double r2 = rx * rx + ry * ry;
                    if (r2 == 0.0) continue;
                    const double r = sqrt(r2);
                    const double ec = erfc(a * r), gs = two_over_sqrtpi * a * exp(-a * a * r2);
                    /* with g(r) = erfc(a r)/r: Bt = -g'/r, Ct = g'' - g'/r */
                    const double Bt = ec / (r2 * r) + gs / r2;
                    const double Ct = 3.0 * ec / (r2 * r) + 3.0 * gs / r2 + 2.0 * a * a * gs;
                    xx += Bt - Ct * rx * rx / r2;
                    yy += Bt - Ct * ry * ry / r2;
                    xy += -Ct * rx * ry / r2;
                }
            }
            /* reciprocal part: (1/L^2) sum_{k != 0} (2 pi/|k|) erfc(|k| eta) k_a k_b cos(k . rho) */
            for (int n = -nrecip; n <= nrecip; ++n) {
                for (int m = -nrecip; m <= nrecip; ++m) {
                    if (m == 0 && n == 0) continue;
                    const double kx = 2.0 * PI * m / L, ky = 2.0 * PI * n / L;
                    const double k = sqrt(kx * kx + ky * ky);
                    const double f = 2.0 * PI / k * erfc(k * eta) * cos(kx * px + ky * py) / ((double)L * L);
                    xx += f * kx * kx;
                    yy += f * ky * ky;
                    xy += f * kx * ky;
                }
            }
            if (px == 0 && py == 0) {
                const double self = 4.0 / (3.0 * sqrt(PI)) * a * a * a;
                xx -= self;
                yy -= self;
            }
            const long o = (long)py * L + px;
            W[o] = xx;
            W[N + o] = yy;
            W[2 * N + o] = xy;
            W[3 * N + o] = -(xx + yy);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Local dipolar field h_i = sum_j W(rho_ij) s_j, rho_ij = r_i - r_j.   */
/* ------------------------------------------------------------------ */
void orc_field_site(int L, const double *W, const double *s, long i, double h[3])
{
    const long N = (long)L * L;
    const double *Wxx = W, *Wyy = W + N, *Wxy = W + 2 * N, *Wzz = W + 3 * N;
    const double *sx = s, *sy = s + N, *sz = s + 2 * N;
    long xi = i % L, yi = i / L;
    double hx = 0, hy = 0, hz = 0;
    for (long j = 0; j < N; ++j) {
        long xj = j % L, yj = j / L;
        long rho = imod(yi - yj, L) * L + imod(xi - xj, L);
        hx += Wxx[rho] * sx[j] + Wxy[rho] * sy[j];
        hy += Wxy[rho] * sx[j] + Wyy[rho] * sy[j];
        hz += Wzz[rho] * sz[j];
    }
    h[0] = hx; h[1] = hy; h[2] = hz;
}

void orc_field(int L, const double *W, const double *s, double *h)
{
    const long N = (long)L * L;
    for (long i = 0; i < N; ++i) {
        double hi[3];
        orc_field_site(L, W, s, i, hi);
        h[i] = hi[0]; h[N + i] = hi[1]; h[2 * N + i] = hi[2];
    }
}

/* Table-free field: the literal pair-plus-image sum of eq. (1), no W. */
void orc_field_images(int L, int M, const double *s, double *h)
{
    const long N = (long)L * L;
    for (long i = 0; i < N; ++i) {
        long xi = i % L, yi = i / L;
        double hx = 0, hy = 0, hz = 0;
        for (long j = 0; j < N; ++j) {
            long xj = j % L, yj = j / L;
            for (int b = -M - 1; b <= M + 1; ++b) {
                long ry = (yi - yj) + (long)b * L;
                for (int a = -M - 1; a <= M + 1; ++a) {
                    long rx = (xi - xj) + (long)a * L;
                    /* the box is centred on site i; the image of j at r is
                     * counted with the edge weights of the box */
                    double w = edge_weight(rx, L, M) * edge_weight(ry, L, M);
                    if (w == 0.0 || (rx == 0 && ry == 0)) continue;
                    double D[4];
                    dipole_tensor((double)rx, (double)ry, D);
                    hx += w * (D[0] * s[j] + D[2] * s[N + j]);
                    hy += w * (D[2] * s[j] + D[1] * s[N + j]);
                    hz += w * (D[3] * s[2 * N + j]);
                }
            }
        }
        h[i] = hx; h[N + i] = hy; h[2 * N + i] = hz;
    }
}

/* ------------------------------------------------------------------ */
/* Energies (eqs. (11)-(12) with the readings above).                 */
/* ------------------------------------------------------------------ */
static long nb(int L, long i, int dx, int dy)
{
    long x = i % L, y = i / L;
    return imod(y + dy, L) * L + imod(x + dx, L);
}

void orc_energy(int L, const double *W, const orc_params *p, const double *s, double parts[4])
{
    const long N = (long)L * L;
    double *h = (double *)malloc(sizeof(double) * 3 * N);
    orc_field(L, W, s, h);
    double eex = 0, edip = 0, eani = 0;
    for (long i = 0; i < N; ++i) {
        long ix = nb(L, i, 1, 0), iy = nb(L, i, 0, 1);
        for (int c = 0; c < 3; ++c)
            eex += -p->J * s[c * N + i] * (s[c * N + ix] + s[c * N + iy]);
        for (int c = 0; c < 3; ++c)
            edip += 0.5 * p->g * s[c * N + i] * h[c * N + i];
        double z = s[2 * N + i];
        eani += -(p->K2 * z * z + p->K4 * z * z * z * z);
    }
    free(h);
    parts[0] = eex; parts[1] = edip; parts[2] = eani; parts[3] = eex + edip + eani;
}

/* Exact single-site energy change for s_k -> S:
 *   dE = -J d.(sum of 4 neighbours) + g (d.h_k + 1/2 d^T W(0) d)
 *        - K2 (Sz^2 - sz^2) - K4 (Sz^4 - sz^4),      d = S - s_k,
 * where h is the field of the current state including the self-image term
 * W(0) s_k; the quadratic term accounts for the images of site k moving
 * together with it (Sec. 2.1 eq. (2), second line; Sec. 3.2). */
double orc_delta_e(int L, const double *W, const orc_params *p, const double *s,
                   const double *h, long k, const double S[3])
{
    const long N = (long)L * L;
    long n1 = nb(L, k, 1, 0), n2 = nb(L, k, -1, 0), n3 = nb(L, k, 0, 1), n4 = nb(L, k, 0, -1);
    double d[3], nn[3];
    for (int c = 0; c < 3; ++c) {
        d[c] = S[c] - s[c * N + k];
        nn[c] = s[c * N + n1] + s[c * N + n2] + s[c * N + n3] + s[c * N + n4];
    }
    double dex = -p->J * (d[0] * nn[0] + d[1] * nn[1] + d[2] * nn[2]);
    double W0xx = W[0], W0yy = W[N], W0xy = W[2 * N], W0zz = W[3 * N];
    double dWd = W0xx * d[0] * d[0] + W0yy * d[1] * d[1] + 2.0 * W0xy * d[0] * d[1]
               + W0zz * d[2] * d[2];
    double ddip = p->g * (d[0] * h[k] + d[1] * h[N + k] + d[2] * h[2 * N + k] + 0.5 * dWd);
    double z0 = s[2 * N + k], z1 = S[2];
    double dani = -p->K2 * (z1 * z1 - z0 * z0) - p->K4 * (z1 * z1 * z1 * z1 - z0 * z0 * z0 * z0);
    return dex + ddip + dani;
}

int orc_metropolis_accept(double dE, double T, double u)
{
    if (dE <= 0.0) return 1;
    return u < exp(-dE / T);
}

/* ------------------------------------------------------------------ */
/* Initial state: every site uniform on S^2 from purpose-0 draws.      */
/* ------------------------------------------------------------------ */
void orc_init_spins(int L, uint64_t seed, uint32_t replica, double *s)
{
    const long N = (long)L * L;
    for (long i = 0; i < N; ++i) {
        double u[4], S[3];
        orc_draw(seed, replica, 0, (uint32_t)i, 0, u);
        orc_direction(u[0], u[1], S);
        s[i] = S[0]; s[N + i] = S[1]; s[2 * N + i] = S[2];
    }
}

/* Ising replicas (the appendix on the dipolar Ising model): s_i = (0, 0,
 * +-1), +1 when the purpose-0 draw u0 < 1/2. */
void orc_init_ising(int L, uint64_t seed, uint32_t replica, double *s)
{
    const long N = (long)L * L;
    for (long i = 0; i < N; ++i) {
        double u[4];
        orc_draw(seed, replica, 0, (uint32_t)i, 0, u);
        s[i] = 0.0; s[N + i] = 0.0; s[2 * N + i] = u[0] < 0.5 ? 1.0 : -1.0;
    }
}

/* Trial spin at site k from the site's draws: a uniform direction (Sec. 2.2,
 * Appendix A) for Heisenberg replicas, the reversal s -> -s for Ising ones. */
static void orc_trial(const orc_params *p, const double *s, long N, long k, const double u[4], double S[3])
{
    if (p->model == 1) {
        S[0] = -s[k]; S[1] = -s[N + k]; S[2] = -s[2 * N + k];
    } else {
        orc_direction(u[0], u[1], S);
    }
}

/* ------------------------------------------------------------------ */
/* Sequential single-spin Metropolis with the exact dE (Sec. 2.2):     */
/* sites in index order; h is kept exact by adding W(rho_mk) d to      */
/* every h_m after an accepted move at k.                              */
/* ------------------------------------------------------------------ */
void orc_sweep_sequential(int L, const double *W, const orc_params *p, double *s, double *h,
                          uint32_t sweep0, int nsweeps, uint64_t *accepted)
{
    const long N = (long)L * L;
    const double *Wxx = W, *Wyy = W + N, *Wxy = W + 2 * N, *Wzz = W + 3 * N;
    for (int t = 0; t < nsweeps; ++t) {
        uint32_t sweep = sweep0 + (uint32_t)t;
        for (long k = 0; k < N; ++k) {
            double u[4], S[3];
            orc_draw(p->seed, p->replica_id, sweep, (uint32_t)k, 1, u);
            orc_trial(p, s, N, k, u, S);
            double dE = orc_delta_e(L, W, p, s, h, k, S);
            if (!orc_metropolis_accept(dE, p->T, u[2])) continue;
            double d[3] = {S[0] - s[k], S[1] - s[N + k], S[2] - s[2 * N + k]};
            s[k] = S[0]; s[N + k] = S[1]; s[2 * N + k] = S[2];
            long xk = k % L, yk = k / L;
            for (long m = 0; m < N; ++m) {
                long rho = imod(m / L - yk, L) * L + imod(m % L - xk, L);
                h[m] += Wxx[rho] * d[0] + Wxy[rho] * d[1];
                h[N + m] += Wxy[rho] * d[0] + Wyy[rho] * d[1];
                h[2 * N + m] += Wzz[rho] * d[2];
            }
            if (accepted) ++*accepted;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Checkerboard frozen-field variant (Sec. 3.2 approximation applied   */
/* to a colour class): for each colour the field of the current state  */
/* is computed once, every site of that colour takes its decision with  */
/* that frozen field, then all accepted moves are applied together.    */
/* ------------------------------------------------------------------ */
void orc_trial_energies(int L, const double *W, const orc_params *p, const double *s,
                        const double *h, uint32_t sweep, int color, double *dE, double *u2,
                        double *S_out)
{
    const long N = (long)L * L;
    for (long k = 0; k < N; ++k) {
        long x = k % L, y = k / L;
        if ((int)((x + y) % 2) != color) { dE[k] = NAN; u2[k] = NAN; continue; }
        double u[4], S[3];
        orc_draw(p->seed, p->replica_id, sweep, (uint32_t)k, 1, u);
        orc_trial(p, s, N, k, u, S);
        dE[k] = orc_delta_e(L, W, p, s, h, k, S);
        u2[k] = u[2];
        if (S_out) { S_out[k] = S[0]; S_out[N + k] = S[1]; S_out[2 * N + k] = S[2]; }
    }
}

void orc_sweep_checkerboard(int L, const double *W, const orc_params *p, double *s,
                            uint32_t sweep0, int nsweeps, uint64_t *accepted)
{
    const long N = (long)L * L;
    double *h = (double *)malloc(sizeof(double) * 3 * N);
    double *dE = (double *)malloc(sizeof(double) * N);
    double *u2 = (double *)malloc(sizeof(double) * N);
    double *S = (double *)malloc(sizeof(double) * 3 * N);
    for (int t = 0; t < nsweeps; ++t) {
        uint32_t sweep = sweep0 + (uint32_t)t;
        for (int color = 0; color < 2; ++color) {
            orc_field(L, W, s, h);
            orc_trial_energies(L, W, p, s, h, sweep, color, dE, u2, S);
            for (long k = 0; k < N; ++k) {
                long x = k % L, y = k / L;
                if ((int)((x + y) % 2) != color) continue;
                if (!orc_metropolis_accept(dE[k], p->T, u2[k])) continue;
                s[k] = S[k]; s[N + k] = S[N + k]; s[2 * N + k] = S[2 * N + k];
                if (accepted) ++*accepted;
            }
        }
    }
    free(h); free(dE); free(u2); free(S);
}

/*
 * The paper's own simultaneous-update set (Sec. 3.1): the sites of one coset
 * of the sublattice l Z^2, i = (a l, b l) + i1, are updated at once, every
 * one of them with the dipolar field of the state before the update (the
 * approximation H3 - H1 ~ H2 - H0 of Sec. 3.2).  A sweep visits the l^2
 * cosets i1 = (cx, cy) in the order cy = 0..l-1, cx = 0..l-1, so each site is
 * proposed once per sweep with its (site, sweep) draws.  l >= 2 and l | L;
 * the sites of a coset are then never nearest neighbours.  With l = L each
 * coset is one site and the sweep is exact sequential Metropolis in index
 * order.
 */
void orc_sweep_coset(int L, const double *W, const orc_params *p, double *s, int l,
                     uint32_t sweep0, int nsweeps, uint64_t *accepted)
{
    const long N = (long)L * L;
    double *h = (double *)malloc(sizeof(double) * 3 * N);
    double *S = (double *)malloc(sizeof(double) * 3 * N);
    unsigned char *take = (unsigned char *)malloc((size_t)N);
    for (int t = 0; t < nsweeps; ++t) {
        const uint32_t sweep = sweep0 + (uint32_t)t;
        for (int cy = 0; cy < l; ++cy) {
            for (int cx = 0; cx < l; ++cx) {
                orc_field(L, W, s, h);
                /* decide every site of the coset on the frozen state ... */
                for (long k = 0; k < N; ++k) {
                    take[k] = 0;
                    if ((int)(k % L) % l != cx || (int)(k / L) % l != cy) continue;
                    double u[4], Sk[3];
                    orc_draw(p->seed, p->replica_id, sweep, (uint32_t)k, 1, u);
                    orc_trial(p, s, N, k, u, Sk);
                    const double dE = orc_delta_e(L, W, p, s, h, k, Sk);
                    if (!orc_metropolis_accept(dE, p->T, u[2])) continue;
                    take[k] = 1;
                    S[k] = Sk[0]; S[N + k] = Sk[1]; S[2 * N + k] = Sk[2];
                }
                /* ... then apply the accepted moves together */
                for (long k = 0; k < N; ++k) {
                    if (!take[k]) continue;
                    s[k] = S[k]; s[N + k] = S[N + k]; s[2 * N + k] = S[2 * N + k];
                    if (accepted) ++*accepted;
                }
            }
        }
    }
    free(h); free(S); free(take);
}

/*
 * The error bound of eq. (10) for the coset update (C_D = 1): the largest
 * change of H3 - H1 that the other simultaneously moved sites can cause,
 * 2 / r^3 per partner (the perpendicular maximum D = 2 of eq. (8)).  Reading
 * taken for the ambiguous range of eq. (10): with all_images = 0 every other
 * site of the coset counts once, at its nearest image (the reading that
 * gives the 0.14 % quoted for L = 64, l = 32, T = 0.1); with all_images = 1
 * every image counts, which sums 2/r^3 over l Z^2 minus the origin.
 */
double orc_coset_error(int L, int l, int all_images)
{
    const int n = L / l;
    double eps = 0.0;
    if (!all_images) {
        for (int b = 0; b < n; ++b) {
            for (int a = 0; a < n; ++a) {
                if (a == 0 && b == 0) continue;
                long dx = (long)a * l, dy = (long)b * l;
                if (2 * dx > L) dx -= L;    /* nearest image */
                if (2 * dy > L) dy -= L;
                const double r2 = (double)(dx * dx + dy * dy);
                eps += 2.0 / (r2 * sqrt(r2));
            }
        }
        return eps;
    }
    /* all images: partners at every point of l Z^2 but the origin; the box
     * sum is closed by its continuum tail 4 sqrt(2) / A outside half-width A */
    const int K = 4096;
    double sum = 0.0;
    for (long b = -K; b <= K; ++b) {
        for (long a = -K; a <= K; ++a) {
            if (a == 0 && b == 0) continue;
            const double r2 = (double)(a * a + b * b);
            sum += 1.0 / (r2 * sqrt(r2));
        }
    }
    sum += 4.0 * sqrt(2.0) / (K + 0.5);
    return 2.0 * sum / ((double)l * l * l);
}

/*
 * Replica exchange on a temperature ladder (parallel tempering), the
 * companion of the Sec. 4 temperature scans for the ladder workload: for
 * every pair (r, r + 1) with r = parity mod 2, the two states are exchanged
 * with probability min(1, exp((1/T_r - 1/T_{r+1}) (E_r - E_{r+1}))), E the
 * total energies of the current states (E NaN: no exchange).  The uniform is
 * u0 of counter (r, round_r, replica_id_r, 2) under seed_r, with round_r the
 * pair's round index.  The pair must share J, K2, K4, g and the model.
 * s: [R][3][N]; E: [R]; swaps[r] counts the exchanges of pair (r, r + 1).
 */
void orc_pt_swap(int L, int R, const orc_params *p, double *s, const double *E, const uint32_t *round,
                 int parity, uint64_t *swaps)
{
    const long N3 = 3L * L * L;
    for (int r = parity; r + 1 < R; r += 2) {
        const double delta = (1.0 / p[r].T - 1.0 / p[r + 1].T) * (E[r] - E[r + 1]);
        double u[4];
        orc_draw(p[r].seed, p[r].replica_id, round[r], (uint32_t)r, 2, u);
        if (!(delta >= 0.0 || u[0] < exp(delta))) continue;
        for (long i = 0; i < N3; ++i) {
            const double tmp = s[(long)r * N3 + i];
            s[(long)r * N3 + i] = s[(long)(r + 1) * N3 + i];
            s[(long)(r + 1) * N3 + i] = tmp;
        }
        if (swaps) ++swaps[r];
    }
}

/* ------------------------------------------------------------------ */
/* Observables of one state (Sec. 4.1 eqs. (14)-(17)).                 */
/* ------------------------------------------------------------------ */
static int sgn(double v) { return (v > 0) - (v < 0); }

void orc_observables(int L, const double *W, const orc_params *p, const double *s,
                     double *out, double *eta_acc)
{
    const long N = (long)L * L;
    for (int k = 0; k < ORC_NOBS; ++k) out[k] = 0.0;
    if (W) {
        double parts[4];
        orc_energy(L, W, p, s, parts);
        out[ORC_OBS_E] = parts[3] / (double)N;
        out[ORC_OBS_EEX] = parts[0] / (double)N;
        out[ORC_OBS_EDIP] = parts[1] / (double)N;
        out[ORC_OBS_EANI] = parts[2] / (double)N;
    } else {
        double eex = 0, eani = 0;
        for (long i = 0; i < N; ++i) {
            long ix = nb(L, i, 1, 0), iy = nb(L, i, 0, 1);
            for (int c = 0; c < 3; ++c)
                eex += -p->J * s[c * N + i] * (s[c * N + ix] + s[c * N + iy]);
            double z = s[2 * N + i];
            eani += -(p->K2 * z * z + p->K4 * z * z * z * z);
        }
        out[ORC_OBS_E] = NAN;
        out[ORC_OBS_EEX] = eex / (double)N;
        out[ORC_OBS_EDIP] = NAN;
        out[ORC_OBS_EANI] = eani / (double)N;
    }
    double m[3] = {0, 0, 0};
    for (long i = 0; i < N; ++i)
        for (int c = 0; c < 3; ++c) m[c] += s[c * N + i];
    for (int c = 0; c < 3; ++c) m[c] /= (double)N;
    out[ORC_OBS_MX] = m[0];
    out[ORC_OBS_MY] = m[1];
    out[ORC_OBS_MZ] = m[2];
    out[ORC_OBS_MABS] = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    out[ORC_OBS_MPAR] = sqrt(m[0] * m[0] + m[1] * m[1]);
    out[ORC_OBS_MZABS] = fabs(m[2]);
    /* eq. (14): n_h counts sign changes along +x, n_v along +y */
    for (int c = 0; c < 3; ++c) {
        long nh = 0, nv = 0;
        for (long i = 0; i < N; ++i) {
            long ix = nb(L, i, 1, 0), iy = nb(L, i, 0, 1);
            nh += 1 - sgn(s[c * N + i]) * sgn(s[c * N + ix]);
            nv += 1 - sgn(s[c * N + i]) * sgn(s[c * N + iy]);
        }
        out[ORC_OBS_NH + c] = (double)nh;
        out[ORC_OBS_NV + c] = (double)nv;
        /* eq. (15); a sample with no walls at all contributes 0 */
        out[ORC_OBS_ORIENT + c] = (nh + nv) > 0 ? fabs((double)(nh - nv)) / (double)(nh + nv) : 0.0;
    }
    out[ORC_OBS_WALLDENS] = (out[ORC_OBS_NV + 2] + out[ORC_OBS_NH + 2]) / (4.0 * (double)N);
    /* eq. (17): per-site (theta - pi/2)^2, theta = arccos s_z; and the cone
     * angle of this one state, the thermal average in eq. (17) replaced by
     * the state itself: (1/N) sum_i sqrt((2/pi)^2 (theta_i - pi/2)^2) */
    double q = 0, eta_sum = 0, eta_state = 0;
    for (long i = 0; i < N; ++i) {
        double z = s[2 * N + i];
        if (z > 1.0) z = 1.0;
        if (z < -1.0) z = -1.0;
        double dth = acos(z) - 0.5 * PI;
        q += dth * dth;
        eta_state += sqrt((2.0 / PI) * (2.0 / PI) * dth * dth);
        if (eta_acc) {
            eta_acc[i] += dth * dth;
            eta_sum += sqrt(eta_acc[i]);
        }
    }
    out[ORC_OBS_Q] = q / (double)N;
    out[ORC_OBS_ETASUM] = eta_acc ? eta_sum / (double)N : NAN;
    out[ORC_OBS_ETAS] = eta_state / (double)N;
    /* a health count, not a quantity of the paper: sites whose spin has a
     * NaN or infinite component */
    long nonfinite = 0;
    for (long i = 0; i < N; ++i)
        if (!(isfinite(s[i]) && isfinite(s[N + i]) && isfinite(s[2 * N + i]))) ++nonfinite;
    out[ORC_OBS_NONFINITE] = (double)nonfinite;
    /* stripes of width 1 (the appendix on the dipolar Ising model): with the
     * four sublattices of the 2 x 2 cell, m_h = m1 + m2 - m3 - m4 is the
     * z magnetization staggered along y and m_v = m1 + m4 - m3 - m2 the one
     * staggered along x, normalised per site */
    double mh = 0.0, mv = 0.0;
    for (long i = 0; i < N; ++i) {
        const double z = s[2 * N + i];
        mh += ((i / L) % 2 == 0) ? z : -z;
        mv += ((i % L) % 2 == 0) ? z : -z;
    }
    out[ORC_OBS_MSTH] = mh / (double)N;
    out[ORC_OBS_MSTV] = mv / (double)N;
}

/* ------------------------------------------------------------------ */
/* Fluctuations (Sec. 5, eq. (18)): sigma^2(X) = <(X - <X>)^2>, the    */
/* averages over the nsamp samples obs[nsamp][ORC_NOBS], for X = the    */
/* planar magnetization M_par of each sample (eq. (16)), the z          */
/* orientational order O_z (eq. (15)) and the cone angle eta of each    */
/* sample (eq. (17) over that state); var[0], var[1], var[2].           */
/* ------------------------------------------------------------------ */
void orc_variances(int nsamp, const double *obs, double var[3])
{
    const int slot[3] = {ORC_OBS_MPAR, ORC_OBS_ORIENT + 2, ORC_OBS_ETAS};
    for (int q = 0; q < 3; ++q) {
        double mean = 0.0;
        for (long k = 0; k < nsamp; ++k) mean += obs[k * ORC_NOBS + slot[q]];
        mean /= (double)nsamp;
        double v = 0.0;
        for (long k = 0; k < nsamp; ++k) {
            const double d = obs[k * ORC_NOBS + slot[q]] - mean;
            v += d * d;
        }
        var[q] = v / (double)nsamp;
    }
}

/* ------------------------------------------------------------------ */
/* Staggered susceptibility of the dipolar Ising appendix:             */
/* chi_st = (L^2 / k_B T) (<m_st^2> - <m_st>^2) over nsamp samples     */
/* obs[nsamp][ORC_NOBS], m_st = sqrt(m_h^2 + m_v^2) of each sample.    */
/* ------------------------------------------------------------------ */
double orc_staggered_susceptibility(int L, double T, int nsamp, const double *obs)
{
    double m1 = 0.0, m2 = 0.0;
    for (long k = 0; k < nsamp; ++k) {
        const double mh = obs[k * ORC_NOBS + ORC_OBS_MSTH], mv = obs[k * ORC_NOBS + ORC_OBS_MSTV];
        const double mst = sqrt(mh * mh + mv * mv);
        m1 += mst;
        m2 += mst * mst;
    }
    m1 /= (double)nsamp;
    m2 /= (double)nsamp;
    return (double)L * (double)L / T * (m2 - m1 * m1);
}

/* ------------------------------------------------------------------ */
/* Run driver: burn-in, then one observables sample per sweep.         */
/* mode 0 = sequential exact, 1 = checkerboard frozen field.           */
/* obs: [nsamp][ORC_NOBS]; eta_acc: [nbatch][N] (may be NULL).         */
/* ------------------------------------------------------------------ */
void orc_run(int L, int M, const orc_params *p, double *s, uint32_t sweep0, int nburn, int nsamp,
             int mode, int with_energy, double *obs, int nbatch, double *eta_acc, uint64_t *accepted)
{
    const long N = (long)L * L;
    double *W = (double *)malloc(sizeof(double) * 4 * N);
    double *h = (double *)malloc(sizeof(double) * 3 * N);
    orc_lattice_sum_kernel(L, M, W);
    orc_field(L, W, s, h);
    uint32_t sweep = sweep0;
    for (int t = 0; t < nburn + nsamp; ++t, ++sweep) {
        if (mode == 0) orc_sweep_sequential(L, W, p, s, h, sweep, 1, accepted);
        else orc_sweep_checkerboard(L, W, p, s, sweep, 1, accepted);
        if (t < nburn) continue;
        int k = t - nburn;
        double *acc = NULL;
        if (eta_acc && nbatch > 0) {
            int b = (int)((long)k * nbatch / nsamp);
            acc = eta_acc + (long)b * N;
        }
        orc_observables(L, with_energy ? W : NULL, p, s, obs + (long)k * ORC_NOBS, acc);
    }
    free(W); free(h);
}
