/*
 * ddmc.h -- C ABI of the MI355X (gfx950) hot path of the dipolar Heisenberg
 * Monte Carlo method of Stamps & Ambrose, arXiv:1211.6234.
 *
 * The model is an L x L periodic square lattice of unit spins with
 * nearest-neighbour exchange, second- and fourth-order uniaxial anisotropy
 * and long-range dipole coupling summed over periodic images (Sec. 2.1,
 * eq. (1); Sec. 4, eqs. (11)-(12)).  In exchange units (J = 1, g = C_D/J):
 *
 *   E = -J sum_i s_i.(s_{i+x} + s_{i+y}) + (g/2) sum_i s_i.h_i
 *       - sum_i (K2 s_iz^2 + K4 s_iz^4),           h = W (*) s,
 *
 * where W (*) s is the circular convolution of the spins with the lattice-
 * summed 3x3 dipole tensor W(rho), self-image term W(0) included.
 *
 * Common conventions of every call:
 *  - Lattice site i = y*L + x (x fastest).  Colour of a site (x + y) mod 2.
 *  - Spin and field arrays are device memory, replica-major and component-
 *    planar: s[R][3][L][L] (planes x, y, z), element type double for a plan
 *    of precision DDMC_F64 and float for DDMC_F32.  Spins are unit vectors.
 *  - W64 is device memory, double [4][L][L], planes xx, yy, xy, zz
 *    (xz = yz = 0: every image vector lies in the film plane).
 *  - Every buffer is owned by the caller; the library never frees caller
 *    memory.  A plan owns only its derived kernel forms and workspace.
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream) except ddmc_plan_create and ddmc_plan_destroy, which
 *    synchronize; argument validation runs on the host before anything is
 *    enqueued.  Calls made
 *    with one plan must be ordered on one stream: the plan's workspace is
 *    shared by its calls.
 *  - Errors: no call throws across the ABI.  DDMC_EINVAL for null pointers,
 *    impossible sizes or parameters; DDMC_EUNSUPPORTED for a size the chosen
 *    algorithm does not handle; DDMC_ENOMEM when workspace allocation fails;
 *    DDMC_EHIP when a HIP call fails.  ddmc_last_error() returns a message for
 *    the last non-OK status of the calling thread.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key = the
 * replica's 64-bit seed (low word first) and counter = (site, sweep,
 * replica_id, purpose); purpose 0 draws initial spins, purpose 1 the
 * Metropolis moves.  Uniforms u = (x + 1/2) 2^-32 in FP64; the FP32 path
 * uses u = (floor(x / 2^9) + 1/2) 2^-23.
 */
#ifndef DDMC_H
#define DDMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DDMC_OK = 0,
    DDMC_EINVAL = 1,
    DDMC_EUNSUPPORTED = 2,
    DDMC_ENOMEM = 3,
    DDMC_EHIP = 4
} ddmc_status;

typedef enum {
    DDMC_F64 = 0,   /* spins, field and arithmetic in double */
    DDMC_F32 = 1    /* spins, field and arithmetic in float  */
} ddmc_prec;

typedef enum {
    DDMC_FIELD_AUTO = 0,    /* FFT where supported, else direct           */
    DDMC_FIELD_DIRECT = 1,  /* direct O(N^2) circular convolution          */
    DDMC_FIELD_FFT = 2,     /* FFT circular convolution: L = 2^a in
                               [8, 512] or 3 * 2^a in [24, 384] (FP64: not
                               512)                                        */
    DDMC_FIELD_FFT_LDS = 3  /* the FFT field, with metropolis_sweep,
                               metropolis_sweep_dev and metropolis_sample
                               run as one launch per call, each replica's
                               lattice, spectrum and transforms held in one
                               workgroup's LDS for every sweep of the call:
                               L in {8, 16, 24, 32, 48, 64} (FP64: up to
                               48).  Every other call of such a plan is that
                               of DDMC_FIELD_FFT.                           */
} ddmc_field_algo;

/* Parameters of one replica (an independent simulation).  Exchange units. */
typedef struct {
    double T;             /* temperature (k_B = 1), > 0                      */
    double J;             /* nearest-neighbour exchange, > 0 ferromagnetic  */
    double K2, K4;        /* anisotropy energy -K2 sz^2 - K4 sz^4 per site   */
    double g;             /* dipole strength C_D / J                         */
    uint64_t seed;        /* Philox key                                      */
    uint32_t replica_id;  /* Philox counter word 2                           */
    uint32_t model;       /* DDMC_HEISENBERG or DDMC_ISING                   */
} ddmc_replica_params;

/* Spin model of a replica.  Heisenberg: unit vectors, the trial spin uniform
 * on the sphere (Sec. 2.2, Appendix A).  Ising (the appendix on the dipolar
 * Ising model): s = (0, 0, +-1), the trial spin the reversal -s, the same
 * energy (anisotropy then constant) and acceptance rule. */
enum { DDMC_HEISENBERG = 0, DDMC_ISING = 1 };

/* Slots of one replica's row of `observables` output (Sec. 4.1). */
enum {
    DDMC_OBS_E = 0,         /* total energy per site (NaN when h == NULL)   */
    DDMC_OBS_EEX = 1,       /* exchange energy per site                     */
    DDMC_OBS_EDIP = 2,      /* dipole energy per site (NaN when h == NULL)  */
    DDMC_OBS_EANI = 3,      /* anisotropy energy per site                   */
    DDMC_OBS_MX = 4,        /* M = (1/N) sum_i s_i                           */
    DDMC_OBS_MY = 5,
    DDMC_OBS_MZ = 6,
    DDMC_OBS_MABS = 7,      /* |M|                                          */
    DDMC_OBS_MPAR = 8,      /* sqrt(Mx^2 + My^2), eq. (16) before averaging */
    DDMC_OBS_MZABS = 9,     /* |Mz|                                          */
    DDMC_OBS_NH = 10,       /* 10..12: n_h^x, n_h^y, n_h^z of eq. (14)       */
    DDMC_OBS_NV = 13,       /* 13..15: n_v^x, n_v^y, n_v^z                   */
    DDMC_OBS_ORIENT = 16,   /* 16..18: |n_h - n_v|/(n_h + n_v), eq. (15); 0 when no walls */
    DDMC_OBS_WALLDENS = 19, /* (n_v^z + n_h^z) / (4N)                        */
    DDMC_OBS_Q = 20,        /* (1/N) sum_i (arccos s_iz - pi/2)^2            */
    DDMC_OBS_ETASUM = 21,   /* (1/N) sum_i sqrt(eta_acc_i) after this sample */
    DDMC_OBS_MSTH = 22,     /* (1/N) sum_i s_iz (-1)^y: width-1 horizontal stripes (m_h) */
    DDMC_OBS_MSTV = 23,     /* (1/N) sum_i s_iz (-1)^x: width-1 vertical stripes (m_v);
                               m_st = sqrt(m_h^2 + m_v^2) (Ising appendix)   */
    DDMC_OBS_ETAS = 24,     /* (2/pi)(1/N) sum_i |arccos s_iz - pi/2|: the cone
                               angle of eq. (17) with the thermal average taken
                               over this one state, whose variance over samples
                               is the sigma^2_eta of eq. (18)                */
    DDMC_OBS_NONFINITE = 25,/* number of sites whose spin has a NaN or infinite
                               component, 0 for a healthy state; such a spin
                               also turns the energies and sums it enters into
                               NaN, and no update accepts a NaN energy change */
    DDMC_NOBS = 26
};

typedef struct ddmc_plan ddmc_plan;

/*
 * lattice_sum_kernel -- the lattice-summed dipole tensor (Sec. 2.1: the
 * periodic tiling of images G = (aL, bL), eq. (1) with C_D = 1, the sum over
 * images computed in advance for every separation).
 *
 *   W_ab(rho) = sum_{r = rho mod L, r in B, r != 0} w(r) (d_ab - 3 r_a r_b / r^2) / r^3
 *
 * with B the square |r_x|, |r_y| <= (M + 1/2) L centred on the field point,
 * w(r) = 1/2 per coordinate lying on the edge of B (1/4 at corners), 1
 * inside.  The truncation keeps W(rho) = W(-rho) and the square symmetry.
 * M = 8 sums |a|, |b| <= 8.
 *
 * M = DDMC_M_ALL (-1) sums every image, W_ab(rho) = sum over all G of the
 * tensor at rho + G (G = 0 omitted at rho = 0), by the Ewald-Harris split of
 * Sec. 2.1 (eqs. (3)-(5) at z = 0): screened real-space images plus the
 * reciprocal-lattice sum of the smooth remainder, W_zz = -(W_xx + W_yy).
 * It is the M -> infinity limit of the box sums (their error falls like
 * 1/M), e.g. W(0) = (S/L^3) diag(-1/2, -1/2, 1), S = 4 zeta(3/2) beta(3/2).
 *
 * L >= 1, M = -1 or 0 <= M <= 1024.  W64: device, double [4][L][L], written
 * in full.  Computed in FP64 on the GPU.
 */
#define DDMC_M_ALL (-1)

ddmc_status lattice_sum_kernel(int32_t L, int32_t M, double *W64, void *stream);

/*
 * ddmc_plan_create -- derive the kernel forms a field algorithm needs from
 * W64 (the output of lattice_sum_kernel for the same L) and allocate the
 * workspace for up to R_max replicas.  Synchronous.  L >= 2; the sweep calls
 * need L even.  DDMC_FIELD_FFT needs L = 2^a in [8, 512] or L = 3 * 2^a in
 * [24, 384] (FP64: not 512), else DDMC_EUNSUPPORTED; DDMC_FIELD_AUTO takes
 * the FFT where it is supported and the direct sum elsewhere.
 * *out receives the plan; destroy it with ddmc_plan_destroy.
 */
ddmc_status ddmc_plan_create(int32_t L, int32_t M, int32_t R_max, ddmc_prec prec,
                             ddmc_field_algo algo, const double *W64, ddmc_plan **out);
ddmc_status ddmc_plan_destroy(ddmc_plan *plan);

/*
 * ddmc_plan_device_bytes -- the device bytes ddmc_plan_create allocates and
 * keeps for a plan of these arguments (derived kernel forms and workspace;
 * the caller's spin, field and parameter arrays are not included), computed
 * without allocating, with AUTO resolved as plan creation resolves it: what a
 * caller that budgets HBM charges for a plan.  Plan creation also holds a
 * temporary FP64 scratch of 8 L (L/2 + 1) doubles while it builds the
 * kernel spectrum.  EINVAL / EUNSUPPORTED as ddmc_plan_create.
 */
ddmc_status ddmc_plan_device_bytes(int32_t L, int32_t R_max, ddmc_prec prec, ddmc_field_algo algo,
                                   uint64_t *bytes);

/* The plan's algorithm after AUTO is resolved (DDMC_FIELD_DIRECT or _FFT). */
ddmc_status ddmc_plan_algo(const ddmc_plan *plan, ddmc_field_algo *algo);

/*
 * replica_params_upload -- validate R host-side parameter records and copy
 * them to the device array dev_params (ddmc_replica_params[R]).  EINVAL if a
 * temperature is not > 0, a parameter is not finite (T = +inf is allowed:
 * every move is then accepted) or an unknown model; nothing is
 * copied then.  The records are handed to the device as the arguments of
 * small store kernels enqueued on `stream` (32 records per launch), which
 * capture them at enqueue time: the host array may be reused on return, the
 * call never waits for the stream (work already queued on it keeps running),
 * and the device array is written in stream order.
 */
ddmc_status replica_params_upload(int32_t R, const ddmc_replica_params *host_params,
                                  ddmc_replica_params *dev_params, void *stream);

/*
 * local_field -- h = W (*) s for R replicas (Sec. 2.1, eq. (2): the field of
 * all spins and their images at every site, self images included):
 *   h_x = Wxx (*) s_x + Wxy (*) s_y,  h_y = Wxy (*) s_x + Wyy (*) s_y,
 *   h_z = Wzz (*) s_z,   (A (*) b)_i = sum_j A(r_i - r_j mod L) b_j.
 * color = -1 writes every site; 0 or 1 writes only the sites of that colour
 * and leaves the others untouched.  s, h: device [R][3][L][L] of the plan's
 * precision, non-overlapping.  1 <= R <= R_max (R = 0 is a no-op).
 */
ddmc_status local_field(ddmc_plan *plan, int32_t R, const void *s, void *h, int32_t color,
                        void *stream);

/*
 * init_spins -- every site of every replica uniform on the unit sphere from
 * the replica's purpose-0 draws (counter (site, 0, replica_id, 0)); Ising
 * replicas get s = (0, 0, +1) where the first draw u0 < 1/2, else (0, 0, -1).
 * params: device ddmc_replica_params[R].  s: device [R][3][L][L].
 */
ddmc_status init_spins(ddmc_plan *plan, int32_t R, const ddmc_replica_params *params, void *s,
                       void *stream);

/*
 * metropolis_sweep -- nsweeps checkerboard sweeps, sweep indices
 * sweep0 .. sweep0 + nsweeps - 1 (each < 2^32).  Each sweep is two half-
 * sweeps, colour 0 then colour 1.  A half-sweep computes the dipolar field
 * of the current state at the sites of its colour, then every site k of the
 * colour proposes S uniform on the sphere and accepts with the Metropolis
 * rule (Sec. 2.2, eq. (7)) using the energy change
 *   dE = -J d.(sum of the 4 neighbours) + g (d.h_k + 1/2 d^T W(0) d)
 *        - K2 (Sz^2 - sz^2) - K4 (Sz^4 - sz^4),          d = S - s_k,
 * with the field frozen for the whole half-sweep: the approximation of
 * Sec. 3.2 (H3 - H1 ~ H2 - H0) applied to all same-colour sites at once.
 * Same-colour sites are never nearest neighbours, so the exchange and
 * anisotropy parts are exact.
 * params: device [R].  s: device [R][3][L][L], updated in place.
 * accepted: device uint64[R], incremented by the accepted moves (may be NULL).
 * L must be even.
 */
ddmc_status metropolis_sweep(ddmc_plan *plan, int32_t R, const ddmc_replica_params *params,
                             void *s, uint64_t sweep0, int32_t nsweeps, uint64_t *accepted,
                             void *stream);

/*
 * metropolis_sweep_dev -- metropolis_sweep with each replica's first sweep
 * index read on the device from sweep_counter[r] (device uint64_t[R]) when
 * the kernels run; the call's kernels (on the same stream) add nsweeps to
 * every counter.  Replicas of one call may therefore be at different
 * points of their chains (requests admitted at different times), and every
 * argument is fixed when the call is enqueued, so a sequence of these calls
 * (with observables) can be captured once in a HIP graph and replayed, each
 * replay continuing the chains.  Sweep indices are taken modulo 2^32.
 */
ddmc_status metropolis_sweep_dev(ddmc_plan *plan, int32_t R, const ddmc_replica_params *params,
                                 void *s, uint64_t *sweep_counter, int32_t nsweeps,
                                 uint64_t *accepted, void *stream);

/*
 * metropolis_sweep_multi -- metropolis_sweep_dev for ngroups groups of
 * replicas of different lattice sizes in one launch (1 <= ngroups <=
 * DDMC_MULTI_MAX_GROUPS): group k has R[k] replicas of plans[k]'s size with
 * parameters params[k] (device [R[k]]), spins s[k] (device [R[k]][3][L][L]),
 * device sweep counters sweep_counter[k] ([R[k]], advanced by nsweeps) and
 * accept counts accepted[k] ([R[k]], or accepted / accepted[k] NULL).  The
 * argument arrays themselves are host arrays of ngroups entries.  Every plan
 * must be of DDMC_FIELD_FFT_LDS and of one precision, and each group's
 * replicas follow exactly the chains metropolis_sweep_dev of its plan gives
 * them (one workgroup per replica; the groups do not interact).  R[k] = 0
 * skips a group; R[k] above plans[k]'s R_max is EINVAL.
 */
#define DDMC_MULTI_MAX_GROUPS 8

ddmc_status metropolis_sweep_multi(int32_t ngroups, ddmc_plan *const *plans, const int32_t *R,
                                   const ddmc_replica_params *const *params, void *const *s,
                                   uint64_t *const *sweep_counter, int32_t nsweeps, uint64_t *const *accepted,
                                   void *stream);

/*
 * metropolis_sample -- the sampling loop of Sec. 4: nsweeps sweeps exactly as
 * metropolis_sweep_dev (same states, sweep indices and accept counts), and
 * after each sweep t one sample of the observables of the state it left:
 * obs[t][r] is what `observables` returns for that state with its full field
 * (energies included), and eta_acc, when given, is advanced once per sample.
 * obs: device double [nsweeps][R][DDMC_NOBS] (not NULL).  eta_acc: device
 * double [R][L][L] or NULL.  accepted: device uint64[R] or NULL.  On the FFT
 * path the sums ride in the sweep's own kernels (the colour-0 row kernel of
 * sweep t sums the state after sweep t-1); a DDMC_FIELD_FFT_LDS plan sums
 * each sample inside its one-workgroup sweep, from the field its colour-0
 * half-sweep computes, with one more field evaluation after the last sweep;
 * the direct path runs one local_field and one observables per sweep.  Sums are FP64 in an order that
 * depends only on L, so results do not depend on R or on the other replicas.
 */
ddmc_status metropolis_sample(ddmc_plan *plan, int32_t R, const ddmc_replica_params *params,
                              void *s, uint64_t *sweep_counter, int32_t nsweeps, double *obs,
                              double *eta_acc, uint64_t *accepted, void *stream);

/*
 * metropolis_sweep_coset -- the paper's own simultaneous-update schedule
 * (Sec. 3.1): the sites i = (a l, b l) + i1 of one coset of the sublattice
 * l Z^2 are updated at once with the frozen field of the state before them
 * (the approximation of Sec. 3.2), for the l^2 cosets i1 = (cx, cy) in the
 * order k = cy l + cx = 0 .. l^2 - 1, so that a sweep proposes every site
 * once (the paper draws i1 at random each iteration; the fixed cycle makes a
 * sweep exactly N attempts).  Each site uses the same (site, sweep) draws,
 * proposal and acceptance rule as metropolis_sweep; sweep indices come from
 * sweep_counter[r] (device uint64[R]), advanced by nsweeps by the call's
 * kernels.  2 <= l <= L and l divides L (l need not be a power of two: L = 48
 * takes l = 3, 6, 12, ...).  With l = L every coset is one site and the sweep is exact
 * sequential Metropolis in index order; each coset costs one field
 * evaluation, so a sweep costs l^2 / 2 checkerboard half-sweeps.  When a
 * coset holds at most 16 sites ((L/l)^2 <= 16) and L <= 64, one workgroup per
 * replica runs the whole call instead: it starts from the full field of the
 * state and brings it up to date after each coset from the accepted changes
 * alone (accumulated in FP64), so the decisions agree with the full-field
 * form except where one lies within rounding of its threshold.
 * s: device [R][3][L][L] updated in place; accepted: device uint64[R] or NULL.
 */
ddmc_status metropolis_sweep_coset(ddmc_plan *plan, int32_t R, const ddmc_replica_params *params,
                                   void *s, int32_t l, uint64_t *sweep_counter, int32_t nsweeps,
                                   uint64_t *accepted, void *stream);

/*
 * parallel_tempering_swap -- replica exchange between neighbours of a
 * temperature ladder (the companion of the Sec. 4 temperature scans for the
 * ladder workload): for every pair (r, r + 1) with r = parity mod 2 the two
 * states are exchanged with probability
 *   min(1, exp((1/T_r - 1/T_{r+1}) (E_r - E_{r+1}))),
 * E the total energies N * obs[r][DDMC_OBS_E] of the current states (a NaN
 * energy never exchanges).  The uniform is u0 of Philox counter
 * (r, sweep_counter[r], replica_id_r, 2) under seed_r, so graph replays that
 * advance the counters draw afresh.  Temperatures stay with their replica
 * slots (and so do the per-slot eta accumulators); only the states move.
 * The pair must share J, K2, K4, g and the model.
 * obs: device double [R][DDMC_NOBS], a sample of the current states with
 * energies (metropolis_sample's last row).  sweep_counter: device uint64[R].
 * swaps: device uint64[R], swaps[r] += 1 per exchange of pair (r, r + 1), or
 * NULL.  R < 2 is a no-op.
 */
ddmc_status parallel_tempering_swap(ddmc_plan *plan, int32_t R, const ddmc_replica_params *params,
                                    void *s, const double *obs, const uint64_t *sweep_counter,
                                    int32_t parity, uint64_t *swaps, void *stream);

/*
 * coset_error_bound -- the bound of eq. (10) on the error in H3 - H1 made by
 * the coset update, in units of C_D: 2 / r^3 per simultaneously moved
 * partner (the perpendicular maximum of eq. (8)).  all_images = 0: every other
 * site of the coset once, at its nearest image (the reading that reproduces
 * the 0.14 % the paper quotes for L = 64, l = 32, k_B T = 0.1 C_D, through
 * exp(eps / T) - 1); all_images = 1: every image of every partner,
 * 2 S / l^3 with S = 4 zeta(3/2) beta(3/2).  Host computation.
 */
ddmc_status coset_error_bound(int32_t L, int32_t l, int32_t all_images, double *eps);

/*
 * trial_energies -- diagnostic form of one half-sweep's decisions: for every
 * site of `color`, the proposed spin S, the energy change dE computed with
 * the given field h (normally local_field of s) and the acceptance uniform
 * u, exactly as metropolis_sweep computes them; nothing is applied.
 * dE, u: device [R][L][L] of the plan's precision (sites of the other colour
 * untouched); S: device [R][3][L][L] (may be NULL).
 */
ddmc_status trial_energies(ddmc_plan *plan, int32_t R, const ddmc_replica_params *params,
                           const void *s, const void *h, uint32_t sweep, int32_t color,
                           void *dE, void *u, void *S, void *stream);

/*
 * spins_convert -- copy R states [R][3][L][L] from one precision to the other
 * (device to device, on `stream`), e.g. to take the FP64 energy of an FP32
 * state: spins_convert to FP64, local_field and observables with an FP64
 * plan (the full-energy resync of eqs. (11)-(12) in double precision).
 * src and dst must not overlap.  R = 0 is a no-op.
 */
ddmc_status spins_convert(int32_t R, int32_t L, const void *src, ddmc_prec src_prec, void *dst,
                          ddmc_prec dst_prec, void *stream);

/*
 * observables -- one sample of the observables of Sec. 4.1 for each replica:
 * energies per site, magnetization M, |M|, M_par (eq. (16)), wall counts
 * n_h, n_v (eq. (14), sgn(0) = 0), orientational order (eq. (15)), wall
 * density, and the cone-angle accumulators of eq. (17):
 * eta_acc[r][i] += (arccos s_iz - pi/2)^2, after which
 * out[DDMC_OBS_ETASUM] = (1/N) sum_i sqrt(eta_acc[r][i]), so that after n
 * samples eta = (2/pi) out[DDMC_OBS_ETASUM] / sqrt(n).
 * h: the field of s (device [R][3][L][L], from local_field with color -1) or
 * NULL to skip the dipole and total energies.  out: device double
 * [R][DDMC_NOBS].  eta_acc: device double [R][L][L] or NULL.  Sums are
 * accumulated in FP64 in a fixed order (bitwise reproducible).
 */
ddmc_status observables(ddmc_plan *plan, int32_t R, const ddmc_replica_params *params,
                        const void *s, const void *h, double *out, double *eta_acc,
                        void *stream);

/*
 * observables_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): `observables` without a plan and without any allocation, the
 * lattice size L (1 <= L <= 4096) and the precision of s and h given
 * directly.  Same arguments, layouts and results (bit for bit) as
 * `observables`, from the same kernels.  The per-block partial sums live in a
 * static device array of the library, DDMC_NOALLOC_R_MAX * 64 * 18 doubles
 * (2.25 MiB on each GPU the library runs on, held until the process ends);
 * every entry a call reads it has written first, so nothing needs clearing.
 * R > DDMC_NOALLOC_R_MAX: DDMC_EINVAL.  Every call on one GPU uses that GPU's
 * array: calls that may overlap (different streams, or different host
 * threads) race and must be ordered by the caller.
 */
#define DDMC_NOALLOC_R_MAX 256

ddmc_status observables_noalloc(int32_t L, ddmc_prec prec, int32_t R, const ddmc_replica_params *params,
                                const void *s, const void *h, double *out, double *eta_acc, void *stream);

/* Kernels timed by the plan's profiler. */
typedef enum {
    DDMC_KERNEL_DIRECT_FIELD = 0,    /* direct field and its split reduction     */
    DDMC_KERNEL_UPDATE = 1,          /* colour update of the direct path; coset  */
                                     /* sweeps of one workgroup per replica      */
    DDMC_KERNEL_FFT_COLUMNS = 2,     /* column FFTs + kernel multiply            */
    DDMC_KERNEL_FFT_ROWS_SWEEP = 3,  /* row FFTs fused with the colour update    */
    DDMC_KERNEL_FFT_ROWS = 4,        /* row FFTs of local_field / sweep start    */
    DDMC_KERNEL_OBSERVABLES = 5,     /* observables passes; final sample of a    */
                                     /* metropolis_sample call                   */
    DDMC_KERNEL_FFT_ROWS_SAMPLE = 6, /* row update that first sums observables   */
    DDMC_KERNEL_COUNT = 7
} ddmc_kernel_id;

/*
 * ddmc_plan_profile -- enable (1) or disable (0) kernel timing for the calls
 * made with this plan: each instrumented launch is bracketed by a pair of HIP
 * events recorded on the launch stream.  Enabling clears the totals.
 * ddmc_plan_profile_read -- waits for the recorded events and returns the
 * total milliseconds and number of launches of one kernel class since the
 * profiler was enabled.  Tracing and timing only; results are unchanged.
 */
ddmc_status ddmc_plan_profile(ddmc_plan *plan, int32_t enable);
ddmc_status ddmc_plan_profile_read(ddmc_plan *plan, int32_t kernel, double *total_ms, int64_t *launches);

/* Message for the last non-OK status returned on the calling thread. */
const char *ddmc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DDMC_H */
