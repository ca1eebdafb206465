// internal.hpp -- plan object and kernel launchers shared by the library's
// translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "ddmc.h"

struct ddmc_prof_pair {
    hipEvent_t start, stop;
    int kernel;
};

struct ddmc_plan {
    int32_t L = 0, M = 0, R_max = 0;
    ddmc_prec prec = DDMC_F64;
    ddmc_field_algo algo = DDMC_FIELD_DIRECT;
    int device = 0;
    double W0[4] = {0, 0, 0, 0};   // self-image tensor W(0): xx, yy, xy, zz
    void *W = nullptr;             // [4][N] kernel in the plan precision
    void *h_ws = nullptr;          // [R_max][3][N] field of the current half-sweep
    void *part_ws = nullptr;       // direct-sum partials [split][R][3][N]
    size_t part_elems = 0;         // capacity of part_ws in elements
    void *spec_ws = nullptr;       // FFT spectra [R_max][3][L][L/2] complex
    void *what = nullptr;          // FFT kernel spectrum [L/2+1][L][4] real
    void *twiddle = nullptr;       // FFT twiddles
    void *obs_ws = nullptr;        // observables partial sums [R_max][OBS_MAX_BLOCKS][OBS_NACC]
    unsigned int *done_ws = nullptr;   // [R_max] completion counters of the last launch of a direct sweep call
    unsigned int *slot_ws = nullptr;   // FFT: [R_max][row blocks] accepted moves per row block
    double *rows_obs_ws = nullptr;     // FFT: [R_max][entries][OBS_NACC] observable sums of a sampling sweep
    bool sweep_lds = false;            // FFT plan whose checkerboard sweeps run one workgroup per replica
    // opt-in kernel timing with HIP events on the launch stream
    mutable bool prof = false;
    mutable std::vector<ddmc_prof_pair> prof_pending;
    mutable std::vector<hipEvent_t> prof_free;
    mutable double prof_ms[DDMC_KERNEL_COUNT] = {};
    mutable int64_t prof_n[DDMC_KERNEL_COUNT] = {};
};

namespace ddmc {

constexpr int OBS_MAX_BLOCKS = 64;
constexpr int OBS_NACC = 18;

void set_error(const std::string &msg);
ddmc_status fail(ddmc_status st, const std::string &msg);
ddmc_status hip_check(hipError_t e, const char *what);

// Records a HIP event pair around the launches made during its lifetime
// when the plan's profiling is on; the pair is resolved lazily.
struct prof_scope {
    const ddmc_plan *p;
    int kernel;
    hipStream_t st;
    hipEvent_t start = nullptr;
    prof_scope(const ddmc_plan *plan, int k, hipStream_t s);
    ~prof_scope();
};
void prof_drain(const ddmc_plan *p, size_t n);

// one element type for every array a plan touches
template <typename T> struct vec4a;
template <> struct __align__(16) vec4a<float> { float a, b, c, d; };
template <> struct __align__(32) vec4a<double> { double a, b, c, d; };

// lattice sum (FP64)
hipError_t launch_lattice_sum(int L, int M, double *W64, hipStream_t st);
// W64 -> plan precision copy
template <typename T> hipError_t launch_convert_kernel(int L, const double *W64, T *W, hipStream_t st);

hipError_t launch_spins_convert(long n, const void *src, bool src64, void *dst, bool dst64, hipStream_t st);

// direct field
template <typename T>
ddmc_status direct_field(ddmc_plan *p, int R, const T *s, T *h, int color, hipStream_t st);
size_t direct_partial_elems(int L, int R_max, size_t elem);

// FFT field
template <typename T>
ddmc_status fft_plan_init(ddmc_plan *p, const double *W64);
template <typename T>
ddmc_status fft_field(ddmc_plan *p, int R, const T *s, T *h, int color, hipStream_t st);
template <typename T>
ddmc_status fft_sweep(ddmc_plan *p, int R, const ddmc_replica_params *params, T *s, uint64_t *sweep_ctr,
                      uint64_t sweep0, int nsweeps, uint64_t *accepted, double *obs, double *eta_acc,
                      hipStream_t st);
template <typename T>
ddmc_status fft_sweep_coset(ddmc_plan *p, int R, const ddmc_replica_params *params, T *s, int l,
                            uint64_t *sweep_ctr, int nsweeps, uint64_t *accepted, hipStream_t st);
void fft_plan_free(ddmc_plan *p);
// device bytes fft_plan_init allocates for (L, R_max, prec) (0: size not supported)
size_t fft_plan_bytes(int L, int R_max, ddmc_prec prec);
bool fft_supported(int L, ddmc_prec prec);

// the l-coset schedule with one workgroup per replica and an incrementally
// updated field, for cosets of at most 16 sites and L <= 64
bool coset_local_ok(int L, int l, ddmc_prec prec);
template <typename T>
ddmc_status coset_local_sweep(ddmc_plan *p, int R, const ddmc_replica_params *params, T *s, int l,
                              uint64_t *sweep_ctr, int nsweeps, uint64_t *accepted, hipStream_t st);

// replica records to the device through kernel arguments (asynchronous, no host wait)
hipError_t launch_params_store(int R, const ddmc_replica_params *host, ddmc_replica_params *dev, hipStream_t st);

// checkerboard sweeps with each replica's lattice in one workgroup's LDS for
// a whole call (L <= 64 FP32, L <= 48 FP64), several plans (lattice sizes)
// per launch; ctr NULL: sweep indices sweep0 + t; obs (single group only):
// one observables sample after each sweep, [nsweeps][R][DDMC_NOBS], with the
// cone-angle accumulators eta_acc [R][N] or NULL
bool lds_sweep_ok(int L, ddmc_prec prec);
template <typename T>
ddmc_status lds_sweep(int ngroups, ddmc_plan *const *plans, const int *R, const ddmc_replica_params *const *params,
                      T *const *s, uint64_t *const *ctr, uint64_t sweep0, int nsweeps, uint64_t *const *accepted,
                      double *obs, double *eta_acc, hipStream_t st);

// sweep kernels
template <typename T>
hipError_t launch_init_spins(const ddmc_plan *p, int R, const ddmc_replica_params *params, T *s,
                             hipStream_t st);
struct sweep_book;
// accept-count / sweep-counter bookkeeping of one half-sweep launch
sweep_book make_book(const ddmc_plan *p, uint64_t *accepted, uint64_t *ctr, int finalize, uint64_t advance);

// colour half-sweep (coset_l = 0, color 0/1) or coset k = color of the l-spaced update (coset_l = l)
template <typename T>
hipError_t launch_update(const ddmc_plan *p, int R, const ddmc_replica_params *params, T *s,
                         const T *h, int color, uint64_t *sweep_ctr, uint32_t sweep, uint64_t *accepted,
                         int finalize, uint64_t advance, hipStream_t st, int coset_l = 0);
template <typename T>
hipError_t launch_trial(const ddmc_plan *p, int R, const ddmc_replica_params *params, const T *s,
                        const T *h, int color, uint32_t sweep, T *dE, T *u, T *S, hipStream_t st);
// reduction of nblk observable partial sums per replica into out[R][NOBS]
// (partial may be NULL) and / or the fold of nslot accept slots per replica
hipError_t launch_obs_final(const ddmc_plan *p, int R, int nblk, const double *partial, int have_h, int have_eta,
                            double *out, const unsigned int *slots, int nslot, uint64_t *accepted, hipStream_t st);
// replica exchange between ladder neighbours (r, r + 1), r = parity mod 2
template <typename T>
hipError_t launch_pt_swap(const ddmc_plan *p, int R, const ddmc_replica_params *params, T *s, const double *obs,
                          const uint64_t *ctr, int parity, uint64_t *swaps, hipStream_t st);
template <typename T>
hipError_t launch_observables(const ddmc_plan *p, int R, const ddmc_replica_params *params,
                              const T *s, const T *h, double *out, double *eta_acc, hipStream_t st);
// the same passes with the partial sums in the library's static device array
// (DDMC_NOALLOC_R_MAX replicas); no allocation
template <typename T>
hipError_t launch_observables_noalloc(int L, int R, const ddmc_replica_params *params, const T *s, const T *h,
                                      double *out, double *eta_acc, hipStream_t st);

}  // namespace ddmc
