// k_observables.hip -- one sample of the observables of Sec. 4.1 per replica:
// energies, magnetization, planar magnetization (eq. (16)), wall counts
// (eq. (14)), orientational order (eq. (15)) and the cone-angle accumulators
// of eq. (17).  Each replica's sites are split into a fixed number of
// contiguous chunks (a function of N only); a block sums one chunk in FP64
// with wave shuffles and a fixed LDS order, and a second kernel adds the
// chunk sums in chunk order, so results are bitwise reproducible and do not
// depend on which other replicas share the launch.
#include <mutex>

#include "obs_common.hpp"

namespace ddmc {

namespace {

constexpr int OBS_THREADS = 256;
constexpr int NACC = obs::NACC;

// Pass 1: block b of replica r sums its contiguous chunk of sites into
// partial[r][b][NACC] (per-thread FP64 sums, wave shuffles, fixed LDS order).
template <typename T>
__global__ void __launch_bounds__(OBS_THREADS)
k_obs_partial(int L, int nblk, const ddmc_replica_params *__restrict__ params, const T *__restrict__ s,
              const T *__restrict__ h, double *__restrict__ eta_acc, double *__restrict__ partial)
{
    __shared__ double red[OBS_THREADS / 64][NACC];
    const long N = (long)L * L;
    const int b = blockIdx.x, r = blockIdx.y;
    const long chunk = (N + nblk - 1) / nblk;
    const long i0 = (long)b * chunk, i1 = min(N, i0 + chunk);
    const ddmc_replica_params p = params[r];
    const T *sr = s + (long)r * 3 * N;
    const T *hr = h ? h + (long)r * 3 * N : nullptr;
    double *acc_r = eta_acc ? eta_acc + (long)r * N : nullptr;
    double a[NACC];
#pragma unroll
    for (int k = 0; k < NACC; ++k) a[k] = 0.0;
    for (long i = i0 + threadIdx.x; i < i1; i += OBS_THREADS) obs::site<T>(a, L, N, sr, hr, acc_r, i, p);
    obs::block_sum<OBS_THREADS>(a, red, partial + ((long)r * nblk + b) * NACC);
}

// Pass 2: per replica, add the block partials (fixed order) and form the
// outputs; optionally add a sweep's per-block accept counts to accepted[r].
constexpr int FINAL_THREADS = 256;
__global__ void __launch_bounds__(FINAL_THREADS)
k_obs_final(int L, int nblk, const double *__restrict__ partial, int have_h, int have_eta,
            double *__restrict__ out, const unsigned int *__restrict__ slots, int nslot,
            unsigned long long *__restrict__ accepted)
{
    __shared__ double tot[NACC];
    const int r = blockIdx.x;
    if (slots && accepted) obs::fold_slots(slots + (long)r * nslot, nslot, accepted + r);
    if (!partial) return;
    obs::partial_sum<FINAL_THREADS / 64>(partial + (long)r * nblk * NACC, nblk, tot);
    if (threadIdx.x == 0) obs::finish(L, tot, have_h != 0, have_eta != 0, out + (long)r * DDMC_NOBS);
}

}  // namespace

static int obs_blocks(long N)
{
    long b = N / 512;
    if (b < 1) b = 1;
    if (b > OBS_MAX_BLOCKS) b = OBS_MAX_BLOCKS;
    return (int)b;
}

// Both passes with the partial sums in `partial` ([R][obs_blocks(N)][NACC]).
template <typename T>
static hipError_t obs_passes(int L, int R, const ddmc_replica_params *params, const T *s, const T *h, double *out,
                             double *eta_acc, double *partial, hipStream_t st)
{
    const long N = (long)L * L;
    const int nblk = obs_blocks(N);
    hipLaunchKernelGGL(k_obs_partial<T>, dim3(nblk, R), dim3(OBS_THREADS), 0, st, L, nblk, params, s, h, eta_acc,
                       partial);
    hipLaunchKernelGGL(k_obs_final, dim3(R), dim3(FINAL_THREADS), 0, st, L, nblk, partial,
                       h != nullptr ? 1 : 0, eta_acc != nullptr ? 1 : 0, out, nullptr, 0, nullptr);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_observables(const ddmc_plan *p, int R, const ddmc_replica_params *params, const T *s,
                              const T *h, double *out, double *eta_acc, hipStream_t st)
{
    prof_scope ps(p, DDMC_KERNEL_OBSERVABLES, st);
    return obs_passes<T>(p->L, R, params, s, h, out, eta_acc, reinterpret_cast<double *>(p->obs_ws), st);
}

// ---- the allocation-free form: the partial sums in a static device array.
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is taken once per device with hipGetSymbolAddress (with the
// device current) and only that address is passed to kernels.
static __device__ __align__(256) double scratch[(size_t)DDMC_NOALLOC_R_MAX * OBS_MAX_BLOCKS * OBS_NACC];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[MAX_DEVICES] = {};
}  // namespace

// Device address of the calling thread's current device's copy of `scratch`.
static hipError_t scratch_address(double **ptr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = reinterpret_cast<double *>(a);
    }
    *ptr = g_scratch_dev[dev];
    return hipSuccess;
}

template <typename T>
hipError_t launch_observables_noalloc(int L, int R, const ddmc_replica_params *params, const T *s, const T *h,
                                      double *out, double *eta_acc, hipStream_t st)
{
    double *partial = nullptr;
    const hipError_t e = scratch_address(&partial);
    if (e != hipSuccess) return e;
    return obs_passes<T>(L, R, params, s, h, out, eta_acc, partial, st);
}

template hipError_t launch_observables_noalloc<float>(int, int, const ddmc_replica_params *, const float *,
                                                      const float *, double *, double *, hipStream_t);
template hipError_t launch_observables_noalloc<double>(int, int, const ddmc_replica_params *, const double *,
                                                       const double *, double *, double *, hipStream_t);

hipError_t launch_obs_final(const ddmc_plan *p, int R, int nblk, const double *partial, int have_h, int have_eta,
                            double *out, const unsigned int *slots, int nslot, uint64_t *accepted, hipStream_t st)
{
    prof_scope ps(p, DDMC_KERNEL_OBSERVABLES, st);
    hipLaunchKernelGGL(k_obs_final, dim3(R), dim3(FINAL_THREADS), 0, st, p->L, nblk, partial, have_h, have_eta, out,
                       slots, nslot, reinterpret_cast<unsigned long long *>(accepted));
    return hipGetLastError();
}

template hipError_t launch_observables<float>(const ddmc_plan *, int, const ddmc_replica_params *, const float *,
                                              const float *, double *, double *, hipStream_t);
template hipError_t launch_observables<double>(const ddmc_plan *, int, const ddmc_replica_params *,
                                               const double *, const double *, double *, double *, hipStream_t);

}  // namespace ddmc
