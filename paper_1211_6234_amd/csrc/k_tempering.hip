// k_tempering.hip -- replica exchange between neighbours of a temperature
// ladder (parallel tempering), the companion of the Sec. 4 temperature scans
// for the ladder workload.  One launch treats every pair (r, r + 1) with
// r = parity mod 2: each block of a pair recomputes the pair's decision (one
// Philox draw) and, when the exchange is taken, swaps its chunk of the two
// states, so no block waits for another.
#include "device_common.hpp"
#include "internal.hpp"

namespace ddmc {

namespace {

constexpr int PT_THREADS = 256;

template <typename T>
__global__ void __launch_bounds__(PT_THREADS)
k_pt_swap(int R, long N, long chunk, const ddmc_replica_params *__restrict__ params, T *__restrict__ s,
          const double *__restrict__ obs, const unsigned long long *__restrict__ ctr, int parity,
          unsigned long long *__restrict__ swaps)
{
    const int r = 2 * (int)blockIdx.y + parity;
    if (r + 1 >= R) return;
    const ddmc_replica_params a = params[r], b = params[r + 1];
    // total energies of the current states; a NaN energy never exchanges
    const double ea = obs[(long)r * DDMC_NOBS + DDMC_OBS_E] * (double)N;
    const double eb = obs[(long)(r + 1) * DDMC_NOBS + DDMC_OBS_E] * (double)N;
    const double delta = (1.0 / a.T - 1.0 / b.T) * (ea - eb);
    const u32x4 d = draw(a.seed, a.replica_id, (uint32_t)ctr[r], (uint32_t)r, 2u);
    if (!(delta >= 0.0 || to_unit<double>(d.v[0]) < exp(delta))) return;
    if (blockIdx.x == 0 && threadIdx.x == 0 && swaps) swaps[r] += 1ull;
    const long n3 = 3 * N;
    T *sa = s + (long)r * n3, *sb = sa + n3;
    const long i0 = (long)blockIdx.x * chunk, i1 = min(n3, i0 + chunk);
    for (long i = i0 + threadIdx.x; i < i1; i += PT_THREADS) {
        const T t = sa[i];
        sa[i] = sb[i];
        sb[i] = t;
    }
}

}  // namespace

template <typename T>
hipError_t launch_pt_swap(const ddmc_plan *p, int R, const ddmc_replica_params *params, T *s, const double *obs,
                          const uint64_t *ctr, int parity, uint64_t *swaps, hipStream_t st)
{
    const long N = (long)p->L * p->L;
    const long n3 = 3 * N;
    const long chunk = 16L * PT_THREADS;
    const long nchunk = (n3 + chunk - 1) / chunk;
    const int npairs = (R - parity) / 2;
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pt_swap<T>, dim3((unsigned)nchunk, (unsigned)npairs), dim3(PT_THREADS), 0, st, R, N, chunk,
                       params, s, obs, reinterpret_cast<const unsigned long long *>(ctr), parity,
                       reinterpret_cast<unsigned long long *>(swaps));
    return hipGetLastError();
}

template hipError_t launch_pt_swap<float>(const ddmc_plan *, int, const ddmc_replica_params *, float *,
                                          const double *, const uint64_t *, int, uint64_t *, hipStream_t);
template hipError_t launch_pt_swap<double>(const ddmc_plan *, int, const ddmc_replica_params *, double *,
                                           const double *, const uint64_t *, int, uint64_t *, hipStream_t);

}  // namespace ddmc
