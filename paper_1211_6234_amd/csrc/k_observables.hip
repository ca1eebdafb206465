// k_observables.hip -- one sample of the observables of Sec. 4.1 per replica:
// energies, magnetization, planar magnetization (eq. (16)), wall counts
// (eq. (14)), orientational order (eq. (15)) and the cone-angle accumulators
// of eq. (17).  Each replica's sites are split into a fixed number of
// contiguous chunks (a function of N only); a block sums one chunk in FP64
// with wave shuffles and a fixed LDS order, and a second kernel adds the
// chunk sums in chunk order, so results are bitwise reproducible and do not
// depend on which other replicas share the launch.
#include "device_common.hpp"
#include "internal.hpp"

namespace ddmc {

namespace {

constexpr int OBS_THREADS = 256;
constexpr int NACC = OBS_NACC;   // ex, dip, ani, mx, my, mz, nh[3], nv[3], q, etasum

__device__ __forceinline__ int sgn_of(double v) { return (v > 0.0) - (v < 0.0); }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// outputs of one replica from its 14 totals
__device__ void finish(int L, int r, const double *t, bool have_h, bool have_eta, double *__restrict__ out)
{
    const double N = (double)L * (double)L;
    const double invN = 1.0 / N;
    double *o = out + (long)r * DDMC_NOBS;
    for (int k = 0; k < DDMC_NOBS; ++k) o[k] = 0.0;
    const double nanv = __longlong_as_double(0x7ff8000000000000ll);
    o[DDMC_OBS_EEX] = t[0] * invN;
    o[DDMC_OBS_EDIP] = have_h ? t[1] * invN : nanv;
    o[DDMC_OBS_EANI] = t[2] * invN;
    o[DDMC_OBS_E] = have_h ? (t[0] + t[1] + t[2]) * invN : nanv;
    const double mx = t[3] * invN, my = t[4] * invN, mz = t[5] * invN;
    o[DDMC_OBS_MX] = mx;
    o[DDMC_OBS_MY] = my;
    o[DDMC_OBS_MZ] = mz;
    o[DDMC_OBS_MABS] = sqrt(mx * mx + my * my + mz * mz);
    o[DDMC_OBS_MPAR] = sqrt(mx * mx + my * my);
    o[DDMC_OBS_MZABS] = fabs(mz);
    for (int c = 0; c < 3; ++c) {
        const double nh = t[6 + c], nv = t[9 + c];
        o[DDMC_OBS_NH + c] = nh;
        o[DDMC_OBS_NV + c] = nv;
        o[DDMC_OBS_ORIENT + c] = (nh + nv) > 0.0 ? fabs(nh - nv) / (nh + nv) : 0.0;
    }
    o[DDMC_OBS_WALLDENS] = (t[11] + t[8]) / (4.0 * N);
    o[DDMC_OBS_Q] = t[12] * invN;
    o[DDMC_OBS_ETASUM] = have_eta ? t[13] * invN : nanv;
}


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
    const double HALF_PI = 1.57079632679489661923;

    double a[NACC];
#pragma unroll
    for (int k = 0; k < NACC; ++k) a[k] = 0.0;

    for (long i = i0 + threadIdx.x; i < i1; i += OBS_THREADS) {
        const int x = (int)(i % L), y = (int)(i / L);
        const long ix = (long)y * L + (x + 1 == L ? 0 : x + 1);
        const long iy = (long)(y + 1 == L ? 0 : y + 1) * L + x;
        const double sx = sr[i], sy = sr[N + i], sz = sr[2 * N + i];
        const double xx = sr[ix], xy = sr[N + ix], xz = sr[2 * N + ix];
        const double yx = sr[iy], yy = sr[N + iy], yz = sr[2 * N + iy];
        a[0] += -p.J * (sx * (xx + yx) + sy * (xy + yy) + sz * (xz + yz));
        if (hr) a[1] += 0.5 * p.g * (sx * (double)hr[i] + sy * (double)hr[N + i] + sz * (double)hr[2 * N + i]);
        const double z2 = sz * sz;
        a[2] += -(p.K2 * z2 + p.K4 * z2 * z2);
        a[3] += sx;
        a[4] += sy;
        a[5] += sz;
        a[6] += (double)(1 - sgn_of(sx) * sgn_of(xx));
        a[7] += (double)(1 - sgn_of(sy) * sgn_of(xy));
        a[8] += (double)(1 - sgn_of(sz) * sgn_of(xz));
        a[9] += (double)(1 - sgn_of(sx) * sgn_of(yx));
        a[10] += (double)(1 - sgn_of(sy) * sgn_of(yy));
        a[11] += (double)(1 - sgn_of(sz) * sgn_of(yz));
        const double zc = fmin(1.0, fmax(-1.0, sz));
        const double dth = acos(zc) - HALF_PI;
        a[12] += dth * dth;
        if (acc_r) {
            const double v = acc_r[i] + dth * dth;
            acc_r[i] = v;
            a[13] += sqrt(v);
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
        const double v = wave_sum(a[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NACC) {
        double v = 0.0;
        for (int w = 0; w < OBS_THREADS / 64; ++w) v += red[w][threadIdx.x];
        partial[((long)r * nblk + b) * NACC + threadIdx.x] = v;
    }
}

// Pass 2: per replica, add the block partials in block order and form the outputs.
__global__ void k_obs_final(int L, int nblk, const double *__restrict__ partial, int have_h, int have_eta,
                            double *__restrict__ out)
{
    __shared__ double tot[NACC];
    const int r = blockIdx.x;
    if (threadIdx.x < NACC) {
        double v = 0.0;
        for (int b = 0; b < nblk; ++b) v += partial[((long)r * nblk + b) * NACC + threadIdx.x];
        tot[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) finish(L, r, tot, have_h != 0, have_eta != 0, out);
}

}  // namespace

static int obs_blocks(long N)
{
    long b = N / 512;
    if (b < 1) b = 1;
    if (b > OBS_MAX_BLOCKS) b = OBS_MAX_BLOCKS;
    return (int)b;
}

template <typename T>
hipError_t launch_observables(const ddmc_plan *p, int R, const ddmc_replica_params *params, const T *s,
                              const T *h, double *out, double *eta_acc, hipStream_t st)
{
    const long N = (long)p->L * p->L;
    const int nblk = obs_blocks(N);
    double *partial = reinterpret_cast<double *>(p->obs_ws);
    prof_scope ps(p, DDMC_KERNEL_OBSERVABLES, st);
    hipLaunchKernelGGL(k_obs_partial<T>, dim3(nblk, R), dim3(OBS_THREADS), 0, st, p->L, nblk, params, s, h, eta_acc,
                       partial);
    hipLaunchKernelGGL(k_obs_final, dim3(R), dim3(64), 0, st, p->L, nblk, partial, h != nullptr ? 1 : 0,
                       eta_acc != nullptr ? 1 : 0, out);
    return hipGetLastError();
}

template hipError_t launch_observables<float>(const ddmc_plan *, int, const ddmc_replica_params *, const float *,
                                              const float *, double *, double *, hipStream_t);
template hipError_t launch_observables<double>(const ddmc_plan *, int, const ddmc_replica_params *,
                                               const double *, const double *, double *, double *, hipStream_t);

}  // namespace ddmc
