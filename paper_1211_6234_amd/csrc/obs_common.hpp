// obs_common.hpp -- per-site accumulation and block reduction of the
// observables of Sec. 4.1 (eqs. (14)-(17)), shared by the standalone
// observables kernels and by the column kernel of the fused sampling sweep.
#pragma once

#include "device_common.hpp"
#include "internal.hpp"

namespace ddmc {
namespace obs {

constexpr int NACC = OBS_NACC;   // ex, dip, ani, mx, my, mz, nh[3], nv[3], q, etasum

__device__ __forceinline__ int sgn_of(double v) { return (v > 0.0) - (v < 0.0); }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Adds the contributions of site i of one replica to a[NACC]: bonds to +x and
// +y, energies, magnetization, wall counts (sgn(0) = 0), (theta - pi/2)^2,
// and, when acc_r is given, the site's cone-angle accumulator.
template <typename T>
__device__ __forceinline__ void site(double (&a)[NACC], int L, long N, const T *__restrict__ sr,
                                     const T *__restrict__ hr, double *__restrict__ acc_r, long i,
                                     const ddmc_replica_params &p)
{
    const double HALF_PI = 1.57079632679489661923;
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

// Block sum of a[NACC] (threads of a one-dimensional block of NTHR): wave
// shuffles, then the waves in order; thread k < NACC writes total k to out[k].
template <int NTHR>
__device__ __forceinline__ void block_sum(double (&a)[NACC], double (*red)[NACC], double *__restrict__ out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
        const double v = wave_sum(a[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NACC) {
        double v = 0.0;
        for (int w = 0; w < NTHR / 64; ++w) v += red[w][threadIdx.x];
        out[threadIdx.x] = v;
    }
}

// Sums nblk partial rows of NACC in order into t[NACC] (threads 0..NACC-1).
__device__ __forceinline__ void partial_sum(const double *__restrict__ partial, int nblk, double *t)
{
    if (threadIdx.x < NACC) {
        double v = 0.0;
        for (int b = 0; b < nblk; ++b) v += partial[(long)b * NACC + threadIdx.x];
        t[threadIdx.x] = v;
    }
}

// outputs of one replica from its NACC totals
__device__ inline void finish(int L, const double *t, bool have_h, bool have_eta, double *__restrict__ o)
{
    const double N = (double)L * (double)L;
    const double invN = 1.0 / N;
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

}  // namespace obs
}  // namespace ddmc
