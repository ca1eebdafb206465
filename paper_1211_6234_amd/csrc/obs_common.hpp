// obs_common.hpp -- per-site accumulation and block reduction of the
// observables of Sec. 4.1 (eqs. (14)-(17)), shared by the standalone
// observables kernels and by the column kernel of the fused sampling sweep.
#pragma once

#include "device_common.hpp"
#include "internal.hpp"

namespace ddmc {
namespace obs {

constexpr int NACC = OBS_NACC;   // ex, dip, ani, mx, my, mz, nh[3], nv[3], q, etasum, m_h, m_v, |dtheta|, non-finite

__device__ __forceinline__ int sgn_of(double v) { return (v > 0.0) - (v < 0.0); }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ int sgn_of(float v) { return (v > 0.0f) - (v < 0.0f); }

// arccos at the precision of the path
__device__ __forceinline__ double acos_t(double z) { return acos(z); }
__device__ __forceinline__ float acos_t(float z) { return acosf(z); }
__device__ __forceinline__ double sqrt_acc(double v, double) { return sqrt(v); }
__device__ __forceinline__ double sqrt_acc(double v, float) { return (double)sqrtf((float)v); }

// The terms of one site that need no neighbour: anisotropy energy,
// magnetization, s_z staggered along y and along x (sy, sx = +-1, the site's
// row and column parity), (theta - pi/2)^2, |theta - pi/2|, whether a spin
// component is NaN or infinite, and, when
// have_acc, the site's cone-angle accumulator acc (FP64) advanced by
// (theta - pi/2)^2 with its square root added.  The per-site terms are
// formed in the path's precision T and added to accumulators of type A:
// FP64 in the standalone kernels (exact for the magnetizations), and in the
// row kernels the path's precision, whose wave totals are summed in FP64.
template <typename T, typename A>
__device__ __forceinline__ void site_terms(A (&a)[NACC], const T (&s)[3], const ddmc_replica_params &p,
                                           bool have_acc, double &acc, A sy, A sx)
{
    const T HALF_PI = (T)1.57079632679489661923;
    const A z2 = (A)(s[2] * s[2]);
    a[2] += -((A)p.K2 * z2 + (A)p.K4 * z2 * z2);
    a[3] += (A)s[0];
    a[4] += (A)s[1];
    a[5] += (A)s[2];
    a[14] += sy * (A)s[2];
    a[15] += sx * (A)s[2];
    const T zc = fmin(T(1), fmax(T(-1), s[2]));
    const T dth = acos_t(zc) - HALF_PI;
    const T q = dth * dth;
    a[12] += (A)q;
    a[16] += (A)fabs(dth);
    a[17] += (isfinite(s[0]) && isfinite(s[1]) && isfinite(s[2])) ? A(0) : A(1);
    if (have_acc) {
        const double v = acc + (double)q;
        acc = v;
        a[13] += (A)sqrt_acc(v, T(0));
    }
}

// Domain-wall indicator 1 - sgn(s) sgn(n) (sgn(0) = 0) of one spin component
// across the bond between a site (s) and its neighbour (n)
__device__ __forceinline__ int wall(float s, float n) { return 1 - sgn_of(s) * sgn_of(n); }
__device__ __forceinline__ int wall(double s, double n) { return 1 - sgn_of(s) * sgn_of(n); }

// Adds one site's contributions to a[NACC] from its spin s, its neighbours
// at +x and +y, and its field h (when have_h): the bonds to +x and +y, the
// three energies, the magnetization, the wall counts and the per-site terms
// of site_terms.
template <typename T>
__device__ __forceinline__ void accumulate(double (&a)[NACC], const T (&s)[3], const T (&px)[3], const T (&py)[3],
                                           bool have_h, const T (&h)[3], const ddmc_replica_params &p,
                                           bool have_acc, double &acc, double sy, double sx)
{
    const T bond = s[0] * (px[0] + py[0]) + s[1] * (px[1] + py[1]) + s[2] * (px[2] + py[2]);
    a[0] += -p.J * (double)bond;
    if (have_h) a[1] += 0.5 * p.g * (double)(s[0] * h[0] + s[1] * h[1] + s[2] * h[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        a[6 + c] += (double)wall(s[c], px[c]);
        a[9 + c] += (double)wall(s[c], py[c]);
    }
    site_terms<T, double>(a, s, p, have_acc, acc, sy, sx);
}

// Site i of one replica read from HBM: the spins of the site and its +x and
// +y neighbours (periodic), the field when hr is given.
template <typename T>
__device__ __forceinline__ void site(double (&a)[NACC], int L, long N, const T *__restrict__ sr,
                                     const T *__restrict__ hr, double *__restrict__ acc_r, long i,
                                     const ddmc_replica_params &p)
{
    const int x = (int)i % L, y = (int)i / L;   // N <= 2^24
    const long ix = (long)y * L + (x + 1 == L ? 0 : x + 1);
    const long iy = (long)(y + 1 == L ? 0 : y + 1) * L + x;
    T s[3], px[3], py[3], h[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        s[c] = sr[c * N + i];
        px[c] = sr[c * N + ix];
        py[c] = sr[c * N + iy];
        if (hr) h[c] = hr[c * N + i];
    }
    double av = acc_r ? acc_r[i] : 0.0;
    accumulate<T>(a, s, px, py, hr != nullptr, h, p, acc_r != nullptr, av, (y & 1) ? -1.0 : 1.0,
                  (x & 1) ? -1.0 : 1.0);
    if (acc_r) acc_r[i] = av;
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

// Lane exchanges of a double as two 32-bit halves.  swap32 / swap16: the
// gfx950 half-wave swaps (lanes 32-63 of x with lanes 0-31 of y; odd 16-lane
// rows of x with even rows of y); returns x' + y', so that lanes whose lane
// bit 5 (4) is clear hold x summed with the partner half's x, the others y
// summed likewise.  dpp<CTRL>: the value of the lane selected by a DPP
// pattern of the lane's 16-lane row.
__device__ __forceinline__ double swap_add32(double x, double y)
{
    const unsigned long long ux = __double_as_longlong(x), uy = __double_as_longlong(y);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ux, (unsigned)uy, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ux >> 32), (unsigned)(uy >> 32), false, false);
    return __longlong_as_double(((unsigned long long)hi[0] << 32) | lo[0]) +
           __longlong_as_double(((unsigned long long)hi[1] << 32) | lo[1]);
}
__device__ __forceinline__ double swap_add16(double x, double y)
{
    const unsigned long long ux = __double_as_longlong(x), uy = __double_as_longlong(y);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ux, (unsigned)uy, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ux >> 32), (unsigned)(uy >> 32), false, false);
    return __longlong_as_double(((unsigned long long)hi[0] << 32) | lo[0]) +
           __longlong_as_double(((unsigned long long)hi[1] << 32) | lo[1]);
}
template <int CTRL> __device__ __forceinline__ double dpp(double x)
{
    const unsigned long long u = __double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_update_dpp(0u, (unsigned)u, CTRL, 0xF, 0xF, false);
    const unsigned hi = __builtin_amdgcn_update_dpp(0u, (unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ float swap_add32(float x, float y)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap_add16(float x, float y)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
template <int CTRL> __device__ __forceinline__ float dpp(float x)
{
    return __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(x), CTRL, 0xF, 0xF, false));
}
constexpr int DPP_ROW_ROR8 = 0x128;          // lane i of a row <- lane i ^ 8
constexpr int DPP_ROW_HALF_MIRROR = 0x141;   // lane i of an 8-lane half row <- lane 7 - i
constexpr int DPP_QUAD_XOR2 = 0x4E;          // quad_perm [2, 3, 0, 1]
constexpr int DPP_QUAD_XOR1 = 0xB1;          // quad_perm [1, 0, 3, 2]

// Sums the first 16 values of a[NACC] over the 64 lanes of a wave.  The first four steps
// each halve the values a lane carries: the lane keeps the half selected by
// one of its lane bits (5, 4, 3, 2) and adds the copy of it held by a partner
// lane whose bit differs (half-wave swaps for bits 5 and 4, DPP patterns for
// bits 3 and 2).  Lane l is then left with value k = l >> 2 summed over the 16
// lanes that share l's bits 0-1; two DPP steps within the quad complete the
// sum.  Every lane returns the wave total of value l >> 2.  All 64 lanes must
// be active.
template <typename A> __device__ __forceinline__ A wave_sum16(const A (&a)[NACC])
{
    static_assert(NACC >= 16, "four halving steps over a[0 .. 15]");
    const int lane = threadIdx.x & 63;
    A v8[8], v4[4], v2[2];
#pragma unroll
    for (int i = 0; i < 8; ++i) v8[i] = swap_add32(a[i], a[8 + i]);
#pragma unroll
    for (int i = 0; i < 4; ++i) v4[i] = swap_add16(v8[i], v8[4 + i]);
    {
        const bool hi = (lane & 8) != 0;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const A keep = hi ? v4[2 + i] : v4[i], give = hi ? v4[i] : v4[2 + i];
            v2[i] = keep + dpp<DPP_ROW_ROR8>(give);
        }
    }
    const bool hi = (lane & 4) != 0;
    A v = (hi ? v2[1] : v2[0]) + dpp<DPP_ROW_HALF_MIRROR>(hi ? v2[0] : v2[1]);
    v += dpp<DPP_QUAD_XOR2>(v);
    v += dpp<DPP_QUAD_XOR1>(v);
    return v;
}

// Sums nblk partial rows of NACC (partial[b][k]) into tot[k] in LDS with the
// NW waves of the block: wave w takes k = w, w + NW, ...; lane l adds rows
// l, l + 64, ... and the wave reduces with shuffles.  The order depends only
// on nblk.  Ends with a barrier; every thread of the block must call it.
template <int NW>
__device__ __forceinline__ void partial_sum(const double *__restrict__ partial, int nblk, double *tot)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int KPW = (NACC + NW - 1) / NW;
    double v[KPW];
#pragma unroll
    for (int j = 0; j < KPW; ++j) v[j] = 0.0;
    for (int b = lane; b < nblk; b += 64) {
#pragma unroll
        for (int j = 0; j < KPW; ++j) {
            const int k = wave + j * NW;
            if (k < NACC) v[j] += partial[(long)b * NACC + k];
        }
    }
#pragma unroll
    for (int j = 0; j < KPW; ++j) {
        const int k = wave + j * NW;
        const double s = wave_sum(v[j]);
        if (k < NACC && lane == 0) tot[k] = s;
    }
    __syncthreads();
}

// Adds nslot per-block accept counts of one replica (slots[k]) to *accepted
// with the first wave of the block.
__device__ __forceinline__ void fold_slots(const unsigned int *__restrict__ slots, int nslot,
                                           unsigned long long *__restrict__ accepted)
{
    if (threadIdx.x >= 64) return;
    unsigned long long v = 0ull;
    for (int k = threadIdx.x; k < nslot; k += 64) v += slots[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (threadIdx.x == 0) *accepted += v;
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
    o[DDMC_OBS_MSTH] = t[14] * invN;
    o[DDMC_OBS_MSTV] = t[15] * invN;
    o[DDMC_OBS_ETAS] = 0.63661977236758134308 * t[16] * invN;   // 2/pi
    o[DDMC_OBS_NONFINITE] = t[17];
}

}  // namespace obs
}  // namespace ddmc
