// device_common.hpp -- device helpers shared by the sweep kernels: the
// counter-based generator, the trial move, the single-site energy change.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ddmc.h"

namespace ddmc {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11).  Each round multiplies words 0 and 2 by the two
// round multipliers, swaps the high/low halves across the pairs and xors in
// the round key; the key advances by the golden-ratio and sqrt(3)-1 Weyl
// increments between rounds.
// ---------------------------------------------------------------------------
struct u32x4 {
    uint32_t v[4];
};

__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1)
{
    constexpr uint32_t MUL_A = 0xD2511F53u, MUL_B = 0xCD9E8D57u;
    constexpr uint32_t WEYL_A = 0x9E3779B9u, WEYL_B = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit multiply per product (a single v_mad_u64_u32)
        const uint64_t pa = (uint64_t)MUL_A * c0, pb = (uint64_t)MUL_B * c2;
        const uint32_t a_hi = (uint32_t)(pa >> 32), a_lo = (uint32_t)pa;
        const uint32_t b_hi = (uint32_t)(pb >> 32), b_lo = (uint32_t)pb;
        const uint32_t n0 = b_hi ^ c1 ^ k0;
        const uint32_t n2 = a_hi ^ c3 ^ k1;
        c0 = n0; c1 = b_lo; c2 = n2; c3 = a_lo;
        k0 += WEYL_A; k1 += WEYL_B;
    }
    u32x4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// draws of one (site, sweep, replica, purpose) counter under a replica seed
__device__ __forceinline__ u32x4 draw(uint64_t seed, uint32_t replica_id, uint32_t sweep,
                                      uint32_t site, uint32_t purpose)
{
    return philox10(site, sweep, replica_id, purpose, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// uniform on (0, 1) at the precision of the path
template <typename T> __device__ __forceinline__ T to_unit(uint32_t x);
template <> __device__ __forceinline__ double to_unit<double>(uint32_t x)
{
    return ((double)x + 0.5) * 0x1p-32;
}
template <> __device__ __forceinline__ float to_unit<float>(uint32_t x)
{
    return ((float)(x >> 9) + 0.5f) * 0x1p-23f;
}

template <typename T> struct vec3 {
    T x, y, z;
};

__device__ __forceinline__ void sincos_2pi(double u, double *s, double *c) { sincospi(2.0 * u, s, c); }
__device__ __forceinline__ void sincos_2pi(float u, float *s, float *c) { sincospif(2.0f * u, s, c); }

// Uniform direction on the unit sphere from two uniforms (Archimedes: the
// height z is uniform on [-1, 1]; the azimuth uniform on [0, 2 pi)).
template <typename T> __device__ __forceinline__ vec3<T> sphere_point(T u0, T u1)
{
    T sn, cs;
    sincos_2pi(u1, &sn, &cs);
    const T rho = T(2) * sqrt(u0 * (T(1) - u0));   // = sqrt(1 - z^2)
    vec3<T> S;
    S.x = rho * cs;
    S.y = rho * sn;
    S.z = T(1) - T(2) * u0;
    return S;
}

// Trial spin of one site from its draws: uniform on the sphere for
// Heisenberg replicas, the reversal of the current spin for Ising ones.
template <typename T>
__device__ __forceinline__ vec3<T> trial_spin(uint32_t model, vec3<T> s, const u32x4 &d)
{
    if (model == DDMC_ISING) return vec3<T>{-s.x, -s.y, -s.z};
    return sphere_point<T>(to_unit<T>(d.v[0]), to_unit<T>(d.v[1]));
}

// Per-replica constants of the energy change, in the arithmetic type.
template <typename T> struct site_consts {
    T J, K2, K4, g, T_;
    T w0xx, w0yy, w0xy, w0zz;   // self-image tensor W(0)
};

// Energy change of s -> S at one site given the neighbour sum nb and the
// frozen dipolar field h at the site (self-image term W(0) s included in h):
//   -J d.nb + g (d.h + d^T W(0) d / 2) - K2 (Sz^2 - sz^2) - K4 (Sz^4 - sz^4).
template <typename T>
__device__ __forceinline__ T energy_change(const site_consts<T> &c, vec3<T> s, vec3<T> S,
                                           vec3<T> nb, vec3<T> h)
{
    const T dx = S.x - s.x, dy = S.y - s.y, dz = S.z - s.z;
    const T exch = -c.J * (dx * nb.x + dy * nb.y + dz * nb.z);
    const T quad = c.w0xx * dx * dx + c.w0yy * dy * dy + T(2) * c.w0xy * dx * dy + c.w0zz * dz * dz;
    const T dip = c.g * (dx * h.x + dy * h.y + dz * h.z + T(0.5) * quad);
    const T z2n = S.z * S.z, z2o = s.z * s.z;
    const T ani = -c.K2 * (z2n - z2o) - c.K4 * (z2n * z2n - z2o * z2o);
    return exch + dip + ani;
}

// Metropolis rule: accept a lowering (or equal) energy, else with
// probability exp(-dE/T); a NaN energy change is rejected.
__device__ __forceinline__ bool metropolis(double dE, double T, double u)
{
    return dE <= 0.0 || u < exp(-dE / T);
}
__device__ __forceinline__ bool metropolis(float dE, float T, float u)
{
    return dE <= 0.0f || u < expf(-dE / T);
}

// ---------------------------------------------------------------------------
// Accept counting and sweep-counter advance.  Every block of a half-sweep
// launch reduces its accepted moves in LDS and adds the total to accepted[r]
// with one integer atomic (a few dozen per replica and launch, instead of one
// per wave).  On the last launch of a call each block then bumps its
// replica's completion counter; the block that completes last advances the
// replica's device sweep counter and resets the completion counter.  No block
// waits on another, and no device-wide fence is needed: the only value the
// finishing block publishes is the counter, which every other block of the
// launch has already read (its read precedes its completion atomic by data
// dependence), and the next launch sees it after the kernel boundary.
// ---------------------------------------------------------------------------
struct sweep_book {
    unsigned int *done;             // [R] completion counters, zero between calls
    unsigned long long *accepted;   // caller's [R] totals, may be NULL
    unsigned long long *ctr;        // caller's [R] device sweep counters, may be NULL
    unsigned long long advance;     // added to ctr[r] by the finishing block
    int finalize;                   // 1 on the last launch of a call with a counter
};

// Called by every thread of the block after a barrier that follows the
// block's updates; block_count is the block's accepted moves (LDS).
__device__ __forceinline__ void book_block(const sweep_book &b, int r, unsigned int nblk_r, unsigned int block_count)
{
    if (threadIdx.x != 0 || threadIdx.y != 0) return;
    if (b.accepted && block_count) atomicAdd(&b.accepted[r], (unsigned long long)block_count);
    if (!b.finalize) return;
    const unsigned int prev = atomicAdd(&b.done[r], 1u);
    if (prev != nblk_r - 1) return;
    b.ctr[r] += b.advance;
    atomicExch(&b.done[r], 0u);
}

}  // namespace ddmc
