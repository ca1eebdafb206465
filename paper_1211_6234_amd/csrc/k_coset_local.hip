// k_coset_local.hip -- the l-coset simultaneous update of Sec. 3.1 for small
// cosets, with a whole replica in one workgroup.
//
// The schedule updates the (L/l)^2 sites of one coset of l Z^2 at once with
// the frozen field of the state before them (Sec. 3.2), the l^2 cosets in
// turn.  When a coset holds few sites, recomputing the full field after each
// coset (two launches per coset on the FFT path) is dominated by the launch
// cost: the paper's L = 64, l = 32 case is 2048 launches per sweep.  Here one
// workgroup (1024 threads, 512 in FP64) owns one replica for all the sweeps
// of a call: the spins (and, when they fit, the kernel W) live in LDS, each
// thread keeps the field of its own sites in FP64 registers, and after each
// coset the field is brought up to date by the changes alone,
// h(x) += W(x - i) (S_i - s_i) over the coset's accepted sites i (self-image
// term included), the coset's terms summed in the working precision.  The
// field at the start of a call is the full convolution computed by the plan's
// field path.  One launch per call after it.
#include "device_common.hpp"
#include "internal.hpp"

namespace ddmc {

namespace {

constexpr int MAX_N = 4096;     // sites of the largest lattice handled here
constexpr int MAX_NC = 16;      // sites per coset handled here
// threads of the workgroup (a power of two) and own sites per thread; FP64
// takes half the threads so that each may hold twice the registers
template <typename T> constexpr int CT = sizeof(T) < sizeof(double) ? 1024 : 512;
template <typename T> constexpr int MAX_NS = MAX_N / CT<T>;
// Component stride of the spins in LDS: in FP32 a fixed MAX_N, so that the y
// and z components of a site sit at constant offsets (16 and 32 KiB, inside a
// DS instruction's immediate offset) from its x component and one address
// serves all three; in FP64 N, to leave room for the kernel W.
template <typename T> constexpr int SPIN_STRIDE = sizeof(T) < sizeof(double) ? MAX_N : 0;
template <typename T> __host__ __device__ inline int spin_stride(int N) { return SPIN_STRIDE<T> ? SPIN_STRIDE<T> : N; }
constexpr size_t COSET_LDS_MAX = 150 * 1024;   // dynamic LDS of one workgroup (160 KB per CU)

template <typename T> struct coset_args {
    int L, l, nsweeps;
    const ddmc_replica_params *params;
    T *s;                          // [R][3][N]
    const T *h0;                   // [R][3][N] field of the starting state
    const T *W;                    // [4][N] planes xx, yy, xy, zz
    double w0[4];                  // W(0)
    unsigned long long *ctr;       // [R] sweep counters, advanced by nsweeps
    unsigned long long *accepted;  // [R] or NULL
};

// W(rho) as (xx, yy, xy, zz): from the LDS copy or from the plan's planes
template <typename T, bool W_LDS>
__device__ __forceinline__ vec4a<T> w_at(const vec4a<T> *wl, const T *W, int N, int rho)
{
    if constexpr (W_LDS) {
        return wl[rho];
    } else {
        vec4a<T> w;
        w.a = W[rho];
        w.b = W[N + rho];
        w.c = W[2 * N + rho];
        w.d = W[3 * N + rho];
        return w;
    }
}

// The same energy change split for moves whose trial spin is known before the
// neighbours are: site_change holds the terms of the site alone,
// g d^T W(0) d / 2 - K2 (Sz^2 - sz^2) - K4 (Sz^4 - sz^4), and
// neighbour_change the rest, -J d.nb + g d.h.
template <typename T>
__device__ __forceinline__ T site_change(const site_consts<T> &c, vec3<T> s, vec3<T> S)
{
    const T dx = S.x - s.x, dy = S.y - s.y, dz = S.z - s.z;
    const T quad = c.w0xx * dx * dx + c.w0yy * dy * dy + T(2) * c.w0xy * dx * dy + c.w0zz * dz * dz;
    const T z2n = S.z * S.z, z2o = s.z * s.z;
    return c.g * T(0.5) * quad - c.K2 * (z2n - z2o) - c.K4 * (z2n * z2n - z2o * z2o);
}
template <typename T>
__device__ __forceinline__ T neighbour_change(const site_consts<T> &c, vec3<T> s, vec3<T> S, vec3<T> nb, vec3<T> h)
{
    const T dx = S.x - s.x, dy = S.y - s.y, dz = S.z - s.z;
    return -c.J * (dx * nb.x + dy * nb.y + dz * nb.z) + c.g * (dx * h.x + dy * h.y + dz * h.z);
}

// Metropolis rule in threshold form: for 0 < u < 1 and T > 0, "dE <= 0 or
// u < exp(-dE/T)" holds exactly when dE < -T ln u.  With the site's own terms
// moved to the threshold, a move is accepted when
// neighbour_change < accept_threshold; NaN on either side rejects it.
template <typename T>
__device__ __forceinline__ T accept_threshold(const site_consts<T> &c, vec3<T> s, vec3<T> S, T u)
{
    T lu;
    if constexpr (sizeof(T) < sizeof(double)) lu = logf(u);
    else lu = log(u);
    return -c.T_ * lu - site_change<T>(c, s, S);
}

// One accepted move of a coset: S - s and the site (x | y << 8)
template <typename T> struct alignas(4 * sizeof(T)) coset_chg {
    T d[3];
    int xy;
};

// An own site in one word: x + L (bits 0-7), y + L (bits 8-15), its coset
// (bits 16-27; 0xfff for a thread with no site in that block, which no coset
// index reaches since such a lattice has N < 4096 sites) and its index within
// the coset (bits 28-31).  With L <= 64 the biased coordinates fit a byte, and
// subtracting a change's (x | y << 8) from the low half gives x - x' + L and
// y - y' + L in [1, 2L), with no borrow between the bytes.
__device__ __forceinline__ int site_coset(uint32_t w) { return (int)((w >> 16) & 0xfffu); }

// own site of thread tid in block q of CT sites: site q CT + j belongs to
// thread (j + 64 q) mod CT
template <typename T> __device__ __forceinline__ int own_site(int tid, int q)
{
    return q * CT<T> + ((tid - 64 * q) & (CT<T> - 1));
}

// P2: L is a power of two, so coordinate differences wrap with a mask
template <typename T, bool W_LDS, bool P2>
__global__ void __launch_bounds__(CT<T>) k_coset_local(coset_args<T> a)
{
    extern __shared__ __align__(32) unsigned char smem[];
    // changes S - s of the coset's accepted sites, double-buffered by coset
    // parity so that one barrier per coset suffices: the owners of coset k+1
    // write one buffer while slower threads may still read coset k's
    __shared__ coset_chg<T> chg[2][MAX_NC];
    // bit m: site m of the coset moved.  Three masks in turn: the owners of
    // coset g set bits of mask g mod 3, every thread reads it after the
    // barrier, and thread 0 clears mask (g + 1) mod 3 while coset g is being
    // decided (its last readers, coset g - 2, passed the barrier before).
    __shared__ unsigned amask[3];
    const int L = a.L, l = a.l, N = L * L;
    const int lgL = 31 - __builtin_clz((unsigned)L);   // log2 L when P2
    const int r = blockIdx.x, tid = threadIdx.x;
    const int C = spin_stride<T>(N);
    T *sl = reinterpret_cast<T *>(smem);   // [3][C], the first N of each component used
    const size_t woff = ((size_t)3 * C * sizeof(T) + sizeof(vec4a<T>) - 1) / sizeof(vec4a<T>) * sizeof(vec4a<T>);
    vec4a<T> *wl = reinterpret_cast<vec4a<T> *>(smem + woff);   // [N] (W_LDS)
    T *sg = a.s + (size_t)r * 3 * N;
    const T *hg = a.h0 + (size_t)r * 3 * N;

    for (int c = 0; c < 3; ++c)
        for (int e = tid; e < N; e += CT<T>) sl[c * C + e] = sg[c * N + e];
    if constexpr (W_LDS) {
        for (int e = tid; e < N; e += CT<T>) {
            vec4a<T> w;
            w.a = a.W[e];
            w.b = a.W[N + e];
            w.c = a.W[2 * N + e];
            w.d = a.W[3 * N + e];
            wl[e] = w;
        }
    }
    // Own sites: one per block of CT sites, rotated by one wave per block
    // (site i = q CT + j belongs to thread (j + 64 q) mod CT), so that the
    // sites of one coset fall on different waves or lanes and are decided
    // together.  Their field is kept in FP64.
    double hr[MAX_NS<T>][3];
    uint32_t wo[MAX_NS<T>];
    const int per = L / l;
#pragma unroll
    for (int q = 0; q < MAX_NS<T>; ++q) {
        const int i = own_site<T>(tid, q);
        const int ic = i < N ? i : N - 1;
        const int x = ic % L, y = ic / L;
        const uint32_t k = i < N ? (uint32_t)((y % l) * l + x % l) : 0xfffu;
        wo[q] = (uint32_t)(x + L) | ((uint32_t)(y + L) << 8) | (k << 16) |
                ((uint32_t)((y / l) * per + x / l) << 28);
#pragma unroll
        for (int c = 0; c < 3; ++c) hr[q][c] = (double)hg[c * N + ic];
    }
    if (tid < 3) amask[tid] = 0u;
    // accepted moves of the call: the bits of the coset masks, summed by
    // every thread alike (a wave-uniform value)
    unsigned long long count = 0ull;
    const ddmc_replica_params p = a.params[r];
    site_consts<T> cst;
    cst.J = (T)p.J; cst.K2 = (T)p.K2; cst.K4 = (T)p.K4; cst.g = (T)p.g; cst.T_ = (T)p.T;
    cst.w0xx = (T)a.w0[0]; cst.w0yy = (T)a.w0[1]; cst.w0xy = (T)a.w0[2]; cst.w0zz = (T)a.w0[3];
    const unsigned long long ctr0 = a.ctr[r];
    __syncthreads();

    // In FP32 the trial spins of a sweep are drawn for all own sites at its
    // start, off the per-coset critical path: they depend only on (site,
    // sweep) and on the site's own spin, which changes only at the site's own
    // decision.  For the same reason the terms of dE that involve the site
    // alone are known then; they are folded with the uniform into an
    // acceptance threshold, so that a decision forms only the neighbour and
    // field terms and compares (no division or exponential on the chain).
    // FP64 has no registers to spare for either and applies the rule as is.
    constexpr bool PRE = sizeof(T) < sizeof(double);
    constexpr int NP = PRE ? MAX_NS<T> : 1;
    vec3<T> Sp[NP];
    T thr[NP];
    int buf = 0, b3 = 0;
    for (int t = 0; t < a.nsweeps; ++t) {
        const uint32_t sweep = (uint32_t)(ctr0 + (unsigned long long)t);
        if constexpr (PRE) {
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                int i = min(own_site<T>(tid, q), N - 1);
                // an opaque copy of the site index keeps each draw whole inside
                // the sweep loop: hoisted, the sweep-independent products of its
                // first round would hold registers through every coset
                asm volatile("" : "+v"(i));
                const vec3<T> so = {sl[i], sl[C + i], sl[2 * C + i]};
                const u32x4 d = draw(p.seed, p.replica_id, sweep, (uint32_t)i, 1u);
                Sp[q] = trial_spin<T>(p.model, so, d);
                thr[q] = accept_threshold<T>(cst, so, Sp[q], to_unit<T>(d.v[2]));
            }
        }
        for (int cy = 0; cy < l; ++cy) {
            for (int cx = 0; cx < l; ++cx) {
                // the owners of the coset's sites decide their moves with the
                // field and spins of the state before the coset
                const int k = cy * l + cx;
                unsigned own = 0u;
#pragma unroll
                for (int q = 0; q < MAX_NS<T>; ++q) own |= (site_coset(wo[q]) == k ? 1u : 0u) << q;
                while (own) {
                    const int q = __builtin_ctz(own);
                    own &= own - 1u;
                    const int i = own_site<T>(tid, q);
                    uint32_t w = wo[0];
                    vec3<T> hv{(T)hr[0][0], (T)hr[0][1], (T)hr[0][2]};
#pragma unroll
                    for (int qq = 1; qq < MAX_NS<T>; ++qq)
                        if (qq == q) {
                            w = wo[qq];
                            hv = vec3<T>{(T)hr[qq][0], (T)hr[qq][1], (T)hr[qq][2]};
                        }
                    const int x = (int)(w & 0xffu) - L, y = (int)((w >> 8) & 0xffu) - L, m = (int)(w >> 28);
                    const int xp = (x + 1 == L) ? 0 : x + 1, xm = (x == 0) ? L - 1 : x - 1;
                    const int yp = (y + 1 == L) ? 0 : y + 1, ym = (y == 0) ? L - 1 : y - 1;
                    const int n0 = y * L + xp, n1 = y * L + xm, n2 = yp * L + x, n3 = ym * L + x;
                    vec3<T> nb;
                    nb.x = sl[n0] + sl[n1] + sl[n2] + sl[n3];
                    nb.y = sl[C + n0] + sl[C + n1] + sl[C + n2] + sl[C + n3];
                    nb.z = sl[2 * C + n0] + sl[2 * C + n1] + sl[2 * C + n2] + sl[2 * C + n3];
                    const vec3<T> so = {sl[i], sl[C + i], sl[2 * C + i]};
                    vec3<T> S;
                    bool acc;
                    if constexpr (PRE) {
                        S = Sp[0];
                        T th = thr[0];
#pragma unroll
                        for (int qq = 1; qq < NP; ++qq)
                            if (qq == q) {
                                S = Sp[qq];
                                th = thr[qq];
                            }
                        acc = neighbour_change<T>(cst, so, S, nb, hv) < th;
                    } else {
                        const u32x4 d = draw(p.seed, p.replica_id, sweep, (uint32_t)i, 1u);
                        S = trial_spin<T>(p.model, so, d);
                        acc = metropolis(energy_change<T>(cst, so, S, nb, hv), cst.T_, to_unit<T>(d.v[2]));
                    }
                    if (acc) {
                        sl[i] = S.x;
                        sl[C + i] = S.y;
                        sl[2 * C + i] = S.z;
                        chg[buf][m] = coset_chg<T>{{S.x - so.x, S.y - so.y, S.z - so.z}, x | (y << 8)};
                        atomicOr(&amask[b3], 1u << m);
                    }
                }
                if (tid == 0) amask[b3 == 2 ? 0 : b3 + 1] = 0u;
                __syncthreads();
                // field of the own sites brought up to date by the accepted
                // changes (summed over the coset in T, then added in FP64); a
                // thread's next decisions read only its own field
                constexpr bool SUM_T = sizeof(T) < sizeof(double);
                // the coset's moved sites in increasing m; nothing to do when
                // none moved
                unsigned am = __builtin_amdgcn_readfirstlane(amask[b3]);
                count += (unsigned long long)__popc(am);
                if (am) {
                    T ax[MAX_NS<T>], ay[MAX_NS<T>], az[MAX_NS<T>];
#pragma unroll
                    for (int q = 0; q < MAX_NS<T>; ++q) ax[q] = ay[q] = az[q] = T(0);
                    while (am) {
                        const int m = __builtin_ctz(am);
                        am &= am - 1u;
                        const coset_chg<T> c = chg[buf][m];
                        // the kernel at every own site's offset first, so that
                        // the reads are in flight together
                        vec4a<T> wq[MAX_NS<T>];
#pragma unroll
                        for (int q = 0; q < MAX_NS<T>; ++q) {
                            const int dxy = (int)(wo[q] & 0xffffu) - c.xy;
                            int rho;
                            if constexpr (P2) {
                                rho = (((dxy >> 8) & (L - 1)) << lgL) | (dxy & (L - 1));
                            } else {
                                int rx = dxy & 0xff, ry = (dxy >> 8) & 0xff;
                                if (rx >= L) rx -= L;
                                if (ry >= L) ry -= L;
                                rho = ry * L + rx;
                            }
                            wq[q] = w_at<T, W_LDS>(wl, a.W, N, rho);
                        }
#pragma unroll
                        for (int q = 0; q < MAX_NS<T>; ++q) {
                            const vec4a<T> w = wq[q];
                            if constexpr (SUM_T) {
                                ax[q] += w.a * c.d[0] + w.c * c.d[1];
                                ay[q] += w.c * c.d[0] + w.b * c.d[1];
                                az[q] += w.d * c.d[2];
                            } else {
                                hr[q][0] += w.a * c.d[0] + w.c * c.d[1];
                                hr[q][1] += w.c * c.d[0] + w.b * c.d[1];
                                hr[q][2] += w.d * c.d[2];
                            }
                        }
                    }
                    if constexpr (SUM_T) {
#pragma unroll
                        for (int q = 0; q < MAX_NS<T>; ++q) {
                            hr[q][0] += (double)ax[q];
                            hr[q][1] += (double)ay[q];
                            hr[q][2] += (double)az[q];
                        }
                    }
                }
                buf ^= 1;
                b3 = b3 == 2 ? 0 : b3 + 1;
            }
        }
    }
    __syncthreads();
    for (int c = 0; c < 3; ++c)
        for (int e = tid; e < N; e += CT<T>) sg[c * N + e] = sl[c * C + e];
    if (tid == 0) {
        a.ctr[r] = ctr0 + (unsigned long long)a.nsweeps;
        if (a.accepted) a.accepted[r] += count;
    }
}

template <typename T> size_t spin_bytes(int L) { return (size_t)3 * spin_stride<T>(L * L) * sizeof(T); }
template <typename T> size_t w_offset(int L)
{
    return (spin_bytes<T>(L) + sizeof(vec4a<T>) - 1) / sizeof(vec4a<T>) * sizeof(vec4a<T>);
}
template <typename T> bool w_in_lds(int L) { return w_offset<T>(L) + (size_t)L * L * sizeof(vec4a<T>) <= COSET_LDS_MAX; }

}  // namespace

bool coset_local_ok(int L, int l, ddmc_prec prec)
{
    if (l < 2 || L % l != 0) return false;
    const int per = L / l;
    if (per * per > MAX_NC || L * L > MAX_N) return false;
    const size_t spins = prec == DDMC_F64 ? spin_bytes<double>(L) : spin_bytes<float>(L);
    return spins <= COSET_LDS_MAX;
}

template <typename T>
ddmc_status coset_local_sweep(ddmc_plan *p, int R, const ddmc_replica_params *params, T *s, int l,
                              uint64_t *sweep_ctr, int nsweeps, uint64_t *accepted, hipStream_t st)
{
    const int L = p->L;
    T *h = reinterpret_cast<T *>(p->h_ws);
    ddmc_status e = p->algo == DDMC_FIELD_FFT ? fft_field<T>(p, R, s, h, -1, st) : direct_field<T>(p, R, s, h, -1, st);
    if (e != DDMC_OK) return e;
    coset_args<T> a;
    a.L = L;
    a.l = l;
    a.nsweeps = nsweeps;
    a.params = params;
    a.s = s;
    a.h0 = h;
    a.W = reinterpret_cast<const T *>(p->W);
    for (int c = 0; c < 4; ++c) a.w0[c] = p->W0[c];
    a.ctr = reinterpret_cast<unsigned long long *>(sweep_ctr);
    a.accepted = reinterpret_cast<unsigned long long *>(accepted);
    const bool wl = w_in_lds<T>(L);
    const size_t lds = wl ? w_offset<T>(L) + (size_t)L * L * sizeof(vec4a<T>) : spin_bytes<T>(L);
    const bool p2 = (L & (L - 1)) == 0;
    const void *fn = wl ? (p2 ? reinterpret_cast<const void *>(&k_coset_local<T, true, true>)
                              : reinterpret_cast<const void *>(&k_coset_local<T, true, false>))
                        : (p2 ? reinterpret_cast<const void *>(&k_coset_local<T, false, true>)
                              : reinterpret_cast<const void *>(&k_coset_local<T, false, false>));
    hipError_t he = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (he != hipSuccess) return hip_check(he, "coset kernel LDS size");
    prof_scope ps(p, DDMC_KERNEL_UPDATE, st);
    if (wl && p2)
        hipLaunchKernelGGL((k_coset_local<T, true, true>), dim3(R), dim3(CT<T>), lds, st, a);
    else if (wl)
        hipLaunchKernelGGL((k_coset_local<T, true, false>), dim3(R), dim3(CT<T>), lds, st, a);
    else if (p2)
        hipLaunchKernelGGL((k_coset_local<T, false, true>), dim3(R), dim3(CT<T>), lds, st, a);
    else
        hipLaunchKernelGGL((k_coset_local<T, false, false>), dim3(R), dim3(CT<T>), lds, st, a);
    return hip_check(hipGetLastError(), "coset kernel launch");
}

template ddmc_status coset_local_sweep<float>(ddmc_plan *, int, const ddmc_replica_params *, float *, int,
                                              uint64_t *, int, uint64_t *, hipStream_t);
template ddmc_status coset_local_sweep<double>(ddmc_plan *, int, const ddmc_replica_params *, double *, int,
                                               uint64_t *, int, uint64_t *, hipStream_t);

}  // namespace ddmc
