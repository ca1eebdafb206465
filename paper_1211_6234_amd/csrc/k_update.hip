// k_update.hip -- the colour half-sweep of the checkerboard Metropolis sweep
// (Sec. 2.2 eq. (7) with the frozen-field approximation of Sec. 3.2) or one
// coset of the l-spaced simultaneous update (Sec. 3.1), the initial uniform
// state, and the diagnostic trial-energy kernel.
//
// One thread per site of the colour; spins and field are component planes
// of one replica, so every load and store of a wave is a coalesced stride-2
// access within a lattice row.  The accepted-move count is reduced within
// each wave with a ballot and added with one integer atomic per wave.
#include "device_common.hpp"
#include "internal.hpp"

namespace ddmc {

namespace {

template <typename T>
__device__ __forceinline__ site_consts<T> load_consts(const ddmc_replica_params &p, const double *W0)
{
    site_consts<T> c;
    c.J = (T)p.J;
    c.K2 = (T)p.K2;
    c.K4 = (T)p.K4;
    c.g = (T)p.g;
    c.T_ = (T)p.T;
    c.w0xx = (T)W0[0];
    c.w0yy = (T)W0[1];
    c.w0xy = (T)W0[2];
    c.w0zz = (T)W0[3];
    return c;
}

struct w0_arg {
    double v[4];
};

// site of colour `color` with index j in [0, N/2): row y, column 2 (j mod L/2) + ((color + y) & 1)
__device__ __forceinline__ void colour_site(int L, long j, int color, int &x, int &y)
{
    const int half = L >> 1;
    y = (int)(j / half);
    x = 2 * (int)(j - (long)y * half) + ((color + y) & 1);
}

// site j in [0, N / l^2) of the coset (cx, cy) + l Z^2, k = cy l + cx
__device__ __forceinline__ void coset_site(int L, int l, long j, int k, int &x, int &y)
{
    const int per = L / l;
    const int jy = (int)(j / per), jx = (int)(j - (long)jy * per);
    x = k % l + l * jx;
    y = k / l + l * jy;
}

template <typename T>
__device__ __forceinline__ vec3<T> neighbour_sum(const T *__restrict__ s, long N, int L, int x, int y)
{
    const int xp = (x + 1 == L) ? 0 : x + 1, xm = (x == 0) ? L - 1 : x - 1;
    const int yp = (y + 1 == L) ? 0 : y + 1, ym = (y == 0) ? L - 1 : y - 1;
    const long a = (long)y * L + xp, b = (long)y * L + xm, c = (long)yp * L + x, d = (long)ym * L + x;
    vec3<T> n;
    n.x = s[a] + s[b] + s[c] + s[d];
    n.y = s[N + a] + s[N + b] + s[N + c] + s[N + d];
    n.z = s[2 * N + a] + s[2 * N + b] + s[2 * N + c] + s[2 * N + d];
    return n;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_update(int L, const ddmc_replica_params *__restrict__ params, T *__restrict__ s, const T *__restrict__ h,
         int color, int coset_l, uint32_t sweep_off, w0_arg w0, sweep_book book)
{
    __shared__ unsigned int block_count;
    const long N = (long)L * L;
    const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    const uint32_t sweep = (uint32_t)((book.ctr ? book.ctr[r] : 0ull) + sweep_off);
    if (threadIdx.x == 0) block_count = 0u;
    __syncthreads();
    bool acc = false;
    const long nsites = coset_l ? N / ((long)coset_l * coset_l) : N / 2;
    if (j < nsites) {
        const ddmc_replica_params p = params[r];
        const site_consts<T> c = load_consts<T>(p, w0.v);
        int x, y;
        if (coset_l)
            coset_site(L, coset_l, j, color, x, y);
        else
            colour_site(L, j, color, x, y);
        const long i = (long)y * L + x;
        T *sr = s + (long)r * 3 * N;
        const T *hr = h + (long)r * 3 * N;
        const u32x4 d = draw(p.seed, p.replica_id, sweep, (uint32_t)i, 1u);
        const T u2 = to_unit<T>(d.v[2]);
        const vec3<T> so = {sr[i], sr[N + i], sr[2 * N + i]};
        const vec3<T> S = trial_spin<T>(p.model, so, d);
        const vec3<T> hv = {hr[i], hr[N + i], hr[2 * N + i]};
        const vec3<T> nb = neighbour_sum<T>(sr, N, L, x, y);
        const T dE = energy_change<T>(c, so, S, nb, hv);
        acc = metropolis(dE, c.T_, u2);
        if (acc) {
            sr[i] = S.x;
            sr[N + i] = S.y;
            sr[2 * N + i] = S.z;
        }
    }
    if (book.accepted) {
        const unsigned long long mask = __ballot(acc);
        if ((threadIdx.x & (warpSize - 1)) == 0 && mask != 0ull) atomicAdd(&block_count, (unsigned int)__popcll(mask));
    }
    __syncthreads();
    book_block(book, r, gridDim.x, block_count);
}

template <typename T>
__global__ void k_trial(int L, const ddmc_replica_params *__restrict__ params, const T *__restrict__ s,
                        const T *__restrict__ h, int color, uint32_t sweep, w0_arg w0, T *__restrict__ dE_out,
                        T *__restrict__ u_out, T *__restrict__ S_out)
{
    const long N = (long)L * L;
    const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (j >= N / 2) return;
    const ddmc_replica_params p = params[r];
    const site_consts<T> c = load_consts<T>(p, w0.v);
    int x, y;
    colour_site(L, j, color, x, y);
    const long i = (long)y * L + x;
    const T *sr = s + (long)r * 3 * N;
    const T *hr = h + (long)r * 3 * N;
    const u32x4 d = draw(p.seed, p.replica_id, sweep, (uint32_t)i, 1u);
    const T u2 = to_unit<T>(d.v[2]);
    const vec3<T> so = {sr[i], sr[N + i], sr[2 * N + i]};
    const vec3<T> S = trial_spin<T>(p.model, so, d);
    const vec3<T> hv = {hr[i], hr[N + i], hr[2 * N + i]};
    const vec3<T> nb = neighbour_sum<T>(sr, N, L, x, y);
    dE_out[(long)r * N + i] = energy_change<T>(c, so, S, nb, hv);
    u_out[(long)r * N + i] = u2;
    if (S_out) {
        T *o = S_out + (long)r * 3 * N;
        o[i] = S.x;
        o[N + i] = S.y;
        o[2 * N + i] = S.z;
    }
}

template <typename T>
__global__ void k_init(int L, const ddmc_replica_params *__restrict__ params, T *__restrict__ s)
{
    const long N = (long)L * L;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= N) return;
    const ddmc_replica_params p = params[r];
    const u32x4 d = draw(p.seed, p.replica_id, 0u, (uint32_t)i, 0u);
    vec3<T> S;
    if (p.model == DDMC_ISING)
        S = vec3<T>{T(0), T(0), to_unit<T>(d.v[0]) < T(0.5) ? T(1) : T(-1)};
    else
        S = sphere_point<T>(to_unit<T>(d.v[0]), to_unit<T>(d.v[1]));
    T *sr = s + (long)r * 3 * N;
    sr[i] = S.x;
    sr[N + i] = S.y;
    sr[2 * N + i] = S.z;
}

w0_arg w0_of(const ddmc_plan *p)
{
    w0_arg a;
    for (int k = 0; k < 4; ++k) a.v[k] = p->W0[k];
    return a;
}

}  // namespace

template <typename T>
hipError_t launch_init_spins(const ddmc_plan *p, int R, const ddmc_replica_params *params, T *s,
                             hipStream_t st)
{
    const long N = (long)p->L * p->L;
    const int bs = 256;
    hipLaunchKernelGGL(k_init<T>, dim3((unsigned)((N + bs - 1) / bs), R), dim3(bs), 0, st, p->L, params, s);
    return hipGetLastError();
}

namespace {

// Replica records travel to the device as the arguments of a store kernel:
// the launch copies them when it is enqueued, so the caller's host array is
// free on return and no host call waits for the stream (a copy from pageable
// host memory would).  1792 bytes of records per launch.
constexpr int PARAMS_PER_LAUNCH = 32;
struct params_chunk {
    ddmc_replica_params v[PARAMS_PER_LAUNCH];
};

__global__ void __launch_bounds__(64) k_params_store(params_chunk c, int n, ddmc_replica_params *__restrict__ dst)
{
    const int t = threadIdx.x;
    if (t < n) dst[t] = c.v[t];
}

}  // namespace

hipError_t launch_params_store(int R, const ddmc_replica_params *host, ddmc_replica_params *dev, hipStream_t st)
{
    for (int r0 = 0; r0 < R; r0 += PARAMS_PER_LAUNCH) {
        const int n = R - r0 < PARAMS_PER_LAUNCH ? R - r0 : PARAMS_PER_LAUNCH;
        params_chunk c;
        for (int k = 0; k < n; ++k) c.v[k] = host[r0 + k];
        for (int k = n; k < PARAMS_PER_LAUNCH; ++k) c.v[k] = ddmc_replica_params{};
        hipLaunchKernelGGL(k_params_store, dim3(1), dim3(64), 0, st, c, n, dev + r0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

sweep_book make_book(const ddmc_plan *p, uint64_t *accepted, uint64_t *ctr, int finalize, uint64_t advance)
{
    sweep_book b;
    b.done = p->done_ws;
    b.accepted = reinterpret_cast<unsigned long long *>(accepted);
    b.ctr = reinterpret_cast<unsigned long long *>(ctr);
    b.advance = advance;
    b.finalize = (finalize && ctr) ? 1 : 0;
    return b;
}

template <typename T>
hipError_t launch_update(const ddmc_plan *p, int R, const ddmc_replica_params *params, T *s,
                         const T *h, int color, uint64_t *sweep_ctr, uint32_t sweep, uint64_t *accepted,
                         int finalize, uint64_t advance, hipStream_t st, int coset_l)
{
    const long N = (long)p->L * p->L;
    const long nsites = coset_l ? N / ((long)coset_l * coset_l) : N / 2;
    const int bs = 256;
    prof_scope ps(p, DDMC_KERNEL_UPDATE, st);
    hipLaunchKernelGGL(k_update<T>, dim3((unsigned)((nsites + bs - 1) / bs), R), dim3(bs), 0, st, p->L, params,
                       s, h, color, coset_l, sweep, w0_of(p), make_book(p, accepted, sweep_ctr, finalize, advance));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_trial(const ddmc_plan *p, int R, const ddmc_replica_params *params, const T *s,
                        const T *h, int color, uint32_t sweep, T *dE, T *u, T *S, hipStream_t st)
{
    const long half = (long)p->L * p->L / 2;
    const int bs = 256;
    hipLaunchKernelGGL(k_trial<T>, dim3((unsigned)((half + bs - 1) / bs), R), dim3(bs), 0, st, p->L, params,
                       s, h, color, sweep, w0_of(p), dE, u, S);
    return hipGetLastError();
}

#define DDMC_INST(T)                                                                                      \
    template hipError_t launch_init_spins<T>(const ddmc_plan *, int, const ddmc_replica_params *, T *,   \
                                             hipStream_t);                                               \
    template hipError_t launch_update<T>(const ddmc_plan *, int, const ddmc_replica_params *, T *,       \
                                         const T *, int, uint64_t *, uint32_t, uint64_t *, int, uint64_t, \
                                         hipStream_t, int);                                              \
    template hipError_t launch_trial<T>(const ddmc_plan *, int, const ddmc_replica_params *, const T *,  \
                                        const T *, int, uint32_t, T *, T *, T *, hipStream_t);
DDMC_INST(float)
DDMC_INST(double)
#undef DDMC_INST

}  // namespace ddmc
