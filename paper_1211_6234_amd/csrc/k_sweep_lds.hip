// k_sweep_lds.hip -- checkerboard sweeps of small lattices with a whole
// replica in one workgroup for every sweep of a call.
//
// For L <= 64 in FP32 (L <= 48 in FP64) a replica's spins, its half spectrum
// and the transform scratch fit in one CU's LDS.  One workgroup (1024
// threads, 512 in FP64) then runs every half-sweep of the call: the FFT field of the
// current state (forward row transforms, column transforms with the kernel
// multiply, inverse row transforms: the same real-to-complex scheme and
// kernel spectrum W^ as the multi-launch FFT path) and the Metropolis update
// of the colour's sites with that frozen field (Sec. 3.2), separated by
// workgroup barriers instead of kernel launches.  The state is read from HBM
// once at the start of a call and written once at the end; W^ is read from
// L2 each half-sweep.
//
// One launch serves several groups of replicas (lattice sizes), each with
// its own plan data: blocks [block0, block0 + R) of a launch belong to one
// group, and each block runs the body compiled for its group's L.
//
// Sampling (metropolis_sample on such a plan): after each sweep the
// observables of the state it left, as the observables call defines them
// with the full field.  The colour-0 half-sweep of sweep t computes the full
// field of the state after sweep t - 1 anyway; the sample of that state is
// summed from it before the update.  The state after the last sweep gets one
// more field evaluation at the end of the call.
#include "fft_reg.hpp"
#include "device_common.hpp"
#include "internal.hpp"
#include "obs_common.hpp"

namespace ddmc {

namespace {

// threads of a workgroup: FP64 takes half, so that each thread may hold
// twice the registers (the FP64 transforms of L = 48 need them)
template <typename T> constexpr int LT = sizeof(T) == 8 ? 512 : 1024;
// dynamic LDS of one workgroup: a CU's 160 KiB less room for the kernel's
// static LDS (a 4-byte counter)
constexpr size_t LDS_BUDGET = 160 * 1024 - 256;
constexpr int LDS_MAX_GROUPS = DDMC_MULTI_MAX_GROUPS;

// One group of replicas sharing a lattice size and a plan.
struct lds_group {
    int L, R, block0;                   // size, replicas, first block of the group in the launch
    uint32_t sweep0;                    // first sweep index when ctr is NULL
    const void *what;                   // plan's W^ [L/2 + 1][L] of (xx, yy, xy, zz), 1/L^2 folded in
    const void *tw;                     // plan's twiddles e^{-2 pi i k / L}, [L]
    const ddmc_replica_params *params;  // [R]
    void *s;                            // [R][3][L][L]
    unsigned long long *ctr;            // [R] device sweep counters or NULL
    unsigned long long *accepted;       // [R] or NULL
    double *obs;                        // [nsweeps][R][DDMC_NOBS]: one sample after each sweep, or NULL
    double *eta_acc;                    // [R][L][L] cone-angle accumulators of the samples, or NULL
    double w0[4];                       // W(0): xx, yy, xy, zz
};
struct lds_batch {
    int ngroups, nsweeps;
    lds_group g[LDS_MAX_GROUPS];
};

template <typename T> struct alignas(2 * sizeof(T)) cpx {
    T re, im;
};
template <typename T> __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return {a.re, -a.im}; }

// ---- compile-time layout of one lattice size
template <typename T, int L> struct lds_geom {
    static constexpr int H = L / 2;
    static constexpr int SP = H + 1;              // row stride of the spectrum (odd: column reads hit
                                                  // distinct banks)
    static constexpr int N = L * L;
    using RS = fftreg::split<H>;                  // row transforms (H points)
    using CS = fftreg::split<L>;                  // column transforms (L points)
    static constexpr int ROW_SEQ = RS::n1 * (RS::n2 + 1);   // scratch per transformed sequence
    static constexpr int COL_SEQ = CS::n1 * (CS::n2 + 1);
    // bytes before the scratch: twiddles, spectrum [3][L][SP], spins [3][N]
    static constexpr size_t FIXED = sizeof(cpx<T>) * ((size_t)L + 3 * (size_t)L * SP) + sizeof(T) * 3 * (size_t)N;
    static constexpr int SCR_AVAIL = FIXED < LDS_BUDGET ? (int)((LDS_BUDGET - FIXED) / sizeof(cpx<T>)) : 0;
    // sequences transformed at once: all of them, or equal chunks that fit
    static constexpr int ROW_NCH = SCR_AVAIL > 0 ? (3 * L * ROW_SEQ + SCR_AVAIL - 1) / SCR_AVAIL : 1;
    static constexpr int COL_NCH = SCR_AVAIL > 0 ? (3 * H * COL_SEQ + SCR_AVAIL - 1) / SCR_AVAIL : 1;
    static constexpr int ROW_CH = (3 * L + ROW_NCH - 1) / ROW_NCH;
    static constexpr int COL_CH = (3 * H + COL_NCH - 1) / COL_NCH;
    static constexpr int SCR_FFT = (ROW_CH * ROW_SEQ > COL_CH * COL_SEQ) ? ROW_CH * ROW_SEQ : COL_CH * COL_SEQ;
    // the scratch also stages a sample's block reduction: NACC FP64 sums per
    // wave and the NACC totals
    static constexpr int SCR_OBS =
        (int)(((size_t)(LT<T> / 64 + 1) * obs::NACC * sizeof(double) + sizeof(cpx<T>) - 1) / sizeof(cpx<T>));
    static constexpr int SCR = SCR_FFT > SCR_OBS ? SCR_FFT : SCR_OBS;
    static constexpr size_t BYTES = FIXED + sizeof(cpx<T>) * (size_t)SCR;
    static constexpr bool OK = BYTES <= LDS_BUDGET;
    // untangle inside the forward column pass: needs every column in one
    // chunk, and pays when that pass has enough items to occupy the
    // workgroup (with few, folding lengthens the busy threads' chains: at
    // L = 16 and 32 a pass of its own was faster)
    template <int LTH> static constexpr bool FOLD_UNTANGLE = COL_NCH == 1 && 3 * H * CS::n2 >= LTH / 2;
};

// Element j of the sequence at a[b], stride es, as stored.
template <typename T> struct ld_plain {
    int es;
    __device__ cpx<T> operator()(const cpx<T> *a, int b, int j) const { return a[b + j * es]; }
};

// Element m of the tangled sequence of a half-spectrum row (stride 1):
// Z[m] = (X[m] + conj X[H-m]) + i (X[m] - conj X[H-m]) e^{2 pi i m / L}, and
// for m = 0 the packed pair X0 + i X_{L/2} unpacked as (re + im, re - im).
// Read by the inverse row transform's first pass straight from the spectrum,
// so that the tangle needs no pass and barrier of its own.
template <typename T, int H> struct ld_tangle {
    const cpx<T> *tw;   // e^{-2 pi i k / L}, k < L = 2H
    __device__ cpx<T> operator()(const cpx<T> *a, int b, int m) const
    {
        const cpx<T> x = a[b + m];
        const cpx<T> bc = cconj(a[b + (m == 0 ? 0 : H - m)]);
        const cpx<T> od = cmul(cpx<T>{x.re - bc.re, x.im - bc.im}, cconj(tw[m]));
        const cpx<T> z = {x.re + bc.re - od.im, x.im + bc.im + od.re};
        return m == 0 ? cpx<T>{x.re + x.im, x.re - x.im} : z;
    }
};

// Element y of column kx of the untangled spectrum, from the tangled rows
// Z[y][k] (row-FFT output, stride SP; b = c L SP + kx):
// X[y][kx] = ((Z[kx] + conj Z[H-kx]) - i w^kx (Z[kx] - conj Z[H-kx])) / 2, and
// for kx = 0 the packed pair X0 + i X_{L/2} = (re + im, re - im).  Read by the
// forward column transform's first pass, so that the untangle needs no pass
// and barrier of its own; valid only when every column is read before any is
// written back (all columns in one chunk).
template <typename T, int H, int SP> struct ld_untangle {
    const cpx<T> *tw;   // e^{-2 pi i k / L}
    __device__ cpx<T> operator()(const cpx<T> *a, int b, int y) const
    {
        const int kx = b % SP;
        const cpx<T> z = a[b + y * SP];
        const cpx<T> bc = cconj(a[b + y * SP + (kx == 0 ? 0 : H - 2 * kx)]);
        const cpx<T> d = {z.re - bc.re, z.im - bc.im};
        const cpx<T> od = cmul(tw[kx], cpx<T>{d.im, -d.re});
        const cpx<T> x = {T(0.5) * (z.re + bc.re + od.re), T(0.5) * (z.im + bc.im + od.im)};
        return kx == 0 ? cpx<T>{z.re + z.im, z.re - z.im} : x;
    }
};

// Two-pass transform (fft_reg.hpp) of the sequences f in [f0, f0 + nf) of
// length n; element j of sequence f is ld(a, base(f), j), stored back at
// a[base(f) + j * es].  Pass A: item (f, j2) takes the n1-point DFT of
// x[j1 n2 + j2] and scales output k1 by w_n^(j2 k1) into the scratch; pass B:
// item (f, k1) takes the n2-point DFT of scratch row k1 and writes
// X[k1 + n1 k2] in place.  Two barriers.
template <typename T, int n, int L, bool INV, typename Base, typename Load>
__device__ __forceinline__ void fft2(cpx<T> *a, Base base, int es, int f0, int nf, cpx<T> *sc, const cpx<T> *tw,
                                     Load ld)
{
    using S = fftreg::split<n>;
    constexpr int n1 = S::n1, n2 = S::n2, P = n2 + 1;
    const int tid = threadIdx.x;
    for (int e = tid; e < nf * n2; e += LT<T>) {
        const int fl = e / n2, j2 = e - fl * n2;
        const int b = base(f0 + fl);
        fftreg::cx<T> v[n1];
#pragma unroll
        for (int j1 = 0; j1 < n1; ++j1) {
            const cpx<T> x = ld(a, b, j1 * n2 + j2);
            v[j1] = {x.re, x.im};
        }
        fftreg::dft<T, n1, INV>(v);
#pragma unroll
        for (int k1 = 0; k1 < n1; ++k1) {
            cpx<T> x{v[k1].re, v[k1].im};
            if (k1 > 0) {
                const cpx<T> w = tw[(j2 * k1 * (L / n)) % L];
                x = cmul(x, INV ? cconj(w) : w);
            }
            sc[(fl * n1 + k1) * P + j2] = x;
        }
    }
    __syncthreads();
    for (int e = tid; e < nf * n1; e += LT<T>) {
        const int fl = e / n1, k1 = e - fl * n1;
        const int b = base(f0 + fl);
        fftreg::cx<T> v[n2];
#pragma unroll
        for (int j2 = 0; j2 < n2; ++j2) {
            const cpx<T> x = sc[(fl * n1 + k1) * P + j2];
            v[j2] = {x.re, x.im};
        }
        fftreg::dft<T, n2, INV>(v);
#pragma unroll
        for (int k2 = 0; k2 < n2; ++k2) a[b + (k1 + n1 * k2) * es] = cpx<T>{v[k2].re, v[k2].im};
    }
    __syncthreads();
}

struct lds_rows {   // sequence f = c L + y: row y of component c
    int SP;
    __device__ int operator()(int f) const { return f * SP; }
};
struct lds_cols {   // sequence f = c H + kx: column kx of component c
    int H, LSP;
    __device__ int operator()(int f) const { return (f / H) * LSP + (f % H); }
};

// One call for replica r of group g: nsweeps checkerboard sweeps.
// SAMPLE: the variant that samples the observables (g.obs set); the plain
// sweeps are compiled without that code
template <typename T, int L, bool SAMPLE>
__device__ __forceinline__ void lds_body(const lds_group &g, int r, int nsweeps, unsigned int *nacc_l)
{
    using G = lds_geom<T, L>;
    constexpr int H = G::H, SP = G::SP, N = G::N;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<T> *tw = reinterpret_cast<cpx<T> *>(smem);   // [L]
    cpx<T> *sp = tw + L;                              // [3][L][SP]
    T *sl = reinterpret_cast<T *>(sp + 3 * L * SP);   // [3][N]
    cpx<T> *sc = reinterpret_cast<cpx<T> *>(sl + 3 * N);
    const int tid = threadIdx.x;
    T *sg = reinterpret_cast<T *>(g.s) + (size_t)r * 3 * N;
    const cpx<T> *twg = reinterpret_cast<const cpx<T> *>(g.tw);
    const vec4a<T> *what = reinterpret_cast<const vec4a<T> *>(g.what);
    const ddmc_replica_params p = g.params[r];
    // the replica's draw words and first sweep are wave-uniform: held in
    // scalar registers, as is whatever the compiler hoists from them
    const uint32_t sweep0 = __builtin_amdgcn_readfirstlane(g.ctr ? (uint32_t)g.ctr[r] : g.sweep0);
    const uint32_t rid = __builtin_amdgcn_readfirstlane(p.replica_id);
    const uint32_t model = __builtin_amdgcn_readfirstlane(p.model);
    const uint64_t seed = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(p.seed >> 32)) << 32) |
                          __builtin_amdgcn_readfirstlane((uint32_t)p.seed);
    site_consts<T> cst;
    cst.J = (T)p.J; cst.K2 = (T)p.K2; cst.K4 = (T)p.K4; cst.g = (T)p.g; cst.T_ = (T)p.T;
    cst.w0xx = (T)g.w0[0]; cst.w0yy = (T)g.w0[1]; cst.w0xy = (T)g.w0[2]; cst.w0zz = (T)g.w0[3];

    for (int e = tid; e < L; e += LT<T>) tw[e] = twg[e];
    for (int e = tid; e < 3 * N; e += LT<T>) sl[e] = sg[e];
    if (tid == 0) *nacc_l = 0u;
    __syncthreads();
    unsigned int my_acc = 0u;
    const lds_rows rows{SP};
    const lds_cols cols{H, L * SP};

    // the full field of the current state, h(x, y) component c in row y of
    // component c of the spectrum: z[n] = h(2n) + i h(2n+1)
    auto field = [&]() {
        // ---- forward row transforms: z[n] = s(2n) + i s(2n+1), H points,
        // then the untangle X[k] = E + w^k O into the spectrum rows
        for (int f0 = 0; f0 < 3 * L; f0 += G::ROW_CH) {
            const int nf = min(G::ROW_CH, 3 * L - f0);
            using S = typename G::RS;
            constexpr int n1 = S::n1, n2 = S::n2, P = n2 + 1;
            for (int e = tid; e < nf * n2; e += LT<T>) {
                const int fl = e / n2, j2 = e - fl * n2;
                const T *row = sl + (size_t)(f0 + fl) * L;   // f = c L + y: component c, row y
                fftreg::cx<T> v[n1];
#pragma unroll
                for (int j1 = 0; j1 < n1; ++j1) {
                    const int m = j1 * n2 + j2;
                    v[j1] = {row[2 * m], row[2 * m + 1]};
                }
                fftreg::dft<T, n1, false>(v);
#pragma unroll
                for (int k1 = 0; k1 < n1; ++k1) {
                    cpx<T> x{v[k1].re, v[k1].im};
                    if (k1 > 0) x = cmul(x, tw[(j2 * k1 * (L / H)) % L]);
                    sc[(fl * n1 + k1) * P + j2] = x;
                }
            }
            __syncthreads();
            for (int e = tid; e < nf * n1; e += LT<T>) {
                const int fl = e / n1, k1 = e - fl * n1;
                fftreg::cx<T> v[n2];
#pragma unroll
                for (int j2 = 0; j2 < n2; ++j2) {
                    const cpx<T> x = sc[(fl * n1 + k1) * P + j2];
                    v[j2] = {x.re, x.im};
                }
                fftreg::dft<T, n2, false>(v);
                cpx<T> *o = sp + (f0 + fl) * SP;
#pragma unroll
                for (int k2 = 0; k2 < n2; ++k2) o[k1 + n1 * k2] = cpx<T>{v[k2].re, v[k2].im};
            }
            __syncthreads();
        }
        // ---- untangle, column transforms, kernel multiply, inverse column
        // transforms.  The untangle happens as the forward column pass
        // reads the rows (FOLD_UNTANGLE) or in a pass of its own, one item
        // per pair (k, H - k) of a row.
        if constexpr (G::template FOLD_UNTANGLE<LT<T>>) {
            fft2<T, L, L, false>(sp, cols, SP, 0, 3 * H, sc, tw, ld_untangle<T, H, SP>{tw});
        } else {
            for (int e = tid; e < 3 * L * (H / 2 + 1); e += LT<T>) {
                const int f = e / (H / 2 + 1), k = e - f * (H / 2 + 1);
                cpx<T> *o = sp + f * SP;
                if (k == 0) {
                    const cpx<T> z = o[0];
                    o[0] = cpx<T>{z.re + z.im, z.re - z.im};   // X0 + i X_{L/2}
                } else {
                    const int km = H - k;
                    const cpx<T> zk = o[k], zm = o[km];
                    auto untangle = [&](cpx<T> a, cpx<T> b, int kk) {   // b = Z[H - kk]
                        const cpx<T> bc = cconj(b);
                        const cpx<T> d = {a.re - bc.re, a.im - bc.im};
                        const cpx<T> od = cmul(tw[kk], cpx<T>{d.im, -d.re});   // w^k (-i) (a - conj b)
                        return cpx<T>{T(0.5) * (a.re + bc.re + od.re), T(0.5) * (a.im + bc.im + od.im)};
                    };
                    const cpx<T> xk = untangle(zk, zm, k);
                    if (km != k) o[km] = untangle(zm, zk, km);
                    o[k] = xk;
                }
            }
            __syncthreads();
            for (int f0 = 0; f0 < 3 * H; f0 += G::COL_CH)
                fft2<T, L, L, false>(sp, cols, SP, f0, min(G::COL_CH, 3 * H - f0), sc, tw, ld_plain<T>{SP});
        }
        // multiply: item (kx, ky); the packed column kx = 0 holds the real
        // columns kx = 0 (A) and kx = L/2 (B) as A + i B, one item per pair (ky, L - ky)
        for (int e = tid; e < (H - 1) * L + (L / 2 + 1); e += LT<T>) {
            if (e < (H - 1) * L) {
                const int kx = 1 + e / L, ky = e % L;
                cpx<T> *vx = sp + ky * SP + kx, *vy = vx + L * SP, *vz = vy + L * SP;
                const vec4a<T> w = what[kx * L + ky];
                const cpx<T> a = *vx, b = *vy, c = *vz;
                *vx = cpx<T>{w.a * a.re + w.c * b.re, w.a * a.im + w.c * b.im};
                *vy = cpx<T>{w.c * a.re + w.b * b.re, w.c * a.im + w.b * b.im};
                *vz = cpx<T>{w.d * c.re, w.d * c.im};
            } else {
                const int ky = e - (H - 1) * L, km = (L - ky) % L;
                const vec4a<T> wa = what[ky], wb = what[H * L + ky];
                const vec4a<T> wam = what[km], wbm = what[H * L + km];
                cpx<T> C[3], Cm[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    C[c] = sp[c * L * SP + ky * SP];
                    Cm[c] = sp[c * L * SP + km * SP];
                }
                // result at bin q from C = F[q] and D = F[-q]
                auto apply = [&](const cpx<T> (&Cq)[3], const cpx<T> (&Dq)[3], vec4a<T> a4, vec4a<T> b4,
                                 cpx<T> (&out)[3]) {
                    cpx<T> A[3], B[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const cpx<T> dc = cconj(Dq[c]);
                        const cpx<T> sm = {Cq[c].re + dc.re, Cq[c].im + dc.im};
                        const cpx<T> df = {Cq[c].re - dc.re, Cq[c].im - dc.im};
                        A[c] = {T(0.5) * sm.re, T(0.5) * sm.im};
                        B[c] = {T(0.5) * df.im, -T(0.5) * df.re};   // df / (2i)
                    }
                    const cpx<T> a0 = {a4.a * A[0].re + a4.c * A[1].re, a4.a * A[0].im + a4.c * A[1].im};
                    const cpx<T> a1 = {a4.c * A[0].re + a4.b * A[1].re, a4.c * A[0].im + a4.b * A[1].im};
                    const cpx<T> a2 = {a4.d * A[2].re, a4.d * A[2].im};
                    const cpx<T> b0 = {b4.a * B[0].re + b4.c * B[1].re, b4.a * B[0].im + b4.c * B[1].im};
                    const cpx<T> b1 = {b4.c * B[0].re + b4.b * B[1].re, b4.c * B[0].im + b4.b * B[1].im};
                    const cpx<T> b2 = {b4.d * B[2].re, b4.d * B[2].im};
                    out[0] = {a0.re - b0.im, a0.im + b0.re};   // a + i b
                    out[1] = {a1.re - b1.im, a1.im + b1.re};
                    out[2] = {a2.re - b2.im, a2.im + b2.re};
                };
                cpx<T> o1[3], o2[3];
                apply(C, Cm, wa, wb, o1);
                if (km != ky) apply(Cm, C, wam, wbm, o2);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    sp[c * L * SP + ky * SP] = o1[c];
                    if (km != ky) sp[c * L * SP + km * SP] = o2[c];
                }
            }
        }
        __syncthreads();
        for (int f0 = 0; f0 < 3 * H; f0 += G::COL_CH)
            fft2<T, L, L, true>(sp, cols, SP, f0, min(G::COL_CH, 3 * H - f0), sc, tw, ld_plain<T>{SP});
        // ---- inverse row transforms, each row tangled as it is read
        for (int f0 = 0; f0 < 3 * L; f0 += G::ROW_CH)
            fft2<T, H, L, true>(sp, rows, 1, f0, min(G::ROW_CH, 3 * L - f0), sc, tw, ld_tangle<T, H>{tw});
    };
    // observables of the current state with that field into row `row` of the
    // samples: each thread sums its sites' terms and each wave its threads'
    // sums in the path's precision (as the fused four-launch sampler does),
    // the wave totals are added in FP64, in an order that depends only on L
    auto sample = [&](int row) {
        using A = T;
        A a[obs::NACC];
#pragma unroll
        for (int k = 0; k < obs::NACC; ++k) a[k] = A(0);
        double *eta_r = g.eta_acc ? g.eta_acc + (size_t)r * N : nullptr;
#pragma unroll 1
        for (int i = tid; i < N; i += LT<T>) {
            const int y = i / L, x = i - y * L;
            const int ix = y * L + (x + 1 == L ? 0 : x + 1), iy = (y + 1 == L ? 0 : y + 1) * L + x;
            T s3[3], px[3], py[3], h3[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                s3[c] = sl[c * N + i];
                px[c] = sl[c * N + ix];
                py[c] = sl[c * N + iy];
                const cpx<T> z = sp[(c * L + y) * SP + (x >> 1)];
                h3[c] = (x & 1) ? z.im : z.re;
            }
            const T bond = s3[0] * (px[0] + py[0]) + s3[1] * (px[1] + py[1]) + s3[2] * (px[2] + py[2]);
            a[0] += -cst.J * bond;
            a[1] += T(0.5) * cst.g * (s3[0] * h3[0] + s3[1] * h3[1] + s3[2] * h3[2]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                a[6 + c] += (A)obs::wall(s3[c], px[c]);
                a[9 + c] += (A)obs::wall(s3[c], py[c]);
            }
            double av = eta_r ? eta_r[i] : 0.0;
            obs::site_terms<T, A>(a, s3, p, eta_r != nullptr, av, (y & 1) ? A(-1) : A(1), (x & 1) ? A(-1) : A(1));
            if (eta_r) eta_r[i] = av;
        }
        // wave totals (the first 16 sums at once, as the row kernels take
        // them; the non-finite count by ballots: a thread holds at most NS
        // sites), then the waves in order in FP64
        double *red = reinterpret_cast<double *>(sc);                 // [waves][NACC]
        double *tot = red + (LT<T> / 64) * obs::NACC;                 // [NACC]
        const A v = obs::wave_sum16(a);
        if ((tid & 3) == 0) red[(tid >> 6) * obs::NACC + ((tid & 63) >> 2)] = (double)v;
        static_assert(obs::NACC == 18, "two accumulators beyond the 16 of wave_sum16");
        const A v16 = obs::wave_sum(a[16]);
        constexpr int NS = (N + LT<T> - 1) / LT<T>;   // sites per thread, at most
        int v17 = 0;
#pragma unroll
        for (int j = 0; j < NS; ++j) v17 += __popcll(__ballot(a[17] > A(j) + A(0.5)));
        if ((tid & 63) == 0) {
            red[(tid >> 6) * obs::NACC + 16] = (double)v16;
            red[(tid >> 6) * obs::NACC + 17] = (double)v17;
        }
        __syncthreads();
        if (tid < obs::NACC) {
            double u = 0.0;
#pragma unroll
            for (int w = 0; w < LT<T> / 64; ++w) u += red[w * obs::NACC + tid];
            tot[tid] = u;
        }
        __syncthreads();
        if (tid == 0) obs::finish(L, tot, true, g.eta_acc != nullptr, g.obs + ((size_t)row * g.R + r) * DDMC_NOBS);
        __syncthreads();   // the scratch serves the next transforms
    };

    // with samples, one more pass takes the field of the state after the last
    // sweep (colour 0 of t = nsweeps, no update)
    const int tend = nsweeps + ((SAMPLE && nsweeps > 0) ? 1 : 0);
    for (int t = 0; t < tend; ++t) {
        const uint32_t sweep = sweep0 + (uint32_t)t;
        for (int color = 0; color < 2; ++color) {
            field();
            if constexpr (SAMPLE) {
                if (color == 0 && t > 0) sample(t - 1);   // the state after sweep t - 1
            }
            if (t == nsweeps) break;
            // ---- Metropolis update of the colour's sites with the frozen field
            // (row y of component c holds z[n] = h(2n) + i h(2n+1))
            for (int j = tid; j < N / 2; j += LT<T>) {
                const int y = j / H, x = 2 * (j - y * H) + ((color + y) & 1);
                const int i = y * L + x;
                const int xp = (x + 1 == L) ? 0 : x + 1, xm = (x == 0) ? L - 1 : x - 1;
                const int yp = (y + 1 == L) ? 0 : y + 1, ym = (y == 0) ? L - 1 : y - 1;
                const int a = y * L + xp, b = y * L + xm, c = yp * L + x, d = ym * L + x;
                vec3<T> nb;
                nb.x = sl[a] + sl[b] + sl[c] + sl[d];
                nb.y = sl[N + a] + sl[N + b] + sl[N + c] + sl[N + d];
                nb.z = sl[2 * N + a] + sl[2 * N + b] + sl[2 * N + c] + sl[2 * N + d];
                const vec3<T> so = {sl[i], sl[N + i], sl[2 * N + i]};
                const cpx<T> zx = sp[y * SP + (x >> 1)], zy = sp[(L + y) * SP + (x >> 1)],
                             zz = sp[(2 * L + y) * SP + (x >> 1)];
                const bool odd = x & 1;
                const vec3<T> hv = {odd ? zx.im : zx.re, odd ? zy.im : zy.re, odd ? zz.im : zz.re};
                const u32x4 dr = draw(seed, rid, sweep, (uint32_t)i, 1u);
                const vec3<T> S = trial_spin<T>(model, so, dr);
                const T dE = energy_change<T>(cst, so, S, nb, hv);
                if (metropolis(dE, cst.T_, to_unit<T>(dr.v[2]))) {
                    sl[i] = S.x;
                    sl[N + i] = S.y;
                    sl[2 * N + i] = S.z;
                    ++my_acc;
                }
            }
            __syncthreads();
        }
    }
    for (int e = tid; e < 3 * N; e += LT<T>) sg[e] = sl[e];
    if (g.accepted) {
        const unsigned long long mask = __ballot(my_acc != 0u);
        unsigned int v = my_acc;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if ((tid & 63) == 0 && mask != 0ull) atomicAdd(nacc_l, v);
        __syncthreads();
        if (tid == 0) g.accepted[r] += *nacc_l;
    }
    if (g.ctr && tid == 0) g.ctr[r] += (unsigned long long)nsweeps;
}

template <typename T, bool SAMPLE>
__global__ void __launch_bounds__(LT<T>) k_sweep_lds(lds_batch b)
{
    __shared__ unsigned int nacc;
    int gi = 0;
    while (gi + 1 < b.ngroups && (int)blockIdx.x >= b.g[gi + 1].block0) ++gi;
    const lds_group &g = b.g[gi];
    const int r = (int)blockIdx.x - g.block0;
    switch (g.L) {
    case 8: if constexpr (lds_geom<T, 8>::OK) lds_body<T, 8, SAMPLE>(g, r, b.nsweeps, &nacc); break;
    case 16: if constexpr (lds_geom<T, 16>::OK) lds_body<T, 16, SAMPLE>(g, r, b.nsweeps, &nacc); break;
    case 24: if constexpr (lds_geom<T, 24>::OK) lds_body<T, 24, SAMPLE>(g, r, b.nsweeps, &nacc); break;
    case 32: if constexpr (lds_geom<T, 32>::OK) lds_body<T, 32, SAMPLE>(g, r, b.nsweeps, &nacc); break;
    case 48: if constexpr (lds_geom<T, 48>::OK) lds_body<T, 48, SAMPLE>(g, r, b.nsweeps, &nacc); break;
    case 64: if constexpr (lds_geom<T, 64>::OK) lds_body<T, 64, SAMPLE>(g, r, b.nsweeps, &nacc); break;
    default: break;
    }
}

template <typename T> size_t lds_bytes(int L)
{
    switch (L) {
    case 8: return lds_geom<T, 8>::OK ? lds_geom<T, 8>::BYTES : 0;
    case 16: return lds_geom<T, 16>::OK ? lds_geom<T, 16>::BYTES : 0;
    case 24: return lds_geom<T, 24>::OK ? lds_geom<T, 24>::BYTES : 0;
    case 32: return lds_geom<T, 32>::OK ? lds_geom<T, 32>::BYTES : 0;
    case 48: return lds_geom<T, 48>::OK ? lds_geom<T, 48>::BYTES : 0;
    case 64: return lds_geom<T, 64>::OK ? lds_geom<T, 64>::BYTES : 0;
    default: return 0;
    }
}

}  // namespace

bool lds_sweep_ok(int L, ddmc_prec prec)
{
    return prec == DDMC_F64 ? lds_bytes<double>(L) > 0 : lds_bytes<float>(L) > 0;
}

template <typename T>
ddmc_status lds_sweep(int ngroups, ddmc_plan *const *plans, const int *R, const ddmc_replica_params *const *params,
                      T *const *s, uint64_t *const *ctr, uint64_t sweep0, int nsweeps, uint64_t *const *accepted,
                      double *obs, double *eta_acc, hipStream_t st)
{
    if ((obs || eta_acc) && ngroups != 1) return fail(DDMC_EINVAL, "LDS sweep: samples need a single group");
    if (ngroups < 1 || ngroups > LDS_MAX_GROUPS) return fail(DDMC_EINVAL, "LDS sweep: 1 to 8 groups per launch");
    lds_batch b{};
    b.ngroups = ngroups;
    b.nsweeps = nsweeps;
    size_t lds = 0;
    int blocks = 0;
    for (int k = 0; k < ngroups; ++k) {
        const ddmc_plan *p = plans[k];
        lds_group &g = b.g[k];
        g.L = p->L;
        g.R = R[k];
        g.block0 = blocks;
        g.sweep0 = (uint32_t)sweep0;
        g.what = p->what;
        g.tw = p->twiddle;
        g.params = params[k];
        g.s = s[k];
        g.ctr = ctr ? reinterpret_cast<unsigned long long *>(ctr[k]) : nullptr;
        g.accepted = accepted ? reinterpret_cast<unsigned long long *>(accepted[k]) : nullptr;
        g.obs = obs;
        g.eta_acc = obs ? eta_acc : nullptr;
        for (int c = 0; c < 4; ++c) g.w0[c] = p->W0[c];
        blocks += R[k];
        const size_t need = lds_bytes<T>(p->L);
        if (need == 0) return fail(DDMC_EUNSUPPORTED, "LDS sweep: lattice size not handled in one workgroup");
        if (need > lds) lds = need;
    }
    if (blocks == 0) return DDMC_OK;
    const void *fn = obs ? reinterpret_cast<const void *>(&k_sweep_lds<T, true>)
                         : reinterpret_cast<const void *>(&k_sweep_lds<T, false>);
    hipError_t he = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (he != hipSuccess) return hip_check(he, "LDS sweep kernel LDS size");
    prof_scope ps(plans[0], DDMC_KERNEL_UPDATE, st);
    if (obs)
        hipLaunchKernelGGL((k_sweep_lds<T, true>), dim3(blocks), dim3(LT<T>), lds, st, b);
    else
        hipLaunchKernelGGL((k_sweep_lds<T, false>), dim3(blocks), dim3(LT<T>), lds, st, b);
    return hip_check(hipGetLastError(), "LDS sweep kernel launch");
}

template ddmc_status lds_sweep<float>(int, ddmc_plan *const *, const int *, const ddmc_replica_params *const *,
                                      float *const *, uint64_t *const *, uint64_t, int, uint64_t *const *, double *,
                                      double *, hipStream_t);
template ddmc_status lds_sweep<double>(int, ddmc_plan *const *, const int *, const ddmc_replica_params *const *,
                                       double *const *, uint64_t *const *, uint64_t, int, uint64_t *const *, double *,
                                       double *, hipStream_t);

}  // namespace ddmc
