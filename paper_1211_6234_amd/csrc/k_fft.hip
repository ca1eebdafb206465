// k_fft.hip -- the local dipolar field as an FFT circular convolution, and the
// checkerboard sweep built on it.
//
// W(rho) is even, so its 2D spectrum is real: h^ = W^ s^ is a real 2x2 (xx,
// xy, yy) plus 1x1 (zz) multiply per wave vector.  Spins are real, so only
// half of each spectrum is kept:
//   rows:    a real L-point transform along x through an L/2-point complex
//            FFT of z[n] = s[2n] + i s[2n+1] and an untangling pass; the two
//            real bins k = 0 and k = L/2 are packed as X0 + i X_{L/2};
//   columns: an L-point complex FFT along y of each of the L/2 packed
//            columns; the packed column 0 carries two real-input sequences
//            whose spectra are separated before the kernel multiply.
// Spectra live in HBM as [R][3][ky][kx] complex, kx < L/2 (the same bytes as
// the spins).  The FFTs themselves run in LDS (Stockham autosort, radix 4
// with a final radix-2 stage when log2 n is odd; twiddles from a table).
//
// A half-sweep of colour c is two launches:
//   k_cols  : spectrum of s -> forward y-FFT -> W^ multiply -> inverse y-FFT
//   k_rows  : inverse x-transform -> field h of the RB rows of the block ->
//             Metropolis update of the colour-c sites of those rows (field
//             frozen, Sec. 3.2) -> forward x-transform of the updated rows,
//             which is the spectrum the next half-sweep starts from.
// The field never goes to HBM inside a sweep.  The 1/L^2 of the inverse
// transform is folded into W^.
#include "device_common.hpp"
#include "internal.hpp"

namespace ddmc {

namespace {

template <typename T> struct cplx {
    T re, im;
};
template <typename T> __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.re, -a.im}; }
// multiply by +i or -i
template <typename T> __device__ __forceinline__ cplx<T> mul_i(cplx<T> a) { return {-a.im, a.re}; }
template <typename T> __device__ __forceinline__ cplx<T> mul_mi(cplx<T> a) { return {a.im, -a.re}; }

// twiddle e^{-2 pi i j / L} (forward) from the table tw[j] = e^{-2 pi i j / L}
template <typename T, bool INV>
__device__ __forceinline__ cplx<T> twiddle(const cplx<T> *tw, int j)
{
    const cplx<T> w = tw[j];
    return INV ? cconj(w) : w;
}

// One FFT of length n (a power of two, n | L) on each of nseq sequences
// stored back to back in `a`; `b` is scratch of the same size.  Returns the
// buffer that holds the result.  All threads of the block take part.
template <typename T, bool INV>
__device__ cplx<T> *fft_lds(cplx<T> *a, cplx<T> *b, int n, int nseq, const cplx<T> *tw, int L)
{
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int p = 1; p < n;) {
        const int R = ((n / p) % 4 == 0) ? 4 : 2;
        const int Tn = n / R;              // butterflies per sequence
        const int step = L / (R * p);      // table stride of the stage's root
        const int work = nseq * Tn;
        if (R == 4) {
            for (int e = tid; e < work; e += nthr) {
                const int f = e / Tn, i = e - f * Tn;
                const int k = i & (p - 1);
                const cplx<T> *src = a + f * n;
                cplx<T> u0 = src[i];
                cplx<T> u1 = cmul(src[i + Tn], twiddle<T, INV>(tw, (k * step) % L));
                cplx<T> u2 = cmul(src[i + 2 * Tn], twiddle<T, INV>(tw, (2 * k * step) % L));
                cplx<T> u3 = cmul(src[i + 3 * Tn], twiddle<T, INV>(tw, (3 * k * step) % L));
                const cplx<T> t0 = cadd(u0, u2), t1 = csub(u0, u2);
                const cplx<T> t2 = cadd(u1, u3), t3 = csub(u1, u3);
                cplx<T> *dst = b + f * n + (i - k) * 4 + k;
                dst[0] = cadd(t0, t2);
                dst[2 * p] = csub(t0, t2);
                if (INV) {
                    dst[p] = cadd(t1, mul_i(t3));
                    dst[3 * p] = csub(t1, mul_i(t3));
                } else {
                    dst[p] = cadd(t1, mul_mi(t3));
                    dst[3 * p] = csub(t1, mul_mi(t3));
                }
            }
        } else {
            for (int e = tid; e < work; e += nthr) {
                const int f = e / Tn, i = e - f * Tn;
                const int k = i & (p - 1);
                const cplx<T> *src = a + f * n;
                const cplx<T> u0 = src[i];
                const cplx<T> u1 = cmul(src[i + Tn], twiddle<T, INV>(tw, (k * step) % L));
                cplx<T> *dst = b + f * n + (i - k) * 2 + k;
                dst[0] = cadd(u0, u1);
                dst[p] = csub(u0, u1);
            }
        }
        __syncthreads();
        cplx<T> *t = a;
        a = b;
        b = t;
        p *= R;
    }
    return a;
}

template <typename T> __device__ __forceinline__ void load_twiddles(cplx<T> *tw_lds, const cplx<T> *tw, int L)
{
    for (int j = threadIdx.x; j < L; j += blockDim.x) tw_lds[j] = tw[j];
}

struct w0_pack {
    double v[4];
};

enum { ROWS_FWD = 0, ROWS_INV = 1, ROWS_SWEEP = 2 };

// Rows kernel.  Block = RB consecutive rows of one replica.
//   ROWS_FWD  : s -> spectrum rows (spec_out)
//   ROWS_INV  : spec_in -> field h (sites of `color`, or all when color < 0)
//   ROWS_SWEEP: spec_in -> field -> update colour -> spectrum rows of the new state
template <typename T, int MODE>
__global__ void __launch_bounds__(256)
k_rows(int L, int RB, T *__restrict__ s, const cplx<T> *__restrict__ spec_in, cplx<T> *__restrict__ spec_out,
       T *__restrict__ h, int color, uint32_t sweep, const ddmc_replica_params *__restrict__ params, w0_pack w0,
       const cplx<T> *__restrict__ tw, unsigned long long *__restrict__ accepted, int write_spec)
{
    extern __shared__ unsigned char smem_raw[];
    const int H = L / 2;
    const long N = (long)L * L;
    const int nseq = 3 * RB;
    cplx<T> *tw_l = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *bufA = tw_l + L;
    cplx<T> *bufB = bufA + nseq * H;
    T *srow = reinterpret_cast<T *>(bufB + nseq * H);   // [RB + 2][3][L], row 0 = y0 - 1

    const int r = blockIdx.y;
    const int y0 = blockIdx.x * RB;
    const int tid = threadIdx.x, nthr = blockDim.x;
    T *sr = s + (long)r * 3 * N;
    load_twiddles(tw_l, tw, L);

    cplx<T> *zres = nullptr;   // inverse result: z[n] = h(2n) + i h(2n+1) per (row, comp)
    if (MODE != ROWS_FWD) {
        const cplx<T> *src = spec_in + (long)r * 3 * L * H;
        for (int e = tid; e < nseq * H; e += nthr) {
            const int k = e % H, q = e / H;   // q = row_local * 3 + comp
            const int yl = q / 3, c = q - yl * 3;
            bufA[e] = src[((long)c * L + (y0 + yl)) * H + k];
        }
        __syncthreads();
        // tangle: Z'[k] = (X[k] + conj X[H-k]) + i (X[k] - conj X[H-k]) e^{+2 pi i k / L}
        for (int e = tid; e < nseq * H; e += nthr) {
            const int k = e % H, q = e / H;
            const cplx<T> X = bufA[q * H + k];
            cplx<T> Z;
            if (k == 0) {
                const T X0 = X.re, XH = X.im;
                Z.re = X0 + XH;
                Z.im = X0 - XH;
            } else {
                const cplx<T> Xc = cconj(bufA[q * H + (H - k)]);
                const cplx<T> E = cadd(X, Xc);
                const cplx<T> O = cmul(csub(X, Xc), cconj(tw_l[k]));
                Z = cadd(E, mul_i(O));
            }
            bufB[q * H + k] = Z;
        }
        __syncthreads();
        zres = fft_lds<T, true>(bufB, bufA, H, nseq, tw_l, L);
    }

    if (MODE == ROWS_INV) {
        T *hr = h + (long)r * 3 * N;
        const int per_row = (color < 0) ? L : H;
        for (int e = tid; e < RB * 3 * per_row; e += nthr) {
            const int j = e % per_row, q = e / per_row;
            const int yl = q / 3, c = q - yl * 3;
            const int y = y0 + yl;
            const int x = (color < 0) ? j : 2 * j + ((color + y) & 1);
            const cplx<T> z = zres[q * H + (x >> 1)];
            hr[(long)c * N + (long)y * L + x] = (x & 1) ? z.im : z.re;
        }
        return;
    }

    // stage the spin rows: own rows (and for the sweep one halo row above and below)
    const int halo = (MODE == ROWS_SWEEP) ? 1 : 0;
    const int nrows = RB + 2 * halo;
    for (int e = tid; e < nrows * 3 * L; e += nthr) {
        const int x = e % L, q = e / L;
        const int rl = q / 3, c = q - rl * 3;
        int y = y0 - halo + rl;
        y = (y < 0) ? y + L : (y >= L ? y - L : y);
        srow[((rl + 1 - halo) * 3 + c) * L + x] = sr[(long)c * N + (long)y * L + x];
    }
    __syncthreads();

    if (MODE == ROWS_SWEEP) {
        const ddmc_replica_params p = params[r];
        site_consts<T> cst;
        cst.J = (T)p.J; cst.K2 = (T)p.K2; cst.K4 = (T)p.K4; cst.g = (T)p.g; cst.T_ = (T)p.T;
        cst.w0xx = (T)w0.v[0]; cst.w0yy = (T)w0.v[1]; cst.w0xy = (T)w0.v[2]; cst.w0zz = (T)w0.v[3];
        const int nsite = RB * H;
        const int rounds = (nsite + nthr - 1) / nthr;
        for (int rd = 0; rd < rounds; ++rd) {
            const int e = rd * nthr + tid;
            bool acc = false;
            if (e < nsite) {
                const int yl = e / H, j = e - yl * H;
                const int y = y0 + yl;
                const int x = 2 * j + ((color + y) & 1);
                const long i = (long)y * L + x;
                const T *row = srow + (yl + 1) * 3 * L;
                const T *up = srow + (yl + 2) * 3 * L;    // y + 1
                const T *dn = srow + yl * 3 * L;          // y - 1
                const int xp = (x + 1 == L) ? 0 : x + 1, xm = (x == 0) ? L - 1 : x - 1;
                vec3<T> nb;
                nb.x = row[xp] + row[xm] + up[x] + dn[x];
                nb.y = row[L + xp] + row[L + xm] + up[L + x] + dn[L + x];
                nb.z = row[2 * L + xp] + row[2 * L + xm] + up[2 * L + x] + dn[2 * L + x];
                const vec3<T> so = {row[x], row[L + x], row[2 * L + x]};
                vec3<T> hv;
                {
                    const cplx<T> zx = zres[(yl * 3 + 0) * H + j];
                    const cplx<T> zy = zres[(yl * 3 + 1) * H + j];
                    const cplx<T> zz = zres[(yl * 3 + 2) * H + j];
                    const bool odd = x & 1;
                    hv.x = odd ? zx.im : zx.re;
                    hv.y = odd ? zy.im : zy.re;
                    hv.z = odd ? zz.im : zz.re;
                }
                const u32x4 d = draw(p.seed, p.replica_id, sweep, (uint32_t)i, 1u);
                const T u0 = to_unit<T>(d.v[0]), u1 = to_unit<T>(d.v[1]), u2 = to_unit<T>(d.v[2]);
                const vec3<T> S = sphere_point<T>(u0, u1);
                const T dE = energy_change<T>(cst, so, S, nb, hv);
                acc = metropolis(dE, cst.T_, u2);
                if (acc) {
                    // rows of one block never neighbour each other within the colour
                    T *rw = srow + (yl + 1) * 3 * L;
                    rw[x] = S.x;
                    rw[L + x] = S.y;
                    rw[2 * L + x] = S.z;
                    sr[i] = S.x;
                    sr[N + i] = S.y;
                    sr[2 * N + i] = S.z;
                }
            }
            if (accepted) {
                const unsigned long long mask = __ballot(acc);
                if ((tid & (warpSize - 1)) == 0 && mask != 0ull)
                    atomicAdd(&accepted[r], (unsigned long long)__popcll(mask));
            }
        }
        __syncthreads();
        if (!write_spec) return;
    }

    // forward: z[n] = s(2n) + i s(2n+1) for each own row and component
    for (int e = tid; e < nseq * H; e += nthr) {
        const int n = e % H, q = e / H;
        const int yl = q / 3, c = q - yl * 3;
        const T *row = srow + ((yl + 1) * 3 + c) * L;   // own row yl is staged at index yl + 1
        bufA[e] = cplx<T>{row[2 * n], row[2 * n + 1]};
    }
    __syncthreads();
    const cplx<T> *Z = fft_lds<T, false>(bufA, bufB, H, nseq, tw_l, L);
    // untangle: X[k] = E + w^k O with E = (Z[k] + conj Z[H-k])/2, O = -i (Z[k] - conj Z[H-k])/2
    cplx<T> *dst = spec_out + (long)r * 3 * L * H;
    for (int e = tid; e < nseq * H; e += nthr) {
        const int k = e % H, q = e / H;
        const int yl = q / 3, c = q - yl * 3;
        const cplx<T> Zk = Z[q * H + k];
        cplx<T> X;
        if (k == 0) {
            X.re = Zk.re + Zk.im;   // X[0]
            X.im = Zk.re - Zk.im;   // X[L/2]
        } else {
            const cplx<T> Zc = cconj(Z[q * H + (H - k)]);
            const cplx<T> E = cadd(Zk, Zc);
            const cplx<T> O = mul_mi(csub(Zk, Zc));
            const cplx<T> v = cadd(E, cmul(tw_l[k], O));
            X.re = T(0.5) * v.re;
            X.im = T(0.5) * v.im;
        }
        dst[((long)c * L + (y0 + yl)) * H + k] = X;
    }
}

// Columns kernel: block = KC packed columns of one replica, all 3 components.
template <typename T>
__global__ void __launch_bounds__(256)
k_cols(int L, int KC, const cplx<T> *__restrict__ spec_in, cplx<T> *__restrict__ spec_out,
       const T *__restrict__ what, const cplx<T> *__restrict__ tw)
{
    extern __shared__ unsigned char smem_raw[];
    const int H = L / 2;
    const int nseq = 3 * KC;
    cplx<T> *tw_l = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *bufA = tw_l + L;
    cplx<T> *bufB = bufA + nseq * L;
    const int r = blockIdx.y;
    const int kx0 = blockIdx.x * KC;
    const int tid = threadIdx.x, nthr = blockDim.x;
    load_twiddles(tw_l, tw, L);
    const cplx<T> *src = spec_in + (long)r * 3 * L * H;
    // gather: sequence (c, j) holds column kx0 + j of component c, indexed by ky
    for (int e = tid; e < nseq * L; e += nthr) {
        const int j = e % KC, q = e / KC;      // q = c * L + ky
        const int c = q / L, ky = q - c * L;
        bufA[(c * KC + j) * L + ky] = src[((long)c * L + ky) * H + kx0 + j];
    }
    __syncthreads();
    const cplx<T> *F = fft_lds<T, false>(bufA, bufB, L, nseq, tw_l, L);
    cplx<T> *G = (F == bufA) ? bufB : bufA;
    const long WP = (long)L * (H + 1);   // plane stride of what[4][L][H + 1]
    for (int e = tid; e < KC * L; e += nthr) {
        const int ky = e % L, j = e / L;
        const int kx = kx0 + j;
        const cplx<T> vx = F[(0 * KC + j) * L + ky];
        const cplx<T> vy = F[(1 * KC + j) * L + ky];
        const cplx<T> vz = F[(2 * KC + j) * L + ky];
        if (kx != 0) {
            const long o = (long)ky * (H + 1) + kx;
            const T wxx = what[o], wyy = what[WP + o], wxy = what[2 * WP + o], wzz = what[3 * WP + o];
            G[(0 * KC + j) * L + ky] = {wxx * vx.re + wxy * vy.re, wxx * vx.im + wxy * vy.im};
            G[(1 * KC + j) * L + ky] = {wxy * vx.re + wyy * vy.re, wxy * vx.im + wyy * vy.im};
            G[(2 * KC + j) * L + ky] = {wzz * vz.re, wzz * vz.im};
        } else {
            // packed column: C = A + i B with A, B the spectra of the real
            // columns kx = 0 and kx = L/2; separate, multiply, repack
            const int km = (L - ky) % L;
            cplx<T> A[3], B[3];
            for (int c = 0; c < 3; ++c) {
                const cplx<T> C = F[(c * KC + j) * L + ky];
                const cplx<T> Cm = cconj(F[(c * KC + j) * L + km]);
                const cplx<T> s = cadd(C, Cm), d = csub(C, Cm);
                A[c] = {T(0.5) * s.re, T(0.5) * s.im};
                B[c] = {T(0.5) * d.im, -T(0.5) * d.re};   // d / (2i)
            }
            const long o0 = (long)ky * (H + 1), oH = o0 + H;
            const T axx = what[o0], ayy = what[WP + o0], axy = what[2 * WP + o0], azz = what[3 * WP + o0];
            const T bxx = what[oH], byy = what[WP + oH], bxy = what[2 * WP + oH], bzz = what[3 * WP + oH];
            cplx<T> a2[3], b2[3];
            a2[0] = {axx * A[0].re + axy * A[1].re, axx * A[0].im + axy * A[1].im};
            a2[1] = {axy * A[0].re + ayy * A[1].re, axy * A[0].im + ayy * A[1].im};
            a2[2] = {azz * A[2].re, azz * A[2].im};
            b2[0] = {bxx * B[0].re + bxy * B[1].re, bxx * B[0].im + bxy * B[1].im};
            b2[1] = {bxy * B[0].re + byy * B[1].re, bxy * B[0].im + byy * B[1].im};
            b2[2] = {bzz * B[2].re, bzz * B[2].im};
            for (int c = 0; c < 3; ++c) G[(c * KC + j) * L + ky] = cadd(a2[c], mul_i(b2[c]));
        }
    }
    __syncthreads();
    cplx<T> *other = (G == bufA) ? bufB : bufA;
    const cplx<T> *Hc = fft_lds<T, true>(G, other, L, nseq, tw_l, L);
    cplx<T> *dst = spec_out + (long)r * 3 * L * H;
    for (int e = tid; e < nseq * L; e += nthr) {
        const int j = e % KC, q = e / KC;
        const int c = q / L, ky = q - c * L;
        dst[((long)c * L + ky) * H + kx0 + j] = Hc[(c * KC + j) * L + ky];
    }
}

// ---- plan-time kernels (FP64): twiddles and the real kernel spectrum
template <typename T> __global__ void k_twiddles(int L, cplx<T> *tw)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= L) return;
    double sn, cs;
    sincospi(2.0 * (double)j / (double)L, &sn, &cs);
    tw[j] = cplx<T>{(T)cs, (T)(-sn)};
}

// x-pass of the kernel spectrum: Tx[c][y][kx] = sum_x W[c][y][x] e^{-2 pi i kx x / L}, kx <= L/2
__global__ void k_what_x(int L, const double *__restrict__ W, double *__restrict__ tx)
{
    const int H1 = L / 2 + 1;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 4L * L * H1) return;
    const int kx = (int)(e % H1);
    const long q = e / H1;           // c * L + y
    const double *row = W + q * L;
    double re = 0.0, im = 0.0;
    for (int x = 0; x < L; ++x) {
        const long m = ((long)kx * x) % L;
        double sn, cs;
        sincospi(2.0 * (double)m / (double)L, &sn, &cs);
        re += row[x] * cs;
        im -= row[x] * sn;
    }
    tx[2 * e] = re;
    tx[2 * e + 1] = im;
}

// y-pass: What[c][ky][kx] = Re sum_y Tx[c][y][kx] e^{-2 pi i ky y / L}, scaled by 1/L^2
template <typename T>
__global__ void k_what_y(int L, const double *__restrict__ tx, T *__restrict__ what)
{
    const int H1 = L / 2 + 1;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 4L * L * H1) return;
    const int kx = (int)(e % H1);
    const long q = e / H1;           // c * L + ky
    const int c = (int)(q / L), ky = (int)(q % L);
    double re = 0.0;
    for (int y = 0; y < L; ++y) {
        const long m = ((long)ky * y) % L;
        double sn, cs;
        sincospi(2.0 * (double)m / (double)L, &sn, &cs);
        const long o = ((long)c * L + y) * H1 + kx;
        re += tx[2 * o] * cs + tx[2 * o + 1] * sn;   // Re[(a + ib)(cs - i sn)]
    }
    what[e] = (T)(re / ((double)L * (double)L));
}

int rows_per_block(int L)
{
    int rb = 256 / (L / 2);
    if (rb < 1) rb = 1;
    if (rb > L) rb = L;
    return rb;
}

int cols_per_block(int L, int R, size_t celem)
{
    const int H = L / 2;
    // LDS: 2 buffers of 3 KC L complex, at most 48 KiB
    int kc = 1;
    while (kc * 2 <= H && (size_t)2 * 3 * (kc * 2) * L * celem <= 49152) kc *= 2;
    // keep enough blocks to fill the chip
    while (kc > 1 && (H / kc) * R < 512) kc /= 2;
    return kc;
}

template <typename T> size_t rows_lds(int L, int RB)
{
    const int H = L / 2;
    return sizeof(cplx<T>) * ((size_t)L + 2 * 3 * RB * H) + sizeof(T) * (size_t)(RB + 2) * 3 * L;
}

template <typename T> size_t cols_lds(int L, int KC)
{
    return sizeof(cplx<T>) * ((size_t)L + 2 * 3 * (size_t)KC * L);
}

w0_pack w0_of(const ddmc_plan *p)
{
    w0_pack a;
    for (int k = 0; k < 4; ++k) a.v[k] = p->W0[k];
    return a;
}

template <typename T, int MODE>
hipError_t launch_rows(const ddmc_plan *p, int R, T *s, const cplx<T> *in, cplx<T> *out, T *h, int color,
                       uint32_t sweep, const ddmc_replica_params *params, uint64_t *accepted, int write_spec,
                       hipStream_t st)
{
    const int L = p->L;
    const int RB = rows_per_block(L);
    dim3 grid(L / RB, R);
    hipLaunchKernelGGL((k_rows<T, MODE>), grid, dim3(256), rows_lds<T>(L, RB), st, L, RB, s, in, out, h, color,
                       sweep, params, w0_of(p), reinterpret_cast<const cplx<T> *>(p->twiddle),
                       reinterpret_cast<unsigned long long *>(accepted), write_spec);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cols(const ddmc_plan *p, int R, const cplx<T> *in, cplx<T> *out, hipStream_t st)
{
    const int L = p->L;
    const int KC = cols_per_block(L, R, sizeof(cplx<T>));
    dim3 grid((L / 2) / KC, R);
    hipLaunchKernelGGL(k_cols<T>, grid, dim3(256), cols_lds<T>(L, KC), st, L, KC, in, out,
                       reinterpret_cast<const T *>(p->what), reinterpret_cast<const cplx<T> *>(p->twiddle));
    return hipGetLastError();
}

template <typename T> cplx<T> *spec_a(ddmc_plan *p) { return reinterpret_cast<cplx<T> *>(p->spec_ws); }
template <typename T> cplx<T> *spec_b(ddmc_plan *p)
{
    return reinterpret_cast<cplx<T> *>(p->spec_ws) + (size_t)p->R_max * 3 * p->L * (p->L / 2);
}

}  // namespace

bool fft_supported(int L) { return L >= 8 && L <= 512 && (L & (L - 1)) == 0; }

void fft_plan_free(ddmc_plan *p)
{
    hipFree(p->spec_ws);
    hipFree(p->what);
    hipFree(p->twiddle);
    p->spec_ws = p->what = p->twiddle = nullptr;
}

template <typename T> ddmc_status fft_plan_init(ddmc_plan *p, const double *W64)
{
    const int L = p->L, H1 = L / 2 + 1;
    const size_t cbytes = sizeof(cplx<T>);
    if (hipMalloc(&p->spec_ws, 2 * (size_t)p->R_max * 3 * L * (L / 2) * cbytes) != hipSuccess ||
        hipMalloc(&p->what, 4 * (size_t)L * H1 * sizeof(T)) != hipSuccess ||
        hipMalloc(&p->twiddle, (size_t)L * cbytes) != hipSuccess)
        return fail(DDMC_ENOMEM, "ddmc_plan_create: cannot allocate FFT workspace");
    double *tx = nullptr;
    if (hipMalloc(&tx, 2 * 4 * (size_t)L * H1 * sizeof(double)) != hipSuccess)
        return fail(DDMC_ENOMEM, "ddmc_plan_create: cannot allocate FFT scratch");
    const long n = 4L * L * H1;
    hipLaunchKernelGGL(k_twiddles<T>, dim3((L + 255) / 256), dim3(256), 0, nullptr, L,
                       reinterpret_cast<cplx<T> *>(p->twiddle));
    hipLaunchKernelGGL(k_what_x, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, nullptr, L, W64, tx);
    hipLaunchKernelGGL(k_what_y<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, nullptr, L, tx,
                       reinterpret_cast<T *>(p->what));
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    hipFree(tx);
    if (e != hipSuccess) return hip_check(e, "FFT plan set-up");
    // kernels with large dynamic LDS
    const int RB = rows_per_block(L);
    const int KC = cols_per_block(L, 1, cbytes);
    if (rows_lds<T>(L, RB) > 65536 || cols_lds<T>(L, KC) > 65536)
        return fail(DDMC_EUNSUPPORTED, "FFT field: lattice too large for the LDS budget");
    return DDMC_OK;
}

template <typename T> ddmc_status fft_field(ddmc_plan *p, int R, const T *s, T *h, int color, hipStream_t st)
{
    cplx<T> *A = spec_a<T>(p), *B = spec_b<T>(p);
    hipError_t e = launch_rows<T, ROWS_FWD>(p, R, const_cast<T *>(s), nullptr, A, nullptr, -1, 0, nullptr,
                                            nullptr, 1, st);
    if (e == hipSuccess) e = launch_cols<T>(p, R, A, B, st);
    if (e == hipSuccess)
        e = launch_rows<T, ROWS_INV>(p, R, const_cast<T *>(s), B, nullptr, h, color, 0, nullptr, nullptr, 0, st);
    return hip_check(e, "FFT field launch");
}

template <typename T>
ddmc_status fft_sweep(ddmc_plan *p, int R, const ddmc_replica_params *params, T *s, uint64_t sweep0, int nsweeps,
                      uint64_t *accepted, hipStream_t st)
{
    cplx<T> *A = spec_a<T>(p), *B = spec_b<T>(p);
    hipError_t e = launch_rows<T, ROWS_FWD>(p, R, s, nullptr, A, nullptr, -1, 0, nullptr, nullptr, 1, st);
    for (int t = 0; t < nsweeps && e == hipSuccess; ++t) {
        const uint32_t sweep = (uint32_t)(sweep0 + (uint64_t)t);
        for (int color = 0; color < 2 && e == hipSuccess; ++color) {
            const bool last = (t == nsweeps - 1) && color == 1;
            e = launch_cols<T>(p, R, A, B, st);
            if (e == hipSuccess)
                e = launch_rows<T, ROWS_SWEEP>(p, R, s, B, A, nullptr, color, sweep, params, accepted, last ? 0 : 1,
                                               st);
        }
    }
    return hip_check(e, "FFT sweep launch");
}

template ddmc_status fft_plan_init<float>(ddmc_plan *, const double *);
template ddmc_status fft_plan_init<double>(ddmc_plan *, const double *);
template ddmc_status fft_field<float>(ddmc_plan *, int, const float *, float *, int, hipStream_t);
template ddmc_status fft_field<double>(ddmc_plan *, int, const double *, double *, int, hipStream_t);
template ddmc_status fft_sweep<float>(ddmc_plan *, int, const ddmc_replica_params *, float *, uint64_t, int,
                                      uint64_t *, hipStream_t);
template ddmc_status fft_sweep<double>(ddmc_plan *, int, const ddmc_replica_params *, double *, uint64_t, int,
                                       uint64_t *, hipStream_t);

}  // namespace ddmc
