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
// The FFTs run as register two-pass transforms n = n1 n2 (fft_reg.hpp) with
// one padded LDS exchange between the passes, with the lattice size a
// compile-time constant (2^a or 3 * 2^a) so that all index arithmetic is
// shifts, masks or multiplications by constants.
//
// Two spectrum buffers per plan, the same bytes as the spins each:
//   S^ (spin spectrum after the row pass), column-blocked
//        [R][3][L/2 / KC][ky][KC] so the column kernel reads contiguous tiles;
//   h^ (field spectrum after the column pass), row-blocked
//        [R][3][L / HB][L/2][HB]: HB consecutive rows ky interleaved, so that
//        a row block (a multiple of HB rows) reads contiguous memory and a
//        column tile writes whole runs of KC x HB elements (128 bytes at
//        L = 128 in FP32) instead of one KC-element piece per row;
// and the real kernel spectrum W^ [L/2 + 1][L][4] (xx, yy, xy, zz of a wave
// vector together), ky contiguous.
//
// A half-sweep of colour c is two launches:
//   k_cols : S^ -> forward y-FFT -> W^ multiply -> inverse y-FFT -> h^
//   k_rows : h^ -> inverse x-transform -> field of the block's RB rows ->
//            Metropolis update of their colour-c sites with the frozen field
//            (Sec. 3.2) -> forward x-transform of the updated rows -> S^,
//            the spectrum the next half-sweep starts from.
// The field itself never goes to HBM inside a sweep.  The 1/L^2 of the
// inverse transform is folded into W^.
//
// Bookkeeping rides in kernels that run anyway: the first row kernel of a
// call advances the device sweep counters; each row-update block stores its
// accepted-move count in a slot of its own, and the next column launch adds
// the slots of a replica to its total in one extra block.  When sampling, the
// state after sweep t-1 is summed while sweep t starts: the colour-0 row
// kernel sums every observable of its rows from the spins it holds in LDS
// and the field it has just inverted, before its update, and the extra block
// of the colour-1 column launch reduces the sums.  No atomics to global
// memory and no device-wide fences on the sweep path.
#include "fft_reg.hpp"
#include "obs_common.hpp"

namespace ddmc {

namespace {

constexpr int NT = 256;   // threads per block of every FFT kernel

// aligned to its size, so that a complex value moves as one 64-bit (FP32)
// or 128-bit (FP64) LDS or global access rather than two separate words
template <typename T> struct alignas(2 * sizeof(T)) cplx {
    T re, im;
};
template <typename T> __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.re, -a.im}; }
template <typename T> __device__ __forceinline__ cplx<T> mul_i(cplx<T> a) { return {-a.im, a.re}; }
template <typename T> __device__ __forceinline__ cplx<T> mul_mi(cplx<T> a) { return {a.im, -a.re}; }
template <typename T> __device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return {a.re * s, a.im * s}; }

// Stores of the spectra and spins a launch hands to the next one.  With
// `stream` set they carry the non-temporal hint, which lets them drain to
// memory while the kernel runs, where ordinary stores sit dirty in L2 until
// the write-back at the end of the kernel; the launch wrappers set it when a
// launch's output is small (STREAM_MAX_BYTES), where that write-back is a
// visible part of a short kernel.  On larger launches the partial cache lines
// these stores leave (32-byte pieces, single spins) are better merged in L2
// first.  Visibility to the next launch is the same either way.
constexpr size_t STREAM_MAX_BYTES = (size_t)8 << 20;
template <typename T> __device__ __forceinline__ void st_out(cplx<T> *p, cplx<T> v, int stream)
{
    if (stream) {
        typedef T v2 __attribute__((ext_vector_type(2)));
        v2 w;
        w.x = v.re;
        w.y = v.im;
        __builtin_nontemporal_store(w, reinterpret_cast<v2 *>(p));
    } else {
        *p = v;
    }
}
template <typename T> __device__ __forceinline__ void st_out(T *p, T v, int stream)
{
    if (stream) {
        __builtin_nontemporal_store(v, p);
    } else {
        *p = v;
    }
}

// ---- compile-time geometry of one lattice size (L = 2^a or 3 * 2^a)
constexpr int largest_divisor_upto(int n, int cap)
{
    int best = 1;
    for (int d = 1; d <= n && d <= cap; ++d)
        if (n % d == 0) best = d;
    return best;
}

template <int L> struct geom {
    static constexpr int H = L / 2;
    // rows per block of k_rows: 3 RB sequences of H points, about NT butterfly slots
    static constexpr int RB = largest_divisor_upto(L, (NT / H) < 1 ? 1 : NT / H);
};

// LDS bank layout.  The LDS has 64 banks of 4 bytes, and a 64-bit access of
// a wave is served in two halves of 32 lanes: 32 complex FP32 values (or 16
// complex FP64 values per quarter of a 128-bit access) at consecutive
// addresses meet no conflict, while lanes whose addresses differ by a
// multiple of 256 bytes collide.  A transform pass has runs of n2 (pass A) or
// n1 (pass B) consecutive lanes on consecutive elements of one sequence, the
// next run in the next sequence; sequences are therefore laid out with a
// stride that is an odd multiple of n2, so that the runs of one half wave
// fall into disjoint banks.
template <int n> constexpr int seq_stride()
{
    constexpr int n2 = fftreg::split<n>::n2;
    return (n2 >= 32 || (n / n2) % 2 == 1) ? n : n + n2;
}

// Register two-pass FFT (see fft_reg.hpp) of NSEQ sequences of length n
// stored with stride seq_stride<n>() in `a`; `b` is scratch of
// NSEQ * n1 * (n2 + 1) elements.  Pass A is done by threads (f, j2) =
// (e / n2, e % n2), e < NSEQ n2, pass B by threads (f, k1) = (e / n1, e % n1).
// A kernel that has a thread's pass-A inputs in registers already (loaded
// from HBM, or formed from other LDS data) calls fft_pass_a itself and skips
// one LDS round trip and one barrier.

// Pass A of thread (f, j2): the n1-point DFT of v[j1] = x_f[j1 n2 + j2], each
// output k1 > 0 scaled by w_n^{j2 k1} (w[k1] = the forward twiddle, conjugated
// here for the inverse), into b.
template <typename T, int n, bool INV>
__device__ __forceinline__ void fft_pass_a(fftreg::cx<T> (&v)[fftreg::split<n>::n1],
                                           const cplx<T> (&w)[fftreg::split<n>::n1], int f, int j2, cplx<T> *b)
{
    constexpr int n1 = fftreg::split<n>::n1, P = fftreg::split<n>::n2 + 1;
    fftreg::dft<T, n1, INV>(v);
#pragma unroll
    for (int k1 = 0; k1 < n1; ++k1) {
        const cplx<T> x{v[k1].re, v[k1].im};
        b[(f * n1 + k1) * P + j2] = (k1 == 0) ? x : cmul(x, INV ? cconj(w[k1]) : w[k1]);
    }
}

// Pass A twiddles of thread j2: w_n^{j2 k1} = tw[(j2 k1 L / n) mod L], k1 < n1
template <typename T, int n, int L>
__device__ __forceinline__ void fft_twiddles_a(cplx<T> (&w)[fftreg::split<n>::n1], int j2, const cplx<T> *tw)
{
#pragma unroll
    for (int k1 = 0; k1 < fftreg::split<n>::n1; ++k1) w[k1] = tw[(j2 * k1 * (L / n)) % L];
}

// Pass B: every thread (f, k1) takes the n2-point DFT of b[f][k1][.] into
// a[f][k1 + n1 k2].  Ends with a barrier.
template <typename T, int n, bool INV, int NSEQ>
__device__ __forceinline__ void fft_pass_b(cplx<T> *a, const cplx<T> *b)
{
    using fftreg::cx;
    constexpr int n1 = fftreg::split<n>::n1, n2 = fftreg::split<n>::n2, P = n2 + 1;
    constexpr int WB = NSEQ * n1, SA = seq_stride<n>();
    const int tid = threadIdx.x;
#pragma unroll
    for (int e0 = 0; e0 < WB; e0 += NT) {
        const int e = e0 + tid;
        if ((WB % NT) == 0 || e < WB) {
            const int f = e / n1, k1 = e % n1;
            cx<T> v[n2];
#pragma unroll
            for (int j2 = 0; j2 < n2; ++j2) {
                const cplx<T> x = b[(f * n1 + k1) * P + j2];
                v[j2] = cx<T>{x.re, x.im};
            }
            fftreg::dft<T, n2, INV>(v);
#pragma unroll
            for (int k2 = 0; k2 < n2; ++k2) a[f * SA + k1 + n1 * k2] = cplx<T>{v[k2].re, v[k2].im};
        }
    }
    __syncthreads();
}

// Both passes, inputs and twiddles from LDS.  The result replaces the input
// in `a`.
template <typename T, int n, int L, bool INV, int NSEQ>
__device__ __forceinline__ cplx<T> *fft_two_pass(cplx<T> *a, cplx<T> *b, const cplx<T> *tw)
{
    using fftreg::cx;
    constexpr int n1 = fftreg::split<n>::n1, n2 = fftreg::split<n>::n2;
    constexpr int WA = NSEQ * n2, SA = seq_stride<n>();
    const int tid = threadIdx.x;
#pragma unroll
    for (int e0 = 0; e0 < WA; e0 += NT) {
        const int e = e0 + tid;
        if ((WA % NT) == 0 || e < WA) {
            const int f = e / n2, j2 = e % n2;
            cx<T> v[n1];
#pragma unroll
            for (int j1 = 0; j1 < n1; ++j1) {
                const cplx<T> x = a[f * SA + j1 * n2 + j2];
                v[j1] = cx<T>{x.re, x.im};
            }
            cplx<T> w[n1];
            fft_twiddles_a<T, n, L>(w, j2, tw);
            fft_pass_a<T, n, INV>(v, w, f, j2, b);
        }
    }
    __syncthreads();
    fft_pass_b<T, n, INV, NSEQ>(a, b);
    return a;
}

// elements of an LDS buffer that holds NSEQ sequences of length n (with
// their stride) and can also serve as the scratch of their transform
template <int n, int NSEQ> constexpr int fft_buf()
{
    constexpr int seqs = NSEQ * seq_stride<n>();
    constexpr int scratch = NSEQ * fftreg::split<n>::n1 * (fftreg::split<n>::n2 + 1);
    return seqs > scratch ? seqs : scratch;
}

// Spin rows in LDS: per (row, component) a segment with the even sites at
// [0, H) and the odd sites at [PO, PO + H), so that the sites of one colour
// are contiguous (the sweep reads every second site), with PO = 32 modulo 64
// so that a wave storing 64 consecutive sites of a row meets no conflict.
// The segment stride SEG is an odd multiple of the row transform's n2, so
// that the forward pass A, whose runs of n2 lanes read one segment each,
// meets none either.
template <int L> struct srow_layout {
    static constexpr int H = L / 2;
    static constexpr int PO = H + ((32 - H % 64) + 64) % 64;
    static constexpr int N2 = fftreg::split<H>::n2;
    static constexpr int SEG0 = PO + H;
    static constexpr int SEG1 = (SEG0 + N2 - 1) / N2 * N2;
    static constexpr int SEG = (N2 >= 64 || (SEG1 / N2) % 2 == 1) ? SEG1 : SEG1 + N2;
    static __device__ __forceinline__ int at(int x) { return (x & 1) * PO + (x >> 1); }
};

struct w0_pack {
    double v[4];
};

// Index arithmetic with wave-uniform parts.  Element e = it * NT + 64 * wave
// + lane of a row-major array with rows of n elements lies in row e / n,
// column e % n; when n is a multiple of 64 the 64 lanes of a wave share the
// row, so that the row, and everything derived from it, is a scalar of the
// wave.  CNT is the element count (iterations past it are clamped to the last
// element for loads, and skipped by in_range).
struct rc_t {
    int row, col;
};
__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }
template <int n, int CNT> __device__ __forceinline__ rc_t elem_rc(int it, int wave, int lane)
{
    if constexpr (n % 64 == 0 && CNT % 64 == 0) {
        const int chunk = min(it * (NT / 64) + wave, CNT / 64 - 1);
        return rc_t{chunk / (n / 64), (chunk % (n / 64)) * 64 + lane};
    } else {
        const int e = min(it * NT + wave * 64 + lane, CNT - 1);
        return rc_t{e / n, e % n};
    }
}
template <int CNT> __device__ __forceinline__ bool in_range(int it, int wave, int lane)
{
    if constexpr (CNT % NT == 0) {
        return true;
    } else if constexpr (CNT % 64 == 0) {
        return it * (NT / 64) + wave < CNT / 64;
    } else {
        return it * NT + wave * 64 + lane < CNT;
    }
}

// (replica r, block b) of a one-dimensional grid of R * nb blocks.  The
// hardware deals consecutive workgroups round robin to the eight XCDs; when R
// is a multiple of 8 all blocks of a replica go to one XCD, so that the cache
// lines several of its blocks share (the 32-byte pieces of a spectrum tile,
// the halo rows of the spins) meet in one L2.  Measured on a copy with the
// column pass's access pattern at L = 128, R = 32: 3.2 us per launch with
// this mapping against 5.2 us without.  R is passed by the caller, so that
// no dependent load of the grid size precedes the kernel's first loads.
__device__ __forceinline__ void xcd_coords(int nb, int R, int &r, int &b)
{
    const unsigned w = blockIdx.x, ub = (unsigned)nb;
    if ((R & 7) == 0) {
        const unsigned k = w >> 3;
        r = (int)((w & 7u) + 8u * (k / ub));
        b = (int)(k % ub);
    } else {
        r = (int)(w / ub);
        b = (int)(w % ub);
    }
}

enum { ROWS_FWD = 0, ROWS_INV = 1, ROWS_SWEEP = 2, ROWS_OBS = 3, ROWS_COSET = 4, ROWS_SAMPLE = 5 };

// Side inputs and outputs of a row launch (all may be NULL).
struct rows_aux {
    unsigned long long *ctr;       // [R] device sweep counters; the sweep index is ctr[r] + sweep_off
    unsigned long long advance;    // ROWS_FWD: block 0 of replica r adds it to ctr[r]
    unsigned int *slots;           // ROWS_SWEEP, ROWS_SAMPLE, ROWS_COSET: [R][row blocks] accepted moves of each block
    double *obs_partial;           // ROWS_SAMPLE, ROWS_OBS: observable sums of the state the launch
                                   // starts from, [R][row blocks][NACC]
    double *eta_acc;               // ROWS_SAMPLE, ROWS_OBS: [R][N] cone-angle accumulators (may be NULL)
    int coset_l;                   // ROWS_COSET: the spacing l of the coset `color`
};

// Side work of a column launch: one extra block per replica, after the
// transform blocks, that folds the accept slots of the previous row launch
// and / or reduces the observable sums of a sample.
struct cols_aux {
    const unsigned int *slots;     // accepted[r] += sum of slots[r][0 .. nslot)
    int nslot;
    unsigned long long *accepted;
    const double *obs_partial;     // obs_out[r] = outputs of the sums obs_partial[r][0 .. nobs)
    int nobs;
    int have_eta;
    double *obs_out;               // [R][DDMC_NOBS]
};

template <typename T, int L, int KC> constexpr size_t cols_lds_bytes_kc()
{
    return sizeof(cplx<T>) * ((size_t)L + 2 * (size_t)fft_buf<L, 3 * KC>());
}

// Packed columns per block of k_cols (also the tile width of S^): up to
// L = 128 the largest divisor of L/2 up to 512/L; above, the widest of 4, 2,
// 1 columns whose transform buffers fit in 64 KB of LDS in this precision
// (an FP32 block keeps 4 columns, about 192 of its threads busy in each
// pass, where the FP64 one must take fewer).
template <typename T, int L> constexpr int col_tile()
{
    constexpr int H = geom<L>::H;
    if constexpr (512 / L >= 4) {
        return largest_divisor_upto(H, 512 / L);
    } else if constexpr (H % 4 == 0 && cols_lds_bytes_kc<T, L, 4>() <= 65536) {
        return 4;
    } else if constexpr (H % 2 == 0 && cols_lds_bytes_kc<T, L, 2>() <= 65536) {
        return 2;
    } else {
        return 1;
    }
}

// Offset of S^(c, ky, kx) in the column-blocked layout of one replica,
// ((c (H / KC) + kx / KC) L + ky) KC + kx % KC, as the sum of a part that
// depends on (c, ky) and one that depends on kx.
template <typename T, int L> __device__ __forceinline__ long sblk_row(int c, int ky)
{
    constexpr int H = geom<L>::H, KC = col_tile<T, L>();
    return ((long)c * (H / KC) * L + ky) * KC;
}
template <typename T, int L> __device__ __forceinline__ int sblk_col(int kx)
{
    constexpr int KC = col_tile<T, L>();
    return (kx / KC) * L * KC + kx % KC;
}

// Rows interleaved in the row-blocked layout of h^: the largest of 4, 2, 1
// that divides the rows of a row block.
template <int L> constexpr int hspec_rows()
{
    constexpr int RB = geom<L>::RB;
    return (RB % 4 == 0) ? 4 : (RB % 2 == 0) ? 2 : 1;
}
// Element e of the h^ rows of a row block (RB rows starting at a multiple of
// HB) in memory order: e = (g H + kx) HB + y is bin kx of row g HB + y, so
// that consecutive lanes read consecutive elements.  CNT = RB H; past it the
// element is clamped to the last one (for loads).
struct hb_elem {
    int row, col, off;   // row within the block, bin kx, offset from the block's first element
};
template <int L, int CNT> __device__ __forceinline__ hb_elem hspec_elem(int it, int tid)
{
    constexpr int H = geom<L>::H, HB = hspec_rows<L>();
    const int e = min(it * NT + tid, CNT - 1);
    const int y = e % HB, kx = (e / HB) % H, g = e / (HB * H);
    return hb_elem{g * HB + y, kx, e};
}
// offset of h^(c, ky, kx) in one replica: ((c (L / HB) + ky / HB) H + kx) HB + ky % HB
template <int L> __device__ __forceinline__ long hblk(int c, int ky, int kx)
{
    constexpr int H = geom<L>::H, HB = hspec_rows<L>();
    return (((long)c * (L / HB) + ky / HB) * H + kx) * HB + ky % HB;
}

template <typename T, int L> constexpr size_t rows_lds_bytes()
{
    constexpr int H = geom<L>::H, RB = geom<L>::RB;
    return sizeof(cplx<T>) * ((size_t)L + 2 * (size_t)fft_buf<H, 3 * RB>()) +
           sizeof(T) * (size_t)(RB + 2) * 3 * srow_layout<L>::SEG + sizeof(double) * (NT / 64) * OBS_NACC;
}

// Packed columns per block of k_cols: the tile width, or half a tile where
// an FP32 block of a whole 4-column tile needs more than 48 KB of LDS (L =
// 256: two such blocks per CU, five of half the width).  Then the two blocks
// of a tile, consecutive and so on one XCD, each read half of every 32-byte
// run of S^; the row kernels keep writing whole tiles.  (Measured: at L = 192
// half tiles were 3 % slower, at 384 and 512 single columns 13-26 %.)
template <typename T, int L> constexpr int col_block()
{
    constexpr int KS = col_tile<T, L>();
    if constexpr (sizeof(T) < sizeof(double) && KS >= 4 && KS % 2 == 0 && cols_lds_bytes_kc<T, L, KS>() > 49152)
        return KS / 2;
    else
        return KS;
}

template <typename T, int L> constexpr size_t cols_lds_bytes()
{
    return cols_lds_bytes_kc<T, L, col_block<T, L>()>();
}

// Rows kernel.  Block = RB consecutive rows of one replica.
//   ROWS_FWD  : s -> S^ rows
//   ROWS_INV  : h^ -> field h at the sites of `color` (all sites when color < 0)
//   ROWS_SWEEP: h^ -> field -> colour update of s -> S^ rows of the new state
//   ROWS_SAMPLE: ROWS_SWEEP (colour 0) that first sums every observable of s
//   ROWS_OBS  : h^ -> field -> observable sums of s
//   ROWS_COSET: ROWS_SWEEP for the sites of one coset of l Z^2
template <typename T, int L, int MODE>
__global__ void __launch_bounds__(NT)
k_rows(T *__restrict__ s, const cplx<T> *__restrict__ spec_in, const cplx<T> *__restrict__ tw, int nrep, int color,
       uint32_t sweep_off, cplx<T> *__restrict__ spec_out, T *__restrict__ h,
       const ddmc_replica_params *__restrict__ params, int stream, rows_aux aux, int write_spec, w0_pack w0)
{
    __shared__ unsigned int block_count;
    constexpr int H = geom<L>::H, RB = geom<L>::RB;
    constexpr int NSEQ = 3 * RB;
    constexpr long N = (long)L * L;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *tw_l = reinterpret_cast<cplx<T> *>(smem_raw);
    constexpr int SH = seq_stride<H>();                // sequence stride in bufA
    using SL_ = srow_layout<L>;
    constexpr int SEG = SL_::SEG;
    cplx<T> *bufA = tw_l + L;                          // transforms in place: [3 RB][SH]
    cplx<T> *bufB = bufA + fft_buf<H, NSEQ>();         // transform scratch
    T *srow = reinterpret_cast<T *>(bufB + fft_buf<H, NSEQ>());   // [RB + 2][3][SEG]; own row yl at index yl + 1
    double *red = reinterpret_cast<double *>(srow + (RB + 2) * 3 * SEG);   // [NT / 64][NACC] wave sums

    constexpr int NRB = L / RB;
    int r, rb;
    xcd_coords(NRB, nrep, r, rb);
    const int y0 = rb * RB;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = wave_index();
    T *sr = s + (long)r * 3 * N;
    constexpr bool UPDATE = (MODE == ROWS_SWEEP || MODE == ROWS_COSET || MODE == ROWS_SAMPLE);
    constexpr bool OBS = (MODE == ROWS_SAMPLE || MODE == ROWS_OBS);

    // ---- prologue: every global load of the block is issued into registers
    // before the first LDS store, so that all of them are in flight together;
    // their addresses need only the first line of the kernel arguments, and
    // the per-replica scalars (parameters, sweep counter) are read after them.
    // Spin rows: own rows, plus one halo row on each side for the sweep and
    // the observables.
    constexpr int HALO = (UPDATE || OBS) ? 1 : 0;
    constexpr int NROWS = RB + 2 * HALO;
    // Per component c (the outer, compile-time index of the loops below) the
    // spins are NROWS rows of L and the spectrum RB rows of H; iteration jt of
    // a component covers elements jt NT + tid of them.
    constexpr int SCNT = (MODE == ROWS_INV) ? 0 : NROWS * L;      // spins per component
    constexpr int SITC = (SCNT + NT - 1) / NT;
    constexpr int SIT = 3 * SITC;
    // spectrum rows X[k] with their mirror X[H - k] for the tangle
    constexpr int ZCNT = (MODE == ROWS_FWD) ? 0 : RB * H;         // spectrum elements per component
    constexpr int ZITC = (ZCNT + NT - 1) / NT;
    constexpr int ZIT = 3 * ZITC;
    constexpr int WIT = (L + NT - 1) / NT;
    T sv[SIT > 0 ? SIT : 1];
    cplx<T> xa[ZIT > 0 ? ZIT : 1], xb[ZIT > 0 ? ZIT : 1], wv[ZIT > 0 ? ZIT : 1], twv[WIT];
#pragma unroll
    for (int it = 0; it < WIT; ++it) twv[it] = tw[(it * NT + tid) % L];
    // (loads are unconditional, out-of-range threads reload the last element,
    // so that no branch separates them; only the LDS stores are guarded)
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
        const int c = it / SITC;
        const rc_t e = elem_rc<L, SCNT>(it % SITC, wave, lane);
        const int x = e.col, rl = e.row;
        int y = y0 - HALO + rl;
        y += (y < 0) ? L : 0;
        y -= (y >= L) ? L : 0;
        sv[it] = sr[(unsigned)c * (unsigned)N + (unsigned)y * (unsigned)L + (unsigned)x];
    }
    if constexpr (MODE != ROWS_FWD) {
        const cplx<T> *src = spec_in + (long)r * 3 * L * H;
#pragma unroll
        for (int it = 0; it < ZIT; ++it) {
            const int c = it / ZITC;
            const hb_elem e = hspec_elem<L, ZCNT>(it % ZITC, tid);
            const int k = e.col;
            constexpr int HB = hspec_rows<L>();
            const cplx<T> *blk = src + hblk<L>(c, y0, 0);   // the block's rows of component c
            xa[it] = blk[e.off];
            xb[it] = blk[e.off + HB * (((H - k) % H) - k)];
            wv[it] = tw[k];
        }
    }
    ddmc_replica_params p{};
    uint32_t sweep = 0;
    if constexpr (UPDATE || OBS) p = params[r];
    if constexpr (UPDATE) sweep = (uint32_t)(aux.ctr ? aux.ctr[r] : 0ull) + sweep_off;
    if (UPDATE && tid == 0) block_count = 0u;
    if (MODE == ROWS_FWD && aux.ctr && rb == 0 && tid == 0) aux.ctr[r] += aux.advance;
    // observables: thread e < RB H takes the horizontal pair (2j, 2j + 1) of
    // own row e / H, j = e % H; its two cone-angle accumulators
    constexpr int NPAIR = RB * H;
    static_assert(!OBS || NPAIR <= NT, "one pair per thread");
    double2 eta2 = {0.0, 0.0};
    if constexpr (OBS) {
        if (aux.eta_acc) {
            const rc_t e = elem_rc<H, NPAIR>(0, wave, lane);
            const unsigned i = (unsigned)(y0 + e.row) * (unsigned)L + 2u * (unsigned)e.col;
            eta2 = *reinterpret_cast<const double2 *>(aux.eta_acc + (long)r * N + i);
        }
    }
    // colour update: thread e < RB H takes site 2j + ((color + y) & 1) of own
    // row e / H, j = e % H.  Its draws depend only on the counter, so they
    // (and the uniform trial direction of a Heisenberg replica) are computed
    // here, while the loads above are in flight.
    constexpr bool COLOUR = (MODE == ROWS_SWEEP || MODE == ROWS_SAMPLE);
    static_assert(!COLOUR || RB * H <= NT, "one site per thread");
    vec3<T> trial_h{T(0), T(0), T(0)};
    T u_acc = T(0);
    if constexpr (COLOUR) {
        const rc_t e = elem_rc<H, RB * H>(0, wave, lane);
        const int y = y0 + e.row, x = 2 * e.col + ((color + y) & 1);
        const u32x4 d = draw(p.seed, p.replica_id, sweep, (uint32_t)(y * L + x), 1u);
        u_acc = to_unit<T>(d.v[2]);
        if (p.model != DDMC_ISING) trial_h = sphere_point<T>(to_unit<T>(d.v[0]), to_unit<T>(d.v[1]));
    }
#pragma unroll
    for (int it = 0; it < WIT; ++it) tw_l[(it * NT + tid) % L] = twv[it];   // L < NT: equal values
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
        if (in_range<SCNT>(it % SITC, wave, lane)) {
            const int c = it / SITC;
            const rc_t e = elem_rc<L, SCNT>(it % SITC, wave, lane);
            const int x = e.col, rl = e.row;
            srow[((rl + 1 - HALO) * 3 + c) * SEG + SL_::at(x)] = sv[it];
        }
    }
    if constexpr (MODE != ROWS_FWD) {
        // tangle: Z'[k] = (X[k] + conj X[H-k]) + i (X[k] - conj X[H-k]) e^{+2 pi i k / L}
#pragma unroll
        for (int it = 0; it < ZIT; ++it) {
            if (ZCNT % NT == 0 || (it % ZITC) * NT + tid < ZCNT) {
                const int c = it / ZITC;
                const hb_elem e = hspec_elem<L, ZCNT>(it % ZITC, tid);
                const int q = e.row * 3 + c;   // sequence of (row, component)
                // both forms are computed and one selected, so that the mirror
                // and twiddle loads stay unconditional
                const cplx<T> X = xa[it];
                const cplx<T> Xc = cconj(xb[it]);
                const cplx<T> O = cmul(csub(X, Xc), cconj(wv[it]));
                const cplx<T> Zg = cadd(cadd(X, Xc), mul_i(O));
                const bool dc = e.col == 0;   // bin 0 carries X0 + i X_{L/2}
                bufA[q * SH + e.col] = cplx<T>{dc ? X.re + X.im : Zg.re, dc ? X.re - X.im : Zg.im};
            }
        }
    }
    __syncthreads();

    cplx<T> *zres = nullptr;   // inverse result: z[n] = h(2n) + i h(2n+1) per (row, comp)
    if constexpr (MODE != ROWS_FWD) {
        zres = fft_two_pass<T, H, L, true, NSEQ>(bufA, bufB, tw_l);
    }

    if constexpr (MODE == ROWS_INV) {
        T *hr = h + (long)r * 3 * N;
        const int per_row = (color < 0) ? L : H;
        for (int e = tid; e < RB * 3 * per_row; e += NT) {
            const int j = e % per_row, q = e / per_row;
            const int yl = q / 3, c = q - yl * 3;
            const int y = y0 + yl;
            const int x = (color < 0) ? j : 2 * j + ((color + y) & 1);
            const cplx<T> z = zres[q * SH + (x >> 1)];
            hr[(long)c * N + (long)y * L + x] = (x & 1) ? z.im : z.re;
        }
        return;
    }

    // ---- observables of the staged state (before this launch's update) over
    // the block's rows.  Per pair: the per-site terms and g/2 s.h of both
    // sites, and the four bonds of its colour-0 member.  The neighbours of a
    // colour-0 site are colour-1 sites, which no block of a colour-0 launch
    // changes, so the halo values read here are those of the staged state
    // whatever the order of the blocks; and every bond of the lattice has
    // exactly one colour-0 end, so each is counted once.  The colour-0 site
    // of a pair is updated below by the same thread, after these reads.
    if constexpr (OBS) {
        // per-pair terms and their wave totals in the path's precision (for
        // FP32: a wave sums 128 sites, about 1e-7 relative), the wave totals
        // in FP64 from there on
        using A = T;
        A a[obs::NACC];
#pragma unroll
        for (int k = 0; k < obs::NACC; ++k) a[k] = A(0);
        if (tid < NPAIR) {
            const rc_t e = elem_rc<H, NPAIR>(0, wave, lane);
            const int yl = e.row, j = e.col, y = y0 + yl;
            const T *row = srow + (yl + 1) * 3 * SEG;
            const T *up = srow + (yl + 2) * 3 * SEG;   // y + 1
            const T *dn = srow + yl * 3 * SEG;         // y - 1
            const int x0 = 2 * j + (y & 1);            // colour-0 member
            const int i0 = SL_::at(x0), i1 = SL_::at(x0 ^ 1);
            const int il = SL_::at((x0 + L - 1) % L), ir = SL_::at((x0 + 1) % L);
            T s0[3], s1[3], nl[3], nr[3], nu[3], nd[3], h0[3], h1[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                s0[c] = row[c * SEG + i0];
                s1[c] = row[c * SEG + i1];
                nl[c] = row[c * SEG + il];
                nr[c] = row[c * SEG + ir];
                nu[c] = up[c * SEG + i0];
                nd[c] = dn[c * SEG + i0];
                const cplx<T> z = zres[(yl * 3 + c) * SH + j];   // h(2j) + i h(2j + 1)
                h0[c] = (y & 1) ? z.im : z.re;
                h1[c] = (y & 1) ? z.re : z.im;
            }
            T bond = T(0);
            int wh[3], wv[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                bond += s0[c] * ((nl[c] + nr[c]) + (nu[c] + nd[c]));
                wh[c] = obs::wall(s0[c], nl[c]) + obs::wall(s0[c], nr[c]);
                wv[c] = obs::wall(s0[c], nu[c]) + obs::wall(s0[c], nd[c]);
            }
            a[0] = -(A)p.J * (A)bond;
            A dot = A(0);
#pragma unroll
            for (int c = 0; c < 3; ++c) dot += (A)s0[c] * (A)h0[c] + (A)s1[c] * (A)h1[c];
            a[1] = (A)(0.5 * p.g) * dot;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                a[6 + c] = (A)wh[c];
                a[9 + c] = (A)wv[c];
            }
            const bool have_acc = aux.eta_acc != nullptr;
            const A sy = (y & 1) ? A(-1) : A(1);
            // the pair's sites in x order carry eta2.x and eta2.y
            double acc0 = (y & 1) ? eta2.y : eta2.x, acc1 = (y & 1) ? eta2.x : eta2.y;
            obs::site_terms<T, A>(a, s0, p, have_acc, acc0, sy, (x0 & 1) ? A(-1) : A(1));
            obs::site_terms<T, A>(a, s1, p, have_acc, acc1, sy, (x0 & 1) ? A(1) : A(-1));
            if (have_acc) {
                const unsigned i = (unsigned)y * (unsigned)L + 2u * (unsigned)j;
                *reinterpret_cast<double2 *>(aux.eta_acc + (long)r * N + i) =
                    (y & 1) ? double2{acc1, acc0} : double2{acc0, acc1};
            }
        }
        const A v = obs::wave_sum16(a);
        if ((tid & 3) == 0) red[(tid >> 6) * obs::NACC + ((tid & 63) >> 2)] = (double)v;
        static_assert(obs::NACC == 18, "two accumulators beyond the 16 of wave_sum16");
        const A v16 = obs::wave_sum(a[16]);
        // the non-finite count of a thread is 0, 1 or 2: two ballots count it
        const int v17 = __popcll(__ballot(a[17] > A(0.5))) + __popcll(__ballot(a[17] > A(1.5)));
        if ((tid & 63) == 0) {
            red[(tid >> 6) * obs::NACC + 16] = (double)v16;
            red[(tid >> 6) * obs::NACC + 17] = (double)v17;
        }
        if constexpr (MODE == ROWS_OBS) {
            __syncthreads();
            if (tid < obs::NACC) {
                double u = 0.0;
#pragma unroll
                for (int w = 0; w < NT / 64; ++w) u += red[w * obs::NACC + tid];
                aux.obs_partial[((long)r * NRB + rb) * obs::NACC + tid] = u;
            }
            return;
        }
    }

    if constexpr (UPDATE) {
        site_consts<T> cst;
        cst.J = (T)p.J; cst.K2 = (T)p.K2; cst.K4 = (T)p.K4; cst.g = (T)p.g; cst.T_ = (T)p.T;
        cst.w0xx = (T)w0.v[0]; cst.w0yy = (T)w0.v[1]; cst.w0xy = (T)w0.v[2]; cst.w0zz = (T)w0.v[3];
        // Metropolis at site (y0 + yl, x) with the frozen field; the sites updated
        // by one launch are never neighbours, so no other thread reads the entry
        // written here
        // trial_h: the uniform direction (Heisenberg), u: the acceptance uniform
        auto try_site = [&](int yl, int x, vec3<T> trial_h, T u) -> bool {
            const int y = y0 + yl;
            const long i = (long)y * L + x;
            T *row = srow + (yl + 1) * 3 * SEG;
            const T *up = srow + (yl + 2) * 3 * SEG;    // y + 1
            const T *dn = srow + yl * 3 * SEG;          // y - 1
            const int ix = SL_::at(x), xp = SL_::at((x + 1) % L), xm = SL_::at((x + L - 1) % L);
            vec3<T> nb;
            nb.x = row[xp] + row[xm] + up[ix] + dn[ix];
            nb.y = row[SEG + xp] + row[SEG + xm] + up[SEG + ix] + dn[SEG + ix];
            nb.z = row[2 * SEG + xp] + row[2 * SEG + xm] + up[2 * SEG + ix] + dn[2 * SEG + ix];
            const vec3<T> so = {row[ix], row[SEG + ix], row[2 * SEG + ix]};
            const int j = x >> 1;
            const cplx<T> zx = zres[(yl * 3 + 0) * SH + j];
            const cplx<T> zy = zres[(yl * 3 + 1) * SH + j];
            const cplx<T> zz = zres[(yl * 3 + 2) * SH + j];
            const bool odd = x & 1;
            const vec3<T> hv = {odd ? zx.im : zx.re, odd ? zy.im : zy.re, odd ? zz.im : zz.re};
            const vec3<T> S = (p.model == DDMC_ISING) ? vec3<T>{-so.x, -so.y, -so.z} : trial_h;
            const T dE = energy_change<T>(cst, so, S, nb, hv);
            const bool acc = metropolis(dE, cst.T_, u);
            if (acc) {
                row[ix] = S.x;
                row[SEG + ix] = S.y;
                row[2 * SEG + ix] = S.z;
                st_out(sr + i, S.x, stream);
                st_out(sr + N + i, S.y, stream);
                st_out(sr + 2 * N + i, S.z, stream);
            }
            return acc;
        };
        auto count = [&](bool acc) {
            if (aux.slots) {
                const unsigned long long mask = __ballot(acc);
                if ((tid & (warpSize - 1)) == 0 && mask != 0ull)
                    atomicAdd(&block_count, (unsigned int)__popcll(mask));
            }
        };
        if constexpr (COLOUR) {
            // colour `color`: column 2j + ((color + y) & 1) of every own row
            bool acc = false;
            if (tid < RB * H) {
                const rc_t e = elem_rc<H, RB * H>(0, wave, lane);
                const int yl = e.row, j = e.col;
                acc = try_site(yl, 2 * j + ((color + y0 + yl) & 1), trial_h, u_acc);
            }
            count(acc);
        } else {
            // coset k = color = cy l + cx of l Z^2: columns cx + l j of the own rows with y = cy mod l
            const int l = aux.coset_l, cx = color % l, cy = color / l, per = L / l;
            const int nsite = RB * per;
            for (int e0 = 0; e0 < nsite; e0 += NT) {
                const int e = e0 + tid;
                bool acc = false;
                if (e < nsite) {
                    const int yl = e / per;
                    if ((y0 + yl) % l == cy) {
                        const int x = cx + l * (e - yl * per);
                        const u32x4 d = draw(p.seed, p.replica_id, sweep, (uint32_t)((y0 + yl) * L + x), 1u);
                        const vec3<T> th = (p.model == DDMC_ISING)
                                               ? vec3<T>{T(0), T(0), T(0)}
                                               : sphere_point<T>(to_unit<T>(d.v[0]), to_unit<T>(d.v[1]));
                        acc = try_site(yl, x, th, to_unit<T>(d.v[2]));
                    }
                }
                count(acc);
            }
        }
        __syncthreads();
        if (aux.slots && tid == 0) aux.slots[(long)r * NRB + rb] = block_count;
        if constexpr (MODE == ROWS_SAMPLE) {
            // the wave sums of the observables pass, written before the barrier above
            if (tid < obs::NACC) {
                double u = 0.0;
#pragma unroll
                for (int w = 0; w < NT / 64; ++w) u += red[w * obs::NACC + tid];
                aux.obs_partial[((long)r * NRB + rb) * obs::NACC + tid] = u;
            }
        }
        if (!write_spec) return;
    }

    // forward pass A straight from the spin rows: z[n] = s(2n) + i s(2n+1),
    // n = j1 N2 + j2, for thread (f, j2) = (e / N2, e % N2), sequence
    // f = row_local * 3 + comp (the rows are final: a barrier precedes this)
    {
        constexpr int N1 = fftreg::split<H>::n1, N2 = fftreg::split<H>::n2, WA = NSEQ * N2;
        static_assert(WA <= NT, "one pass-A item per thread");
        if (tid < WA) {
            const int fa = tid / N2, j2a = tid % N2;
            const int yl = fa / 3, c = fa - yl * 3;
            const T *row = srow + ((yl + 1) * 3 + c) * SEG;
            fftreg::cx<T> v[N1];
#pragma unroll
            for (int j1 = 0; j1 < N1; ++j1) {
                const int n = j1 * N2 + j2a;
                v[j1] = fftreg::cx<T>{row[n], row[SL_::PO + n]};
            }
            cplx<T> w[N1];
            fft_twiddles_a<T, H, L>(w, j2a, tw_l);
            fft_pass_a<T, H, false>(v, w, fa, j2a, bufB);
        }
    }
    __syncthreads();
    fft_pass_b<T, H, false, NSEQ>(bufA, bufB);
    const cplx<T> *Z = bufA;
    // untangle: X[k] = E + w^k O, E = (Z[k] + conj Z[H-k])/2, O = -i (Z[k] - conj Z[H-k])/2
    cplx<T> *dst = spec_out + (long)r * 3 * L * H;
    constexpr int UITC = (RB * H + NT - 1) / NT;   // iterations per component
#pragma unroll
    for (int it = 0; it < 3 * UITC; ++it) {
        if (in_range<RB * H>(it % UITC, wave, lane)) {
            const int c = it / UITC;
            const rc_t e = elem_rc<H, RB * H>(it % UITC, wave, lane);
            const int k = e.col, yl = e.row, q = yl * 3 + c;
            const cplx<T> Zk = Z[q * SH + k];
            cplx<T> X;
            if (k == 0) {
                X.re = Zk.re + Zk.im;   // X[0]
                X.im = Zk.re - Zk.im;   // X[L/2]
            } else {
                const cplx<T> Zc = cconj(Z[q * SH + (H - k)]);
                const cplx<T> v = cadd(cadd(Zk, Zc), cmul(tw_l[k], mul_mi(csub(Zk, Zc))));
                X = cscale(v, T(0.5));
            }
            st_out(dst + sblk_row<T, L>(c, y0 + yl) + sblk_col<T, L>(k), X, stream);
        }
    }
}

// Columns kernel: block = KC packed columns of one replica, all 3 components.
// Side work runs in one extra block per replica (tile index H / KC).
template <typename T, int L>
__global__ void __launch_bounds__(NT)
k_cols(const cplx<T> *__restrict__ spec_in, const T *__restrict__ what, const cplx<T> *__restrict__ tw, int nrep,
       int side, cplx<T> *__restrict__ spec_out, int aux_stream, cols_aux aux)
{
    constexpr int H = geom<L>::H, KC = col_block<T, L>(), KS = col_tile<T, L>();
    constexpr int NSEQ = 3 * KC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int r, kb;                             // replica, column tile (or extra block when side != 0)
    xcd_coords(H / KC + side, nrep, r, kb);
    const int tid = threadIdx.x;
    if (kb >= H / KC) {
        if (aux.slots && aux.accepted) obs::fold_slots(aux.slots + (long)r * aux.nslot, aux.nslot, aux.accepted + r);
        if (aux.obs_partial) {
            double *tot = reinterpret_cast<double *>(smem_raw);
            obs::partial_sum<NT / 64>(aux.obs_partial + (long)r * aux.nobs * obs::NACC, aux.nobs, tot);
            if (tid == 0) obs::finish(L, tot, true, aux.have_eta != 0, aux.obs_out + (long)r * DDMC_NOBS);
        }
        return;
    }
    cplx<T> *tw_l = reinterpret_cast<cplx<T> *>(smem_raw);
    constexpr int SL = seq_stride<L>();                 // sequence stride in bufA and bufB
    cplx<T> *bufA = tw_l + L;                           // [3 KC][SL]
    cplx<T> *bufB = bufA + fft_buf<L, NSEQ>();
    const int kx0 = kb * KC;
    // ---- prologue: twiddles, kernel multipliers and the spectrum tile are
    // all loaded into registers before the first LDS store
    constexpr int WIT = (L + NT - 1) / NT;
    cplx<T> twv[WIT];
#pragma unroll
    for (int it = 0; it < WIT; ++it) twv[it] = tw[(it * NT + tid) % L];
    constexpr int NITEM = (KC * L + NT - 1) / NT;
    vec4a<T> wk[NITEM], wn[NITEM];   // (xx, yy, xy, zz) at kx, and at L/2 for the packed column
    // (loads are unconditional, out-of-range threads reload the last element)
    const vec4a<T> *what4 = reinterpret_cast<const vec4a<T> *>(what);
#pragma unroll
    for (int it = 0; it < NITEM; ++it) {
        const int e = min(it * NT + tid, KC * L - 1);
        const int ky = e % L, j = e / L;
        const unsigned o = (unsigned)(kx0 + j) * L + ky;   // consecutive threads: consecutive ky
        wk[it] = what4[o];
        // the packed column also needs the multipliers at kx = L/2
        wn[it] = what4[(kx0 + j == 0) ? (unsigned)H * L + ky : o];
    }
    // Forward pass A runs from registers: thread e < WA is (f, j2) = (e / N2,
    // e % N2), sequence f = c KC + j (column kx0 + j of component c), and
    // loads its elements ky = j1 N2 + j2 of the tile [ky][KS] of component c
    // (the 64 lanes of a wave read consecutive elements) and its twiddles.
    constexpr int N1 = fftreg::split<L>::n1, N2 = fftreg::split<L>::n2, WA = NSEQ * N2;
    static_assert(WA <= NT, "one pass-A item per thread");
    const int ea = min(tid, WA - 1), fa = ea / N2, j2a = ea % N2;
    const cplx<T> *src = spec_in + (long)r * 3 * L * H;
    cplx<T> twa[N1], ga[N1];
    fft_twiddles_a<T, L, L>(twa, j2a, tw);
    {
        const int c = fa / KC, j = fa % KC;
        // column kx0 + j in the tile layout of S^ (tiles of KS columns; a
        // block of half a tile reads the half it owns)
        const unsigned tile = KC == KS ? (unsigned)kb : (unsigned)(kx0 + j) / KS;
        const unsigned jj = KC == KS ? (unsigned)j : (unsigned)(kx0 + j) % KS;
#pragma unroll
        for (int j1 = 0; j1 < N1; ++j1)
            ga[j1] = src[(((unsigned)c * (H / KS) + tile) * L + (unsigned)(j1 * N2 + j2a)) * KS + jj];
    }
    if (tid < WA) {
        fftreg::cx<T> v[N1];
#pragma unroll
        for (int j1 = 0; j1 < N1; ++j1) v[j1] = fftreg::cx<T>{ga[j1].re, ga[j1].im};
        fft_pass_a<T, L, false>(v, twa, fa, j2a, bufB);
    }
    // the twiddle table for the inverse passes, stored only now: a store
    // ahead of the pass above would make the tile loads wait for the
    // twiddle load
#pragma unroll
    for (int it = 0; it < WIT; ++it) tw_l[(it * NT + tid) % L] = twv[it];   // L < NT: equal values
    __syncthreads();
    fft_pass_b<T, L, false, NSEQ>(bufA, bufB);
    const cplx<T> *F = bufA;
    cplx<T> *G = bufB;
#pragma unroll
    for (int it = 0; it < NITEM; ++it) {
        const int e = it * NT + tid;
        if (e < KC * L) {
            const int ky = e % L, j = e / L;
            const int kx = kx0 + j;
            if (kx != 0) {
                const cplx<T> vx = F[(0 * KC + j) * SL + ky];
                const cplx<T> vy = F[(1 * KC + j) * SL + ky];
                const cplx<T> vz = F[(2 * KC + j) * SL + ky];
                const T wxx = wk[it].a, wyy = wk[it].b, wxy = wk[it].c, wzz = wk[it].d;
                G[(0 * KC + j) * SL + ky] = {wxx * vx.re + wxy * vy.re, wxx * vx.im + wxy * vy.im};
                G[(1 * KC + j) * SL + ky] = {wxy * vx.re + wyy * vy.re, wxy * vx.im + wyy * vy.im};
                G[(2 * KC + j) * SL + ky] = {wzz * vz.re, wzz * vz.im};
            } else {
                // packed column: C = A + i B, A and B the spectra of the real
                // columns kx = 0 and kx = L/2; separate, multiply, repack
                const int km = (L - ky) % L;
                cplx<T> A[3], B[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const cplx<T> C = F[(c * KC + j) * SL + ky];
                    const cplx<T> Cm = cconj(F[(c * KC + j) * SL + km]);
                    const cplx<T> sm = cadd(C, Cm), df = csub(C, Cm);
                    A[c] = cscale(sm, T(0.5));
                    B[c] = {T(0.5) * df.im, -T(0.5) * df.re};   // df / (2i)
                }
                const T axx = wk[it].a, ayy = wk[it].b, axy = wk[it].c, azz = wk[it].d;
                const T bxx = wn[it].a, byy = wn[it].b, bxy = wn[it].c, bzz = wn[it].d;
                const cplx<T> a0 = {axx * A[0].re + axy * A[1].re, axx * A[0].im + axy * A[1].im};
                const cplx<T> a1 = {axy * A[0].re + ayy * A[1].re, axy * A[0].im + ayy * A[1].im};
                const cplx<T> a2 = {azz * A[2].re, azz * A[2].im};
                const cplx<T> b0 = {bxx * B[0].re + bxy * B[1].re, bxx * B[0].im + bxy * B[1].im};
                const cplx<T> b1 = {bxy * B[0].re + byy * B[1].re, bxy * B[0].im + byy * B[1].im};
                const cplx<T> b2 = {bzz * B[2].re, bzz * B[2].im};
                G[(0 * KC + j) * SL + ky] = cadd(a0, mul_i(b0));
                G[(1 * KC + j) * SL + ky] = cadd(a1, mul_i(b1));
                G[(2 * KC + j) * SL + ky] = cadd(a2, mul_i(b2));
            }
        }
    }
    __syncthreads();
    const cplx<T> *Hc = fft_two_pass<T, L, L, true, NSEQ>(G, bufA, tw_l);
    cplx<T> *dst = spec_out + (long)r * 3 * L * H;
    // thread e writes element (c, ky = HB g + y, kx0 + j) of the tile, with
    // e = ((c (L / HB) + g) KC + j) HB + y: KC HB consecutive elements of h^
    // per (c, g)
    constexpr int HB = hspec_rows<L>();
#pragma unroll
    for (int e0 = 0; e0 < NSEQ * L; e0 += NT) {
        const int e = e0 + tid;
        if (e < NSEQ * L) {
            const int y = e % HB, j = (e / HB) % KC, cg = e / (HB * KC);   // cg = c (L / HB) + g
            const int c = cg / (L / HB), ky = (cg % (L / HB)) * HB + y;
            st_out(dst + ((long)cg * H + kx0 + j) * HB + y, Hc[(c * KC + j) * SL + ky], aux_stream);
        }
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

// y-pass: What[c][kx][ky] = Re sum_y Tx[c][y][kx] e^{-2 pi i ky y / L}, scaled
// by 1/L^2; stored as [kx][ky][c] (ky consecutive, the order the column
// kernel reads, and the four planes of a wave vector in one vector load)
template <typename T>
__global__ void k_what_y(int L, const double *__restrict__ tx, T *__restrict__ what)
{
    const int H1 = L / 2 + 1;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 4L * L * H1) return;
    const int ky = (int)(e % L);
    const long q = e / L;            // c * H1 + kx
    const int c = (int)(q / H1), kx = (int)(q % H1);
    double re = 0.0;
    for (int y = 0; y < L; ++y) {
        const long m = ((long)ky * y) % L;
        double sn, cs;
        sincospi(2.0 * (double)m / (double)L, &sn, &cs);
        const long o = ((long)c * L + y) * H1 + kx;
        re += tx[2 * o] * cs + tx[2 * o + 1] * sn;   // Re[(a + ib)(cs - i sn)]
    }
    what[((long)kx * L + ky) * 4 + c] = (T)(re / ((double)L * (double)L));
}

w0_pack w0_of(const ddmc_plan *p)
{
    w0_pack a;
    for (int k = 0; k < 4; ++k) a.v[k] = p->W0[k];
    return a;
}

template <typename T> cplx<T> *spec_a(ddmc_plan *p) { return reinterpret_cast<cplx<T> *>(p->spec_ws); }
template <typename T> cplx<T> *spec_b(ddmc_plan *p)
{
    return reinterpret_cast<cplx<T> *>(p->spec_ws) + (size_t)p->R_max * 3 * p->L * (p->L / 2);
}

// ---- launchers for one compile-time lattice size
template <typename T, int L> struct fft_impl {
    static constexpr int NRB = L / geom<L>::RB;   // row blocks per replica
    // streaming stores when the spectrum a launch writes is small
    static bool stream_out(int R) { return (size_t)R * 3 * L * (L / 2) * sizeof(cplx<T>) <= STREAM_MAX_BYTES; }
    static bool lds_ok() { return rows_lds_bytes<T, L>() <= 65536 && cols_lds_bytes<T, L>() <= 65536; }

    template <int MODE>
    static hipError_t rows(const ddmc_plan *p, int R, T *s, const cplx<T> *in, cplx<T> *out, T *h, int color,
                           uint32_t sweep_off, const ddmc_replica_params *params, const rows_aux &aux, int write_spec,
                           hipStream_t st)
    {
        dim3 grid(NRB * R);
        const int kid = (MODE == ROWS_SWEEP || MODE == ROWS_COSET) ? DDMC_KERNEL_FFT_ROWS_SWEEP
                        : MODE == ROWS_SAMPLE                       ? DDMC_KERNEL_FFT_ROWS_SAMPLE
                        : MODE == ROWS_OBS                          ? DDMC_KERNEL_OBSERVABLES
                                                                    : DDMC_KERNEL_FFT_ROWS;
        prof_scope ps(p, kid, st);
        hipLaunchKernelGGL((k_rows<T, L, MODE>), grid, dim3(NT), (rows_lds_bytes<T, L>()), st, s, in,
                           reinterpret_cast<const cplx<T> *>(p->twiddle), R, color, sweep_off, out, h, params,
                           stream_out(R) ? 1 : 0, aux, write_spec, w0_of(p));
        return hipGetLastError();
    }

    static hipError_t cols(const ddmc_plan *p, int R, const cplx<T> *in, cplx<T> *out, const cols_aux &aux,
                           hipStream_t st)
    {
        const bool side = (aux.slots && aux.accepted) || aux.obs_partial;
        dim3 grid(((L / 2) / col_block<T, L>() + (side ? 1 : 0)) * R);
        prof_scope ps(p, DDMC_KERNEL_FFT_COLUMNS, st);
        hipLaunchKernelGGL((k_cols<T, L>), grid, dim3(NT), (cols_lds_bytes<T, L>()), st, in,
                           reinterpret_cast<const T *>(p->what), reinterpret_cast<const cplx<T> *>(p->twiddle), R,
                           side ? 1 : 0, out, stream_out(R) ? 1 : 0, aux);
        return hipGetLastError();
    }

    static hipError_t field(ddmc_plan *p, int R, const T *s, T *h, int color, hipStream_t st)
    {
        cplx<T> *A = spec_a<T>(p), *B = spec_b<T>(p);
        const rows_aux none{};
        hipError_t e = rows<ROWS_FWD>(p, R, const_cast<T *>(s), nullptr, A, nullptr, -1, 0, nullptr, none, 1, st);
        if (e == hipSuccess) e = cols(p, R, A, B, cols_aux{}, st);
        if (e == hipSuccess)
            e = rows<ROWS_INV>(p, R, const_cast<T *>(s), B, nullptr, h, color, 0, nullptr, none, 0, st);
        return e;
    }

    // nsweeps sweeps of the l-coset schedule: cosets k = cy l + cx in order
    static hipError_t sweep_coset(ddmc_plan *p, int R, const ddmc_replica_params *params, T *s, int l,
                                  uint64_t *sweep_ctr, int nsweeps, uint64_t *accepted, hipStream_t st)
    {
        cplx<T> *A = spec_a<T>(p), *B = spec_b<T>(p);
        auto *ctr = reinterpret_cast<unsigned long long *>(sweep_ctr);
        auto *acc = reinterpret_cast<unsigned long long *>(accepted);
        unsigned int *slots = accepted ? p->slot_ws : nullptr;
        const uint32_t base = (uint32_t)(0u - (uint32_t)nsweeps);
        rows_aux fwd{};
        fwd.ctr = ctr;
        fwd.advance = (unsigned long long)nsweeps;
        hipError_t e = rows<ROWS_FWD>(p, R, s, nullptr, A, nullptr, -1, 0, nullptr, fwd, 1, st);
        bool slots_pending = false;
        const int ncos = l * l;
        for (int t = 0; t < nsweeps && e == hipSuccess; ++t) {
            for (int k = 0; k < ncos && e == hipSuccess; ++k) {
                cols_aux ca{};
                if (slots_pending) {
                    ca.slots = slots;
                    ca.nslot = NRB;
                    ca.accepted = acc;
                }
                e = cols(p, R, A, B, ca, st);
                if (e != hipSuccess) break;
                rows_aux ra{};
                ra.ctr = ctr;
                ra.slots = slots;
                ra.coset_l = l;
                const bool last = (t == nsweeps - 1) && k == ncos - 1;
                e = rows<ROWS_COSET>(p, R, s, B, A, nullptr, k, base + (uint32_t)t, params, ra, last ? 0 : 1, st);
                slots_pending = slots != nullptr;
            }
        }
        if (e == hipSuccess && slots_pending) e = launch_obs_final(p, R, 0, nullptr, 0, 0, nullptr, slots, NRB, accepted, st);
        return e;
    }

    // nsweeps sweeps; with obs, one observables sample after each sweep
    // (obs[t][r][DDMC_NOBS], eta_acc advanced once per sample).
    static hipError_t sweep(ddmc_plan *p, int R, const ddmc_replica_params *params, T *s, uint64_t *sweep_ctr,
                            uint64_t sweep0, int nsweeps, uint64_t *accepted, double *obs, double *eta_acc,
                            hipStream_t st)
    {
        cplx<T> *A = spec_a<T>(p), *B = spec_b<T>(p);
        auto *ctr = reinterpret_cast<unsigned long long *>(sweep_ctr);
        auto *acc = reinterpret_cast<unsigned long long *>(accepted);
        unsigned int *slots = accepted ? p->slot_ws : nullptr;
        double *part = p->rows_obs_ws;
        const long obs_stride = (long)R * DDMC_NOBS;
        // sweep index of sweep t: ctr[r] (already advanced by nsweeps) - nsweeps + t, or sweep0 + t
        const uint32_t base = ctr ? (uint32_t)(0u - (uint32_t)nsweeps) : (uint32_t)sweep0;
        rows_aux fwd{};
        fwd.ctr = ctr;
        fwd.advance = (unsigned long long)nsweeps;
        hipError_t e = rows<ROWS_FWD>(p, R, s, nullptr, A, nullptr, -1, 0, nullptr, fwd, 1, st);
        bool slots_pending = false, obs_pending = false;
        for (int t = 0; t < nsweeps && e == hipSuccess; ++t) {
            for (int color = 0; color < 2 && e == hipSuccess; ++color) {
                cols_aux ca{};
                if (slots_pending) {
                    ca.slots = slots;
                    ca.nslot = NRB;
                    ca.accepted = acc;
                }
                if (obs_pending) {   // sums of the state after sweep t-1, made by rows (t, colour 0)
                    ca.obs_partial = part;
                    ca.nobs = NRB;
                    ca.have_eta = eta_acc != nullptr;
                    ca.obs_out = obs + (t - 1) * obs_stride;
                }
                e = cols(p, R, A, B, ca, st);
                if (e != hipSuccess) break;
                rows_aux ra{};
                ra.ctr = ctr;
                ra.slots = slots;
                const bool sample = obs && color == 0 && t > 0;
                const bool last = (t == nsweeps - 1) && color == 1;
                if (sample) {
                    ra.obs_partial = part;
                    ra.eta_acc = eta_acc;
                    e = rows<ROWS_SAMPLE>(p, R, s, B, A, nullptr, color, base + (uint32_t)t, params, ra, 1, st);
                } else {
                    e = rows<ROWS_SWEEP>(p, R, s, B, A, nullptr, color, base + (uint32_t)t, params, ra,
                                         (last && !obs) ? 0 : 1, st);
                }
                slots_pending = slots != nullptr;
                obs_pending = sample;
            }
        }
        if (e != hipSuccess) return e;
        if (obs) {   // sample of the final state: field, sums, reduction
            cols_aux ca{};
            if (slots_pending) {
                ca.slots = slots;
                ca.nslot = NRB;
                ca.accepted = acc;
            }
            e = cols(p, R, A, B, ca, st);
            rows_aux ra{};
            ra.obs_partial = part;
            ra.eta_acc = eta_acc;
            if (e == hipSuccess) e = rows<ROWS_OBS>(p, R, s, B, nullptr, nullptr, -1, 0, params, ra, 0, st);
            if (e == hipSuccess)
                e = launch_obs_final(p, R, NRB, part, 1, eta_acc != nullptr, obs + (nsweeps - 1) * obs_stride,
                                     nullptr, 0, nullptr, st);
        } else if (slots_pending) {
            e = launch_obs_final(p, R, 0, nullptr, 0, 0, nullptr, slots, NRB, accepted, st);
        }
        return e;
    }
};

// run F<T, L>::f(args...) for the plan's lattice size
#define DDMC_FFT_DISPATCH(L_, EXPR)                \
    switch (L_) {                                  \
    case 8: { constexpr int LL = 8; EXPR; } break;     \
    case 16: { constexpr int LL = 16; EXPR; } break;   \
    case 24: { constexpr int LL = 24; EXPR; } break;   \
    case 32: { constexpr int LL = 32; EXPR; } break;   \
    case 48: { constexpr int LL = 48; EXPR; } break;   \
    case 64: { constexpr int LL = 64; EXPR; } break;   \
    case 96: { constexpr int LL = 96; EXPR; } break;   \
    case 128: { constexpr int LL = 128; EXPR; } break; \
    case 192: { constexpr int LL = 192; EXPR; } break; \
    case 256: { constexpr int LL = 256; EXPR; } break; \
    case 384: { constexpr int LL = 384; EXPR; } break; \
    case 512: { constexpr int LL = 512; EXPR; } break; \
    default: break;                                \
    }

}  // namespace

bool fft_supported(int L, ddmc_prec prec)
{
    bool ok = false;
    if (prec == DDMC_F64) {
        DDMC_FFT_DISPATCH(L, ok = (fft_impl<double, LL>::lds_ok()));
    } else {
        DDMC_FFT_DISPATCH(L, ok = (fft_impl<float, LL>::lds_ok()));
    }
    return ok;
}

void fft_plan_free(ddmc_plan *p)
{
    hipFree(p->spec_ws);
    hipFree(p->what);
    hipFree(p->twiddle);
    hipFree(p->slot_ws);
    hipFree(p->rows_obs_ws);
    p->spec_ws = p->what = p->twiddle = nullptr;
    p->slot_ws = nullptr;
    p->rows_obs_ws = nullptr;
}

// bytes of the FFT workspace of a plan: both spectra, the kernel spectrum,
// twiddles, accept slots and observable partial sums
struct fft_sizes {
    size_t spec, what, twiddle, slots, obs;
    size_t total() const { return spec + what + twiddle + slots + obs; }
};

template <typename T> fft_sizes fft_sizes_of(int L, int R_max, int nrb)
{
    const size_t cbytes = sizeof(cplx<T>);
    fft_sizes z;
    z.spec = 2 * (size_t)R_max * 3 * L * (L / 2) * cbytes;
    z.what = 4 * (size_t)L * (L / 2 + 1) * sizeof(T);
    z.twiddle = (size_t)L * cbytes;
    z.slots = (size_t)R_max * nrb * sizeof(unsigned int);
    z.obs = (size_t)R_max * nrb * OBS_NACC * sizeof(double);
    return z;
}

size_t fft_plan_bytes(int L, int R_max, ddmc_prec prec)
{
    int nrb = 0;
    if (prec == DDMC_F64) {
        DDMC_FFT_DISPATCH(L, (nrb = fft_impl<double, LL>::NRB));
        return nrb ? fft_sizes_of<double>(L, R_max, nrb).total() : 0;
    }
    DDMC_FFT_DISPATCH(L, (nrb = fft_impl<float, LL>::NRB));
    return nrb ? fft_sizes_of<float>(L, R_max, nrb).total() : 0;
}

template <typename T> ddmc_status fft_plan_init(ddmc_plan *p, const double *W64)
{
    const int L = p->L, H1 = L / 2 + 1;
    bool ok = false;
    int nrb = 0;
    DDMC_FFT_DISPATCH(L, (ok = fft_impl<T, LL>::lds_ok(), nrb = fft_impl<T, LL>::NRB));
    if (!ok) return fail(DDMC_EUNSUPPORTED, "FFT field: this lattice size exceeds the LDS budget in this precision");
    const fft_sizes z = fft_sizes_of<T>(L, p->R_max, nrb);
    if (hipMalloc(&p->spec_ws, z.spec) != hipSuccess || hipMalloc(&p->what, z.what) != hipSuccess ||
        hipMalloc(&p->twiddle, z.twiddle) != hipSuccess ||
        hipMalloc((void **)&p->slot_ws, z.slots) != hipSuccess ||
        hipMalloc((void **)&p->rows_obs_ws, z.obs) != hipSuccess)
        return fail(DDMC_ENOMEM, "ddmc_plan_create: cannot allocate FFT workspace");
    double *tx = nullptr;
    if (hipMalloc(&tx, 2 * 4 * (size_t)L * H1 * sizeof(double)) != hipSuccess)
        return fail(DDMC_ENOMEM, "ddmc_plan_create: cannot allocate FFT scratch");
    const long n = 4L * L * H1;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_twiddles<T>, dim3((L + 255) / 256), dim3(256), 0, nullptr, L,
                       reinterpret_cast<cplx<T> *>(p->twiddle));
    hipLaunchKernelGGL(k_what_x, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, nullptr, L, W64, tx);
    hipLaunchKernelGGL(k_what_y<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, nullptr, L, tx,
                       reinterpret_cast<T *>(p->what));
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    hipFree(tx);
    return hip_check(e, "FFT plan set-up");
}

template <typename T> ddmc_status fft_field(ddmc_plan *p, int R, const T *s, T *h, int color, hipStream_t st)
{
    hipError_t e = hipErrorInvalidValue;
    DDMC_FFT_DISPATCH(p->L, e = (fft_impl<T, LL>::field(p, R, s, h, color, st)));
    return hip_check(e, "FFT field launch");
}

template <typename T>
ddmc_status fft_sweep(ddmc_plan *p, int R, const ddmc_replica_params *params, T *s, uint64_t *sweep_ctr,
                      uint64_t sweep0, int nsweeps, uint64_t *accepted, double *obs, double *eta_acc, hipStream_t st)
{
    hipError_t e = hipErrorInvalidValue;
    DDMC_FFT_DISPATCH(p->L, e = (fft_impl<T, LL>::sweep(p, R, params, s, sweep_ctr, sweep0, nsweeps, accepted, obs,
                                                         eta_acc, st)));
    return hip_check(e, "FFT sweep launch");
}

template <typename T>
ddmc_status fft_sweep_coset(ddmc_plan *p, int R, const ddmc_replica_params *params, T *s, int l, uint64_t *sweep_ctr,
                            int nsweeps, uint64_t *accepted, hipStream_t st)
{
    hipError_t e = hipErrorInvalidValue;
    DDMC_FFT_DISPATCH(p->L, e = (fft_impl<T, LL>::sweep_coset(p, R, params, s, l, sweep_ctr, nsweeps, accepted, st)));
    return hip_check(e, "FFT coset sweep launch");
}

template ddmc_status fft_sweep_coset<float>(ddmc_plan *, int, const ddmc_replica_params *, float *, int, uint64_t *,
                                            int, uint64_t *, hipStream_t);
template ddmc_status fft_sweep_coset<double>(ddmc_plan *, int, const ddmc_replica_params *, double *, int,
                                             uint64_t *, int, uint64_t *, hipStream_t);
template ddmc_status fft_plan_init<float>(ddmc_plan *, const double *);
template ddmc_status fft_plan_init<double>(ddmc_plan *, const double *);
template ddmc_status fft_field<float>(ddmc_plan *, int, const float *, float *, int, hipStream_t);
template ddmc_status fft_field<double>(ddmc_plan *, int, const double *, double *, int, hipStream_t);
template ddmc_status fft_sweep<float>(ddmc_plan *, int, const ddmc_replica_params *, float *, uint64_t *,
                                      uint64_t, int, uint64_t *, double *, double *, hipStream_t);
template ddmc_status fft_sweep<double>(ddmc_plan *, int, const ddmc_replica_params *, double *, uint64_t *,
                                       uint64_t, int, uint64_t *, double *, double *, hipStream_t);

}  // namespace ddmc
