// fft_reg.hpp -- register-resident FFT passes for the LDS transforms.
//
// A length-n complex DFT with n = n1 n2 is done in two register passes
// (the "four-step" factorization): pass A, one thread per j2 < n2, loads the
// n1 points x[j1 n2 + j2], takes their n1-point DFT in registers and scales
// output k1 by w_n^(j2 k1); pass B, one thread per k1 < n1, loads the n2
// values of row k1, takes their n2-point DFT and writes X[k1 + n1 k2].  The
// intermediate rows are padded by one element so that neither pass meets LDS
// bank conflicts.  Two barriers per transform instead of one per radix-4
// stage.  Small DFTs are unrolled radix-2 networks with the roots as
// compile-time constants (exact for the multiples of pi/4), with one radix-3
// stage for lengths 3 * 2^k.
#pragma once

#include <hip/hip_runtime.h>

namespace ddmc {
namespace fftreg {

// cos and sin of 2 pi k / 96, k = 0 .. 95 (96 = lcm of the radices 2^5 and 3)
__device__ constexpr double ROOT96[96][2] = {
    {1.0, 0.0},
    {0.9978589232386035, 0.06540312923014306},
    {0.9914448613738104, 0.13052619222005157},
    {0.9807852804032304, 0.19509032201612825},
    {0.9659258262890683, 0.25881904510252074},
    {0.9469301294951057, 0.3214394653031616},
    {0.9238795325112867, 0.3826834323650898},
    {0.8968727415326884, 0.44228869021900125},
    {0.8660254037844387, 0.49999999999999994},
    {0.8314696123025452, 0.5555702330196022},
    {0.7933533402912352, 0.6087614290087207},
    {0.7518398074789774, 0.6593458151000688},
    {0.7071067811865476, 0.7071067811865475},
    {0.6593458151000688, 0.7518398074789774},
    {0.6087614290087207, 0.7933533402912352},
    {0.5555702330196024, 0.8314696123025451},
    {0.5000000000000001, 0.8660254037844386},
    {0.44228869021900125, 0.8968727415326884},
    {0.38268343236508984, 0.9238795325112867},
    {0.3214394653031617, 0.9469301294951056},
    {0.25881904510252074, 0.9659258262890683},
    {0.19509032201612833, 0.9807852804032304},
    {0.1305261922200517, 0.9914448613738104},
    {0.06540312923014327, 0.9978589232386035},
    {6.123233995736766e-17, 1.0},
    {-0.06540312923014314, 0.9978589232386035},
    {-0.1305261922200516, 0.9914448613738104},
    {-0.1950903220161282, 0.9807852804032304},
    {-0.25881904510252063, 0.9659258262890683},
    {-0.3214394653031616, 0.9469301294951057},
    {-0.3826834323650895, 0.9238795325112868},
    {-0.44228869021900113, 0.8968727415326884},
    {-0.4999999999999998, 0.8660254037844387},
    {-0.5555702330196023, 0.8314696123025451},
    {-0.6087614290087207, 0.7933533402912352},
    {-0.6593458151000688, 0.7518398074789774},
    {-0.7071067811865475, 0.7071067811865476},
    {-0.7518398074789773, 0.659345815100069},
    {-0.793353340291235, 0.6087614290087209},
    {-0.831469612302545, 0.5555702330196025},
    {-0.8660254037844387, 0.49999999999999994},
    {-0.8968727415326881, 0.4422886902190017},
    {-0.9238795325112867, 0.3826834323650899},
    {-0.9469301294951056, 0.32143946530316175},
    {-0.9659258262890682, 0.258819045102521},
    {-0.9807852804032304, 0.19509032201612816},
    {-0.9914448613738104, 0.130526192220052},
    {-0.9978589232386035, 0.06540312923014312},
    {-1.0, 1.2246467991473532e-16},
    {-0.9978589232386035, -0.06540312923014287},
    {-0.9914448613738104, -0.13052619222005177},
    {-0.9807852804032305, -0.19509032201612792},
    {-0.9659258262890683, -0.2588190451025208},
    {-0.9469301294951057, -0.32143946530316153},
    {-0.9238795325112868, -0.38268343236508967},
    {-0.8968727415326883, -0.44228869021900147},
    {-0.8660254037844388, -0.4999999999999997},
    {-0.8314696123025455, -0.555570233019602},
    {-0.7933533402912352, -0.6087614290087207},
    {-0.7518398074789775, -0.6593458151000688},
    {-0.7071067811865479, -0.7071067811865471},
    {-0.6593458151000691, -0.7518398074789773},
    {-0.6087614290087209, -0.7933533402912349},
    {-0.5555702330196022, -0.8314696123025452},
    {-0.5000000000000004, -0.8660254037844384},
    {-0.44228869021900136, -0.8968727415326883},
    {-0.3826834323650895, -0.9238795325112868},
    {-0.3214394653031618, -0.9469301294951056},
    {-0.25881904510252063, -0.9659258262890683},
    {-0.19509032201612866, -0.9807852804032303},
    {-0.13052619222005163, -0.9914448613738104},
    {-0.06540312923014273, -0.9978589232386035},
    {-1.8369701987210297e-16, -1.0},
    {0.06540312923014237, -0.9978589232386036},
    {0.13052619222005127, -0.9914448613738105},
    {0.1950903220161283, -0.9807852804032304},
    {0.2588190451025203, -0.9659258262890684},
    {0.3214394653031615, -0.9469301294951057},
    {0.38268343236508917, -0.923879532511287},
    {0.442288690219001, -0.8968727415326885},
    {0.5000000000000001, -0.8660254037844386},
    {0.5555702330196018, -0.8314696123025455},
    {0.6087614290087199, -0.7933533402912357},
    {0.6593458151000691, -0.7518398074789772},
    {0.7071067811865474, -0.7071067811865477},
    {0.7518398074789775, -0.6593458151000687},
    {0.7933533402912349, -0.6087614290087209},
    {0.8314696123025448, -0.555570233019603},
    {0.8660254037844384, -0.5000000000000004},
    {0.8968727415326883, -0.4422886902190014},
    {0.9238795325112868, -0.38268343236508956},
    {0.9469301294951056, -0.32143946530316186},
    {0.9659258262890681, -0.25881904510252157},
    {0.9807852804032303, -0.19509032201612872},
    {0.9914448613738104, -0.13052619222005168},
    {0.9978589232386035, -0.0654031292301428},
};

template <typename T> struct cx {
    T re, im;
};

// e^{-/+ 2 pi i k / R} for R | 96 (forward / inverse); with R and k known
// at compile time after unrolling, the table entry folds to a constant
template <typename T, bool INV>
__device__ __forceinline__ cx<T> root(int R, int k)
{
    const int m = (k % R) * (96 / R);
    return cx<T>{(T)ROOT96[m][0], INV ? (T)ROOT96[m][1] : -(T)ROOT96[m][1]};
}

// b * e^{-/+ 2 pi i k / R}.  After unrolling, k and R are constants: the
// multiples of pi/2 become exact sign swaps and the odd multiples of pi/4
// two additions and one scaling, so only the other roots cost a full
// complex multiply.
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rotate(cx<T> b, int R, int k)
{
    const int m = (k % R) * (96 / R);   // angle in units of 2 pi / 96
    const T h = (T)0.70710678118654752440;
    if (m == 0) return b;
    if (m == 48) return cx<T>{-b.re, -b.im};
    // forward multiplies by e^{-i a}, inverse by e^{+i a}
    if (m == 24) return INV ? cx<T>{-b.im, b.re} : cx<T>{b.im, -b.re};
    if (m == 72) return INV ? cx<T>{b.im, -b.re} : cx<T>{-b.im, b.re};
    if (m == 12) return INV ? cx<T>{h * (b.re - b.im), h * (b.re + b.im)} : cx<T>{h * (b.re + b.im), h * (b.im - b.re)};
    if (m == 36)
        return INV ? cx<T>{-h * (b.re + b.im), h * (b.re - b.im)} : cx<T>{h * (b.im - b.re), -h * (b.re + b.im)};
    const cx<T> t = root<T, INV>(R, k);
    return cx<T>{b.re * t.re - b.im * t.im, b.re * t.im + b.im * t.re};
}

template <int R> __device__ constexpr int bitrev(int k)
{
    int r = 0;
    for (int b = 1, c = R >> 1; b < R; b <<= 1, c >>= 1)
        if (k & b) r |= c;
    return r;
}

template <typename T, int R, bool INV> __device__ __forceinline__ void dft(cx<T> (&v)[R]);

// R = 3 m: decimation in time into the three subsequences v[3j + r], their
// m-point DFTs, the twiddles w_R^{r k} and one 3-point DFT per k
// (w_3 = -1/2 -/+ i sqrt(3)/2).
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_radix3(cx<T> (&v)[R])
{
    constexpr int m = R / 3;
    const T s3 = (T)0.86602540378443864676;   // sqrt(3) / 2
    cx<T> a0[m], a1[m], a2[m];
#pragma unroll
    for (int j = 0; j < m; ++j) {
        a0[j] = v[3 * j];
        a1[j] = v[3 * j + 1];
        a2[j] = v[3 * j + 2];
    }
    if constexpr (m > 1) {
        dft<T, m, INV>(a0);
        dft<T, m, INV>(a1);
        dft<T, m, INV>(a2);
    }
#pragma unroll
    for (int k = 0; k < m; ++k) {
        const cx<T> b0 = a0[k], b1 = rotate<T, INV>(a1[k], R, k), b2 = rotate<T, INV>(a2[k], R, 2 * k);
        const cx<T> s = {b1.re + b2.re, b1.im + b2.im}, d = {b1.re - b2.re, b1.im - b2.im};
        const cx<T> c = {b0.re - (T)0.5 * s.re, b0.im - (T)0.5 * s.im};
        // -/+ i sqrt(3)/2 d for the forward / inverse transform
        const cx<T> e = INV ? cx<T>{-s3 * d.im, s3 * d.re} : cx<T>{s3 * d.im, -s3 * d.re};
        v[k] = {b0.re + s.re, b0.im + s.im};
        v[k + m] = {c.re + e.re, c.im + e.im};
        v[k + 2 * m] = {c.re - e.re, c.im - e.im};
    }
}

// In-place R-point DFT of registers v: R a power of two up to 32 (radix-2
// network), or 3 times such a power (one radix-3 stage on top).
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(cx<T> (&v)[R])
{
    if constexpr (R % 3 == 0) {
        dft_radix3<T, R, INV>(v);
        return;
    }
    cx<T> w[R];
#pragma unroll
    for (int k = 0; k < R; ++k) w[k] = v[bitrev<R>(k)];
#pragma unroll
    for (int half = 1; half < R; half <<= 1) {
#pragma unroll
        for (int g = 0; g < R; g += 2 * half) {
#pragma unroll
            for (int j = 0; j < half; ++j) {
                const cx<T> a = w[g + j];
                const cx<T> bt = rotate<T, INV>(w[g + j + half], 2 * half, j);
                w[g + j] = {a.re + bt.re, a.im + bt.im};
                w[g + j + half] = {a.re - bt.re, a.im - bt.im};
            }
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = w[k];
}

// factorization n = n1 n2 used by the passes: powers of two, and 3 times a
// power of two (the factor 3 inside n1)
template <int n> struct split {
    static constexpr bool tri = (n % 3) == 0;
    static constexpr int p = tri ? n / 3 : n;   // the power-of-two part
    static constexpr int n1 = tri ? (p >= 32 ? 3 * (p / 16 > 2 ? 8 : 4) : (p >= 4 ? 3 * (p / 2 >= 4 ? 4 : p / 2) : 3))
                                  : ((n >= 256) ? 16 * (n / 256 > 1 ? 2 : 1)
                                                : (n >= 16 ? 8 : (n >= 4 ? n / 2 : 1)));
    static constexpr int n2 = n / n1;
    static_assert(n1 * n2 == n, "factorization");
};

}  // namespace fftreg
}  // namespace ddmc
