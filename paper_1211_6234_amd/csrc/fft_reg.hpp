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
// compile-time constants (exact for the multiples of pi/4).
#pragma once

#include <hip/hip_runtime.h>

namespace ddmc {
namespace fftreg {

// cos and sin of 2 pi k / 32, k = 0 .. 31
__device__ constexpr double ROOT32[32][2] = {
    {1, 0},
    {0.98078528040323043, 0.19509032201612825},
    {0.92387953251128674, 0.38268343236508978},
    {0.83146961230254524, 0.55557023301960218},
    {0.70710678118654757, 0.70710678118654746},
    {0.55557023301960229, 0.83146961230254524},
    {0.38268343236508984, 0.92387953251128674},
    {0.19509032201612833, 0.98078528040323043},
    {6.123233995736766e-17, 1},
    {-0.19509032201612819, 0.98078528040323043},
    {-0.38268343236508973, 0.92387953251128674},
    {-0.55557023301960196, 0.83146961230254546},
    {-0.70710678118654746, 0.70710678118654757},
    {-0.83146961230254535, 0.55557023301960218},
    {-0.92387953251128674, 0.38268343236508989},
    {-0.98078528040323043, 0.19509032201612861},
    {-1, 1.2246467991473532e-16},
    {-0.98078528040323043, -0.19509032201612836},
    {-0.92387953251128685, -0.38268343236508967},
    {-0.83146961230254546, -0.55557023301960196},
    {-0.70710678118654768, -0.70710678118654746},
    {-0.55557023301960218, -0.83146961230254524},
    {-0.38268343236509034, -0.92387953251128652},
    {-0.19509032201612866, -0.98078528040323032},
    {-1.8369701987210297e-16, -1},
    {0.1950903220161283, -0.98078528040323043},
    {0.38268343236509, -0.92387953251128663},
    {0.55557023301960184, -0.83146961230254546},
    {0.70710678118654735, -0.70710678118654768},
    {0.83146961230254524, -0.55557023301960218},
    {0.92387953251128652, -0.38268343236509039},
    {0.98078528040323032, -0.19509032201612872},
};

template <typename T> struct cx {
    T re, im;
};

// e^{-/+ 2 pi i k / R} for R | 32 (forward / inverse); with R and k known
// at compile time after unrolling, the table entry folds to a constant
template <typename T, bool INV>
__device__ __forceinline__ cx<T> root(int R, int k)
{
    const int m = (k % R) * (32 / R);
    return cx<T>{(T)ROOT32[m][0], INV ? (T)ROOT32[m][1] : -(T)ROOT32[m][1]};
}

// b * e^{-/+ 2 pi i k / R}.  After unrolling, k and R are constants: the
// multiples of pi/2 become exact sign swaps and the odd multiples of pi/4
// two additions and one scaling, so only the other roots cost a full
// complex multiply.
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rotate(cx<T> b, int R, int k)
{
    const int m = (k % R) * (32 / R);   // angle in units of 2 pi / 32
    const T h = (T)0.70710678118654752440;
    if (m == 0) return b;
    if (m == 16) return cx<T>{-b.re, -b.im};
    // forward multiplies by e^{-i a}, inverse by e^{+i a}
    if (m == 8) return INV ? cx<T>{-b.im, b.re} : cx<T>{b.im, -b.re};
    if (m == 24) return INV ? cx<T>{b.im, -b.re} : cx<T>{-b.im, b.re};
    if (m == 4) return INV ? cx<T>{h * (b.re - b.im), h * (b.re + b.im)} : cx<T>{h * (b.re + b.im), h * (b.im - b.re)};
    if (m == 12)
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

// In-place R-point DFT of registers v (R a power of two, R <= 32).
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(cx<T> (&v)[R])
{
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

// factorization of n used by the passes
template <int n> struct split {
    static constexpr int n1 = (n >= 256) ? 16 * (n / 256 > 1 ? 2 : 1) : (n >= 128 ? 16 : (n >= 16 ? 8 : (n >= 4 ? n / 2 : 1)));
    static constexpr int n2 = n / n1;
};

}  // namespace fftreg
}  // namespace ddmc
