// k_lattice.hip -- the lattice-summed dipole tensor W(rho) in FP64 (Sec. 2.1:
// the sum over periodic images G = (aL, bL) of the dipole tensor of eq. (1),
// precomputed once per lattice size), over a square box of images or over
// all of them.
#include "internal.hpp"

namespace ddmc {

// Weight of an image coordinate c in the square |c| <= (M + 1/2) L, in
// units of the lattice constant: 2|c| < (2M+1)L inside, == on the edge.
__device__ __forceinline__ double box_weight(long c, long edge2)
{
    const long a2 = 2 * (c < 0 ? -c : c);
    return a2 < edge2 ? 1.0 : (a2 == edge2 ? 0.5 : 0.0);
}

// One thread per separation rho = (px, py); sums the images r = rho + (aL, bL)
// of the in-plane dipole tensor (delta_ab r^2 - 3 r_a r_b) / r^5.
__global__ void k_lattice_sum(int L, int M, double *__restrict__ W)
{
    const long N = (long)L * L;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const long px = i % L, py = i / L;
    const long edge2 = (long)(2 * M + 1) * L;
    double sxx = 0.0, syy = 0.0, sxy = 0.0, szz = 0.0;
    for (int b = -M - 1; b <= M + 1; ++b) {
        const long ry = py + (long)b * L;
        const double wy = box_weight(ry, edge2);
        if (wy == 0.0) continue;
        for (int a = -M - 1; a <= M + 1; ++a) {
            const long rx = px + (long)a * L;
            const double w = wy * box_weight(rx, edge2);
            if (w == 0.0 || (rx == 0 && ry == 0)) continue;
            const double x = (double)rx, y = (double)ry;
            const double r2 = x * x + y * y;
            const double inv_r = 1.0 / sqrt(r2);
            const double inv_r3 = inv_r * inv_r * inv_r;
            const double inv_r5 = inv_r3 / r2;
            sxx += w * (r2 - 3.0 * x * x) * inv_r5;
            syy += w * (r2 - 3.0 * y * y) * inv_r5;
            sxy += w * (-3.0 * x * y) * inv_r5;
            szz += w * inv_r3;
        }
    }
    W[i] = sxx;
    W[N + i] = syy;
    W[2 * N + i] = sxy;
    W[3 * N + i] = szz;
}

// All images (M < 0): the Ewald-Harris split of Sec. 2.1 (eqs. (3)-(5) at
// z = 0).  With 1/r = erfc(r/2e)/r + erf(r/2e)/r, the screened part is summed
// over images in real space and the smooth part over the reciprocal lattice
// k = 2 pi (m, n) / L through its in-plane transform (2 pi / |k|) erfc(|k| e).
// The tensor is minus the second derivatives of each part; at rho = 0 the
// smooth part of the excluded self term contributes (4/(3 sqrt(pi))) (1/2e)^3
// to xx and yy and is taken off.  W_zz = -(W_xx + W_yy) (every image term is
// trace-free).  One thread per separation; the phase k.rho is reduced exactly
// in integers before the cosine.
__global__ void k_lattice_ewald(int L, double e, int nreal, int nrecip, double *__restrict__ W)
{
    const long N = (long)L * L;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int px = (int)(i % L), py = (int)(i / L);
    const double a = 0.5 / e;
    const double c_gauss = 2.0 * a * 0.56418958354775628695;   // 2 a / sqrt(pi)
    double sxx = 0.0, syy = 0.0, sxy = 0.0;
    for (int b = -nreal; b <= nreal; ++b) {
        const double y = (double)py + (double)b * L;
        for (int c = -nreal; c <= nreal; ++c) {
            const double x = (double)px + (double)c * L;
            const double r2 = x * x + y * y;
            if (r2 == 0.0) continue;
            const double inv_r = 1.0 / sqrt(r2);
            const double q = erfc(a * r2 * inv_r) * inv_r * inv_r * inv_r;    // erfc(a r) / r^3
            const double gz = c_gauss * exp(-a * a * r2);                   // (2a/sqrt(pi)) e^{-a^2 r^2}
            // -d_a d_b [erfc(a r)/r] = u delta_ab - v r_a r_b / r^2
            const double u = q + gz * inv_r * inv_r;
            const double v = 3.0 * q + (3.0 * inv_r * inv_r + 2.0 * a * a) * gz;
            const double xr = x * inv_r, yr = y * inv_r;
            sxx += u - v * xr * xr;
            syy += u - v * yr * yr;
            sxy -= v * xr * yr;
        }
    }
    const double scale = 2.0 * 3.14159265358979323846 / ((double)L * (double)L);
    for (int n = -nrecip; n <= nrecip; ++n) {
        for (int m = -nrecip; m <= nrecip; ++m) {
            if (m == 0 && n == 0) continue;
            const double kx = 2.0 * 3.14159265358979323846 * m / L, ky = 2.0 * 3.14159265358979323846 * n / L;
            const double k = sqrt(kx * kx + ky * ky);
            const int ph = (int)((((long)m * px + (long)n * py) % L + L) % L);   // k.rho = 2 pi ph / L
            const double w = scale * erfc(k * e) / k * cospi(2.0 * ph / (double)L);
            sxx += w * kx * kx;
            syy += w * ky * ky;
            sxy += w * kx * ky;
        }
    }
    if (i == 0) {
        const double self = 4.0 * 0.56418958354775628695 / 3.0 * a * a * a;
        sxx -= self;
        syy -= self;
    }
    W[i] = sxx;
    W[N + i] = syy;
    W[2 * N + i] = sxy;
    W[3 * N + i] = -(sxx + syy);
}

hipError_t launch_lattice_sum(int L, int M, double *W64, hipStream_t st)
{
    const long N = (long)L * L;
    const int bs = 256;
    const long nb = (N + bs - 1) / bs;
    if (M < 0) {
        // split length L/4: images with a r < 6.5 (|G| <= 3.25 L + rho) and wave
        // vectors with |k| e < 6.5 (|m|, |n| <= 4.2) carry everything above 1e-19
        const double e = 0.25 * L;
        const int nreal = 5, nrecip = 6;
        hipLaunchKernelGGL(k_lattice_ewald, dim3((unsigned)nb), dim3(bs), 0, st, L, e, nreal, nrecip, W64);
    } else {
        hipLaunchKernelGGL(k_lattice_sum, dim3((unsigned)nb), dim3(bs), 0, st, L, M, W64);
    }
    return hipGetLastError();
}

template <typename T>
__global__ void k_convert(long n, const double *__restrict__ src, T *__restrict__ dst)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (T)src[i];
}

template <typename T> hipError_t launch_convert_kernel(int L, const double *W64, T *W, hipStream_t st)
{
    const long n = 4L * L * L;
    const int bs = 256;
    hipLaunchKernelGGL(k_convert<T>, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st, n, W64, W);
    return hipGetLastError();
}

template <typename S, typename D>
__global__ void k_convert_any(long n, const S *__restrict__ src, D *__restrict__ dst)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (D)src[i];
}

hipError_t launch_spins_convert(long n, const void *src, bool src64, void *dst, bool dst64, hipStream_t st)
{
    const int bs = 256;
    const dim3 g((unsigned)((n + bs - 1) / bs));
    if (src64 && dst64)
        hipLaunchKernelGGL((k_convert_any<double, double>), g, dim3(bs), 0, st, n, (const double *)src, (double *)dst);
    else if (src64)
        hipLaunchKernelGGL((k_convert_any<double, float>), g, dim3(bs), 0, st, n, (const double *)src, (float *)dst);
    else if (dst64)
        hipLaunchKernelGGL((k_convert_any<float, double>), g, dim3(bs), 0, st, n, (const float *)src, (double *)dst);
    else
        hipLaunchKernelGGL((k_convert_any<float, float>), g, dim3(bs), 0, st, n, (const float *)src, (float *)dst);
    return hipGetLastError();
}

template hipError_t launch_convert_kernel<float>(int, const double *, float *, hipStream_t);
template hipError_t launch_convert_kernel<double>(int, const double *, double *, hipStream_t);

}  // namespace ddmc
