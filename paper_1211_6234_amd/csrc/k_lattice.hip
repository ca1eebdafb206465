// k_lattice.hip -- the lattice-summed dipole tensor W(rho) in FP64 (Sec. 2.1:
// the sum over periodic images G = (aL, bL) of the dipole tensor of eq. (1),
// precomputed once per lattice size).
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

hipError_t launch_lattice_sum(int L, int M, double *W64, hipStream_t st)
{
    const long N = (long)L * L;
    const int bs = 256;
    const long nb = (N + bs - 1) / bs;
    hipLaunchKernelGGL(k_lattice_sum, dim3((unsigned)nb), dim3(bs), 0, st, L, M, W64);
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
