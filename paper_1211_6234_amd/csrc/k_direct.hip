// k_direct.hip -- the local dipolar field by direct summation (Sec. 2.1:
// N interactions per site), h_i = sum_j W(r_i - r_j) s_j, on VALU.
//
// Work decomposition.  A block owns RY output rows of one replica and a range
// of input rows (split-K over input rows keeps a single replica's field
// spread over the whole chip; partial sums are added in a fixed order by a
// second kernel; the split depends on L only, so results do not depend on
// the batch).  Input rows are staged in LDS in chunks of VC rows, together
// with the band of RY + VC - 1 kernel rows they need (rho_y = y - v).
// Each thread accumulates XB outputs of one row spaced D apart (D = 2 when
// only one colour is wanted); the kernel entries of its outputs for
// consecutive inputs of one parity form a sliding window, kept in registers
// as a ring buffer so that each step loads one new kernel entry and one
// broadcast spin for 5 XB fused multiply-adds.
#include "internal.hpp"

namespace ddmc {

namespace {

constexpr int VC = 2;   // input rows per LDS chunk

template <typename T> struct acc3 {
    T x, y, z;
};

template <typename T, int XB, int D>
__global__ void __launch_bounds__(1024)
k_direct(int L, int R, const T *__restrict__ W, const T *__restrict__ s, T *__restrict__ out,
         int color, int RY, int VK, long split_stride)
{
    using V4 = vec4a<T>;
    extern __shared__ unsigned char smem_raw[];
    V4 *sp = reinterpret_cast<V4 *>(smem_raw);          // [VC][L] spins
    V4 *wb = sp + VC * L;                                // [RY + VC - 1][L] kernel rows

    const long N = (long)L * L;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int nthr = blockDim.x * blockDim.y, tid = ty * blockDim.x + tx;
    const int y0 = blockIdx.x * RY;
    const int kb = blockIdx.y;
    const int r = blockIdx.z;
    const int v_begin = kb * VK;
    const int v_end = min(L, v_begin + VK);

    const T *sr = s + (long)r * 3 * N;
    const T *Wxx = W, *Wyy = W + N, *Wxy = W + 2 * N, *Wzz = W + 3 * N;

    const int y = y0 + ty;
    const bool row_ok = y < L;
    const int p = (D == 2) ? ((color + y) & 1) : 0;
    const int base = p + D * tx * XB;

    acc3<T> acc[XB];
#pragma unroll
    for (int k = 0; k < XB; ++k) acc[k] = acc3<T>{T(0), T(0), T(0)};

    for (int vc0 = v_begin; vc0 < v_end; vc0 += VC) {
        const int nv = min(VC, v_end - vc0);
        // stage the spins of input rows vc0 .. vc0 + nv - 1
        for (int e = tid; e < nv * L; e += nthr) {
            const int vi = e / L, u = e - vi * L;
            const long j = (long)(vc0 + vi) * L + u;
            V4 t;
            t.a = sr[j]; t.b = sr[N + j]; t.c = sr[2 * N + j]; t.d = T(0);
            sp[vi * L + u] = t;
        }
        // stage kernel rows rho_y = y0 - vc0 - (VC - 1) + t, t < RY + VC - 1
        const int nrow = RY + VC - 1;
        for (int e = tid; e < nrow * L; e += nthr) {
            const int t = e / L, u = e - t * L;
            int ry = (y0 - vc0 - (VC - 1) + t) % L;
            if (ry < 0) ry += L;
            const long q = (long)ry * L + u;
            V4 w;
            w.a = Wxx[q]; w.b = Wyy[q]; w.c = Wxy[q]; w.d = Wzz[q];
            wb[t * L + u] = w;
        }
        __syncthreads();
        if (row_ok) {
            for (int vi = 0; vi < nv; ++vi) {
                const V4 *wrow = wb + (ty - vi + (VC - 1)) * L;
                const V4 *srow = sp + vi * L;
#pragma unroll
                for (int q = 0; q < D; ++q) {
                    // window for step m holds k-th output's entry in slot (k - m) mod XB
                    V4 win[XB];
                    int idx = base - q;
                    if (idx < 0) idx += L;
#pragma unroll
                    for (int k = 0; k < XB; ++k) {
                        int ik = idx + D * k;
                        if (ik >= L) ik -= L;
                        win[k] = wrow[ik];
                    }
                    const int steps = L / D;
                    for (int mc = 0; mc < steps; mc += XB) {
#pragma unroll
                        for (int mm = 0; mm < XB; ++mm) {
                            if (mm > 0 || mc > 0) {
                                idx -= D;
                                if (idx < 0) idx += L;
                                win[(XB - mm) % XB] = wrow[idx];
                            }
                            const V4 sv = srow[q + D * (mc + mm)];
#pragma unroll
                            for (int k = 0; k < XB; ++k) {
                                const V4 w = win[(k - mm + XB) % XB];
                                acc[k].x += w.a * sv.a + w.c * sv.b;
                                acc[k].y += w.c * sv.a + w.b * sv.b;
                                acc[k].z += w.d * sv.c;
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (!row_ok) return;
    T *o = out + (long)kb * split_stride + (long)r * 3 * N;
#pragma unroll
    for (int k = 0; k < XB; ++k) {
        const long i = (long)y * L + base + D * k;
        o[i] = acc[k].x;
        o[N + i] = acc[k].y;
        o[2 * N + i] = acc[k].z;
    }
}

// h = sum over splits of the partials, sites of one colour (or all)
template <typename T>
__global__ void k_split_sum(int L, int R, int nsplit, long split_stride, const T *__restrict__ part,
                            T *__restrict__ h, int color)
{
    const long N = (long)L * L;
    const long per = (color < 0) ? N : N / 2;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= per * 3 * R) return;
    const long r = e / (3 * per);
    const long rem = e - r * 3 * per;
    const long c = rem / per;
    const long j = rem - c * per;
    long i;
    if (color < 0) {
        i = j;
    } else {
        const long half = L / 2;
        const long yy = j / half;
        i = yy * L + 2 * (j - yy * half) + ((color + yy) & 1);
    }
    const long off = r * 3 * N + c * N + i;
    T acc = part[off];
    for (int k = 1; k < nsplit; ++k) acc += part[(long)k * split_stride + off];
    h[off] = acc;
}

int pick_xb(int cols)
{
    if (cols % 4 == 0) return 4;
    if (cols % 2 == 0) return 2;
    return 1;
}

// Split count over input rows: enough blocks to cover the chip for a single
// replica.  It depends on L only, so a replica's summation order (and hence
// its field, bit for bit) does not depend on how many replicas share a call.
int pick_split(int L, int row_blocks)
{
    const int target = 2048;
    int k = (target + row_blocks - 1) / row_blocks;
    const int kmax = (L + 3) / 4;   // at least 4 input rows per block
    if (k > kmax) k = kmax;
    if (k > 32) k = 32;
    if (k < 1) k = 1;
    return k;
}

int pick_ry(int L, size_t elem)
{
    // LDS: (VC + RY + VC - 1) rows of L vec4 elements, at most 64 KiB
    const size_t row_bytes = (size_t)L * 4 * elem;
    int ry = 8;
    while (ry > 1 && (size_t)(2 * VC - 1 + ry) * row_bytes > 65536) ry /= 2;
    return ry;
}

template <typename T, int XB, int D>
hipError_t launch_direct_t(int L, int R, const T *W, const T *s, T *out, int color, int RY, int ksplit,
                           long split_stride, hipStream_t st)
{
    const int cols = L / D / XB;
    dim3 block(cols, RY);
    const int VK = (L + ksplit - 1) / ksplit;
    dim3 grid((L + RY - 1) / RY, ksplit, R);
    const size_t lds = (size_t)(2 * VC - 1 + RY) * L * sizeof(vec4a<T>);
    hipLaunchKernelGGL((k_direct<T, XB, D>), grid, block, lds, st, L, R, W, s, out, color, RY, VK,
                       split_stride);
    return hipGetLastError();
}

}  // namespace

size_t direct_partial_elems(int L, int R_max, size_t elem)
{
    const int ry = pick_ry(L, elem);
    const int k = pick_split(L, (L + ry - 1) / ry);
    return k > 1 ? (size_t)k * R_max * 3 * (size_t)L * L : 0;
}

template <typename T>
ddmc_status direct_field(ddmc_plan *p, int R, const T *s, T *h, int color, hipStream_t st)
{
    const int L = p->L;
    const int D = (color < 0) ? 1 : 2;
    const int cols = L / D;
    const int XB = pick_xb(cols);
    const int RY = pick_ry(L, sizeof(T));
    if (cols / XB * RY > 1024)
        return fail(DDMC_EUNSUPPORTED, "direct field: lattice too large for one block row");
    const int row_blocks = (L + RY - 1) / RY;
    const int ksplit = pick_split(L, row_blocks);
    const long N = (long)L * L;
    if (ksplit > 1 && (size_t)ksplit * R * 3 * N > p->part_elems)
        return fail(DDMC_ENOMEM, "direct field: split workspace smaller than R_max needs");
    T *dst = (ksplit > 1) ? reinterpret_cast<T *>(p->part_ws) : h;
    const long split_stride = (long)R * 3 * N;
    const T *W = reinterpret_cast<const T *>(p->W);
    prof_scope ps(p, DDMC_KERNEL_DIRECT_FIELD, st);
    hipError_t e = hipSuccess;
#define DDMC_DIRECT_CASE(XBV, DV)                                                                  \
    if (XB == XBV && D == DV)                                                                      \
        e = launch_direct_t<T, XBV, DV>(L, R, W, s, dst, color, RY, ksplit, split_stride, st);
    DDMC_DIRECT_CASE(4, 1)
    DDMC_DIRECT_CASE(2, 1)
    DDMC_DIRECT_CASE(1, 1)
    DDMC_DIRECT_CASE(4, 2)
    DDMC_DIRECT_CASE(2, 2)
    DDMC_DIRECT_CASE(1, 2)
#undef DDMC_DIRECT_CASE
    if (e != hipSuccess) return hip_check(e, "direct field launch");
    if (ksplit > 1) {
        const long per = (color < 0) ? N : N / 2;
        const long total = per * 3 * R;
        const int bs = 256;
        hipLaunchKernelGGL(k_split_sum<T>, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, st, L, R,
                           ksplit, split_stride, dst, h, color);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_check(e, "direct field reduction launch");
    }
    return DDMC_OK;
}

template ddmc_status direct_field<float>(ddmc_plan *, int, const float *, float *, int, hipStream_t);
template ddmc_status direct_field<double>(ddmc_plan *, int, const double *, double *, int, hipStream_t);

}  // namespace ddmc
