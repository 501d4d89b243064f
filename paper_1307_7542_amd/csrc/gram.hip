// Dense Gram matrix G = Q^T Q of m stored Lanczos vectors on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64): the orthogonality check of the
// reorthogonalised Lanczos recurrence (Sec. IV; the paper's own runs use no
// reorthogonalisation, Sec. V).
//
// Q is n x m, one n-long vector (FP32 or FP64) per column, and is read from
// HBM once.  Each workgroup takes a contiguous range of rows and stages RB
// rows x m columns in LDS (row-major, odd pitch so the column-wise stores do
// not collide in the banks); each wavefront accumulates its share of the
// upper-triangle 16 x 16 tiles of G over those rows.  For tile (I, J) and MFMA
// step s, lane i + 16 k supplies A = Q[r0 + 4 s + k, 16 I + i] and
// B = Q[r0 + 4 s + k, 16 J + i], and lane l receives G[16 I + l / 16 + 4 r,
// 16 J + l % 16] in accumulator slot r (the instruction's lane layout, checked
// on the device).  FP32 vectors are widened to FP64 exactly, so every product
// is exact and the sums are FP64.  The per-workgroup tiles are summed by a
// second kernel in workgroup order, so G does not depend on timing.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace hub {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int GB = 1024;        // lanes per workgroup (16 wavefronts)
constexpr int GW = GB / 64;     // wavefronts
constexpr int TPW = 5;          // tiles per wavefront and pass (20 FP64 accumulators)
constexpr int RB = 64;          // rows staged per block
constexpr int kTilesPerPass = GW * TPW;

__device__ __forceinline__ void tri_tile(int t, int nt, int &I, int &J)
{
    // t-th (I, J) with I <= J, row by row
    I = 0;
    int row_len = nt;
    while (t >= row_len) {
        t -= row_len;
        ++I;
        --row_len;
    }
    J = I + t;
}

template <typename T>
__global__ __launch_bounds__(GB) void k_gram_mfma(const T *const *__restrict__ Q, int m, int64_t n,
                                                  int64_t rows_per_wg, int pitch, int t0, int ntiles,
                                                  double *__restrict__ part)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *xs = reinterpret_cast<T *>(smem_raw);  // RB x pitch
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int nt = (m + 15) / 16, ncol = 16 * nt;
    d4 acc[TPW];
    int tij[TPW];  // column offsets 16 I | (16 J << 16) of the wavefront's tiles
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        acc[u] = d4{0.0, 0.0, 0.0, 0.0};
        const int t = wave + GW * u;
        int I = 0, J = 0;
        if (t < ntiles) tri_tile(t0 + t, nt, I, J);
        tij[u] = 16 * I | (16 * J << 16);
    }
    const int64_t r_begin = (int64_t)blockIdx.x * rows_per_wg;
    const int64_t r_end = min(n, r_begin + rows_per_wg);
    for (int64_t r0 = r_begin; r0 < r_end; r0 += RB) {
        const int nr = (int)min((int64_t)RB, r_end - r0);
        __syncthreads();  // the previous block's operands are consumed
        // consecutive lanes take consecutive rows of one column (coalesced reads)
        for (int idx = (int)threadIdx.x; idx < RB * ncol; idx += GB) {
            const int c = idx / RB, r = idx - c * RB;
            T v = (T)0;
            if (c < m && r < nr) v = Q[c][r0 + r];
            xs[r * pitch + c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            if (wave + GW * u >= ntiles) continue;  // uniform over the wavefront
            const T *ra = xs + (tij[u] & 0xFFFF) + (lane & 15);
            const T *rb = xs + (tij[u] >> 16) + (lane & 15);
            d4 a4 = acc[u];
#pragma unroll 4
            for (int s = 0; s < RB / 4; ++s) {
                const int r = 4 * s + (lane >> 4);
                a4 = __builtin_amdgcn_mfma_f64_16x16x4f64((double)ra[r * pitch], (double)rb[r * pitch], a4, 0, 0, 0);
            }
            acc[u] = a4;
        }
    }
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int t = wave + GW * u;
        if (t >= ntiles) continue;
        double *dst = part + ((int64_t)blockIdx.x * ntiles + t) * 256;
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[((lane >> 4) + 4 * r) * 16 + (lane & 15)] = acc[u][r];
    }
}

// G[i][j] (ld x ld, both triangles) = sum over workgroups, in order, of their tiles
__global__ void k_gram_reduce(const double *__restrict__ part, int nwg, int t0, int ntiles, int nt, int ld,
                              double *__restrict__ G)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)ntiles * 256) return;
    const int t = (int)(e / 256), w = (int)(e % 256);
    double s = 0.0;
    for (int g = 0; g < nwg; ++g) s += part[((int64_t)g * ntiles + t) * 256 + w];
    int I, J;
    tri_tile(t0 + t, nt, I, J);
    const int i = 16 * I + w / 16, j = 16 * J + w % 16;
    G[(int64_t)i * ld + j] = s;
    G[(int64_t)j * ld + i] = s;
}

template <typename T>
hub_status gram_t(const void *const *dq, int m, int64_t n, double *dG, int ld, hipStream_t st)
{
    const int nt = (m + 15) / 16;
    const int ntri = nt * (nt + 1) / 2;
    const int pitch = 16 * nt + 1;
    const size_t lds = (size_t)RB * pitch * sizeof(T);
    // workgroups: at most 256, each with whole blocks of rows
    int nwg = (int)std::min<int64_t>(256, std::max<int64_t>(1, (n + 16 * RB - 1) / (16 * RB)));
    const int64_t rows = ((n + nwg - 1) / nwg + RB - 1) / RB * RB;
    nwg = (int)((n + rows - 1) / rows);
    double *part = nullptr;
    const int per_pass = std::min(ntri, kTilesPerPass);
    HUB_HIP(hipMalloc((void **)&part, sizeof(double) * 256 * (size_t)nwg * (size_t)per_pass));
    struct Free {
        void *p;
        ~Free() { (void)hipFree(p); }
    } fr{part};
    HUB_HIP(hipFuncSetAttribute((const void *)k_gram_mfma<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    for (int t0 = 0; t0 < ntri; t0 += per_pass) {
        const int nti = std::min(per_pass, ntri - t0);
        hipLaunchKernelGGL(k_gram_mfma<T>, dim3((unsigned)nwg), dim3(GB), lds, st, (const T *const *)dq, m, n, rows,
                           pitch, t0, nti, part);
        hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((nti * 256 + 255) / 256)), dim3(256), 0, st, part, nwg, t0,
                           nti, nt, ld, dG);
        HUB_HIP(hipGetLastError());
    }
    // the stream must not run past the workspace's free
    HUB_HIP(hipStreamSynchronize(st));
    return HUB_OK;
}

}  // namespace

hub_status gram_mfma(int dtype, const void *const *dq, int m, int64_t n, double *dG, int ld, hipStream_t st)
{
    if (m <= 0 || n <= 0) return HUB_OK;
    if (ld < 16 * ((m + 15) / 16)) {
        set_error("Gram: leading dimension below the padded size");
        return HUB_ERR_INVALID_ARG;
    }
    if ((size_t)RB * (16 * ((m + 15) / 16) + 1) * (dtype == HUB_F64 ? 8 : 4) > 160 * 1024) {
        set_error("Gram: too many vectors for one staged block (m <= 304 in FP64, 624 in FP32)");
        return HUB_ERR_UNSUPPORTED;
    }
    if (dtype == HUB_F64) return gram_t<double>(dq, m, n, dG, ld, st);
    return gram_t<float>(dq, m, n, dG, ld, st);
}

}  // namespace hub
