// Adjoint of the Kronecker-sum product with respect to the model parameters.
//
// H depends linearly on every t_b, U_i and eps_i (Eq. count1 with per-bond and
// per-site parameters), so g^T (dH/dtheta) x is a bilinear form that reuses the
// structure of the product (Sec. IV A):
//   - bond b, spin up:   sum over entries (a, l) of H_up with bond b of
//                        (-esign) <g[a, :], x[l, :]>   (row dot products of V),
//   - bond b, spin down: sum over entries (b', l) of H_dn with bond b of
//                        (-esign) <g[:, b'], x[:, l]>  (column dot products),
//   - U_i:   sum_{a,b} n_i(up_a & dn_b) g[a,b] x[a,b],
//   - eps_i: sum_{a,b} (n_i(up_a) + n_i(dn_b)) g[a,b] x[a,b].
// Every reduction has a fixed order (per-entry partial sums over fixed column
// chunks, LDS trees, then in-order sums), so the result is reproducible.
#include <vector>

#include "internal.h"

namespace hub {
namespace {

constexpr int AB = 256;

__device__ __forceinline__ double block_sum_a(double v, double *s)
{
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = AB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < (unsigned)off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double neg_esign(uint32_t x, int i, int j)
{
    // -esign for a hop across bond (i < j) from state x: esign = (-1)^(occupied strictly between)
    const uint32_t below_j = (j >= 32) ? 0xFFFFFFFFu : ((1u << j) - 1u);
    const uint32_t upto_i = (i >= 31) ? 0xFFFFFFFFu : ((1u << (i + 1)) - 1u);
    return (__popc(x & below_j & ~upto_i) & 1) ? 1.0 : -1.0;
}

// Site terms: per block partial sums of the 2M site accumulators.
__global__ __launch_bounds__(AB) void k_site_terms(const double *__restrict__ g, const double *__restrict__ x,
                                                   int cu, int cd, int M, const uint32_t *__restrict__ up,
                                                   const uint32_t *__restrict__ dn, double *__restrict__ partial)
{
    __shared__ double s[AB];
    double aU[kMaxSites], aE[kMaxSites];
#pragma unroll
    for (int i = 0; i < kMaxSites; ++i) { aU[i] = 0.0; aE[i] = 0.0; }
    for (int b = blockIdx.x; b < cd; b += gridDim.x) {
        const uint32_t db = dn[b];
        for (int a = threadIdx.x; a < cu; a += AB) {
            const int64_t idx = (int64_t)b * cu + a;
            const double gx = g[idx] * x[idx];
            const uint32_t ua = up[a];
            const uint32_t both = ua & db;
#pragma unroll
            for (int i = 0; i < kMaxSites; ++i) {
                aU[i] += ((both >> i) & 1u) ? gx : 0.0;
                aE[i] += (double)(((ua >> i) & 1u) + ((db >> i) & 1u)) * gx;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kMaxSites; ++i) {
        if (i < M) {
            const double rU = block_sum_a(aU[i], s);
            const double rE = block_sum_a(aE[i], s);
            if (threadIdx.x == 0) {
                partial[(int64_t)blockIdx.x * 2 * kMaxSites + i] = rU;
                partial[(int64_t)blockIdx.x * 2 * kMaxSites + kMaxSites + i] = rE;
            }
        }
    }
}

// Down-spin entries: one block per row b of H_dn, a column dot product per entry.
__global__ __launch_bounds__(AB) void k_dn_terms(const double *__restrict__ g, const double *__restrict__ x, int cu,
                                                 const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                 const int32_t *__restrict__ bond, const uint32_t *__restrict__ basis,
                                                 const int32_t *__restrict__ bi, const int32_t *__restrict__ bj,
                                                 double *__restrict__ wout)
{
    __shared__ double s[AB];
    const int b = blockIdx.x;
    const double *gb = g + (int64_t)b * cu;
    for (int k = rp[b]; k < rp[b + 1]; ++k) {
        const double *xl = x + (int64_t)col[k] * cu;
        double acc = 0.0;
        for (int a = threadIdx.x; a < cu; a += AB) acc += gb[a] * xl[a];
        const double r = block_sum_a(acc, s);
        if (threadIdx.x == 0) {
            const int e = bond[k];
            wout[k] = neg_esign(basis[b], bi[e], bj[e]) * r;
        }
    }
}

// Up-spin entries: blocks own column chunks; a lane owns row a and keeps one
// accumulator per entry of that row (in windows of UW entries).
constexpr int UW = 16;

__global__ __launch_bounds__(AB) void k_up_terms(const double *__restrict__ g, const double *__restrict__ x, int cu,
                                                 int cd, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ col, int max_row, int nchunk,
                                                 double *__restrict__ partial, int64_t nnz)
{
    const int chunk = blockIdx.x;
    const int cols_per = (cd + nchunk - 1) / nchunk;
    const int b0 = chunk * cols_per;
    const int b1 = min(cd, b0 + cols_per);
    for (int a = blockIdx.y * AB + threadIdx.x; a < cu; a += gridDim.y * AB) {
        const int s0 = rp[a], len = rp[a + 1] - s0;
        for (int w0 = 0; w0 < len; w0 += UW) {
            double acc[UW];
            int cl[UW];
#pragma unroll
            for (int u = 0; u < UW; ++u) {
                acc[u] = 0.0;
                cl[u] = (w0 + u < len) ? col[s0 + w0 + u] : 0;
            }
            for (int b = b0; b < b1; ++b) {
                const double ga = g[(int64_t)b * cu + a];
                const double *xb = x + (int64_t)b * cu;
#pragma unroll
                for (int u = 0; u < UW; ++u)
                    if (w0 + u < len) acc[u] += ga * xb[cl[u]];
            }
#pragma unroll
            for (int u = 0; u < UW; ++u)
                if (w0 + u < len) partial[(int64_t)chunk * nnz + s0 + w0 + u] = acc[u];
        }
    }
    (void)max_row;
}

__global__ void k_up_finish(const double *__restrict__ partial, int nchunk, int64_t nnz, int cu,
                            const int32_t *__restrict__ rp, const int32_t *__restrict__ bond,
                            const uint32_t *__restrict__ basis, const int32_t *__restrict__ bi,
                            const int32_t *__restrict__ bj, double *__restrict__ wout)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= cu) return;
    for (int k = rp[a]; k < rp[a + 1]; ++k) {
        double acc = 0.0;
        for (int c = 0; c < nchunk; ++c) acc += partial[(int64_t)c * nnz + k];
        const int e = bond[k];
        wout[k] = neg_esign(basis[a], bi[e], bj[e]) * acc;
    }
}

}  // namespace

hub_status param_bilinear(const hub_sector *s, const double *g, const double *x, double *dbond, double *dU,
                          double *deps, hipStream_t st)
{
    const SpinTables &U = s->spin[0];
    const SpinTables &D = s->spin[1];
    const int cu = (int)U.count, cd = (int)D.count, M = s->M;
    const int nsite_blocks = cd < 1024 ? cd : 1024;
    const int nchunk = cd < 64 ? cd : 64;
    const int64_t nnz_u = U.nnz, nnz_d = D.nnz;

    struct Buf {
        void *p = nullptr;
        ~Buf() { if (p) (void)hipFree(p); }
    } b_site, b_wu, b_wd, b_part;
    HUB_HIP(hipMalloc(&b_site.p, sizeof(double) * (size_t)nsite_blocks * 2 * kMaxSites));
    HUB_HIP(hipMalloc(&b_wu.p, sizeof(double) * (size_t)(nnz_u > 0 ? nnz_u : 1)));
    HUB_HIP(hipMalloc(&b_wd.p, sizeof(double) * (size_t)(nnz_d > 0 ? nnz_d : 1)));
    HUB_HIP(hipMalloc(&b_part.p, sizeof(double) * (size_t)nchunk * (size_t)(nnz_u > 0 ? nnz_u : 1)));

    hipLaunchKernelGGL(k_site_terms, dim3(nsite_blocks), dim3(AB), 0, st, g, x, cu, cd, M, U.basis, D.basis,
                       (double *)b_site.p);
    if (nnz_d > 0)
        hipLaunchKernelGGL(k_dn_terms, dim3(cd), dim3(AB), 0, st, g, x, cu, D.rp, D.col, D.bond, D.basis, s->d_bi,
                           s->d_bj, (double *)b_wd.p);
    if (nnz_u > 0) {
        const int gy = (cu + AB - 1) / AB < 64 ? (cu + AB - 1) / AB : 64;
        hipLaunchKernelGGL(k_up_terms, dim3(nchunk, gy), dim3(AB), 0, st, g, x, cu, cd, U.rp, U.col, U.max_row,
                           nchunk, (double *)b_part.p, nnz_u);
        hipLaunchKernelGGL(k_up_finish, dim3((cu + 255) / 256), dim3(256), 0, st, (const double *)b_part.p, nchunk,
                           nnz_u, cu, U.rp, U.bond, U.basis, s->d_bi, s->d_bj, (double *)b_wu.p);
    }
    HUB_HIP(hipGetLastError());

    std::vector<double> site((size_t)nsite_blocks * 2 * kMaxSites), wu((size_t)nnz_u), wd((size_t)nnz_d);
    std::vector<int32_t> bu((size_t)nnz_u), bd((size_t)nnz_d);
    HUB_HIP(hipMemcpyAsync(site.data(), b_site.p, sizeof(double) * site.size(), hipMemcpyDeviceToHost, st));
    if (nnz_u > 0) {
        HUB_HIP(hipMemcpyAsync(wu.data(), b_wu.p, sizeof(double) * nnz_u, hipMemcpyDeviceToHost, st));
        HUB_HIP(hipMemcpyAsync(bu.data(), U.bond, sizeof(int32_t) * nnz_u, hipMemcpyDeviceToHost, st));
    }
    if (nnz_d > 0) {
        HUB_HIP(hipMemcpyAsync(wd.data(), b_wd.p, sizeof(double) * nnz_d, hipMemcpyDeviceToHost, st));
        HUB_HIP(hipMemcpyAsync(bd.data(), D.bond, sizeof(int32_t) * nnz_d, hipMemcpyDeviceToHost, st));
    }
    HUB_HIP(hipStreamSynchronize(st));

    std::vector<double> acc_b((size_t)s->nb, 0.0);
    for (int64_t k = 0; k < nnz_u; ++k) acc_b[bu[k]] += wu[k];
    for (int64_t k = 0; k < nnz_d; ++k) acc_b[bd[k]] += wd[k];
    if (dbond)
        for (int b = 0; b < s->nb; ++b) dbond[b] = acc_b[b];
    for (int i = 0; i < M; ++i) {
        double su = 0.0, se = 0.0;
        for (int blk = 0; blk < nsite_blocks; ++blk) {
            su += site[(size_t)blk * 2 * kMaxSites + i];
            se += site[(size_t)blk * 2 * kMaxSites + kMaxSites + i];
        }
        if (dU) dU[i] = su;
        if (deps) deps[i] = se;
    }
    return HUB_OK;
}

}  // namespace hub
