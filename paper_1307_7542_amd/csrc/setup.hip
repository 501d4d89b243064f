// Sector set-up kernels: one-spin bases, ranks, hopping matrices H_sigma in CSR,
// per-state on-site energy sums.
//
// Basis (Sec. II, Algorithm I of Appendix A): the states of N electrons on M
// sites, as occupation integers in ascending order.  Instead of scanning 2^M
// integers, lane r builds the r-th state directly by the combinatorial number
// system: the ascending order of N-bit integers is the colexicographic order of
// their set-bit positions b_1 < ... < b_N, and the position of such an integer is
//     rank(x) = sum_{k=1..N} C(b_k, k).
// Unrank picks, for k = N down to 1, the largest c with C(c, k) <= r.
//
// Hopping matrix (Sec. III A, Sec. IV A): for state p and a canonical bond (i, j)
// with exactly one end occupied, the hopped state is l = p xor (2^i | 2^j), the
// sign is esign = (-1)^(popcount of p strictly between i and j), and the stored
// element is -t_ij * esign in column rank(l).  Rows are built in two passes
// (count, exclusive scan, fill); within a row entries are placed by the numeric
// order of the hopped states, which is their column order because rank is
// monotone.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace hub {
namespace {

__device__ __forceinline__ int64_t d_rank(uint32_t x, const uint64_t *__restrict__ C)
{
    int64_t r = 0;
    int k = 1;
    while (x) {
        const int b = __builtin_ctz(x);
        r += (int64_t)C[b * kBinomN + k];
        ++k;
        x &= x - 1u;
    }
    return r;
}

__global__ void k_unrank(uint32_t *__restrict__ basis, int64_t count, int M, int N,
                         const uint64_t *__restrict__ C)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count) return;
    uint64_t rem = (uint64_t)r;
    uint32_t x = 0;
    int c = M - 1;
    for (int k = N; k >= 1; --k) {
        while (C[c * kBinomN + k] > rem) --c;  // stops at c >= k-1 since C(k-1, k) = 0
        x |= 1u << c;
        rem -= C[c * kBinomN + k];
        --c;
    }
    basis[r] = x;
}

__global__ void k_rank(const uint64_t *__restrict__ xs, int64_t n, int M, int N, const uint64_t *__restrict__ C,
                       int64_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t x = xs[i];
    const uint64_t lim = (M >= 32) ? (uint64_t)0xFFFFFFFFull : ((1ull << M) - 1ull);
    if ((x & ~lim) != 0 || (int)__popcll(x) != N) {
        out[i] = -1;
        return;
    }
    out[i] = d_rank((uint32_t)x, C);
}

__device__ __forceinline__ uint32_t between_mask(int i, int j)
{
    // bits strictly between i < j
    const uint32_t below_j = (j >= 32) ? 0xFFFFFFFFu : ((1u << j) - 1u);
    const uint32_t upto_i = (i >= 31) ? 0xFFFFFFFFu : ((1u << (i + 1)) - 1u);
    return below_j & ~upto_i;
}

__global__ void k_csr_count(const uint32_t *__restrict__ basis, int64_t count, const int32_t *__restrict__ bi,
                            const int32_t *__restrict__ bj, int nb, int32_t *__restrict__ rowlen)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= count) return;
    const uint32_t x = basis[p];
    int n = 0;
    for (int e = 0; e < nb; ++e) n += (int)(((x >> bi[e]) ^ (x >> bj[e])) & 1u);
    rowlen[p] = n;
}

// Exclusive scan of rowlen into rp[0..count], in three kernels: per-block
// inclusive scan with block totals, a single-block scan of the totals, and the
// addition of the block offsets.
constexpr int kScanBlock = 1024;

__global__ void k_scan_local(const int32_t *__restrict__ in, int64_t n, int64_t *__restrict__ tmp,
                             int64_t *__restrict__ block_sums)
{
    __shared__ int64_t s[kScanBlock];
    const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    s[threadIdx.x] = (i < n) ? (int64_t)in[i] : 0;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int64_t v = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += v;
        __syncthreads();
    }
    if (i < n) tmp[i] = s[threadIdx.x];  // inclusive within the block
    if (threadIdx.x == kScanBlock - 1) block_sums[blockIdx.x] = s[kScanBlock - 1];
}

__global__ void k_scan_sums(int64_t *__restrict__ block_sums, int64_t nblocks)
{
    // single block; sequential carry over chunks of kScanBlock
    __shared__ int64_t s[kScanBlock];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nblocks; base += kScanBlock) {
        const int64_t i = base + threadIdx.x;
        s[threadIdx.x] = (i < nblocks) ? block_sums[i] : 0;
        __syncthreads();
        for (int off = 1; off < kScanBlock; off <<= 1) {
            int64_t v = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += v;
            __syncthreads();
        }
        const int64_t excl = carry + s[threadIdx.x] - ((i < nblocks) ? block_sums[i] : 0);
        __syncthreads();
        if (i < nblocks) block_sums[i] = excl;  // exclusive offset of block i
        if (threadIdx.x == kScanBlock - 1) carry += s[kScanBlock - 1];
        __syncthreads();
    }
}

__global__ void k_scan_finish(const int32_t *__restrict__ in, const int64_t *__restrict__ tmp,
                              const int64_t *__restrict__ block_off, int64_t n, int32_t *__restrict__ rp)
{
    const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    if (i < n) {
        const int64_t incl = tmp[i] + block_off[blockIdx.x];
        rp[i + 1] = (int32_t)incl;
        if (i == 0) rp[0] = 0;
        (void)in;
    }
}

__global__ void k_csr_fill(const uint32_t *__restrict__ basis, int64_t count, const int32_t *__restrict__ bi,
                           const int32_t *__restrict__ bj, const double *__restrict__ t, int nb,
                           const uint64_t *__restrict__ C, const int32_t *__restrict__ rp,
                           int32_t *__restrict__ col, double *__restrict__ val64, float *__restrict__ val32,
                           int32_t *__restrict__ bond)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= count) return;
    const uint32_t x = basis[p];
    const int base = rp[p];
    for (int e = 0; e < nb; ++e) {
        const int i = bi[e], j = bj[e];
        if ((((x >> i) ^ (x >> j)) & 1u) == 0) continue;
        const uint32_t l = x ^ ((1u << i) | (1u << j));
        int pos = 0;
        for (int e2 = 0; e2 < nb; ++e2) {
            const int i2 = bi[e2], j2 = bj[e2];
            if ((((x >> i2) ^ (x >> j2)) & 1u) == 0) continue;
            pos += (int)((x ^ ((1u << i2) | (1u << j2))) < l);
        }
        const int between = __popc(x & between_mask(i, j));
        const double v = (between & 1) ? t[e] : -t[e];  // -t * esign
        col[base + pos] = (int32_t)d_rank(l, C);
        val64[base + pos] = v;
        val32[base + pos] = (float)v;
        bond[base + pos] = e;
    }
}

__global__ void k_site_energy(const uint32_t *__restrict__ basis, int64_t count, int M,
                              const double *__restrict__ eps, double *__restrict__ e64, float *__restrict__ e32)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= count) return;
    const uint32_t x = basis[p];
    double s = 0.0;
    for (int i = 0; i < M; ++i)
        if ((x >> i) & 1u) s += eps[i];
    e64[p] = s;
    e32[p] = (float)s;
}

__global__ void k_max_row(const int32_t *__restrict__ rp, int64_t count, int32_t *__restrict__ out)
{
    __shared__ int32_t s[256];
    int32_t m = 0;
    for (int64_t p = threadIdx.x; p < count; p += 256) m = max(m, rp[p + 1] - rp[p]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < (unsigned)off) s[threadIdx.x] = max(s[threadIdx.x], s[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

__global__ void k_slice_len(const int32_t *__restrict__ rp, int64_t count, int64_t nslices, int32_t *__restrict__ len)
{
    const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= nslices) return;
    int m = 0;
    const int64_t r1 = min(count, (sl + 1) * 64);
    for (int64_t r = sl * 64; r < r1; ++r) m = max(m, rp[r + 1] - rp[r]);
    len[sl] = m;
}

__global__ void k_sell_fill(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                            const double *__restrict__ val, const int32_t *__restrict__ bond,
                            const double *__restrict__ t, int64_t count, const int32_t *__restrict__ sp,
                            int32_t *__restrict__ ecol, float *__restrict__ e32, double *__restrict__ e64,
                            uint2 *__restrict__ pk32, uint4 *__restrict__ pk64, uint32_t *__restrict__ c32)
{
    // one lane per (padded) row of a slice
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t sl = r / 64, lane = r % 64;
    const int64_t base = 64 * (int64_t)sp[sl];
    const int len = sp[sl + 1] - sp[sl];
    const int rl = (r < count) ? rp[r + 1] - rp[r] : 0;
    const int r0 = (r < count) ? rp[r] : 0;
    for (int k = 0; k < len; ++k) {
        const int64_t o = base + 64 * (int64_t)k + lane;
        int32_t c;
        double v;
        uint32_t code = 255u;
        if (k < rl) {
            c = col[r0 + k];
            v = val[r0 + k];
            const int e = bond[r0 + k];
            code = 2u * (uint32_t)e + ((v == t[e] && v != 0.0) ? 1u : 0u);  // val = -t esign
        } else {
            c = (r < count) ? (int32_t)r : 0;
            v = 0.0;
        }
        if (c32) c32[o] = ((uint32_t)c & 0xFFFFFFu) | (code << 24);
        ecol[o] = c;
        e64[o] = v;
        e32[o] = (float)v;
        pk32[o] = make_uint2((uint32_t)c, __float_as_uint((float)v));
        const unsigned long long vb = (unsigned long long)__double_as_longlong(v);
        pk64[o] = make_uint4((uint32_t)c, 0u, (uint32_t)(vb & 0xFFFFFFFFull), (uint32_t)(vb >> 32));
    }
}

// Per row: the sub-range of its (column-sorted) CSR entries with column in [c_lo, c_hi).
__global__ void k_chunk_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t count,
                             int c_lo, int c_hi, int32_t *__restrict__ rstart, int32_t *__restrict__ rlen)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count) return;
    int k0 = rp[r], k1 = rp[r + 1];
    int s0 = k1, s1 = k1;
    for (int k = k0; k < k1; ++k) {
        if (col[k] >= c_lo && s0 == k1) s0 = k;
        if (col[k] >= c_hi) { s1 = k; break; }
    }
    if (s0 > s1) s0 = s1;
    rstart[r] = s0;
    rlen[r] = s1 - s0;
}

__global__ void k_slice_max(const int32_t *__restrict__ len, int64_t count, int64_t nslices, int32_t *__restrict__ out)
{
    const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= nslices) return;
    int m = 0;
    const int64_t r1 = min(count, (sl + 1) * 64);
    for (int64_t r = sl * 64; r < r1; ++r) m = max(m, len[r]);
    out[sl] = m;
}

__global__ void k_chunk_fill(const int32_t *__restrict__ rstart, const int32_t *__restrict__ rlen,
                             const int32_t *__restrict__ col, const double *__restrict__ val,
                             const int32_t *__restrict__ bond, const double *__restrict__ t, int64_t count,
                             const int32_t *__restrict__ sp, int c_lo, uint32_t *__restrict__ out)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t sl = r / 64, lane = r % 64;
    const int64_t base = 64 * (int64_t)sp[sl];
    const int len = sp[sl + 1] - sp[sl];
    const int rl = (r < count) ? rlen[r] : 0;
    const int r0 = (r < count) ? rstart[r] : 0;
    for (int k = 0; k < len; ++k) {
        uint32_t e = 255u << 24;  // padding: column 0 of the chunk, value 0
        if (k < rl) {
            const double v = val[r0 + k];
            const int b = bond[r0 + k];
            const uint32_t code = 2u * (uint32_t)b + ((v == t[b] && v != 0.0) ? 1u : 0u);
            e = ((uint32_t)(col[r0 + k] - c_lo) & 0xFFFFFFu) | (code << 24);
        }
        out[base + 64 * (int64_t)k + lane] = e;
    }
}

template <typename T>
hub_status dalloc(hub_sector *s, T **p, size_t n)
{
    void *q = nullptr;
    const size_t bytes = (n == 0 ? 1 : n) * sizeof(T);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
        return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? HUB_ERR_OOM : HUB_ERR_DEVICE;
    }
    s->owned.push_back(q);
    *p = (T *)q;
    return HUB_OK;
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

hub_status scan_lengths(hub_sector *s, const int32_t *len, int64_t n, int32_t *rp, hipStream_t st)
{
    const int64_t nblk = (n + kScanBlock - 1) / kScanBlock;
    int64_t *tmp = nullptr, *bsum = nullptr;
    HUB_TRY(dalloc(s, &tmp, n));
    HUB_TRY(dalloc(s, &bsum, nblk));
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nblk), dim3(kScanBlock), 0, st, len, n, tmp, bsum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, st, bsum, nblk);
    hipLaunchKernelGGL(k_scan_finish, dim3((unsigned)nblk), dim3(kScanBlock), 0, st, len, tmp, bsum, n, rp);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status build_spin_tables(hub_sector *s, int spin, int N, hipStream_t st)
{
    SpinTables &T = s->spin[spin];
    T.N = N;
    // count = C(M, N) from the host copy of the table row
    uint64_t C[kBinomN][kBinomN] = {};
    for (int n = 0; n < kBinomN; ++n) {
        C[n][0] = 1;
        for (int k = 1; k <= n; ++k) C[n][k] = C[n - 1][k - 1] + (k <= n - 1 ? C[n - 1][k] : 0);
    }
    T.count = (int64_t)C[s->M][N];
    const int64_t count = T.count;
    if ((int64_t)count * (int64_t)(s->nb > 0 ? s->nb : 1) >= ((int64_t)1 << 31)) {
        set_error("hopping matrix would exceed 2^31 entries");
        return HUB_ERR_RANGE;
    }
    HUB_TRY(dalloc(s, &T.basis, count));
    HUB_TRY(dalloc(s, &T.rp, count + 1));
    HUB_TRY(dalloc(s, &T.e64, count));
    HUB_TRY(dalloc(s, &T.e32, count));
    int32_t *rowlen = nullptr;
    int64_t *tmp = nullptr, *bsum = nullptr;
    int32_t *dmax = nullptr;
    const int64_t nblk = (count + kScanBlock - 1) / kScanBlock;
    HUB_TRY(dalloc(s, &rowlen, count));
    HUB_TRY(dalloc(s, &tmp, count));
    HUB_TRY(dalloc(s, &bsum, nblk));
    HUB_TRY(dalloc(s, &dmax, 1));

    const int B = 256;
    hipLaunchKernelGGL(k_unrank, dim3(grid_for(count, B)), dim3(B), 0, st, T.basis, count, s->M, N, s->d_binom);
    hipLaunchKernelGGL(k_csr_count, dim3(grid_for(count, B)), dim3(B), 0, st, T.basis, count, s->d_bi, s->d_bj,
                       s->nb, rowlen);
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nblk), dim3(kScanBlock), 0, st, rowlen, count, tmp, bsum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, st, bsum, nblk);
    hipLaunchKernelGGL(k_scan_finish, dim3((unsigned)nblk), dim3(kScanBlock), 0, st, rowlen, tmp, bsum, count,
                       T.rp);
    HUB_HIP(hipGetLastError());
    int32_t nnz32 = 0;
    HUB_HIP(hipMemcpyAsync(&nnz32, T.rp + count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HUB_HIP(hipStreamSynchronize(st));
    T.nnz = nnz32;
    HUB_TRY(dalloc(s, &T.col, T.nnz));
    HUB_TRY(dalloc(s, &T.val64, T.nnz));
    HUB_TRY(dalloc(s, &T.val32, T.nnz));
    HUB_TRY(dalloc(s, &T.bond, T.nnz));
    hipLaunchKernelGGL(k_csr_fill, dim3(grid_for(count, B)), dim3(B), 0, st, T.basis, count, s->d_bi, s->d_bj,
                       s->d_t, s->nb, s->d_binom, T.rp, T.col, T.val64, T.val32, T.bond);
    hipLaunchKernelGGL(k_site_energy, dim3(grid_for(count, B)), dim3(B), 0, st, T.basis, count, s->M, s->d_eps,
                       T.e64, T.e32);
    hipLaunchKernelGGL(k_max_row, dim3(1), dim3(256), 0, st, T.rp, count, dmax);
    HUB_HIP(hipGetLastError());
    HUB_HIP(hipMemcpyAsync(&T.max_row, dmax, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HUB_HIP(hipStreamSynchronize(st));

    // sliced ELL copy (slices of 64 rows)
    T.nslices = (count + 63) / 64;
    const int64_t ns = T.nslices;
    int32_t *slen = nullptr, *sp = nullptr;
    int64_t *stmp = nullptr, *ssum = nullptr;
    const int64_t snblk = (ns + kScanBlock - 1) / kScanBlock;
    HUB_TRY(dalloc(s, &slen, ns));
    HUB_TRY(dalloc(s, &sp, ns + 1));
    HUB_TRY(dalloc(s, &stmp, ns));
    HUB_TRY(dalloc(s, &ssum, snblk));
    hipLaunchKernelGGL(k_slice_len, dim3(grid_for(ns, B)), dim3(B), 0, st, T.rp, count, ns, slen);
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)snblk), dim3(kScanBlock), 0, st, slen, ns, stmp, ssum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, st, ssum, snblk);
    hipLaunchKernelGGL(k_scan_finish, dim3((unsigned)snblk), dim3(kScanBlock), 0, st, slen, stmp, ssum, ns, sp);
    HUB_HIP(hipGetLastError());
    int32_t slots = 0;
    HUB_HIP(hipMemcpyAsync(&slots, sp + ns, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HUB_HIP(hipStreamSynchronize(st));
    if ((int64_t)slots * 64 >= ((int64_t)1 << 31)) {
        set_error("sliced hopping matrix would exceed 2^31 entries");
        return HUB_ERR_RANGE;
    }
    const int64_t nell = 64 * (int64_t)slots;
    T.sl_off = sp;  // in units of 64 entries
    HUB_TRY(dalloc(s, &T.ell_col, nell));
    HUB_TRY(dalloc(s, &T.ell_v32, nell));
    HUB_TRY(dalloc(s, &T.ell_v64, nell));
    HUB_TRY(dalloc(s, &T.ell_pk32, nell));
    HUB_TRY(dalloc(s, &T.ell_pk64, nell));
    const bool compact = count < (1 << 24) && s->nb <= 127;
    if (compact) {
        HUB_TRY(dalloc(s, &T.ell_c32, nell));
        HUB_TRY(dalloc(s, &T.code_v64, 256));
        HUB_TRY(dalloc(s, &T.code_v32, 256));
        std::vector<double> cv(256, 0.0);
        std::vector<float> cf(256, 0.0f);
        for (int e = 0; e < s->nb; ++e) {
            cv[2 * e] = -s->t[e];  // esign = +1
            cv[2 * e + 1] = s->t[e];
            cf[2 * e] = (float)cv[2 * e];
            cf[2 * e + 1] = (float)cv[2 * e + 1];
        }
        HUB_HIP(hipMemcpy(T.code_v64, cv.data(), 256 * sizeof(double), hipMemcpyHostToDevice));
        HUB_HIP(hipMemcpy(T.code_v32, cf.data(), 256 * sizeof(float), hipMemcpyHostToDevice));
    }
    hipLaunchKernelGGL(k_sell_fill, dim3((unsigned)ns), dim3(64), 0, st, T.rp, T.col, T.val64, T.bond, s->d_t, count,
                       sp, T.ell_col, T.ell_v32, T.ell_v64, T.ell_pk32, T.ell_pk64, T.ell_c32);
    HUB_HIP(hipGetLastError());
    HUB_HIP(hipStreamSynchronize(st));
    return HUB_OK;
}

// Chunk tables of H_spin (see ChunkSet), built on first request and kept for
// the life of the sector.  Called under the sector's cache mutex.
static hub_status build_chunk_set(hub_sector *s, int spin, int chunk_rows, ChunkSet &cs, hipStream_t st)
{
    const SpinTables &T = s->spin[spin];
    if (!T.ell_c32) {
        set_error("chunked products need the compact entry format (count < 2^24, <= 127 bonds)");
        return HUB_ERR_UNSUPPORTED;
    }
    if (chunk_rows < 1) {
        set_error("chunk of fewer than one column");
        return HUB_ERR_INVALID_ARG;
    }
    const int64_t count = T.count, ns = T.nslices;
    const int P = (int)((count + chunk_rows - 1) / chunk_rows);
    // temporaries freed on every path; the tables themselves are owned by the sector
    struct Tmp {
        std::vector<void *> p;
        ~Tmp()
        {
            for (void *q : p) (void)hipFree(q);
        }
    } tmp;
    auto talloc = [&](void **q, size_t bytes) -> hub_status {
        HUB_HIP(hipMalloc(q, bytes == 0 ? 1 : bytes));
        tmp.p.push_back(*q);
        return HUB_OK;
    };
    int32_t *rstart = nullptr, *rlen = nullptr, *slen = nullptr, *offs = nullptr;
    int64_t *stmp = nullptr, *ssum = nullptr;
    const int64_t snblk = (ns + kScanBlock - 1) / kScanBlock;
    HUB_TRY(talloc((void **)&rstart, sizeof(int32_t) * (size_t)count));
    HUB_TRY(talloc((void **)&rlen, sizeof(int32_t) * (size_t)count));
    HUB_TRY(talloc((void **)&slen, sizeof(int32_t) * (size_t)ns));
    HUB_TRY(talloc((void **)&stmp, sizeof(int64_t) * (size_t)ns));
    HUB_TRY(talloc((void **)&ssum, sizeof(int64_t) * (size_t)snblk));
    HUB_TRY(dalloc(s, &offs, (size_t)P * (ns + 1)));
    std::vector<int64_t> base(P + 1, 0);
    const int B = 256;
    for (int p = 0; p < P; ++p) {
        const int c_lo = p * chunk_rows;
        const int c_hi = (int)std::min<int64_t>(count, (int64_t)(p + 1) * chunk_rows);
        int32_t *sp = offs + (size_t)p * (ns + 1);
        hipLaunchKernelGGL(k_chunk_rows, dim3(grid_for(count, B)), dim3(B), 0, st, T.rp, T.col, count, c_lo, c_hi,
                           rstart, rlen);
        hipLaunchKernelGGL(k_slice_max, dim3(grid_for(ns, B)), dim3(B), 0, st, rlen, count, ns, slen);
        hipLaunchKernelGGL(k_scan_local, dim3((unsigned)snblk), dim3(kScanBlock), 0, st, slen, ns, stmp, ssum);
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, st, ssum, snblk);
        hipLaunchKernelGGL(k_scan_finish, dim3((unsigned)snblk), dim3(kScanBlock), 0, st, slen, stmp, ssum, ns, sp);
        HUB_HIP(hipGetLastError());
        int32_t slots = 0;
        HUB_HIP(hipMemcpyAsync(&slots, sp + ns, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HUB_HIP(hipStreamSynchronize(st));
        base[p + 1] = base[p] + 64 * (int64_t)slots;
    }
    if (base[P] >= ((int64_t)1 << 31)) {
        set_error("chunked hopping matrix would exceed 2^31 entries");
        return HUB_ERR_RANGE;
    }
    uint32_t *ell = nullptr;
    int64_t *dbase = nullptr;
    HUB_TRY(dalloc(s, &ell, (size_t)base[P]));
    HUB_TRY(dalloc(s, &dbase, P));
    HUB_HIP(hipMemcpyAsync(dbase, base.data(), sizeof(int64_t) * P, hipMemcpyHostToDevice, st));
    for (int p = 0; p < P; ++p) {
        const int c_lo = p * chunk_rows;
        const int c_hi = (int)std::min<int64_t>(count, (int64_t)(p + 1) * chunk_rows);
        hipLaunchKernelGGL(k_chunk_rows, dim3(grid_for(count, B)), dim3(B), 0, st, T.rp, T.col, count, c_lo, c_hi,
                           rstart, rlen);
        hipLaunchKernelGGL(k_chunk_fill, dim3((unsigned)ns), dim3(64), 0, st, rstart, rlen, T.col, T.val64, T.bond,
                           s->d_t, count, offs + (size_t)p * (ns + 1), c_lo, ell + base[p]);
    }
    HUB_HIP(hipGetLastError());
    HUB_HIP(hipStreamSynchronize(st));
    cs.spin = spin;
    cs.rows = chunk_rows;
    cs.n = P;
    cs.off = offs;
    cs.base = dbase;
    cs.ell = ell;
    return HUB_OK;
}

hub_status chunk_set(const hub_sector *cs, int spin, int rows, const ChunkSet **out, hipStream_t st)
{
    hub_sector *s = const_cast<hub_sector *>(cs);  // the chunk cache is not part of the sector's value
    if (s->shared_spin) spin = 0;
    for (const ChunkSet &c : s->chunks)
        if (c.spin == spin && c.rows == rows) {
            *out = &c;
            return HUB_OK;
        }
    ChunkSet c;
    HUB_TRY(build_chunk_set(s, spin, rows, c, st));
    s->chunks.push_back(c);
    *out = &s->chunks.back();
    return HUB_OK;
}

hub_status rank_device(const hub_sector *s, int spin, const uint64_t *dx, int64_t n, int64_t *dout,
                       hipStream_t st)
{
    if (n <= 0) return HUB_OK;
    const int B = 256;
    hipLaunchKernelGGL(k_rank, dim3(grid_for(n, B)), dim3(B), 0, st, dx, n, s->M, s->spin[spin].N, s->d_binom,
                       dout);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

}  // namespace hub
