// Batches of independent sectors (the impurity problems of an exact-
// diagonalisation DMFT step, Sec. VIII) solved together.
//
// Product: every sector keeps its own tables; a descriptor array gives each
// workgroup's sector, and a work-item list (sector, column tile) covers all
// sectors in one launch.  The kernel is the fused Kronecker-sum product of
// Sec. IV A (LDS-staged columns, sliced-ELL H_up gathers with compact entries,
// H_dn neighbour columns, diagonal from the bit patterns).
//
// Lanczos (Sec. IV): all sectors step in lockstep.  Vector kernels run over a
// "segment" grid (a fixed number of blocks per sector, so per-sector reductions
// are deterministic); alpha and beta live on the device per sector; converged
// sectors are masked out by an active flag.  The vector roles rotate over three
// buffers according to a device-resident step counter, so one step can be
// captured once as a HIP graph and replayed.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <new>
#include <cfloat>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "internal.h"

namespace hub {
namespace {

constexpr int BRB = 256;  // segment block size

template <typename T>
struct BDesc {
    int32_t cu, cd;
    int64_t off;
    const uint32_t *up_basis, *dn_basis;
    const T *e_up, *e_dn;
    const int32_t *dn_rp, *dn_col;
    const T *dn_val;
    const int32_t *sl_off;
    const uint32_t *ell;
    const T *code_v;
    const T *Us;
    T U;
    int32_t uniform;
    uint32_t umask;
};

template <typename T>
__device__ __forceinline__ T bdiag(const BDesc<T> &D, uint32_t both)
{
    if (D.uniform) return D.U * (T)__popc(both);
    T d = (T)0;
    uint32_t m = both & D.umask;
    while (m) {
        const int i = __builtin_ctz(m);
        d += D.Us[i];
        m &= m - 1u;
    }
    return d;
}

// Role of each vector slot at step k: v = V[k % 3], v_prev = V[(k + 2) % 3],
// v_next = V[(k + 1) % 3]; slot 3 of the pointer table is w.
template <typename T>
struct Roles {
    T *v, *vp, *vn, *w;
};

template <typename T>
__device__ __forceinline__ Roles<T> roles(T *const *ptrs, int k)
{
    Roles<T> r;
    r.v = ptrs[k % 3];
    r.vp = ptrs[(k + 2) % 3];
    r.vn = ptrs[(k + 1) % 3];
    r.w = ptrs[3];
    return r;
}

// Batched product.  SEL (the Lanczos step): x = v and y = w from the pointer
// table at the device step counter, and the first update fused in: w = H v -
// beta_k v_prev (rounded as a separate update would be) and this work item's
// partial of <w, v> in ipart[item] (a fixed-order block sum); otherwise x, y
// as given.
template <typename T, int TB, int BS, bool SEL>
__global__ __launch_bounds__(BS) void k_batch_kron(const BDesc<T> *__restrict__ desc, const int2 *__restrict__ items,
                                                   const T *xg, T *yg, T *const *ptrs, const int *step,
                                                   const int *__restrict__ active, const double *__restrict__ beta,
                                                   int kmax, double *__restrict__ ipart)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[SEL ? BS : 1];
    T *tab = reinterpret_cast<T *>(smem_raw);
    T *xs = tab + 256;
    const int2 it = items[blockIdx.x];
    if (active && !active[it.x]) return;
    const BDesc<T> D = desc[it.x];
    const T *x = xg;
    T *y = yg;
    const T *vp = nullptr;
    int k = 0;
    double bt = 0.0;
    if (SEL) {
        k = *step;
        const Roles<T> r = roles(ptrs, k);
        x = r.v;
        y = r.w;
        vp = r.vp + D.off;
        if (k > 0) bt = beta[(int64_t)it.x * kmax + k];
    }
    double dacc = 0.0;
    x += D.off;
    y += D.off;
    const int cu = D.cu, cd = D.cd;
    const int b0 = it.y * TB;
    for (int i = threadIdx.x; i < 256; i += BS) tab[i] = D.code_v[i];
#pragma unroll
    for (int t = 0; t < TB; ++t) {
        const int b = b0 + t;
        const T *xb = x + (int64_t)min(b, cd - 1) * cu;
        for (int a = threadIdx.x; a < cu; a += BS) xs[a * TB + t] = (b < cd) ? xb[a] : (T)0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (int a = threadIdx.x; a < cu; a += BS) {
        const uint32_t ua = D.up_basis[a];
        const T eua = D.e_up[a];
        T acc[TB];
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            const int b = min(b0 + t, cd - 1);
            acc[t] = (bdiag(D, ua & D.dn_basis[b]) + eua + D.e_dn[b]) * xs[a * TB + t];
        }
        const int s = a >> 6;
        const int o0 = D.sl_off[s] * 64 + lane;
        const int len = D.sl_off[s + 1] - D.sl_off[s];
        for (int k = 0; k < len; ++k) {
            const uint32_t e = D.ell[o0 + 64 * k];
            const T v = tab[e >> 24];
            const T *xr = xs + (e & 0xFFFFFFu) * TB;
#pragma unroll
            for (int t = 0; t < TB; ++t) acc[t] += v * xr[t];
        }
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            const int b = b0 + t;
            if (b >= cd) continue;
            T s2 = (T)0;
            for (int kk = D.dn_rp[b]; kk < D.dn_rp[b + 1]; ++kk) s2 += D.dn_val[kk] * x[(int64_t)D.dn_col[kk] * cu + a];
            T o = acc[t] + s2;
            if (SEL) {
                if (k > 0) o = (T)((double)o - bt * (double)vp[(int64_t)b * cu + a]);
                dacc += (double)o * (double)xs[a * TB + t];
            }
            y[(int64_t)b * cu + a] = o;
        }
    }
    if (SEL) {
        red[threadIdx.x] = dacc;
        __syncthreads();
        for (int o2 = BS / 2; o2 > 0; o2 >>= 1) {
            if (threadIdx.x < (unsigned)o2) red[threadIdx.x] += red[threadIdx.x + o2];
            __syncthreads();
        }
        if (threadIdx.x == 0) ipart[blockIdx.x] = red[0];
    }
}

// alpha[p * kmax + step] = the sum of sector p's work-item partials, in item order
__global__ __launch_bounds__(BRB) void k_b_ifinal(const int *__restrict__ istart, const int *__restrict__ icount,
                                                  const double *__restrict__ ipart, double *alpha, int kmax,
                                                  const int *step, const int *__restrict__ active)
{
    __shared__ double sh[BRB];
    const int p = blockIdx.x;
    if (active && !active[p]) return;
    double acc = 0.0;
    for (int j = threadIdx.x; j < icount[p]; j += BRB) acc += ipart[istart[p] + j];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = BRB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) alpha[(int64_t)p * kmax + *step] = sh[0];
}

struct Seg {
    const int32_t *prob;    // [nblocks] sector of the block
    const int32_t *local;   // [nblocks] block index within the sector
    const int32_t *nseg;    // [P] blocks per sector
    const int32_t *start;   // [P] first block of the sector
    const int64_t *off;     // [P + 1] vector offsets
};

__device__ __forceinline__ double bblock_sum(double v, double *s)
{
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = BRB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

#define SEG_LOOP(S, p, i)                                                                    \
    const int p = S.prob[blockIdx.x];                                                        \
    const int64_t n_##p = S.off[p + 1] - S.off[p];                                           \
    const int64_t o_##p = S.off[p];                                                          \
    const int64_t stride_##p = (int64_t)S.nseg[p] * BRB;                                     \
    for (int64_t i = (int64_t)S.local[blockIdx.x] * BRB + threadIdx.x; i < n_##p; i += stride_##p)

// partial[block] = sum over the block's elements of a * b (a == b allowed).
template <typename T>
__global__ __launch_bounds__(BRB) void k_b_dot(Seg S, const T *a, const T *b, double *partial,
                                               const int *__restrict__ active)
{
    __shared__ double sh[BRB];
    const int pp = S.prob[blockIdx.x];
    if (active && !active[pp]) return;
    double acc = 0.0;
    SEG_LOOP(S, p, i) acc += (double)a[o_p + i] * (double)b[o_p + i];
    const double r = bblock_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// out[p * ostride + slot] = (sqrt of) the sum of the sector's partials; slot from the step counter when step != null.
__global__ __launch_bounds__(BRB) void k_b_final(Seg S, const double *partial, double *out, int ostride, int slot,
                                                 const int *step, int step_add, int sqrt_result,
                                                 const int *__restrict__ active)
{
    __shared__ double sh[BRB];
    const int p = blockIdx.x;
    if (active && !active[p]) return;
    double acc = 0.0;
    for (int j = threadIdx.x; j < S.nseg[p]; j += BRB) acc += partial[S.start[p] + j];
    const double r = bblock_sum(acc, sh);
    if (threadIdx.x == 0) {
        const int sl = step ? (*step + step_add) : slot;
        out[(int64_t)p * ostride + sl] = sqrt_result ? sqrt(r) : r;
    }
}

// w -= alpha_k v; partial beta^2 = <w, w>.
template <typename T>
__global__ __launch_bounds__(BRB) void k_b_lz_b(Seg S, T *const *ptrs, const int *step, const double *alpha,
                                                int kmax, double *partial, const int *__restrict__ active)
{
    __shared__ double sh[BRB];
    const int pp = S.prob[blockIdx.x];
    if (active && !active[pp]) return;
    const int k = *step;
    const Roles<T> r = roles(ptrs, k);
    const double al = alpha[(int64_t)pp * kmax + k];
    double acc = 0.0;
    SEG_LOOP(S, p, i)
    {
        const T wi = (T)((double)r.w[o_p + i] - al * (double)r.v[o_p + i]);
        r.w[o_p + i] = wi;
        acc += (double)wi * (double)wi;
    }
    const double s = bblock_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// v_next = w / beta_{k+1} (zero after a breakdown).
template <typename T>
__global__ __launch_bounds__(BRB) void k_b_lz_next(Seg S, T *const *ptrs, const int *step, const double *beta,
                                                   int kmax, const int *__restrict__ active)
{
    const int pp = S.prob[blockIdx.x];
    if (active && !active[pp]) return;
    const int k = *step;
    const Roles<T> r = roles(ptrs, k);
    const double bt = beta[(int64_t)pp * kmax + k + 1];
    SEG_LOOP(S, p, i) r.vn[o_p + i] = (bt > 0.0) ? (T)((double)r.w[o_p + i] / bt) : (T)0;
}

__global__ void k_b_step(int *step, int add, int set)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *step = (set >= 0) ? set : (*step + add);
}

// Start vectors: sector-local SplitMix64 entries (same as a single-sector solve).
template <typename T>
__global__ __launch_bounds__(BRB) void k_b_start(Seg S, T *out, uint64_t seed)
{
    SEG_LOOP(S, p, i)
    {
        uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z = z ^ (z >> 31);
        out[o_p + i] = (T)(-1.0 + 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)));
    }
}

// x /= norm[p] (norms of unit stride per sector)
template <typename T>
__global__ __launch_bounds__(BRB) void k_b_div(Seg S, T *x, const double *nrm)
{
    const int pp = S.prob[blockIdx.x];
    const double f = nrm[pp];
    SEG_LOOP(S, p, i) x[o_p + i] = (f > 0.0) ? (T)((double)x[o_p + i] / f) : (T)0;
}

// Second pass (replay with the stored alpha / beta at step k, explicit k):
// w = H v (done by the product), w = (w - beta_k v_prev) - alpha_k v, v_next = w / beta_{k+1}.
template <typename T>
__global__ __launch_bounds__(BRB) void k_b_replay(Seg S, T *w, const T *v, const T *vp, T *vn, const double *alpha,
                                                  const double *beta, int kmax, int k, const int *__restrict__ mlen)
{
    const int pp = S.prob[blockIdx.x];
    if (k + 1 >= mlen[pp]) return;
    const double bt = (k > 0) ? beta[(int64_t)pp * kmax + k] : 0.0;
    const double al = alpha[(int64_t)pp * kmax + k];
    const double bn = beta[(int64_t)pp * kmax + k + 1];
    SEG_LOOP(S, p, i)
    {
        T wi = w[o_p + i];
        if (k > 0) wi = (T)((double)wi - bt * (double)vp[o_p + i]);
        wi = (T)((double)wi - al * (double)v[o_p + i]);
        vn[o_p + i] = (bn > 0.0) ? (T)((double)wi / bn) : (T)0;
    }
}

template <typename T>
__global__ __launch_bounds__(BRB) void k_b_psi(Seg S, double *psi, const T *v, const double *y, int kmax, int k,
                                               const int *__restrict__ mlen)
{
    const int pp = S.prob[blockIdx.x];
    if (k >= mlen[pp]) return;
    const double c = y[(int64_t)pp * kmax + k];
    SEG_LOOP(S, p, i) psi[o_p + i] = (k == 0 ? 0.0 : psi[o_p + i]) + c * (double)v[o_p + i];
}

// psi *= scale[p]
// Per block: the largest |psi| of the block's elements and its sector-local
// index (ties: the lower index).
__device__ __forceinline__ bool amax_better(double a1, int64_t i1, double a2, int64_t i2)
{
    return a1 > a2 || (a1 == a2 && i1 < i2);
}

__global__ __launch_bounds__(BRB) void k_b_amax(Seg S, const double *psi, double *pa, int64_t *pi)
{
    __shared__ double sa[BRB];
    __shared__ int64_t si[BRB];
    double best = -1.0;
    int64_t bi = INT64_MAX;
    SEG_LOOP(S, p, i)
    {
        const double a = fabs(psi[o_p + i]);
        if (amax_better(a, i, best, bi)) {
            best = a;
            bi = i;
        }
    }
    sa[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int o = BRB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o && amax_better(sa[threadIdx.x + o], si[threadIdx.x + o], sa[threadIdx.x], si[threadIdx.x])) {
            sa[threadIdx.x] = sa[threadIdx.x + o];
            si[threadIdx.x] = si[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pa[blockIdx.x] = sa[0];
        pi[blockIdx.x] = si[0];
    }
}

// One block per sector: scale[p] = sign / ||psi_p|| with the norm from the
// squared-norm partials (k_b_final's order) and the sign of the largest-magnitude
// entry (lowest index on ties), so that k_b_scale_psi leaves a unit vector whose
// largest entry is positive.
__global__ __launch_bounds__(BRB) void k_b_norm_sign(Seg S, const double *partial, const double *pa,
                                                     const int64_t *pi, const double *psi, double *scale)
{
    __shared__ double sh[BRB];
    __shared__ double sa[BRB];
    __shared__ int64_t si[BRB];
    const int p = blockIdx.x;
    double acc = 0.0, best = -1.0;
    int64_t bi = INT64_MAX;
    for (int j = threadIdx.x; j < S.nseg[p]; j += BRB) {
        acc += partial[S.start[p] + j];
        if (amax_better(pa[S.start[p] + j], pi[S.start[p] + j], best, bi)) {
            best = pa[S.start[p] + j];
            bi = pi[S.start[p] + j];
        }
    }
    const double s2 = bblock_sum(acc, sh);
    sa[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int o = BRB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o && amax_better(sa[threadIdx.x + o], si[threadIdx.x + o], sa[threadIdx.x], si[threadIdx.x])) {
            sa[threadIdx.x] = sa[threadIdx.x + o];
            si[threadIdx.x] = si[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double nr = sqrt(s2);
        const int64_t n_p = S.off[p + 1] - S.off[p];
        const double v = (si[0] >= 0 && si[0] < n_p) ? psi[S.off[p] + si[0]] : 0.0;
        scale[p] = (nr > 0.0 ? 1.0 / nr : 0.0) * (v < 0.0 ? -1.0 : 1.0);
    }
}

__global__ __launch_bounds__(BRB) void k_b_scale_psi(Seg S, double *psi, const double *scale)
{
    const int pp = S.prob[blockIdx.x];
    const double f = scale[pp];
    SEG_LOOP(S, p, i) psi[o_p + i] *= f;
}

}  // namespace
}  // namespace hub

// ----------------------------------------------------------------------------

struct hub_batch {
    int device = 0;
    int P = 0;
    std::vector<const hub_sector *> secs;
    std::vector<int64_t> off;  // P + 1
    int max_cu = 0;
    size_t lds_max = 65536;
    std::vector<void *> owned;
    void *desc[2] = {nullptr, nullptr};  // device BDesc<double>[P], BDesc<float>[P]
    // segment tables
    int nblocks = 0;
    int32_t *seg_prob = nullptr, *seg_local = nullptr, *seg_n = nullptr, *seg_start = nullptr;
    int64_t *d_off = nullptr;
    // tuned product per dtype
    bool tuned[2] = {false, false};
    int tb[2] = {1, 1}, bs[2] = {256, 256};
    int2 *items[2] = {nullptr, nullptr};
    int nitems[2] = {0, 0};
    int *istart[2] = {nullptr, nullptr}, *icount[2] = {nullptr, nullptr};  // items of each sector
    double tune_seconds = 0.0;
};

namespace hub {
namespace {

hub_status bfail(hub_status c, const std::string &m)
{
    set_error(m);
    return c;
}

template <typename T>
hub_status balloc(hub_batch *b, T **p, size_t n)
{
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, (n == 0 ? 1 : n) * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return bfail(HUB_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    b->owned.push_back(q);
    *p = (T *)q;
    return HUB_OK;
}

Seg seg_of(const hub_batch *b)
{
    Seg S;
    S.prob = b->seg_prob;
    S.local = b->seg_local;
    S.nseg = b->seg_n;
    S.start = b->seg_start;
    S.off = b->d_off;
    return S;
}

template <typename T>
BDesc<T> make_desc(const hub_sector *s, int64_t off)
{
    const SpinTables &U = s->spin[0], &D = s->spin[1];
    BDesc<T> d;
    d.cu = (int32_t)U.count;
    d.cd = (int32_t)D.count;
    d.off = off;
    d.up_basis = U.basis;
    d.dn_basis = D.basis;
    d.dn_rp = D.rp;
    d.dn_col = D.col;
    d.sl_off = U.sl_off;
    d.ell = U.ell_c32;
    d.uniform = s->uniformU;
    d.umask = s->umask;
    d.U = (T)s->U0;
    if constexpr (sizeof(T) == 8) {
        d.e_up = U.e64;
        d.e_dn = D.e64;
        d.dn_val = D.val64;
        d.code_v = U.code_v64;
        d.Us = s->d_U64;
    } else {
        d.e_up = U.e32;
        d.e_dn = D.e32;
        d.dn_val = D.val32;
        d.code_v = U.code_v32;
        d.Us = s->d_U32;
    }
    return d;
}

template <typename T, int TB, int BS, bool SEL>
hub_status launch_bk(hub_batch *b, int di, const T *x, T *y, T *const *ptrs, const int *step, const int *active,
                     hipStream_t st, const double *beta, int kmax, double *ipart)
{
    const size_t lds = (size_t)(256 + (size_t)b->max_cu * TB) * sizeof(T);
    static std::atomic<bool> attr{false};
    if (!attr) {
        HUB_HIP(hipFuncSetAttribute((const void *)k_batch_kron<T, TB, BS, SEL>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds_max));
        attr = true;
    }
    hipLaunchKernelGGL((k_batch_kron<T, TB, BS, SEL>), dim3(b->nitems[di]), dim3(BS), lds, st,
                       (const BDesc<T> *)b->desc[di], b->items[di], x, y, ptrs, step, active, beta, kmax, ipart);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

// SEL: the Lanczos step (vectors from the pointer table, first update fused,
// item partials of alpha in ipart; beta and kmax as in the solver's arrays)
template <typename T, bool SEL>
hub_status launch_batch_product(hub_batch *b, const T *x, T *y, T *const *ptrs, const int *step, const int *active,
                                hipStream_t st, const double *beta = nullptr, int kmax = 0, double *ipart = nullptr)
{
    const int di = (sizeof(T) == 8) ? 0 : 1;
    const int tb = b->tb[di], bs = b->bs[di];
#define HUB_BK(TBV, BSV)                                                                 \
    if (tb == TBV && bs == BSV)                                                          \
        return launch_bk<T, TBV, BSV, SEL>(b, di, x, y, ptrs, step, active, st, beta, kmax, ipart);
    HUB_BK(1, 256) HUB_BK(2, 256) HUB_BK(4, 256) HUB_BK(8, 256)
    HUB_BK(1, 512) HUB_BK(2, 512) HUB_BK(4, 512) HUB_BK(8, 512)
#undef HUB_BK
    return bfail(HUB_ERR_UNSUPPORTED, "untuned product shape");
}

hub_status build_items(hub_batch *b, int di, int tb)
{
    std::vector<int2> it;
    for (int p = 0; p < b->P; ++p) {
        const int cd = (int)b->secs[p]->spin[1].count;
        for (int t = 0; t * tb < cd; ++t) it.push_back(make_int2(p, t));
    }
    if (b->items[di]) {
        HUB_HIP(hipFree(b->items[di]));
        for (auto &q : b->owned)
            if (q == (void *)b->items[di]) q = nullptr;
        b->items[di] = nullptr;
    }
    HUB_TRY(balloc(b, &b->items[di], it.size()));
    HUB_HIP(hipMemcpy(b->items[di], it.data(), sizeof(int2) * it.size(), hipMemcpyHostToDevice));
    b->nitems[di] = (int)it.size();
    // the items of sector p are [istart[p], istart[p] + icount[p]) (sector-major order)
    std::vector<int> hs(b->P, 0), hc(b->P, 0);
    for (int i = 0; i < (int)it.size(); ++i) {
        if (hc[it[i].x] == 0) hs[it[i].x] = i;
        ++hc[it[i].x];
    }
    if (!b->istart[di]) HUB_TRY(balloc(b, &b->istart[di], (size_t)b->P));
    if (!b->icount[di]) HUB_TRY(balloc(b, &b->icount[di], (size_t)b->P));
    HUB_HIP(hipMemcpy(b->istart[di], hs.data(), sizeof(int) * b->P, hipMemcpyHostToDevice));
    HUB_HIP(hipMemcpy(b->icount[di], hc.data(), sizeof(int) * b->P, hipMemcpyHostToDevice));
    b->tb[di] = tb;
    return HUB_OK;
}

// Autotuner: time every (TB, BS) whose panel fits the LDS on the batch itself.
template <typename T>
hub_status tune(hub_batch *b, hipStream_t st)
{
    const int di = (sizeof(T) == 8) ? 0 : 1;
    if (b->tuned[di]) return HUB_OK;
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = b->off[b->P];
    T *x = nullptr, *y = nullptr;
    HUB_HIP(hipMalloc(&x, sizeof(T) * n));
    if (hipMalloc(&y, sizeof(T) * n) != hipSuccess) {
        (void)hipFree(x);
        return bfail(HUB_ERR_OOM, "tuning buffers");
    }
    struct Free {
        void *a, *c;
        ~Free() { (void)hipFree(a); (void)hipFree(c); }
    } fr{x, y};
    hipLaunchKernelGGL(k_b_start<T>, dim3(b->nblocks), dim3(BRB), 0, st, seg_of(b), x, (uint64_t)1);
    hipEvent_t e0, e1;
    HUB_HIP(hipEventCreate(&e0));
    HUB_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    int btb = 1, bbs = 256;
    for (int tb : {1, 2, 4, 8}) {
        if ((size_t)(256 + (size_t)b->max_cu * tb) * sizeof(T) > b->lds_max) continue;
        HUB_TRY(build_items(b, di, tb));
        for (int bs : {256, 512}) {
            b->bs[di] = bs;
            HUB_TRY((launch_batch_product<T, false>(b, x, y, nullptr, nullptr, nullptr, st)));
            HUB_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < 3; ++r) HUB_TRY((launch_batch_product<T, false>(b, x, y, nullptr, nullptr, nullptr, st)));
            HUB_HIP(hipEventRecord(e1, st));
            HUB_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            HUB_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                btb = tb;
                bbs = bs;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HUB_TRY(build_items(b, di, btb));
    b->bs[di] = bbs;
    b->tuned[di] = true;
    b->tune_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return HUB_OK;
}

template <typename T>
hub_status batch_solve(hub_batch *b, const hub_lanczos_opts *o, double *e0_out, int32_t *iters_out, double *psi,
                       hipStream_t user_st, hub_batch_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const double tune0 = b->tune_seconds;
    const int di = (sizeof(T) == 8) ? 0 : 1;
    const int P = b->P;
    const int64_t n = b->off[P];
    int64_t maxdim = 0;
    for (int p = 0; p < P; ++p) maxdim = std::max<int64_t>(maxdim, b->off[p + 1] - b->off[p]);
    int max_iter = o->max_iter > 0 ? o->max_iter : 400;
    if ((int64_t)max_iter > maxdim) max_iter = (int)maxdim;
    const double tol = o->tol > 0 ? o->tol : (sizeof(T) == 8 ? 1e-12 : 1e-7);
    const int check_every = o->check_every > 0 ? o->check_every : 5;
    const int kmax = max_iter + 2;
    const Seg S = seg_of(b);

    // a private stream for capture, ordered after the caller's stream
    hipStream_t st;
    HUB_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } sg{st};
    hipEvent_t ev;
    HUB_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HUB_HIP(hipEventRecord(ev, user_st));
    HUB_HIP(hipStreamWaitEvent(st, ev, 0));
    HUB_TRY(tune<T>(b, st));
    if (o->refine) HUB_TRY(tune<double>(b, st));

    std::vector<void *> mem;
    struct MemGuard {
        std::vector<void *> &m;
        ~MemGuard() { for (void *q : m) (void)hipFree(q); }
    } mg{mem};
    auto alloc = [&](void **q, size_t bytes) -> hub_status {
        hipError_t e = hipMalloc(q, bytes == 0 ? 1 : bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return bfail(HUB_ERR_OOM, "batch workspace");
        }
        mem.push_back(*q);
        return HUB_OK;
    };
    T *V[4];
    for (int i = 0; i < 4; ++i) HUB_TRY(alloc((void **)&V[i], sizeof(T) * n));
    T **ptrs = nullptr;
    int *step = nullptr, *active = nullptr, *mlen = nullptr;
    double *alpha = nullptr, *beta = nullptr, *partial = nullptr, *nrm = nullptr, *ycoef = nullptr;
    HUB_TRY(alloc((void **)&ptrs, sizeof(T *) * 4));
    HUB_TRY(alloc((void **)&step, sizeof(int) * 4));
    HUB_TRY(alloc((void **)&active, sizeof(int) * P));
    HUB_TRY(alloc((void **)&mlen, sizeof(int) * P));
    HUB_TRY(alloc((void **)&alpha, sizeof(double) * (size_t)P * kmax));
    HUB_TRY(alloc((void **)&beta, sizeof(double) * (size_t)P * kmax));
    HUB_TRY(alloc((void **)&partial, sizeof(double) * (size_t)b->nblocks));
    double *ipart = nullptr;  // alpha partials of the fused product, one per work item
    HUB_TRY(alloc((void **)&ipart, sizeof(double) * (size_t)std::max(1, b->nitems[di])));
    HUB_TRY(alloc((void **)&nrm, sizeof(double) * (size_t)P * 4));
    HUB_TRY(alloc((void **)&ycoef, sizeof(double) * (size_t)P * kmax));
    HUB_HIP(hipMemcpyAsync(ptrs, V, sizeof(T *) * 4, hipMemcpyHostToDevice, st));
    std::vector<int> hact(P, 1);
    HUB_HIP(hipMemcpyAsync(active, hact.data(), sizeof(int) * P, hipMemcpyHostToDevice, st));
    HUB_HIP(hipMemsetAsync(beta, 0, sizeof(double) * (size_t)P * kmax, st));
    HUB_HIP(hipMemsetAsync(alpha, 0, sizeof(double) * (size_t)P * kmax, st));

    // start vectors v0 = x / ||x|| per sector
    auto make_start = [&](T *v) -> hub_status {
        hipLaunchKernelGGL(k_b_start<T>, dim3(b->nblocks), dim3(BRB), 0, st, S, v, o->seed);
        hipLaunchKernelGGL(k_b_dot<T>, dim3(b->nblocks), dim3(BRB), 0, st, S, (const T *)v, (const T *)v, partial,
                           (const int *)nullptr);
        hipLaunchKernelGGL(k_b_final, dim3(P), dim3(BRB), 0, st, S, partial, nrm, 1, 0, (const int *)nullptr, 0, 1,
                           (const int *)nullptr);
        hipLaunchKernelGGL(k_b_div<T>, dim3(b->nblocks), dim3(BRB), 0, st, S, v, (const double *)nrm);
        HUB_HIP(hipGetLastError());
        return HUB_OK;
    };
    HUB_TRY(make_start(V[0]));
    hipLaunchKernelGGL(k_b_step, dim3(1), dim3(64), 0, st, step, 0, 0);

    // one Lanczos step, captured as a graph
    auto one_step = [&]() -> hub_status {
        HUB_TRY((launch_batch_product<T, true>(b, nullptr, nullptr, ptrs, step, active, st, beta, kmax, ipart)));
        hipLaunchKernelGGL(k_b_ifinal, dim3(P), dim3(BRB), 0, st, (const int *)b->istart[di],
                           (const int *)b->icount[di], (const double *)ipart, alpha, kmax, (const int *)step,
                           (const int *)active);
        hipLaunchKernelGGL(k_b_lz_b<T>, dim3(b->nblocks), dim3(BRB), 0, st, S, ptrs, (const int *)step,
                           (const double *)alpha, kmax, partial, (const int *)active);
        hipLaunchKernelGGL(k_b_final, dim3(P), dim3(BRB), 0, st, S, (const double *)partial, beta, kmax, 0,
                           (const int *)step, 1, 1, (const int *)active);
        hipLaunchKernelGGL(k_b_lz_next<T>, dim3(b->nblocks), dim3(BRB), 0, st, S, ptrs, (const int *)step,
                           (const double *)beta, kmax, (const int *)active);
        hipLaunchKernelGGL(k_b_step, dim3(1), dim3(64), 0, st, step, 1, -1);
        HUB_HIP(hipGetLastError());
        return HUB_OK;
    };
    // one eager step first (also sets the kernel attributes outside the capture);
    // the captured graph then replays steps 1, 2, ...
    HUB_TRY(one_step());
    int k = 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // HUB_BATCH_GRAPH=0 replays the step eagerly (same kernels, same order)
    const char *genv = std::getenv("HUB_BATCH_GRAPH");
    bool use_graph = !(genv && genv[0] == '0');
    if (use_graph && hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        hub_status cs = one_step();
        hipError_t ec = hipStreamEndCapture(st, &graph);
        if (cs != HUB_OK || ec != hipSuccess || hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) != hipSuccess)
            use_graph = false;
    } else {
        use_graph = false;
    }
    (void)hipGetLastError();
    // a whole group of check_every steps in one graph as well (one launch per group)
    hipGraph_t graph_g = nullptr;
    hipGraphExec_t gexec_g = nullptr;
    if (use_graph && check_every > 1 && hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        hub_status cs = HUB_OK;
        for (int s2 = 0; s2 < check_every && cs == HUB_OK; ++s2) cs = one_step();
        hipError_t ec = hipStreamEndCapture(st, &graph_g);
        if (cs != HUB_OK || ec != hipSuccess ||
            hipGraphInstantiate(&gexec_g, graph_g, nullptr, nullptr, 0) != hipSuccess)
            gexec_g = nullptr;
    }
    (void)hipGetLastError();
    struct GraphGuard {
        hipGraph_t g;
        hipGraphExec_t x;
        ~GraphGuard() {
            if (x) (void)hipGraphExecDestroy(x);
            if (g) (void)hipGraphDestroy(g);
        }
    } gg{graph, gexec}, gg_group{graph_g, gexec_g};

    std::vector<int> m_final(P, 0), conv(P, 0);
    std::vector<double> theta(P, 0.0);
    std::vector<std::vector<double>> ys(P);
    std::vector<double> tmax(P, 0.0);
    int replays = 0, nactive = P;

    // Convergence checks overlap the GPU: after every group of check_every steps
    // the coefficients are copied into one of two pinned buffers, the next group
    // is enqueued before the host examines the previous copy, and the new active
    // mask (through pinned memory as well) reaches the device one group later.
    // A sector found converged may so run one more group; those steps are never
    // used (its T and psi stop at the step of the test).
    const size_t nab = (size_t)P * kmax;
    double *hab = nullptr;  // [2 slots][alpha | beta]
    int *hmask = nullptr;   // [2][P]
    HUB_HIP(hipHostMalloc((void **)&hab, sizeof(double) * 4 * nab));
    struct PinGuard {
        void *p;
        hipStream_t st;
        ~PinGuard()
        {
            if (!p) return;
            (void)hipStreamSynchronize(st);
            (void)hipHostFree(p);
        }
    } pin_ab{hab, st}, pin_mask{nullptr, st};
    HUB_HIP(hipHostMalloc((void **)&hmask, sizeof(int) * 2 * (size_t)P));
    pin_mask.p = hmask;
    hipEvent_t cev[2] = {nullptr, nullptr};
    HUB_HIP(hipEventCreateWithFlags(&cev[0], hipEventDisableTiming));
    HUB_HIP(hipEventCreateWithFlags(&cev[1], hipEventDisableTiming));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard()
        {
            for (int i = 0; i < 2; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } evg{cev};
    int kslot[2] = {0, 0};
    auto enqueue_copy = [&](int sl) -> hub_status {
        HUB_HIP(hipMemcpyAsync(hab + (size_t)sl * 2 * nab, alpha, sizeof(double) * nab, hipMemcpyDeviceToHost, st));
        HUB_HIP(hipMemcpyAsync(hab + (size_t)sl * 2 * nab + nab, beta, sizeof(double) * nab, hipMemcpyDeviceToHost,
                               st));
        HUB_HIP(hipEventRecord(cev[sl], st));
        kslot[sl] = k;
        return HUB_OK;
    };
    auto enqueue_steps = [&](int nsteps) -> hub_status {
        if (gexec_g && nsteps == check_every) {
            HUB_HIP(hipGraphLaunch(gexec_g, st));
            replays += nsteps;
            k += nsteps;
            return HUB_OK;
        }
        for (int s2 = 0; s2 < nsteps; ++s2) {
            if (use_graph) {
                HUB_HIP(hipGraphLaunch(gexec, st));
                ++replays;
            } else {
                HUB_TRY(one_step());
            }
        }
        k += nsteps;
        return HUB_OK;
    };
    // Ritz test of every active sector on a copy holding kk steps
    auto check_copy = [&](const double *ha, const double *hb, int kk) {
        for (int p = 0; p < P; ++p) {
            if (!hact[p]) continue;
            const double *a = ha + (size_t)p * kmax;
            const double *bb = hb + (size_t)p * kmax;
            const int64_t dimp = b->off[p + 1] - b->off[p];
            int m = (int)std::min<int64_t>(kk, dimp);
            bool brk = false;
            for (int j = 0; j < m; ++j) {
                tmax[p] = std::max(tmax[p], std::fabs(a[j]) + 2.0 * std::fabs(bb[j + 1]));
                const double thr = 64.0 * (sizeof(T) == 8 ? DBL_EPSILON : FLT_EPSILON) * std::max(tmax[p], DBL_MIN);
                if (!(bb[j + 1] > thr)) {
                    m = j + 1;
                    brk = true;
                    break;
                }
            }
            std::vector<double> y;
            const double th = tri_lowest(a, bb + 1, m, y);
            const double res = brk ? 0.0 : std::fabs(bb[m]) * std::fabs(y[m - 1]);
            const double scale = std::fabs(th) > 0 ? std::fabs(th) : 1.0;
            theta[p] = th;
            m_final[p] = m;
            ys[p] = y;
            if (brk || res <= tol * scale || (int64_t)m >= dimp) {
                conv[p] = 1;
                hact[p] = 0;
                --nactive;
            }
        }
    };
    HUB_TRY(enqueue_copy(0));
    int sl = 0, msl = 0;
    while (true) {
        const int nsteps = nactive > 0 ? std::min(check_every, max_iter - k) : 0;
        if (nsteps > 0) {
            HUB_TRY(enqueue_steps(nsteps));
            HUB_TRY(enqueue_copy(sl ^ 1));
        }
        HUB_HIP(hipEventSynchronize(cev[sl]));  // the group just enqueued keeps running
        const double *ha = hab + (size_t)sl * 2 * nab;
        check_copy(ha, ha + nab, kslot[sl]);
        if (nactive == 0 || nsteps == 0) break;
        int *hm = hmask + (size_t)msl * P;
        std::memcpy(hm, hact.data(), sizeof(int) * (size_t)P);
        HUB_HIP(hipMemcpyAsync(active, hm, sizeof(int) * P, hipMemcpyHostToDevice, st));
        msl ^= 1;
        sl ^= 1;
    }
    std::vector<double> e0(theta);

    if (psi && (o->want_vector || o->refine)) {
        // second pass with the stored alpha / beta; psi = sum_j y_j v_j per sector
        int mmax = 0;
        std::vector<double> hy((size_t)P * kmax, 0.0);
        for (int p = 0; p < P; ++p) {
            mmax = std::max(mmax, m_final[p]);
            for (int j = 0; j < m_final[p]; ++j) hy[(size_t)p * kmax + j] = ys[p][j];
        }
        HUB_HIP(hipMemcpyAsync(ycoef, hy.data(), sizeof(double) * hy.size(), hipMemcpyHostToDevice, st));
        HUB_HIP(hipMemcpyAsync(mlen, m_final.data(), sizeof(int) * P, hipMemcpyHostToDevice, st));
        HUB_TRY(make_start(V[0]));
        T *vp = V[2], *vc = V[0], *vn = V[1];
        for (int j = 0; j < mmax; ++j) {
            hipLaunchKernelGGL(k_b_psi<T>, dim3(b->nblocks), dim3(BRB), 0, st, S, psi, (const T *)vc,
                               (const double *)ycoef, kmax, j, (const int *)mlen);
            if (j + 1 >= mmax) break;
            HUB_TRY((launch_batch_product<T, false>(b, vc, V[3], nullptr, nullptr, nullptr, st)));
            hipLaunchKernelGGL(k_b_replay<T>, dim3(b->nblocks), dim3(BRB), 0, st, S, V[3], (const T *)vc,
                               (const T *)vp, vn, (const double *)alpha, (const double *)beta, kmax, j,
                               (const int *)mlen);
            T *tmp = vp;
            vp = vc;
            vc = vn;
            vn = tmp;
        }
        // normalise and fix the sign (largest-magnitude entry positive, lowest index on ties), on the device
        double *pa = nullptr;
        int64_t *pi = nullptr;
        HUB_TRY(alloc((void **)&pa, sizeof(double) * (size_t)b->nblocks));
        HUB_TRY(alloc((void **)&pi, sizeof(int64_t) * (size_t)b->nblocks));
        hipLaunchKernelGGL(k_b_dot<double>, dim3(b->nblocks), dim3(BRB), 0, st, S, (const double *)psi,
                           (const double *)psi, partial, (const int *)nullptr);
        hipLaunchKernelGGL(k_b_amax, dim3(b->nblocks), dim3(BRB), 0, st, S, (const double *)psi, pa, pi);
        hipLaunchKernelGGL(k_b_norm_sign, dim3(P), dim3(BRB), 0, st, S, (const double *)partial,
                           (const double *)pa, (const int64_t *)pi, (const double *)psi, nrm);
        hipLaunchKernelGGL(k_b_scale_psi, dim3(b->nblocks), dim3(BRB), 0, st, S, psi, (const double *)nrm);
        HUB_HIP(hipGetLastError());
        if (o->refine) {
            double *hp = nullptr;
            HUB_TRY(alloc((void **)&hp, sizeof(double) * n));
            HUB_TRY((launch_batch_product<double, false>(b, psi, hp, nullptr, nullptr, nullptr, st)));
            hipLaunchKernelGGL(k_b_dot<double>, dim3(b->nblocks), dim3(BRB), 0, st, S, (const double *)psi,
                               (const double *)hp, partial, (const int *)nullptr);
            hipLaunchKernelGGL(k_b_final, dim3(P), dim3(BRB), 0, st, S, (const double *)partial, nrm + P, 1, 0,
                               (const int *)nullptr, 0, 0, (const int *)nullptr);
            HUB_HIP(hipGetLastError());
            HUB_HIP(hipMemcpyAsync(e0.data(), nrm + P, sizeof(double) * P, hipMemcpyDeviceToHost, st));
        }
        HUB_HIP(hipGetLastError());
    }
    HUB_HIP(hipStreamSynchronize(st));
    HUB_HIP(hipEventRecord(ev, st));
    HUB_HIP(hipStreamWaitEvent(user_st, ev, 0));
    (void)hipEventDestroy(ev);
    for (int p = 0; p < P; ++p) {
        if (e0_out) e0_out[p] = e0[p];
        if (iters_out) iters_out[p] = m_final[p];
    }
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->steps = k;
        info->graph_replays = replays;
        info->tile_columns = b->tb[di];
        info->block_size = b->bs[di];
        info->tune_seconds = b->tune_seconds - tune0;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    for (int p = 0; p < P; ++p)
        if (!conv[p]) return bfail(HUB_ERR_NOT_CONVERGED, "a sector of the batch did not converge");
    return HUB_OK;
}

}  // namespace
}  // namespace hub

using namespace hub;

extern "C" {

hub_status hub_batch_create(const hub_sector *const *sectors, int32_t count, hub_batch **out)
{
    if (!out) return bfail(HUB_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!sectors || count <= 0) return bfail(HUB_ERR_INVALID_ARG, "empty batch");
    hub_batch *b = new (std::nothrow) hub_batch();
    if (!b) return bfail(HUB_ERR_OOM, "host allocation failed");
    struct Guard {
        hub_batch *b;
        ~Guard() {
            if (!b) return;
            for (void *q : b->owned)
                if (q) (void)hipFree(q);
            delete b;
        }
    } guard{b};
    b->P = count;
    b->off.assign(count + 1, 0);
    for (int p = 0; p < count; ++p) {
        const hub_sector *s = sectors[p];
        if (!s) return bfail(HUB_ERR_INVALID_ARG, "NULL sector in batch");
        if (p > 0 && s->device != sectors[0]->device) return bfail(HUB_ERR_INVALID_ARG, "sectors on different devices");
        if (!s->spin[0].ell_c32) return bfail(HUB_ERR_UNSUPPORTED, "sector without compact product tables");
        if (s->k0) return bfail(HUB_ERR_UNSUPPORTED, "translation (k = 0) sectors cannot be batched");
        b->secs.push_back(s);
        b->off[p + 1] = b->off[p] + s->dim;
        b->max_cu = std::max(b->max_cu, (int)s->spin[0].count);
    }
    b->device = sectors[0]->device;
    // dynamic LDS for the product's panel; 4 KB stay for the static reduction array
    // of the fused Lanczos update (up to 512 doubles)
    b->lds_max = sectors[0]->lds_max - 4096;
    HUB_HIP(hipSetDevice(b->device));
    if ((size_t)(256 + (size_t)b->max_cu) * 8 > b->lds_max)
        return bfail(HUB_ERR_UNSUPPORTED, "a sector's column does not fit in LDS for the batched product");
    std::vector<BDesc<double>> d64(count);
    std::vector<BDesc<float>> d32(count);
    for (int p = 0; p < count; ++p) {
        d64[p] = make_desc<double>(sectors[p], b->off[p]);
        d32[p] = make_desc<float>(sectors[p], b->off[p]);
    }
    BDesc<double> *dd64 = nullptr;
    BDesc<float> *dd32 = nullptr;
    HUB_TRY(balloc(b, &dd64, count));
    HUB_TRY(balloc(b, &dd32, count));
    HUB_HIP(hipMemcpy(dd64, d64.data(), sizeof(BDesc<double>) * count, hipMemcpyHostToDevice));
    HUB_HIP(hipMemcpy(dd32, d32.data(), sizeof(BDesc<float>) * count, hipMemcpyHostToDevice));
    b->desc[0] = dd64;
    b->desc[1] = dd32;
    // segment grid: blocks per sector ~ dim / (8 * BRB), between 1 and 64
    std::vector<int32_t> sp, sl, sn(count), ss(count);
    for (int p = 0; p < count; ++p) {
        const int64_t d = b->off[p + 1] - b->off[p];
        int64_t nb = (d + 8 * BRB - 1) / (8 * BRB);
        nb = std::max<int64_t>(1, std::min<int64_t>(64, nb));
        sn[p] = (int32_t)nb;
        ss[p] = (int32_t)sp.size();
        for (int j = 0; j < nb; ++j) {
            sp.push_back(p);
            sl.push_back(j);
        }
    }
    b->nblocks = (int)sp.size();
    HUB_TRY(balloc(b, &b->seg_prob, sp.size()));
    HUB_TRY(balloc(b, &b->seg_local, sl.size()));
    HUB_TRY(balloc(b, &b->seg_n, count));
    HUB_TRY(balloc(b, &b->seg_start, count));
    HUB_TRY(balloc(b, &b->d_off, count + 1));
    HUB_HIP(hipMemcpy(b->seg_prob, sp.data(), sizeof(int32_t) * sp.size(), hipMemcpyHostToDevice));
    HUB_HIP(hipMemcpy(b->seg_local, sl.data(), sizeof(int32_t) * sl.size(), hipMemcpyHostToDevice));
    HUB_HIP(hipMemcpy(b->seg_n, sn.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice));
    HUB_HIP(hipMemcpy(b->seg_start, ss.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice));
    HUB_HIP(hipMemcpy(b->d_off, b->off.data(), sizeof(int64_t) * (count + 1), hipMemcpyHostToDevice));
    guard.b = nullptr;
    *out = b;
    return HUB_OK;
}

void hub_batch_destroy(hub_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    for (void *q : b->owned)
        if (q) (void)hipFree(q);
    delete b;
}

hub_status hub_batch_offsets(const hub_batch *b, int64_t *offsets)
{
    if (!b || !offsets) return bfail(HUB_ERR_INVALID_ARG, "NULL argument");
    for (int p = 0; p <= b->P; ++p) offsets[p] = b->off[p];
    return HUB_OK;
}

hub_status hub_batch_matvec(hub_batch *b, int32_t dtype, const void *dev_x, void *dev_y, void *stream)
{
    if (!b || !dev_x || !dev_y) return bfail(HUB_ERR_INVALID_ARG, "NULL argument");
    if (dtype != HUB_F64 && dtype != HUB_F32) return bfail(HUB_ERR_INVALID_ARG, "bad dtype");
    HUB_HIP(hipSetDevice(b->device));
    const size_t bytes = (size_t)b->off[b->P] * (dtype == HUB_F64 ? 8 : 4);
    const char *x = (const char *)dev_x, *y = (const char *)dev_y;
    if (x < y + bytes && y < x + bytes) return bfail(HUB_ERR_INVALID_ARG, "x and y overlap");
    hipStream_t st = (hipStream_t)stream;
    if (dtype == HUB_F64) {
        HUB_TRY(tune<double>(b, st));
        return launch_batch_product<double, false>(b, (const double *)dev_x, (double *)dev_y, nullptr, nullptr,
                                                   nullptr, st);
    }
    HUB_TRY(tune<float>(b, st));
    return launch_batch_product<float, false>(b, (const float *)dev_x, (float *)dev_y, nullptr, nullptr, nullptr, st);
}

hub_status hub_batch_ground_state(hub_batch *b, const hub_lanczos_opts *opts, double *e0, int32_t *iters,
                                  void *dev_psi, void *stream, hub_batch_info *info)
{
    if (!b || !opts) return bfail(HUB_ERR_INVALID_ARG, "NULL argument");
    if (opts->reorth != 0) return bfail(HUB_ERR_UNSUPPORTED, "the batched solve runs the plain recurrence");
    if (opts->dev_start) return bfail(HUB_ERR_UNSUPPORTED, "the batched solve draws its own start vectors");
    if (opts->vec_dtype != HUB_F64 && opts->vec_dtype != HUB_F32) return bfail(HUB_ERR_INVALID_ARG, "bad dtype");
    if (opts->refine && !dev_psi) return bfail(HUB_ERR_INVALID_ARG, "refine needs dev_psi");
    HUB_HIP(hipSetDevice(b->device));
    if (opts->vec_dtype == HUB_F64)
        return batch_solve<double>(b, opts, e0, iters, (double *)dev_psi, (hipStream_t)stream, info);
    return batch_solve<float>(b, opts, e0, iters, (double *)dev_psi, (hipStream_t)stream, info);
}

}  // extern "C"
