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
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <new>
#include <cfloat>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
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
    uint64_t cu_magic;  // ceil(2^32 / cu): e / cu = (e * cu_magic) >> 32 for e * cu < 2^32
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

// TB consecutive LDS values read as one access (aligned to their size, at most 16 bytes)
template <typename T, int N>
struct __attribute__((aligned(sizeof(T) * N < 16 ? sizeof(T) * N : 16))) BVec {
    T v[N];
};

// The lockstep recurrence keeps its vectors unnormalised, u_k = beta_k v_k
// (u_0 = v_0, beta_0 taken as 1), in three rotating slots: at step k, u_k =
// V[k % 3], u_{k-1} = V[(k + 2) % 3], and w, then u_{k+1} in place, V[(k + 1) % 3].
template <typename T>
struct Roles {
    T *v, *vp, *w;
};

template <typename T>
__device__ __forceinline__ Roles<T> roles(T *const *ptrs, int k)
{
    Roles<T> r;
    r.v = ptrs[k % 3];
    r.vp = ptrs[(k + 2) % 3];
    r.w = ptrs[(k + 1) % 3];
    return r;
}

// 1 / beta (0 after a breakdown)
__device__ __forceinline__ double binv(double b) { return b > 0.0 ? 1.0 / b : 0.0; }

// Batched product.  A work item is `ncol` consecutive columns of one sector,
// taken in groups of TB columns (the last group padded).  The item's columns
// are staged in LDS interleaved by group (element (a, column g TB + t) at
// (g cu + a) TB + t), and its H_dn rows, e_dn and bit patterns beside them.  A
// lane owns TB columns of one row of one group: position f = g cu + a, the
// quotient by a multiply-high with ceil(2^32 / cu) (exact while f cu < 2^32),
// so a sector smaller than the workgroup fills it with several groups; each
// H_up entry is read once for the TB columns (one LDS access gathers them),
// and each lane takes R positions BS apart at a time, so that their loads are
// in flight together (loads unconditional: a position past the end, or an
// entry past its row's length, re-reads a valid one and only the update is
// selected).  Every element is formed as in the single-sector product
// (diagonal, then the H_up entries in sliced-ELL order, then the H_dn entries
// in CSR order, one fused multiply-add each): the two agree bit for bit.
// SEL (the Lanczos step): x = u_k and y = w from the pointer table at the device
// step counter, and the first update fused in: w = (H u_k) / beta_k -
// (beta_k / beta_{k-1}) u_{k-1}, evaluated in FP64 and rounded once, and this
// item's partial of <w, u_k> = beta_k alpha_k in ipart[it.w] (a fixed-order
// block sum, at the item's place in sector-major order); otherwise x, y as given.
template <typename T, int BS, int R, int TB, bool SEL>
__global__ __launch_bounds__(BS) void k_batch_kron(const BDesc<T> *__restrict__ desc, const int4 *__restrict__ items,
                                                   const T *xg, T *yg, T *const *ptrs, const int *step,
                                                   const int *__restrict__ active, const double *__restrict__ beta,
                                                   int kmax, double *__restrict__ ipart, int nitems)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[SEL ? BS : 1];
    T *tab = reinterpret_cast<T *>(smem_raw);
    T *xs = tab + 256;
    // items in launch order (costliest first): with converged sectors masked
    // out, the remaining work stays spread over every XCD
    const int item = (int)blockIdx.x;
    if (item >= nitems) return;
    const int4 it = items[item];
    if (active && !active[it.x]) return;
    const BDesc<T> D = desc[it.x];
    const T *x = xg;
    T *y = yg;
    const T *vp = nullptr;
    int ks = 0;
    double sx = 1.0, bt = 0.0;  // 1 / beta_k and beta_k / beta_{k-1}
    if (SEL) {
        ks = *step;
        const Roles<T> r = roles(ptrs, ks);
        x = r.v;
        y = r.w;
        vp = r.vp + D.off;
        if (ks > 0) {
            const double bk = beta[(int64_t)it.x * kmax + ks];
            sx = binv(bk);
            bt = bk * (ks > 1 ? binv(beta[(int64_t)it.x * kmax + ks - 1]) : 1.0);
        }
    }
    x += D.off;
    y += D.off;
    const int cu = D.cu, b0 = it.y, ncol = it.z;
    const int ng = (ncol + TB - 1) / TB, F = ng * cu;
    const int64_t t0 = (int64_t)b0 * cu;
    const int rp0 = D.dn_rp[b0], nnz = D.dn_rp[b0 + ncol] - rp0;
    T *lval = xs + (int64_t)F * TB;
    T *ledn = lval + nnz;
    int *lcol = reinterpret_cast<int *>(ledn + ncol);
    int *lrp = lcol + nnz;
    uint32_t *ldnb = reinterpret_cast<uint32_t *>(lrp + ncol + 1);
    for (int i = threadIdx.x; i < 256; i += BS) tab[i] = D.code_v[i];
    for (int e = threadIdx.x; e < ng * TB * cu; e += BS) {
        const int c = (int)(((uint64_t)(uint32_t)e * D.cu_magic) >> 32);  // column in the item
        const int a = e - c * cu;
        xs[((c / TB) * cu + a) * TB + c % TB] = (c < ncol) ? x[t0 + e] : (T)0;
    }
    for (int q = threadIdx.x; q < nnz; q += BS) {
        lval[q] = D.dn_val[rp0 + q];
        lcol[q] = D.dn_col[rp0 + q];
    }
    for (int t = threadIdx.x; t <= ncol; t += BS) lrp[t] = D.dn_rp[b0 + t] - rp0;
    for (int t = threadIdx.x; t < ncol; t += BS) {
        ledn[t] = D.e_dn[b0 + t];
        ldnb[t] = D.dn_basis[b0 + t];
    }
    __syncthreads();
    double dacc = 0.0;
    for (int f0 = threadIdx.x; f0 < F; f0 += R * BS) {
        int ra[R], rg[R];  // row, group
        T acc[R][TB];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int f = (f0 + j * BS < F) ? f0 + j * BS : f0;
            rg[j] = (int)(((uint64_t)(uint32_t)f * D.cu_magic) >> 32);
            ra[j] = f - rg[j] * cu;
            const uint32_t ub = D.up_basis[ra[j]];
            const T eu = D.e_up[ra[j]];
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                const int c = min(rg[j] * TB + t, ncol - 1);
                acc[j][t] = (bdiag(D, ub & ldnb[c]) + eu + ledn[c]) * xs[f * TB + t];
            }
        }
        // H_up: entry k of row a at ell[64 sl_off[a / 64] + a % 64 + 64 k]
        int eo[R], el_n[R], lmax = 0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int s = ra[j] >> 6;
            eo[j] = D.sl_off[s] * 64 + (ra[j] & 63);
            el_n[j] = D.sl_off[s + 1] - D.sl_off[s];
            lmax = max(lmax, el_n[j]);
        }
        for (int k = 0; k < lmax; ++k) {
            uint32_t c[R];
#pragma unroll
            for (int j = 0; j < R; ++j) c[j] = D.ell[el_n[j] > 0 ? eo[j] + 64 * min(k, el_n[j] - 1) : 0];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const T v = tab[c[j] >> 24];
                const BVec<T, TB> xv =
                    *reinterpret_cast<const BVec<T, TB> *>(xs + (rg[j] * cu + (int)(c[j] & 0xFFFFFFu)) * TB);
#pragma unroll
                for (int t = 0; t < TB; ++t) {
                    const T f = fma(v, xv.v[t], acc[j][t]);
                    acc[j][t] = (k < el_n[j]) ? f : acc[j][t];
                }
            }
        }
        // H_dn: the row of each column's CSR (from LDS), neighbour columns read
        // from the vector
        int ds[R][TB], dn[R][TB], nmax = 0;
#pragma unroll
        for (int j = 0; j < R; ++j)
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                const int cc = rg[j] * TB + t;
                ds[j][t] = lrp[min(cc, ncol)];
                dn[j][t] = (cc < ncol) ? lrp[cc + 1] - ds[j][t] : 0;
                nmax = max(nmax, dn[j][t]);
            }
        for (int u = 0; u < nmax; ++u) {
            T w[R][TB], xv[R][TB];
#pragma unroll
            for (int j = 0; j < R; ++j)
#pragma unroll
                for (int t = 0; t < TB; ++t) {
                    const int kk = dn[j][t] > 0 ? ds[j][t] + min(u, dn[j][t] - 1) : 0;
                    w[j][t] = lval[kk];
                    xv[j][t] = x[(int64_t)lcol[kk] * cu + ra[j]];
                }
#pragma unroll
            for (int j = 0; j < R; ++j)
#pragma unroll
                for (int t = 0; t < TB; ++t) {
                    const T f = fma(w[j][t], xv[j][t], acc[j][t]);
                    acc[j][t] = (u < dn[j][t]) ? f : acc[j][t];
                }
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (f0 + j * BS >= F) continue;
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                const int cc = rg[j] * TB + t;
                if (cc >= ncol) continue;
                const int64_t o = t0 + (int64_t)cc * cu + ra[j];
                T r = acc[j][t];
                if (SEL) {
                    r = (ks > 0) ? (T)fma(sx, (double)r, -(bt * (double)vp[o])) : (T)(sx * (double)r);
                    dacc += (double)r * (double)xs[(rg[j] * cu + ra[j]) * TB + t];
                }
                y[o] = r;
            }
        }
    }
    if (SEL) {
        red[threadIdx.x] = dacc;
        __syncthreads();
        for (int o2 = BS / 2; o2 > 0; o2 >>= 1) {
            if (threadIdx.x < (unsigned)o2) red[threadIdx.x] += red[threadIdx.x + o2];
            __syncthreads();
        }
        if (threadIdx.x == 0) ipart[it.w] = red[0];
    }
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

// The sum of v[0 .. n) in a fixed order (lane j adds j, j + BRB, ..., then the
// tree of bblock_sum), the same in every block that forms it.
__device__ __forceinline__ double bsum_strided(const double *v, int n, double *sh)
{
    double acc = 0.0;
    for (int j = threadIdx.x; j < n; j += BRB) acc += v[j];
    return bblock_sum(acc, sh);
}

// Lanczos step after the fused product: alpha_k from the sector's work-item
// partials (their sum over beta_k; every block of the sector forms it alike, the
// first stores it), then u_{k+1} = w - (alpha_k / beta_k) u_k in place of w and
// the block's partial of beta_{k+1}^2 = <u_{k+1}, u_{k+1}>.
template <typename T>
__global__ __launch_bounds__(BRB) void k_b_lz_ab(Seg S, T *const *ptrs, const int *step,
                                                 const int *__restrict__ istart, const int *__restrict__ icount,
                                                 const double *__restrict__ ipart, double *alpha,
                                                 const double *__restrict__ beta, int kmax, double *partial,
                                                 const int *__restrict__ active)
{
    __shared__ double sh[BRB];
    const int pp = S.prob[blockIdx.x];
    if (active && !active[pp]) return;
    const int k = *step;
    const double ib = k > 0 ? binv(beta[(int64_t)pp * kmax + k]) : 1.0;
    const double al = bsum_strided(ipart + istart[pp], icount[pp], sh) * ib;
    if (S.local[blockIdx.x] == 0 && threadIdx.x == 0) alpha[(int64_t)pp * kmax + k] = al;
    const double c = al * ib;
    const Roles<T> r = roles(ptrs, k);
    double acc = 0.0;
    SEG_LOOP(S, p, i)
    {
        const T wi = (T)((double)r.w[o_p + i] - c * (double)r.v[o_p + i]);
        r.w[o_p + i] = wi;
        acc += (double)wi * (double)wi;
    }
    const double s2 = bblock_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s2;
}

// One block per sector: beta_{k+1} = sqrt of the sector's <w, w> partials.
// The last block to arrive advances the step counter (every block has read it
// before the barrier that precedes its arrival) and re-arms the arrival
// counter `done`; the next kernel on the stream sees the new value at the
// kernel boundary.  No fence: a device-scope fence per block would write back
// the L2 each time.
__global__ __launch_bounds__(BRB) void k_b_beta(Seg S, int *step, const double *partial, double *beta, int kmax,
                                                const int *__restrict__ active, unsigned int *done)
{
    __shared__ double sh[BRB];
    const int p = blockIdx.x;
    const int k = *step;
    if (!active || active[p]) {
        const double bt = sqrt(bsum_strided(partial + S.start[p], S.nseg[p], sh));
        if (threadIdx.x == 0) beta[(int64_t)p * kmax + k + 1] = bt;
    }
    __syncthreads();
    if (threadIdx.x == 0 && atomicAdd(done, 1u) == gridDim.x - 1u) {
        atomicExch(done, 0u);
        *step = k + 1;
    }
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

// Second pass (replay with the stored alpha / beta at step k, explicit k): y =
// H u_k (done by the product, into the slot of u_{k+1}) becomes w as in the
// product's epilogue and then u_{k+1} = w - (alpha_k / beta_k) u_k as in
// k_b_lz_ab, with the same roundings, so the first pass's vectors come back bit
// for bit.
template <typename T>
__global__ __launch_bounds__(BRB) void k_b_replay(Seg S, T *y, const T *u, const T *up, const double *alpha,
                                                  const double *beta, int kmax, int k, const int *__restrict__ mlen)
{
    const int pp = S.prob[blockIdx.x];
    if (k + 1 >= mlen[pp]) return;
    double sx = 1.0, bt = 0.0, ib = 1.0;
    if (k > 0) {
        const double bk = beta[(int64_t)pp * kmax + k];
        sx = binv(bk);
        ib = sx;
        bt = bk * (k > 1 ? binv(beta[(int64_t)pp * kmax + k - 1]) : 1.0);
    }
    const double c = alpha[(int64_t)pp * kmax + k] * ib;
    SEG_LOOP(S, p, i)
    {
        const T w = (k > 0) ? (T)fma(sx, (double)y[o_p + i], -(bt * (double)up[o_p + i]))
                            : (T)(sx * (double)y[o_p + i]);
        y[o_p + i] = (T)((double)w - c * (double)u[o_p + i]);
    }
}

template <typename T>
__global__ __launch_bounds__(BRB) void k_b_psi(Seg S, double *psi, const T *v, const double *y,
                                               const double *__restrict__ beta, int kmax, int k,
                                               const int *__restrict__ mlen)
{
    const int pp = S.prob[blockIdx.x];
    if (k >= mlen[pp]) return;
    // v_k = u_k / beta_k (beta_0 taken as 1)
    const double c = y[(int64_t)pp * kmax + k] * (k > 0 ? binv(beta[(int64_t)pp * kmax + k]) : 1.0);
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
    int rr[2] = {1, 1}, bs[2] = {256, 256}, tb[2] = {1, 1};  // rows / columns per lane, workgroup size
    int4 *items[2] = {nullptr, nullptr};      // {sector, first column, columns, 0}
    int nitems[2] = {0, 0};
    size_t lds_bytes[2] = {0, 0};             // dynamic LDS of the largest item
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
    d.cu_magic = ((1ull << 32) + (uint64_t)d.cu - 1) / (uint64_t)d.cu;
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

template <typename T, int BS, int R, int TB, bool SEL>
hub_status launch_bk(hub_batch *b, int di, const T *x, T *y, T *const *ptrs, const int *step, const int *active,
                     hipStream_t st, const double *beta, int kmax, double *ipart)
{
    static std::atomic<bool> attr{false};
    if (!attr) {
        HUB_HIP(hipFuncSetAttribute((const void *)k_batch_kron<T, BS, R, TB, SEL>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds_max));
        attr = true;
    }
    const int n = b->nitems[di];
    hipLaunchKernelGGL((k_batch_kron<T, BS, R, TB, SEL>), dim3(n), dim3(BS), b->lds_bytes[di], st,
                       (const BDesc<T> *)b->desc[di], b->items[di], x, y, ptrs, step, active, beta, kmax, ipart, n);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

// The product shapes the tuner tries: {workgroup size, rows per lane, columns per lane}
constexpr int kBatchShapes[][3] = {{256, 4, 1}, {256, 2, 2}, {256, 1, 4}, {256, 2, 4}, {256, 4, 2},
                                   {512, 4, 1}, {512, 2, 2}, {512, 1, 4}, {512, 2, 4}};

// SEL: the Lanczos step (vectors from the pointer table, first update fused,
// item partials of alpha in ipart; beta and kmax as in the solver's arrays)
template <typename T, bool SEL>
hub_status launch_batch_product(hub_batch *b, const T *x, T *y, T *const *ptrs, const int *step, const int *active,
                                hipStream_t st, const double *beta = nullptr, int kmax = 0, double *ipart = nullptr)
{
    const int di = (sizeof(T) == 8) ? 0 : 1;
    const int rr = b->rr[di], bs = b->bs[di], tb = b->tb[di];
#define HUB_BK(BSV, RV, TBV)                                                             \
    if (bs == BSV && rr == RV && tb == TBV)                                              \
        return launch_bk<T, BSV, RV, TBV, SEL>(b, di, x, y, ptrs, step, active, st, beta, kmax, ipart);
    HUB_BK(256, 4, 1) HUB_BK(256, 2, 2) HUB_BK(256, 1, 4) HUB_BK(256, 2, 4) HUB_BK(256, 4, 2)
    HUB_BK(512, 4, 1) HUB_BK(512, 2, 2) HUB_BK(512, 1, 4) HUB_BK(512, 2, 4)
#undef HUB_BK
    return bfail(HUB_ERR_UNSUPPORTED, "untuned product shape");
}

// Work items: each sector's columns in runs of tb x max(1, target / count_up)
// (the last run shorter), at most kItemDnEntries / (the longest H_dn row)
// columns, so that their H_dn rows fit the LDS beside them.
constexpr int kItemDnEntries = 4096;

hub_status build_items(hub_batch *b, int di, int target, int tb)
{
    const size_t es = di == 0 ? sizeof(double) : sizeof(float);
    std::vector<int4> it;
    size_t lds = 0;
    for (int p = 0; p < b->P; ++p) {
        const SpinTables &DN = b->secs[p]->spin[1];
        const int cu = (int)b->secs[p]->spin[0].count, cd = (int)DN.count;
        const int deg = std::max(1, (int)DN.max_row);
        const int per = std::max(1, std::min({cd, tb * std::max(1, target / cu), kItemDnEntries / deg}));
        // the in-kernel quotients by cu are exact while (padded columns of an item) * cu * cu < 2^32
        const uint64_t padded = (uint64_t)((per + tb - 1) / tb * tb);
        if (padded * (uint64_t)cu * (uint64_t)cu >= (1ull << 32))
            return bfail(HUB_ERR_UNSUPPORTED, "sector too large for the batched product");
        for (int b0 = 0; b0 < cd; b0 += per) {
            const int n = std::min(per, cd - b0);
            it.push_back(make_int4(p, b0, n, (int)it.size()));
            const size_t nnz = (size_t)n * (size_t)deg;
            const size_t ncp = (size_t)((n + tb - 1) / tb * tb);
            lds = std::max(lds, (256 + ncp * cu + nnz + n) * es + (nnz + 2 * (size_t)n + 1) * 4);
        }
    }
    if (b->items[di]) {
        HUB_HIP(hipFree(b->items[di]));
        for (auto &q : b->owned)
            if (q == (void *)b->items[di]) q = nullptr;
        b->items[di] = nullptr;
    }
    // launch order: costliest items first (elements times the entries per
    // element), so the last wave of workgroups holds the cheapest ones; .w keeps
    // the item's sector-major index, where its alpha partial goes
    std::vector<int4> lo(it);
    auto cost = [&](const int4 &q) {
        const hub_sector *sp = b->secs[q.x];
        const double cu = (double)sp->spin[0].count, cd = (double)sp->spin[1].count;
        return (double)q.z * cu * (1.0 + (double)sp->spin[0].nnz / cu + (double)sp->spin[1].nnz / cd);
    };
    std::stable_sort(lo.begin(), lo.end(), [&](const int4 &a, const int4 &c) { return cost(a) > cost(c); });
    HUB_TRY(balloc(b, &b->items[di], lo.size()));
    HUB_HIP(hipMemcpy(b->items[di], lo.data(), sizeof(int4) * lo.size(), hipMemcpyHostToDevice));
    b->nitems[di] = (int)it.size();
    b->lds_bytes[di] = lds;
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
    return HUB_OK;
}

// Autotuner: time every (workgroup size, elements per lane) whose items fit
// the LDS on the batch itself; items hold about size x elements-per-lane
// elements.
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
    struct EvFree {
        hipEvent_t a, c;
        ~EvFree() { (void)hipEventDestroy(a); (void)hipEventDestroy(c); }
    } ef{e0, e1};
    float best = 1e30f;
    int bsel = -1;
    const int nshape = (int)(sizeof(kBatchShapes) / sizeof(kBatchShapes[0]));
    for (int i = 0; i < nshape; ++i) {
        const int bs = kBatchShapes[i][0], r = kBatchShapes[i][1], tbv = kBatchShapes[i][2];
        HUB_TRY(build_items(b, di, bs * r, tbv));
        if (b->lds_bytes[di] > b->lds_max) continue;
        b->bs[di] = bs;
        b->rr[di] = r;
        b->tb[di] = tbv;
        HUB_TRY((launch_batch_product<T, false>(b, x, y, nullptr, nullptr, nullptr, st)));
        HUB_HIP(hipEventRecord(e0, st));
        for (int q = 0; q < 3; ++q) HUB_TRY((launch_batch_product<T, false>(b, x, y, nullptr, nullptr, nullptr, st)));
        HUB_HIP(hipEventRecord(e1, st));
        HUB_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        HUB_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
            best = ms;
            bsel = i;
        }
    }
    if (bsel < 0) return bfail(HUB_ERR_UNSUPPORTED, "a sector's columns do not fit in LDS for the batched product");
    b->bs[di] = kBatchShapes[bsel][0];
    b->rr[di] = kBatchShapes[bsel][1];
    b->tb[di] = kBatchShapes[bsel][2];
    HUB_TRY(build_items(b, di, b->bs[di] * b->rr[di], b->tb[di]));
    b->tuned[di] = true;
    b->tune_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return HUB_OK;
}

// Host workers for the per-sector convergence tests (a tridiagonal solve each):
// run(n, f) calls f(0) ... f(n - 1) on the caller and the workers and returns
// when all are done.  The pool lives for one batched solve.
class HostPool {
public:
    explicit HostPool(int nthreads)
    {
        for (int i = 0; i < nthreads; ++i) th_.emplace_back([this] { loop(); });
    }
    ~HostPool()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    void run(int n, const std::function<void(int)> &f)
    {
        if (th_.empty() || n < 2) {
            for (int i = 0; i < n; ++i) f(i);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            job_ = &f;
            n_ = n;
            next_.store(0);
            busy_ = (int)th_.size();
            ++gen_;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [this] { return busy_ == 0; });
        job_ = nullptr;
    }

private:
    void work()
    {
        for (int i = next_.fetch_add(1); i < n_; i = next_.fetch_add(1)) (*job_)(i);
    }
    void loop()
    {
        int seen = 0;
        while (true) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
            }
            work();
            std::lock_guard<std::mutex> lk(mu_);
            if (--busy_ == 0) done_cv_.notify_one();
        }
    }
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int)> *job_ = nullptr;
    int n_ = 0, busy_ = 0, gen_ = 0;
    std::atomic<int> next_{0};
    bool stop_ = false;
};

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
    T *V[3];
    for (int i = 0; i < 3; ++i) HUB_TRY(alloc((void **)&V[i], sizeof(T) * n));
    T **ptrs = nullptr;
    int *step = nullptr, *active = nullptr, *mlen = nullptr;
    double *alpha = nullptr, *beta = nullptr, *partial = nullptr, *nrm = nullptr, *ycoef = nullptr;
    HUB_TRY(alloc((void **)&ptrs, sizeof(T *) * 3));
    HUB_TRY(alloc((void **)&step, sizeof(int) * 4));
    unsigned int *done = reinterpret_cast<unsigned int *>(step + 1);  // arrival counter of k_b_beta
    HUB_TRY(alloc((void **)&active, sizeof(int) * P));
    HUB_TRY(alloc((void **)&mlen, sizeof(int) * P));
    HUB_TRY(alloc((void **)&alpha, sizeof(double) * (size_t)P * kmax));
    HUB_TRY(alloc((void **)&beta, sizeof(double) * (size_t)P * kmax));
    HUB_TRY(alloc((void **)&partial, sizeof(double) * (size_t)b->nblocks));
    double *ipart = nullptr;  // alpha partials of the fused product, one per work item
    HUB_TRY(alloc((void **)&ipart, sizeof(double) * (size_t)std::max(1, b->nitems[di])));
    HUB_TRY(alloc((void **)&nrm, sizeof(double) * (size_t)P * 4));
    HUB_TRY(alloc((void **)&ycoef, sizeof(double) * (size_t)P * kmax));
    HUB_HIP(hipMemcpyAsync(ptrs, V, sizeof(T *) * 3, hipMemcpyHostToDevice, st));
    std::vector<int> hact(P, 1);
    HUB_HIP(hipMemcpyAsync(active, hact.data(), sizeof(int) * P, hipMemcpyHostToDevice, st));
    HUB_HIP(hipMemsetAsync(step, 0, sizeof(int) * 4, st));
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

    // one Lanczos step, captured as a graph: the fused product; alpha and
    // u_{k+1} = w - (alpha / beta_k) u_k; beta_{k+1} and the step counter
    auto one_step = [&]() -> hub_status {
        HUB_TRY((launch_batch_product<T, true>(b, nullptr, nullptr, ptrs, step, active, st, beta, kmax, ipart)));
        hipLaunchKernelGGL(k_b_lz_ab<T>, dim3(b->nblocks), dim3(BRB), 0, st, S, ptrs, (const int *)step,
                           (const int *)b->istart[di], (const int *)b->icount[di], (const double *)ipart, alpha,
                           (const double *)beta, kmax, partial, (const int *)active);
        hipLaunchKernelGGL(k_b_beta, dim3(P), dim3(BRB), 0, st, S, step, (const double *)partial, beta, kmax,
                           (const int *)active, done);
        HUB_HIP(hipGetLastError());
        return HUB_OK;
    };
    // one eager step first (also sets the kernel attributes outside the capture);
    // the captured graph then replays steps 1, 2, ...
    HUB_TRY(one_step());
    int k = 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // opts->batch_no_graph: every step launched eagerly (same kernels, same order)
    bool use_graph = !o->batch_no_graph;
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
    // the coefficients are copied into a ring of pinned buffers, and kAhead
    // further groups are enqueued before the host examines a copy; the new
    // active mask (through pinned memory as well) reaches the device after the
    // groups already queued.  A sector found converged may so run kAhead more
    // groups; those steps are never used (its T and psi stop at the step of the
    // test).  (Two groups ahead left the inter-kernel gaps of the 64-sector
    // batch unchanged: the host test is not what the GPU waits for.)
    constexpr int kAhead = 1, NS = kAhead + 1;
    const size_t nab = (size_t)P * kmax;
    double *hab = nullptr;  // [2 slots][alpha | beta]
    int *hmask = nullptr;   // [2][P]
    HUB_HIP(hipHostMalloc((void **)&hab, sizeof(double) * 2 * NS * nab));
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
    HUB_HIP(hipHostMalloc((void **)&hmask, sizeof(int) * NS * (size_t)P));
    pin_mask.p = hmask;
    hipEvent_t cev[NS] = {};
    for (int i = 0; i < NS; ++i) HUB_HIP(hipEventCreateWithFlags(&cev[i], hipEventDisableTiming));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard()
        {
            for (int i = 0; i < NS; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } evg{cev};
    int kslot[NS] = {};
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
    // the tests of the active sectors run on a few host threads (their tridiagonal
    // solves would otherwise keep the GPU waiting at the end of a group)
    const int nthreads = std::max(0, std::min(7, (int)std::thread::hardware_concurrency() - 1));
    HostPool pool(P > 1 ? nthreads : 0);
    std::vector<int> act;
    auto check_copy = [&](const double *ha, const double *hb, int kk) {
        act.clear();
        for (int p = 0; p < P; ++p)
            if (hact[p]) act.push_back(p);
        const std::function<void(int)> one = [&](int i) {
            const int p = act[(size_t)i];
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
            ys[p] = std::move(y);
            if (brk || res <= tol * scale || (int64_t)m >= dimp) conv[p] = 1;
        };
        pool.run((int)act.size(), one);
        for (const int p : act)
            if (conv[p]) {
                hact[p] = 0;
                --nactive;
            }
    };
    std::deque<int> pend;  // copies enqueued and not yet examined, oldest first
    int next_slot = 0, msl = 0;
    HUB_TRY(enqueue_copy(next_slot));
    pend.push_back(next_slot);
    next_slot = (next_slot + 1) % NS;
    while (true) {
        while ((int)pend.size() <= kAhead && nactive > 0 && k < max_iter) {
            HUB_TRY(enqueue_steps(std::min(check_every, max_iter - k)));
            HUB_TRY(enqueue_copy(next_slot));
            pend.push_back(next_slot);
            next_slot = (next_slot + 1) % NS;
        }
        const int sl = pend.front();
        pend.pop_front();
        HUB_HIP(hipEventSynchronize(cev[sl]));  // the groups enqueued after it keep running
        const double *ha = hab + (size_t)sl * 2 * nab;
        check_copy(ha, ha + nab, kslot[sl]);
        if (nactive == 0 || (pend.empty() && k >= max_iter)) break;
        int *hm = hmask + (size_t)msl * P;
        std::memcpy(hm, hact.data(), sizeof(int) * (size_t)P);
        HUB_HIP(hipMemcpyAsync(active, hm, sizeof(int) * P, hipMemcpyHostToDevice, st));
        msl = (msl + 1) % NS;
    }
    std::vector<double> e0(theta);

    if (psi && (o->want_vector || o->refine)) {
        // second pass with the stored alpha / beta; psi = sum_j (y_j / beta_j) u_j per sector
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
                               (const double *)ycoef, (const double *)beta, kmax, j, (const int *)mlen);
            if (j + 1 >= mmax) break;
            HUB_TRY((launch_batch_product<T, false>(b, vc, vn, nullptr, nullptr, nullptr, st)));
            hipLaunchKernelGGL(k_b_replay<T>, dim3(b->nblocks), dim3(BRB), 0, st, S, vn, (const T *)vc,
                               (const T *)vp, (const double *)alpha, (const double *)beta, kmax, j,
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
        info->rows_per_lane = b->rr[di];
        info->cols_per_lane = b->tb[di];
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
    // the smallest work item (one FP64 column with its H_dn row) must fit
    for (const hub_sector *s : b->secs) {
        const size_t cu = (size_t)s->spin[0].count, deg = (size_t)std::max(1, (int)s->spin[1].max_row);
        if ((256 + cu + deg + 1) * 8 + (deg + 3) * 4 > b->lds_max)
            return bfail(HUB_ERR_UNSUPPORTED, "a sector's column does not fit in LDS for the batched product");
    }
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
    // segment grid: blocks per sector ~ dim / (8 * BRB) (eight elements per
    // lane, so the vector passes keep many loads in flight), between 1 and 1024
    std::vector<int32_t> sp, sl, sn(count), ss(count);
    for (int p = 0; p < count; ++p) {
        const int64_t d = b->off[p + 1] - b->off[p];
        int64_t nb = (d + 8 * BRB - 1) / (8 * BRB);
        nb = std::max<int64_t>(1, std::min<int64_t>(1024, nb));
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
