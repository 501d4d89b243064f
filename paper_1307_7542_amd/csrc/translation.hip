// Translation symmetry, k = 0 (Sec. VI), for lattices invariant under a cyclic
// shift of the site labels by w (w = 1: the periodic chain).
//
// G lowers every bit position of an occupation integer by w (cyclically).  On
// a ket whose creation operators are in increasing site order, G moves the k
// operators of the lowest w sites past the other N - k:
//   G |x> = (-1)^(k (N - k)) |rotr(x, w)>.
// On the two-spin kets of Sec. II (up block, then down block) the two blocks
// are translated separately and the signs multiply.  A k = 0 state obeys
// psi(G c) = g(c) psi(c) with G|c> = g(c)|Gc>.
//
// Layout (differs from the combined representatives of Eq. (count7), which
// are not formed): a k = 0 state is stored as phi[i + b R] = sqrt(P_i) psi(R_i, b)
// for the up representatives R_i (smallest integer of each cycle, ascending;
// P_i its period) and every down state b.  Every two-spin configuration is a
// translate of some (R_i, b), so phi determines psi, and sum |phi|^2 equals the
// full-space norm: Euclidean products of phi are the physical ones.  For
// R_i with P_i < L the amplitudes of row i are tied together by the
// stabiliser G^P_i; the projector onto that consistent subspace runs after
// every product and on start vectors.
//
// The product y = H phi (rows i, columns b):
//   diagonal:  D(R_i, b) phi(i, b) (Sec. III B);
//   H_dn term: sum_b' H_dn[b, b'] phi(i, b')       (whole rows, as in Eq. (count1));
//   H_up term: for each hop R_i -> x' = G^s R_i' (phase e', amplitude -t esign):
//              coef = -t esign e' sqrt(P_i / P_i') times g_s(G^-s b) phi(i', G^-s b).
// The H_up term maps column b to columns of b's own down cycle, so one
// workgroup per down cycle stages that cycle's columns in LDS and reuses every
// hop entry for all members of the cycle.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

namespace hub {
namespace {

__device__ __forceinline__ uint32_t g_rot(uint32_t x, int M, int w)
{
    const uint32_t mask = (M >= 32) ? 0xFFFFFFFFu : ((1u << M) - 1u);
    return ((x >> w) | (x << (M - w))) & mask;
}

__device__ __forceinline__ int g_sign(uint32_t x, int N, int w)
{
    const int k = __popc(x & ((1u << w) - 1u));
    return ((k * (N - k)) & 1) ? -1 : 1;
}

__device__ __forceinline__ int64_t t_rank(uint32_t x, const uint64_t *__restrict__ C)
{
    int64_t r = 0;
    int k = 1;
    while (x) {
        r += (int64_t)C[__builtin_ctz(x) * kBinomN + k];
        ++k;
        x &= x - 1u;
    }
    return r;
}

// Cycle of every basis state: representative (basis index), translation s with
// G^s|R> = e|x>, the phase e, the period and the sign sigma of G^P on the cycle.
__global__ void k_cycles(const uint32_t *__restrict__ basis, int64_t count, int M, int N, int w,
                         const uint64_t *__restrict__ C, int32_t *__restrict__ rep_idx, int32_t *__restrict__ shift,
                         int32_t *__restrict__ phase, int32_t *__restrict__ period, int32_t *__restrict__ sigma,
                         int32_t *__restrict__ is_rep)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const uint32_t x = basis[k];
    uint32_t y = x, best = x;
    int c = 1, cbest = 1, jbest = 0, P = 0;
    while (true) {
        c *= g_sign(y, N, w);
        y = g_rot(y, M, w);
        ++P;
        if (y == x) break;
        if (y < best) {
            best = y;
            cbest = c;
            jbest = P;
        }
    }
    // G^jbest |x> = cbest |R>, G^P |x> = c |x>  =>  G^(P - jbest) |R> = cbest c |x>
    rep_idx[k] = (int32_t)t_rank(best, C);
    shift[k] = (jbest == 0) ? 0 : P - jbest;
    phase[k] = (jbest == 0) ? 1 : cbest * c;
    period[k] = P;
    sigma[k] = c;
    is_rep[k] = (jbest == 0) ? 1 : 0;
}

// Compaction: row[k] = position of basis state k among the representatives.
__global__ void k_rep_rows(const int32_t *__restrict__ is_rep, const int32_t *__restrict__ pos, int64_t count,
                           int32_t *__restrict__ row)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    row[k] = is_rep[k] ? pos[k] : -1;
}

__global__ void k_rep_fill(const uint32_t *__restrict__ basis, const int32_t *__restrict__ is_rep,
                           const int32_t *__restrict__ row, const int32_t *__restrict__ period,
                           const int32_t *__restrict__ sigma, const double *__restrict__ e64, int64_t count,
                           uint32_t *__restrict__ reps, int32_t *__restrict__ rper, int32_t *__restrict__ rsig,
                           double *__restrict__ re64, float *__restrict__ re32)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count || !is_rep[k]) return;
    const int r = row[k];
    reps[r] = basis[k];
    rper[r] = period[k];
    rsig[r] = sigma[k];
    re64[r] = e64[k];
    re32[r] = (float)e64[k];
}

__device__ __forceinline__ uint32_t t_between(int i, int j)
{
    const uint32_t below_j = (j >= 32) ? 0xFFFFFFFFu : ((1u << j) - 1u);
    const uint32_t upto_i = (i >= 31) ? 0xFFFFFFFFu : ((1u << (i + 1)) - 1u);
    return below_j & ~upto_i;
}

__global__ void k_hop_count(const uint32_t *__restrict__ reps, int64_t R, const int32_t *__restrict__ bi,
                            const int32_t *__restrict__ bj, int nb, int32_t *__restrict__ len)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const uint32_t x = reps[r];
    int n = 0;
    for (int e = 0; e < nb; ++e) n += (((x >> bi[e]) ^ (x >> bj[e])) & 1u) ? 1 : 0;
    len[r] = n;
}

__global__ void k_hop_fill(const uint32_t *__restrict__ reps, int64_t R, const int32_t *__restrict__ rper,
                           const int32_t *__restrict__ bi, const int32_t *__restrict__ bj,
                           const double *__restrict__ t, int nb, const uint64_t *__restrict__ C,
                           const int32_t *__restrict__ rep_idx, const int32_t *__restrict__ shift,
                           const int32_t *__restrict__ phase, const int32_t *__restrict__ row,
                           const int32_t *__restrict__ rp, int32_t *__restrict__ hrow, int32_t *__restrict__ hs,
                           double *__restrict__ hc64, float *__restrict__ hc32)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const uint32_t x = reps[r];
    int o = rp[r];
    for (int e = 0; e < nb; ++e) {
        const int i = bi[e], j = bj[e];
        if ((((x >> i) ^ (x >> j)) & 1u) == 0) continue;
        const uint32_t x2 = x ^ ((1u << i) | (1u << j));
        const int es = (__popc(x & t_between(i, j)) & 1) ? -1 : 1;
        const int64_t k2 = t_rank(x2, C);
        const int r2 = row[rep_idx[k2]];
        const double c = -t[e] * (double)es * (double)phase[k2] * sqrt((double)rper[r] / (double)rper[r2]);
        hrow[o] = r2;
        hs[o] = shift[k2];
        hc64[o] = c;
        hc32[o] = (float)c;
        ++o;
    }
}

// Down cycles: member list (cycle order) and the phases c_a.
__global__ void k_orbit_fill(int64_t count, const int32_t *__restrict__ rep_idx, const int32_t *__restrict__ shift,
                             const int32_t *__restrict__ phase, const int32_t *__restrict__ row,
                             const int32_t *__restrict__ orb_off, int32_t *__restrict__ cols,
                             int32_t *__restrict__ sgn)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int j = row[rep_idx[k]];
    const int o = orb_off[j] + shift[k];
    cols[o] = (int32_t)k;
    sgn[o] = phase[k];
}

// Sign g_s(G^-s b) for member m of a cycle of length q with phases c[] and
// sigma; the source member is (m - s) mod q.
__device__ __forceinline__ int cyc_sign(const int32_t *c, int q, int sigma, int m, int s, int *src)
{
    int a = (m - s) % q;
    if (a < 0) a += q;
    *src = a;
    const int tot = a + s;
    const int wraps = tot / q;
    int g = c[a] * c[tot - wraps * q];
    if ((wraps & 1) && sigma < 0) g = -g;
    return g;
}

template <typename T>
struct K0Args {
    const T *x;
    T *y;
    int64_t R;
    int M, L;
    const uint32_t *reps, *dn_basis;
    const T *rep_e, *e_dn;
    int uniform;
    T U;
    uint32_t umask;
    const T *Us;
    const int32_t *hop_rp, *hop_row, *hop_s;
    const T *hop_c;
    const int32_t *dn_rp, *dn_col;
    const T *dn_val;
    const int32_t *orb_off, *orb_cols, *orb_sign, *orb_sigma;
};

template <typename T>
__device__ __forceinline__ T k0_diag(const K0Args<T> &A, uint32_t both)
{
    if (A.uniform) return A.U * (T)__popc(both);
    T d = (T)0;
    uint32_t m = both & A.umask;
    while (m) {
        d += A.Us[__builtin_ctz(m)];
        m &= m - 1u;
    }
    return d;
}

// One workgroup per down cycle j: the cycle's q columns are staged in LDS
// (STAGE; R x q values) or read from global memory; wave w takes members
// m = w, w + NW, ... and its lanes take rows i = lane + 64 r.  Each lane
// computes whole output elements: diagonal, the H_up hops of row i (source
// member (m - s) mod q with its phase, from per-cycle tables in LDS) and the
// H_dn neighbour columns.
template <typename T, int BS, bool STAGE>
__global__ __launch_bounds__(BS) void k_k0_product(K0Args<T> A)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int NW = BS / 64;
    __shared__ int32_t cols[32], csg[32];
    __shared__ int8_t sg[32 * 32];
    __shared__ int8_t srcm[32 * 32];
    T *xs = reinterpret_cast<T *>(smem_raw);
    const int j = blockIdx.x;
    const int o0 = A.orb_off[j];
    const int q = A.orb_off[j + 1] - o0;
    const int sigma = A.orb_sigma[j];
    const int64_t R = A.R;
    if ((int)threadIdx.x < q) {
        cols[threadIdx.x] = A.orb_cols[o0 + threadIdx.x];
        csg[threadIdx.x] = A.orb_sign[o0 + threadIdx.x];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < q * A.L; t += BS) {
        const int m = t / A.L, s = t - (t / A.L) * A.L;
        int a;
        sg[m * 32 + s] = (int8_t)cyc_sign(csg, q, sigma, m, s, &a);
        srcm[m * 32 + s] = (int8_t)a;
    }
    if (STAGE) {
        for (int m = 0; m < q; ++m) {
            const T *xc = A.x + (int64_t)cols[m] * R;
            for (int64_t i = threadIdx.x; i < R; i += BS) xs[(int64_t)m * R + i] = xc[i];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int m = wave; m < q; m += NW) {
        const int b = cols[m];
        const uint32_t db = A.dn_basis[b];
        const T eb = A.e_dn[b];
        const int ks = A.dn_rp[b], ke = A.dn_rp[b + 1];
        for (int64_t i = lane; i < R; i += 64) {
            const T xv = STAGE ? xs[(int64_t)m * R + i] : A.x[(int64_t)b * R + i];
            T acc = (k0_diag(A, A.reps[i] & db) + A.rep_e[i] + eb) * xv;
            for (int h = A.hop_rp[i]; h < A.hop_rp[i + 1]; ++h) {
                const int s = A.hop_s[h];
                const int a = srcm[m * 32 + s];
                const int64_t r2 = A.hop_row[h];
                const T c = A.hop_c[h];
                const T xs2 = STAGE ? xs[(int64_t)a * R + r2] : A.x[(int64_t)cols[a] * R + r2];
                acc += (sg[m * 32 + s] < 0 ? -c : c) * xs2;
            }
            T s2 = (T)0;
            for (int k = ks; k < ke; ++k) s2 += A.dn_val[k] * A.x[(int64_t)A.dn_col[k] * R + i];
            A.y[(int64_t)b * R + i] = acc + s2;
        }
    }
}

// Projector onto the consistent subspace of the rows with P_i < L: one
// 64-lane block per (short row, down cycle); lane m holds member m and
// averages the q members over the stabiliser G^P_i (order L / P_i), in place.
template <typename T>
__global__ __launch_bounds__(64) void k_k0_project(T *x, int64_t R, int L, int64_t n_orb,
                                                   const int32_t *__restrict__ short_rows,
                                                   const int32_t *__restrict__ period,
                                                   const int32_t *__restrict__ short_sigma,
                                                   const int32_t *__restrict__ orb_off,
                                                   const int32_t *__restrict__ orb_cols,
                                                   const int32_t *__restrict__ orb_sign,
                                                   const int32_t *__restrict__ orb_sigma)
{
    __shared__ T v[32];
    __shared__ int32_t c[32];
    const int64_t r = blockIdx.x / n_orb, j = blockIdx.x - (blockIdx.x / n_orb) * n_orb;
    const int64_t i = short_rows[r];
    const int P = period[i];
    const int su = short_sigma[r];
    const int n = L / P;
    const int o0 = orb_off[j];
    const int q = orb_off[j + 1] - o0;
    const int sigma = orb_sigma[j];
    const int m = threadIdx.x;
    int64_t addr = 0;
    if (m < q) {
        addr = (int64_t)orb_cols[o0 + m] * R + i;
        v[m] = x[addr];
        c[m] = orb_sign[o0 + m];
    }
    __syncthreads();
    if (m < q) {
        double acc = 0.0;
        int gu = 1;
        for (int k = 0; k < n; ++k) {
            int a;
            const int g = cyc_sign(c, q, sigma, m, k * P, &a);
            acc += (double)(gu * g) * (double)v[a];
            gu *= su;
        }
        x[addr] = (T)(acc / (double)n);
    }
}

template <typename T>
K0Args<T> k0_args(const hub_sector *s, const void *x, void *y)
{
    const K0Tables &K = *s->k0;
    const SpinTables &Dn = s->spin[1];
    K0Args<T> A;
    A.x = (const T *)x;
    A.y = (T *)y;
    A.R = K.R;
    A.M = s->M;
    A.L = K.L;
    A.reps = K.reps;
    A.dn_basis = Dn.basis;
    A.uniform = s->uniformU;
    A.U = (T)s->U0;
    A.umask = s->umask;
    A.hop_rp = K.hop_rp;
    A.hop_row = K.hop_row;
    A.hop_s = K.hop_s;
    A.dn_rp = Dn.rp;
    A.dn_col = Dn.col;
    A.orb_off = K.orb_off;
    A.orb_cols = K.orb_cols;
    A.orb_sign = K.orb_sign;
    A.orb_sigma = K.orb_sigma;
    if constexpr (sizeof(T) == 8) {
        A.rep_e = K.rep_e64;
        A.e_dn = Dn.e64;
        A.Us = s->d_U64;
        A.hop_c = K.hop_c64;
        A.dn_val = Dn.val64;
    } else {
        A.rep_e = K.rep_e32;
        A.e_dn = Dn.e32;
        A.Us = s->d_U32;
        A.hop_c = (const T *)K.hop_c32;
        A.dn_val = (const T *)Dn.val32;
    }
    return A;
}

template <typename T>
hub_status k0_project_t(const hub_sector *s, void *x, hipStream_t st)
{
    const K0Tables &K = *s->k0;
    if (K.n_short == 0) return HUB_OK;
    const int64_t nb = K.n_short * K.n_orb;
    hipLaunchKernelGGL((k_k0_project<T>), dim3((unsigned)nb), dim3(64), 0, st, (T *)x, K.R, K.L, K.n_orb,
                       K.short_rows, K.period, K.short_sigma, K.orb_off, K.orb_cols, K.orb_sign, K.orb_sigma);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

template <typename T>
hub_status k0_product_t(const hub_sector *s, const void *x, void *y, hipStream_t st)
{
    constexpr int BS = 1024;
    const K0Tables &K = *s->k0;
    const K0Args<T> A = k0_args<T>(s, x, y);
    const size_t lds = (size_t)K.max_q * (size_t)K.R * sizeof(T);
    // the kernel also holds up to 2.2 KB of static LDS (cycle tables)
    const size_t dyn_max = s->lds_max - 4096;
    if (lds <= dyn_max) {
        static std::atomic<bool> attr{false};
        if (!attr) {
            HUB_HIP(hipFuncSetAttribute((const void *)k_k0_product<T, BS, true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_max));
            attr = true;
        }
        hipLaunchKernelGGL((k_k0_product<T, BS, true>), dim3((unsigned)K.n_orb), dim3(BS), lds, st, A);
    } else {
        hipLaunchKernelGGL((k_k0_product<T, BS, false>), dim3((unsigned)K.n_orb), dim3(BS), 0, st, A);
    }
    HUB_HIP(hipGetLastError());
    return k0_project_t<T>(s, y, st);
}

hub_status tfail(hub_status c, const std::string &m)
{
    set_error(m);
    return c;
}

template <typename T>
hub_status talloc(hub_sector *s, T **p, size_t n)
{
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, (n == 0 ? 1 : n) * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return tfail(HUB_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    s->owned.push_back(q);
    *p = (T *)q;
    return HUB_OK;
}

struct CycleTables {
    int32_t *rep_idx = nullptr, *shift = nullptr, *phase = nullptr, *period = nullptr, *sigma = nullptr,
            *is_rep = nullptr, *pos = nullptr, *row = nullptr;
    int64_t nrep = 0;
};

hub_status cycles_of(hub_sector *s, int spin, int w, CycleTables &c, hipStream_t st)
{
    const SpinTables &S = s->spin[spin];
    const int64_t n = S.count;
    HUB_TRY(talloc(s, &c.rep_idx, n));
    HUB_TRY(talloc(s, &c.shift, n));
    HUB_TRY(talloc(s, &c.phase, n));
    HUB_TRY(talloc(s, &c.period, n));
    HUB_TRY(talloc(s, &c.sigma, n));
    HUB_TRY(talloc(s, &c.is_rep, n));
    HUB_TRY(talloc(s, &c.pos, n + 1));
    HUB_TRY(talloc(s, &c.row, n));
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_cycles, dim3(g), dim3(256), 0, st, S.basis, n, s->M, S.N, w, (const uint64_t *)s->d_binom,
                       c.rep_idx, c.shift, c.phase, c.period, c.sigma, c.is_rep);
    HUB_HIP(hipGetLastError());
    HUB_TRY(scan_lengths(s, c.is_rep, n, c.pos, st));
    hipLaunchKernelGGL(k_rep_rows, dim3(g), dim3(256), 0, st, c.is_rep, (const int32_t *)c.pos, n, c.row);
    HUB_HIP(hipGetLastError());
    int32_t nr = 0;
    HUB_HIP(hipMemcpyAsync(&nr, c.pos + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HUB_HIP(hipStreamSynchronize(st));
    c.nrep = nr;
    return HUB_OK;
}

hub_status build_k0(hub_sector *s, int w, hipStream_t st)
{
    const int M = s->M;
    if (w < 1 || w >= M || M % w != 0) return tfail(HUB_ERR_INVALID_ARG, "shift must divide M and be < M");
    // the model must be invariant under i -> i - w (mod M): bonds with equal t, uniform U and eps
    for (int e = 0; e < s->nb; ++e) {
        int a = ((s->bi[e] - w) % M + M) % M, b = ((s->bj[e] - w) % M + M) % M;
        if (a > b) std::swap(a, b);
        bool found = false;
        for (int f = 0; f < s->nb; ++f)
            if (s->bi[f] == a && s->bj[f] == b && s->t[f] == s->t[e]) found = true;
        if (!found) return tfail(HUB_ERR_INVALID_ARG, "the bonds are not invariant under the translation");
    }
    for (int i = 1; i < M; ++i)
        if (s->U[i] != s->U[0] || s->eps[i] != s->eps[0])
            return tfail(HUB_ERR_INVALID_ARG, "U and eps must be uniform for translation symmetry");
    K0Tables *K = new (std::nothrow) K0Tables();
    if (!K) return tfail(HUB_ERR_OOM, "host allocation failed");
    s->k0 = K;
    K->w = w;
    K->L = M / w;
    if (K->L > 32) return tfail(HUB_ERR_UNSUPPORTED, "translation group order above 32");
    CycleTables cu, cd;
    HUB_TRY(cycles_of(s, 0, w, cu, st));
    HUB_TRY(cycles_of(s, 1, w, cd, st));
    const int64_t R = cu.nrep, nu = s->spin[0].count, nd = s->spin[1].count;
    K->R = R;
    K->n_orb = cd.nrep;
    // up representatives
    int32_t *rsig = nullptr;
    HUB_TRY(talloc(s, &K->reps, R));
    HUB_TRY(talloc(s, &K->period, R));
    HUB_TRY(talloc(s, &rsig, R));
    HUB_TRY(talloc(s, &K->rep_e64, R));
    HUB_TRY(talloc(s, &K->rep_e32, R));
    const unsigned gu = (unsigned)((nu + 255) / 256), gd = (unsigned)((nd + 255) / 256);
    hipLaunchKernelGGL(k_rep_fill, dim3(gu), dim3(256), 0, st, s->spin[0].basis, cu.is_rep, cu.row, cu.period,
                       cu.sigma, s->spin[0].e64, nu, K->reps, K->period, rsig, K->rep_e64, K->rep_e32);
    // up hops
    int32_t *len = nullptr;
    HUB_TRY(talloc(s, &len, R));
    HUB_TRY(talloc(s, &K->hop_rp, R + 1));
    const unsigned gr = (unsigned)((R + 255) / 256);
    hipLaunchKernelGGL(k_hop_count, dim3(gr), dim3(256), 0, st, K->reps, R, s->d_bi, s->d_bj, s->nb, len);
    HUB_HIP(hipGetLastError());
    HUB_TRY(scan_lengths(s, len, R, K->hop_rp, st));
    int32_t nnz = 0;
    HUB_HIP(hipMemcpyAsync(&nnz, K->hop_rp + R, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HUB_HIP(hipStreamSynchronize(st));
    K->hop_nnz = nnz;
    HUB_TRY(talloc(s, &K->hop_row, nnz));
    HUB_TRY(talloc(s, &K->hop_s, nnz));
    HUB_TRY(talloc(s, &K->hop_c64, nnz));
    HUB_TRY(talloc(s, &K->hop_c32, nnz));
    hipLaunchKernelGGL(k_hop_fill, dim3(gr), dim3(256), 0, st, K->reps, R, K->period, s->d_bi, s->d_bj, s->d_t,
                       s->nb, (const uint64_t *)s->d_binom, cu.rep_idx, cu.shift, cu.phase, cu.row, K->hop_rp,
                       K->hop_row, K->hop_s, K->hop_c64, K->hop_c32);
    HUB_HIP(hipGetLastError());
    // down cycles: offsets from the representatives' periods
    uint32_t *dreps = nullptr;
    int32_t *dper = nullptr;
    double *de64 = nullptr;
    float *de32 = nullptr;
    HUB_TRY(talloc(s, &dreps, K->n_orb));
    HUB_TRY(talloc(s, &dper, K->n_orb));
    HUB_TRY(talloc(s, &K->orb_sigma, K->n_orb));
    HUB_TRY(talloc(s, &de64, K->n_orb));
    HUB_TRY(talloc(s, &de32, K->n_orb));
    hipLaunchKernelGGL(k_rep_fill, dim3(gd), dim3(256), 0, st, s->spin[1].basis, cd.is_rep, cd.row, cd.period,
                       cd.sigma, s->spin[1].e64, nd, dreps, dper, K->orb_sigma, de64, de32);
    HUB_TRY(talloc(s, &K->orb_off, K->n_orb + 1));
    HUB_TRY(scan_lengths(s, dper, K->n_orb, K->orb_off, st));
    HUB_TRY(talloc(s, &K->orb_cols, nd));
    HUB_TRY(talloc(s, &K->orb_sign, nd));
    hipLaunchKernelGGL(k_orbit_fill, dim3(gd), dim3(256), 0, st, nd, cd.rep_idx, cd.shift, cd.phase, cd.row,
                       K->orb_off, K->orb_cols, K->orb_sign);
    HUB_HIP(hipGetLastError());
    // host: longest down cycle and the short up rows
    std::vector<int32_t> hper(R), hsig(R), hdp(K->n_orb);
    HUB_HIP(hipMemcpyAsync(hper.data(), K->period, sizeof(int32_t) * R, hipMemcpyDeviceToHost, st));
    HUB_HIP(hipMemcpyAsync(hsig.data(), rsig, sizeof(int32_t) * R, hipMemcpyDeviceToHost, st));
    HUB_HIP(hipMemcpyAsync(hdp.data(), dper, sizeof(int32_t) * K->n_orb, hipMemcpyDeviceToHost, st));
    HUB_HIP(hipStreamSynchronize(st));
    for (int32_t q : hdp) K->max_q = std::max(K->max_q, (int)q);
    std::vector<int32_t> sr, ss;
    for (int64_t i = 0; i < R; ++i)
        if (hper[i] < K->L) {
            sr.push_back((int32_t)i);
            ss.push_back(hsig[i]);
        }
    K->n_short = (int64_t)sr.size();
    HUB_TRY(talloc(s, &K->short_rows, sr.size()));
    HUB_TRY(talloc(s, &K->short_sigma, sr.size()));
    if (!sr.empty()) {
        HUB_HIP(hipMemcpy(K->short_rows, sr.data(), sizeof(int32_t) * sr.size(), hipMemcpyHostToDevice));
        HUB_HIP(hipMemcpy(K->short_sigma, ss.data(), sizeof(int32_t) * ss.size(), hipMemcpyHostToDevice));
    }
    if (R * nd >= ((int64_t)1 << 40)) return tfail(HUB_ERR_RANGE, "k = 0 space too large");
    s->dim = R * nd;
    return HUB_OK;
}

}  // namespace

hub_status apply_h(const hub_sector *s, int dtype, const void *x, void *y, hipStream_t st)
{
    if (!s->k0) return launch_matvec(s, dtype, x, y, st);
    if (dtype == HUB_F64) return k0_product_t<double>(s, x, y, st);
    return k0_product_t<float>(s, x, y, st);
}

hub_status k0_project(const hub_sector *s, int dtype, void *x, hipStream_t st)
{
    if (!s->k0) return HUB_OK;
    if (dtype == HUB_F64) return k0_project_t<double>(s, x, st);
    return k0_project_t<float>(s, x, st);
}

}  // namespace hub

using namespace hub;

extern "C" {

hub_status hub_sector_create_k0(const hub_model *model, int32_t n_up, int32_t n_dn, int32_t shift, hub_sector **out)
{
    if (!out) return tfail(HUB_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    hub_sector *s = nullptr;
    HUB_TRY(hub_sector_create(model, n_up, n_dn, &s));
    hipStream_t st = nullptr;
    const hub_status r = build_k0(s, shift, st);
    if (r != HUB_OK) {
        hub_sector_destroy(s);
        return r;
    }
    *out = s;
    return HUB_OK;
}

hub_status hub_k0_layout(const hub_sector *sec, int64_t *n_reps, uint64_t *reps, int32_t *periods)
{
    if (!sec || !n_reps) return tfail(HUB_ERR_INVALID_ARG, "NULL argument");
    if (!sec->k0) return tfail(HUB_ERR_INVALID_ARG, "not a translation (k = 0) sector");
    const K0Tables &K = *sec->k0;
    *n_reps = K.R;
    HUB_HIP(hipSetDevice(sec->device));
    if (reps) {
        std::vector<uint32_t> h(K.R);
        HUB_HIP(hipMemcpy(h.data(), K.reps, sizeof(uint32_t) * K.R, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < K.R; ++i) reps[i] = h[i];
    }
    if (periods) HUB_HIP(hipMemcpy(periods, K.period, sizeof(int32_t) * K.R, hipMemcpyDeviceToHost));
    return HUB_OK;
}

}  // extern "C"
