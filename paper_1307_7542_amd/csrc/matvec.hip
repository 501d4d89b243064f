// Kronecker-sum product of the sector Hamiltonian (Sec. IV A):
//
//     Y = H_up V + V H_dn^T + D o V,   V, Y: count_up x count_dn, column-major.
//
// H_dn is real symmetric, so column b of V H_dn^T is sum_l H_dn[b, l] V[:, l]
// and row a of it is H_dn applied to row a of V.  D(a, b) = U-part(basis_up[a]
// & basis_dn[b]) + e_up[a] + e_dn[b] is generated from the bit patterns (the
// doubly occupied sites of Sec. III B) and never stored.
//
// The two terms want orthogonal access patterns: the H_up term gathers inside
// one column of V, the H_dn term inside one row.  Schedules (hub_schedule in
// hubbard.h; the tuner times the candidates on the first product):
//
//   columns   whole columns of V staged in LDS (k_kron_quad, four rows per
//             lane): the H_up term gathers from LDS; in one pass the H_dn term
//             reads its neighbour columns through L2 / MALL.
//   chunked   columns larger than the LDS (k_kron_chunked_parts): the columns
//             are staged chunk by chunk while the output rows stay in registers.
//   rows      one row per lane (k_kron_fused), for count_up % 4 != 0 or
//             vectors that are not 16-byte aligned.
//   csr       rows of the CSR gathered from global memory (no compact entries).
//
// Every schedule computes each element as: diagonal, then the H_up entries in
// column order, then the H_dn entries in column order, one fused multiply-add
// per term, so all give bit-identical products (tested).
//
// H_up is read from its sliced-ELL copy: lane r of a wavefront owns row
// 64*s + r of slice s and loads entry k from a coalesced address; the default
// entry is {column : 24, code : 8} with the value looked up in a 256-entry
// table in LDS (code = 2 bond + (esign < 0), 255 = padding).
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "internal.h"

namespace hub {
namespace {

template <typename T>
struct MvArgs {
    const T *__restrict__ x;
    T *y;
    int32_t cu, cd;
    const int32_t *__restrict__ up_rp;
    const int32_t *__restrict__ up_col;
    const T *__restrict__ up_val;
    const int32_t *__restrict__ dn_rp;
    const int32_t *__restrict__ dn_col;
    const T *__restrict__ dn_val;
    const uint32_t *__restrict__ up_basis;
    const uint32_t *__restrict__ dn_basis;
    const T *__restrict__ e_up;
    const T *__restrict__ e_dn;
    const T *__restrict__ Us;  // per-site U (non-uniform case)
    T U;
    int32_t uniform;
    uint32_t umask;
    int32_t stream;  // vectors beyond the MALL: data read or written once bypasses retention (k_kron_quad)
};

template <typename T>
using Pk = typename std::conditional<sizeof(T) == 8, uint4, uint2>::type;

__device__ __forceinline__ void unpack(uint2 e, int &c, float &v)
{
    c = (int)e.x;
    v = __uint_as_float(e.y);
}

__device__ __forceinline__ void unpack(uint4 e, int &c, double &v)
{
    c = (int)e.x;
    v = __hiloint2double((int)e.w, (int)e.z);
}

template <typename T>
__device__ __forceinline__ T diag_u(const MvArgs<T> &A, uint32_t both)
{
    if (A.uniform) return A.U * (T)__popc(both);
    T d = (T)0;
    uint32_t m = both & A.umask;
    while (m) {
        const int i = __builtin_ctz(m);
        d += A.Us[i];
        m &= m - 1u;
    }
    return d;
}

template <typename T, int TB>
struct Vec {
    T v[TB];
};

// acc[t] += sum_k val_k * xs[col_k * TB + t] over the sliced-ELL row, 4 entries in flight.
template <typename T, int TB>
__device__ __forceinline__ void up_term(T (&acc)[TB], const T *xs, const Pk<T> *__restrict__ ell, int o0, int len)
{
    int k = 0;
    for (; k + 4 <= len; k += 4) {
        int c0, c1, c2, c3;
        T v0, v1, v2, v3;
        unpack(ell[o0 + 64 * k], c0, v0);
        unpack(ell[o0 + 64 * (k + 1)], c1, v1);
        unpack(ell[o0 + 64 * (k + 2)], c2, v2);
        unpack(ell[o0 + 64 * (k + 3)], c3, v3);
        const Vec<T, TB> x0 = *reinterpret_cast<const Vec<T, TB> *>(xs + c0 * TB);
        const Vec<T, TB> x1 = *reinterpret_cast<const Vec<T, TB> *>(xs + c1 * TB);
        const Vec<T, TB> x2 = *reinterpret_cast<const Vec<T, TB> *>(xs + c2 * TB);
        const Vec<T, TB> x3 = *reinterpret_cast<const Vec<T, TB> *>(xs + c3 * TB);
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            acc[t] += v0 * x0.v[t];
            acc[t] += v1 * x1.v[t];
            acc[t] += v2 * x2.v[t];
            acc[t] += v3 * x3.v[t];
        }
    }
    for (; k < len; ++k) {
        int c0;
        T v0;
        unpack(ell[o0 + 64 * k], c0, v0);
        const Vec<T, TB> x0 = *reinterpret_cast<const Vec<T, TB> *>(xs + c0 * TB);
#pragma unroll
        for (int t = 0; t < TB; ++t) acc[t] += v0 * x0.v[t];
    }
}

// Same with compact entries {column : 24, code : 8}; the values come from the
// per-code table `tab` held in LDS (code 255 = padding, value 0).
template <typename T, int TB>
__device__ __forceinline__ void up_term_c(T (&acc)[TB], const T *xs, const T *tab,
                                          const uint32_t *__restrict__ ell, int o0, int len)
{
    int k = 0;
    for (; k + 4 <= len; k += 4) {
        const uint32_t e0 = ell[o0 + 64 * k], e1 = ell[o0 + 64 * (k + 1)];
        const uint32_t e2 = ell[o0 + 64 * (k + 2)], e3 = ell[o0 + 64 * (k + 3)];
        const T v0 = tab[e0 >> 24], v1 = tab[e1 >> 24], v2 = tab[e2 >> 24], v3 = tab[e3 >> 24];
        const Vec<T, TB> x0 = *reinterpret_cast<const Vec<T, TB> *>(xs + (e0 & 0xFFFFFFu) * TB);
        const Vec<T, TB> x1 = *reinterpret_cast<const Vec<T, TB> *>(xs + (e1 & 0xFFFFFFu) * TB);
        const Vec<T, TB> x2 = *reinterpret_cast<const Vec<T, TB> *>(xs + (e2 & 0xFFFFFFu) * TB);
        const Vec<T, TB> x3 = *reinterpret_cast<const Vec<T, TB> *>(xs + (e3 & 0xFFFFFFu) * TB);
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            acc[t] += v0 * x0.v[t];
            acc[t] += v1 * x1.v[t];
            acc[t] += v2 * x2.v[t];
            acc[t] += v3 * x3.v[t];
        }
    }
    for (; k < len; ++k) {
        const uint32_t e0 = ell[o0 + 64 * k];
        const T v0 = tab[e0 >> 24];
        const Vec<T, TB> x0 = *reinterpret_cast<const Vec<T, TB> *>(xs + (e0 & 0xFFFFFFu) * TB);
#pragma unroll
        for (int t = 0; t < TB; ++t) acc[t] += v0 * x0.v[t];
    }
}

// acc += sum_k H_dn[b, k] x[a + col_k * cu] over row b of H_dn (uniform over the wavefront).
template <typename T>
__device__ __forceinline__ void dn_term(T &acc, const MvArgs<T> &A, int ks, int ke, const T *__restrict__ xa)
{
    const int64_t cu = A.cu;
    for (int k = ks; k < ke; ++k) acc += A.dn_val[k] * xa[(int64_t)A.dn_col[k] * cu];
}

// Block -> tile with every XCD (workgroup i runs on XCD i mod 8) owning a
// contiguous range of tiles; returns -1 for the padding blocks.
__device__ __forceinline__ int xcd_tile(int ntiles)
{
    const int per = (ntiles + 7) >> 3;
    const int t = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    return t < ntiles ? t : -1;
}

template <typename T, int TB>
__device__ __forceinline__ void stage_columns(const MvArgs<T> &A, T *xs, int b0, int bs)
{
#pragma unroll
    for (int t = 0; t < TB; ++t) {
        const int b = b0 + t;
        const T *__restrict__ xb = A.x + (int64_t)min(b, A.cd - 1) * A.cu;
        for (int a = threadIdx.x; a < A.cu; a += bs) xs[a * TB + t] = (b < A.cd) ? xb[a] : (T)0;
    }
}

// ---- 16-byte accesses ---------------------------------------------------
template <typename T>
struct Q4 {
    T v[4];
};

template <typename T>
__device__ __forceinline__ Q4<T> ld_q4(const T *p)
{
    Q4<T> r;
    if constexpr (sizeof(T) == 4) {
        const float4 q = *reinterpret_cast<const float4 *>(p);
        r.v[0] = q.x;
        r.v[1] = q.y;
        r.v[2] = q.z;
        r.v[3] = q.w;
    } else {
        const double2 q0 = reinterpret_cast<const double2 *>(p)[0], q1 = reinterpret_cast<const double2 *>(p)[1];
        r.v[0] = q0.x;
        r.v[1] = q0.y;
        r.v[2] = q1.x;
        r.v[3] = q1.y;
    }
    return r;
}

// streaming (non-temporal) variants for data read or written once
template <typename T>
__device__ __forceinline__ Q4<T> ld_q4_nt(const T *p)
{
    Q4<T> r;
    if constexpr (sizeof(T) == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 q = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(p));
        r.v[0] = q.x;
        r.v[1] = q.y;
        r.v[2] = q.z;
        r.v[3] = q.w;
    } else {
        typedef double d2 __attribute__((ext_vector_type(2)));
        const d2 q0 = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(p));
        const d2 q1 = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(p) + 1);
        r.v[0] = q0.x;
        r.v[1] = q0.y;
        r.v[2] = q1.x;
        r.v[3] = q1.y;
    }
    return r;
}

template <typename T>
__device__ __forceinline__ void st_q4_nt(T *p, const T (&v)[4])
{
    if constexpr (sizeof(T) == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 q = {v[0], v[1], v[2], v[3]};
        __builtin_nontemporal_store(q, reinterpret_cast<f4 *>(p));
    } else {
        typedef double d2 __attribute__((ext_vector_type(2)));
        const d2 q0 = {v[0], v[1]}, q1 = {v[2], v[3]};
        __builtin_nontemporal_store(q0, reinterpret_cast<d2 *>(p));
        __builtin_nontemporal_store(q1, reinterpret_cast<d2 *>(p) + 1);
    }
}

template <typename T>
__device__ __forceinline__ void st_q4(T *p, const T (&v)[4])
{
    if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        reinterpret_cast<double2 *>(p)[0] = make_double2(v[0], v[1]);
        reinterpret_cast<double2 *>(p)[1] = make_double2(v[2], v[3]);
    }
}

// First Lanczos update fused into the product's epilogue: w = (H x) - beta v_prev
// (rounded as the separate update kernel does) and partial sums of w * x.
//
// unnorm: the Lanczos vectors are kept unnormalised, x = beta_k v_k and
// vprev = beta_{k-1} v_{k-1} (beta_0 taken as 1, beta NULL at the first step),
// and the epilogue forms w = (H x) / beta_k - (beta_k / beta_{k-1}) vprev in
// FP64 before the one rounding; the partials are then of <w, x> = beta_k alpha_k.
// Both updates are written as explicit fused multiply-adds, so every tile
// shape (each its own template instance) rounds them the same way.
template <typename T>
struct LzEpi {
    const T *vprev;           // NULL at the first step
    const double *beta;       // beta_k (device)
    double *apart;            // [cd] per-column partials
    int G;                    // lane-quad groups per column: ceil(count_up / 256)
    const double *beta_prev;  // unnorm: beta_{k-1} (device), NULL for beta_0
    int unnorm;
    double *gpart;            // row-chunked product: [cd][G] group partials (summed into apart per column)
};

__device__ __forceinline__ double inv_beta(const double *b)
{
    if (!b) return 1.0;
    const double v = *b;
    return v > 0.0 ? 1.0 / v : 0.0;
}

__device__ __forceinline__ double quad_wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
struct EpiCoef {
    double sx = 1.0, bt = 0.0;
};

template <typename T>
__device__ __forceinline__ EpiCoef<T> epi_coef(const LzEpi<T> &E)
{
    EpiCoef<T> c;
    if (E.unnorm) {
        c.sx = inv_beta(E.beta);
        c.bt = E.vprev ? *E.beta * inv_beta(E.beta_prev) : 0.0;
    } else if (E.vprev) {
        c.bt = *E.beta;
    }
    return c;
}

// w from the product value o and the v_prev value vp (see LzEpi)
template <typename T>
__device__ __forceinline__ T epi_w(const LzEpi<T> &E, const EpiCoef<T> &c, T o, T vp)
{
    if (E.unnorm) {
        if (E.vprev) return (T)fma(c.sx, (double)o, -(c.bt * (double)vp));
        return (T)(c.sx * (double)o);
    }
    if (E.vprev) return (T)fma(-c.bt, (double)vp, (double)o);
    return o;
}

// ---- whole columns in LDS, four consecutive rows per lane -----------------
// One workgroup per TB output columns; lane q owns rows 4q .. 4q+3 (count_up %
// 4 == 0): the column staging, the H_dn neighbour reads and the stores are
// 16-byte (FP32) or 2 x 16-byte (FP64) accesses, and the four rows' sliced-ELL
// entries k are four consecutive lanes of the slice, read with one 16-byte
// load.  XC: XCD-contiguous tile order (workgroup i on XCD i mod 8 takes the
// i-th tile of that XCD's range) or plain launch order.  EPI: the first
// Lanczos update, each group of 64 lane-quads (256 rows) summed by one
// wavefront in a fixed order, then the groups of a column in increasing order,
// so the per-column partials do not depend on the tile shape.
template <typename T, int TB, int BS, bool XC, bool EPI>
__global__ __launch_bounds__(BS) void k_kron_quad(MvArgs<T> A, const int32_t *__restrict__ sl_off,
                                                  const uint32_t *__restrict__ ellc, const T *__restrict__ code_v,
                                                  int ntiles, LzEpi<T> E)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tab = reinterpret_cast<T *>(smem_raw);  // 256 code values
    T *xs = tab + 256;                         // TB staged columns, interleaved
    double *gpart = reinterpret_cast<double *>(xs + TB * A.cu);  // EPI: TB x G group partials
    int tile;
    if (XC) {
        tile = xcd_tile(ntiles);
    } else {
        tile = (int)blockIdx.x < ntiles ? (int)blockIdx.x : -1;
    }
    if (tile < 0) return;
    const int cu = A.cu, cd = A.cd, nq = cu >> 2;
    const int b0 = tile * TB;
    for (int i = threadIdx.x; i < 256; i += BS) tab[i] = code_v[i];
#pragma unroll
    for (int t = 0; t < TB; ++t) {
        const T *__restrict__ xb = A.x + (int64_t)min(b0 + t, cd - 1) * cu;
        for (int q = threadIdx.x; q < nq; q += BS) {
            const Q4<T> v = ld_q4(xb + 4 * q);
#pragma unroll
            for (int r = 0; r < 4; ++r) xs[(4 * q + r) * TB + t] = v.v[r];
        }
    }
    __syncthreads();
    int ds[TB], de[TB];
    uint32_t dnb[TB];
    T edn[TB];
#pragma unroll
    for (int t = 0; t < TB; ++t) {
        const int b = min(b0 + t, cd - 1);
        ds[t] = A.dn_rp[b];
        de[t] = (b0 + t < cd) ? A.dn_rp[b + 1] : ds[t];
        dnb[t] = A.dn_basis[b];
        edn[t] = A.e_dn[b];
    }
    const int64_t cu64 = cu;
    const int lane = threadIdx.x & 63;
    EpiCoef<T> ec;
    if (EPI) ec = epi_coef(E);
    // with the epilogue every lane of a wavefront runs the same iterations (it
    // reduces over the wavefront); without it a lane stops after its last quad
    for (int q = threadIdx.x; EPI ? (q - lane < nq) : (q < nq); q += BS) {
        const bool live = !EPI || q < nq;
        const int a0 = 4 * (live ? q : 0);
        T acc[4][TB];
        // the epilogue's v_prev rows are loaded first: a lane runs only one or
        // two iterations, so a load issued after the gathers leaves its latency exposed
        Q4<T> vpq[EPI ? TB : 1];
        if (EPI && live && E.vprev) {
#pragma unroll
            for (int t = 0; t < TB; ++t)
                vpq[t] = A.stream ? ld_q4_nt(E.vprev + (int64_t)min(b0 + t, cd - 1) * cu64 + a0)
                                  : ld_q4(E.vprev + (int64_t)min(b0 + t, cd - 1) * cu64 + a0);
        }
        const uint4 ub = *reinterpret_cast<const uint4 *>(A.up_basis + a0);
        const uint32_t uu[4] = {ub.x, ub.y, ub.z, ub.w};
        const Q4<T> eu = ld_q4(A.e_up + a0);
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int t = 0; t < TB; ++t)
                acc[r][t] = (diag_u(A, uu[r] & dnb[t]) + eu.v[r] + edn[t]) * xs[(a0 + r) * TB + t];
        // H_up term: entries k of rows a0 .. a0+3 are lanes (a0 & 63) .. +3 of slice a0 >> 6
        const int s = a0 >> 6;
        const uint4 *__restrict__ e4 = reinterpret_cast<const uint4 *>(ellc + (int64_t)sl_off[s] * 64 + (a0 & 63));
        const int len = sl_off[s + 1] - sl_off[s];
        int k = 0;
        for (; k + 2 <= len; k += 2) {
            const uint4 ea = e4[16 * k], eb = e4[16 * (k + 1)];
            const uint32_t e[8] = {ea.x, ea.y, ea.z, ea.w, eb.x, eb.y, eb.z, eb.w};
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const T v = tab[e[i] >> 24];
                const T *xr = xs + (e[i] & 0xFFFFFFu) * TB;
#pragma unroll
                for (int t = 0; t < TB; ++t) acc[i & 3][t] += v * xr[t];
            }
        }
        if (k < len) {
            const uint4 ea = e4[16 * k];
            const uint32_t e[4] = {ea.x, ea.y, ea.z, ea.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const T v = tab[e[i] >> 24];
                const T *xr = xs + (e[i] & 0xFFFFFFu) * TB;
#pragma unroll
                for (int t = 0; t < TB; ++t) acc[i][t] += v * xr[t];
            }
        }
        // H_dn term: whole neighbour columns, four rows per load
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            int kk = ds[t];
            for (; kk + 4 <= de[t]; kk += 4) {
                Q4<T> v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = ld_q4(A.x + (int64_t)A.dn_col[kk + u] * cu64 + a0);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const T w = A.dn_val[kk + u];
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[r][t] += w * v[u].v[r];
                }
            }
            for (; kk < de[t]; ++kk) {
                const Q4<T> v = ld_q4(A.x + (int64_t)A.dn_col[kk] * cu64 + a0);
                const T w = A.dn_val[kk];
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r][t] += w * v.v[r];
            }
        }
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            if (b0 + t >= cd) continue;
            T o[4] = {acc[0][t], acc[1][t], acc[2][t], acc[3][t]};
            if (EPI) {
                double part = 0.0;
                if (live) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) o[r] = epi_w(E, ec, o[r], E.vprev ? vpq[t].v[r] : (T)0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) part += (double)o[r] * (double)xs[(a0 + r) * TB + t];
                }
                part = quad_wave_sum(part);
                if (lane == 0) gpart[t * E.G + (q >> 6)] = part;
            }
            if (live) {
                if (A.stream) st_q4_nt(A.y + (int64_t)(b0 + t) * cu64 + a0, o);
                else st_q4(A.y + (int64_t)(b0 + t) * cu64 + a0, o);
            }
        }
    }
    if (EPI) {
        // one partial per column: its groups summed in increasing order
        __syncthreads();
        if (threadIdx.x < TB && b0 + (int)threadIdx.x < cd) {
            double sum = 0.0;
            for (int g = 0; g < E.G; ++g) sum += gpart[threadIdx.x * E.G + g];
            E.apart[b0 + threadIdx.x] = sum;
        }
    }
}

// ---- columns larger than the LDS: row-chunked staging --------------------
// Work item (tile of TB columns, row part j) owns quads [j BS QPL, (j+1) BS
// QPL) of its columns, QPL per lane.  It stages every row chunk of its columns
// in turn (interleaved, element (a, t) at a TB + t) and accumulates the chunk's
// H_up entries of its rows, each entry serving the TB columns; then the H_dn
// term and one store.  No partial results go through memory.  Tiles are
// interleaved over the XCDs (tile = 8 k + xcd) and row parts dispatched in
// turn (every tile's first part, then every tile's second, ...), so the
// neighbour rows the H_dn term reads at a time are one part's (2x9 ladder:
// FP32 30.6 -> 30.0 ms, FP64 57.8 -> 56.1 ms against the parts of a tile
// dispatched together).
//
// EPI: the first Lanczos update fused into the store, as in k_kron_quad: each
// wavefront's 64 lane-quads (one group of 256 rows of a column) are summed in
// the same fixed order into E.gpart[column][group]; k_epi_colsum then adds a
// column's groups in increasing order, so the per-column partials equal the
// columns schedule's bit for bit.
template <typename T, int BS, int QPL, int TB, bool EPI>
__global__ __launch_bounds__(BS) void k_kron_chunked_parts(MvArgs<T> A, const int32_t *__restrict__ ch_off,
                                                           const int64_t *__restrict__ ch_base,
                                                           const uint32_t *__restrict__ ch_ell,
                                                           const T *__restrict__ code_v, int nchunks,
                                                           int chunk_rows, int nslices, int P, LzEpi<T> E)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tab = reinterpret_cast<T *>(smem_raw);
    T *xs = tab + 256;
    const int xcd = (int)(blockIdx.x & 7), r = (int)(blockIdx.x >> 3);
    const int cd = A.cd;
    const int ntiles = (cd + TB - 1) / TB;
    const int n8 = (ntiles + 7) / 8;
    const int tile = 8 * (r % n8) + xcd, part = r / n8;
    if (tile >= ntiles) return;
    const int b0 = tile * TB;
    const int cu = A.cu, nq = cu >> 2;
    const int64_t cu64 = cu;
    const int qa = part * BS * QPL;
    for (int i = threadIdx.x; i < 256; i += BS) tab[i] = code_v[i];
    const T *xb[TB];
    uint32_t dnb[TB];
    T edn[TB];
    int ds[TB], de[TB];
#pragma unroll
    for (int t = 0; t < TB; ++t) {
        const int b = min(b0 + t, cd - 1);
        xb[t] = A.x + (int64_t)b * cu;
        dnb[t] = A.dn_basis[b];
        edn[t] = A.e_dn[b];
        ds[t] = A.dn_rp[b];
        de[t] = (b0 + t < cd) ? A.dn_rp[b + 1] : ds[t];
    }
    T acc[QPL][4][TB];
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
        const int q = qa + (int)threadIdx.x + i * BS;
        if (q < nq) {
            const int a0 = 4 * q;
            const uint4 ub = *reinterpret_cast<const uint4 *>(A.up_basis + a0);
            const uint32_t uu[4] = {ub.x, ub.y, ub.z, ub.w};
            const Q4<T> eu = ld_q4(A.e_up + a0);
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                const Q4<T> xv = ld_q4(xb[t] + a0);
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
                    acc[i][rr][t] = (diag_u(A, uu[rr] & dnb[t]) + eu.v[rr] + edn[t]) * xv.v[rr];
            }
        }
    }
    for (int p = 0; p < nchunks; ++p) {
        const int q0 = (p * chunk_rows) >> 2;
        const int q1 = min(nq, q0 + (chunk_rows >> 2));
        __syncthreads();  // previous chunk done with xs
#pragma unroll
        for (int t = 0; t < TB; ++t)
            for (int q = q0 + threadIdx.x; q < q1; q += BS) {
                const Q4<T> v = ld_q4(xb[t] + 4 * q);
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) xs[(4 * (q - q0) + rr) * TB + t] = v.v[rr];
            }
        __syncthreads();
        const int32_t *off = ch_off + (int64_t)p * (nslices + 1);
        const uint32_t *ell = ch_ell + ch_base[p];
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            const int q = qa + (int)threadIdx.x + i * BS;
            if (q >= nq) continue;
            const int a0 = 4 * q;
            const int sl = a0 >> 6;
            const uint4 *__restrict__ e4 = reinterpret_cast<const uint4 *>(ell + (int64_t)off[sl] * 64 + (a0 & 63));
            const int len = off[sl + 1] - off[sl];
            int k = 0;
            for (; k + 2 <= len; k += 2) {
                const uint4 ea = e4[16 * k], eb = e4[16 * (k + 1)];
                const uint32_t e[8] = {ea.x, ea.y, ea.z, ea.w, eb.x, eb.y, eb.z, eb.w};
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const T v = tab[e[u] >> 24];
                    const T *xr = xs + (e[u] & 0xFFFFFFu) * TB;
#pragma unroll
                    for (int t = 0; t < TB; ++t) acc[i][u & 3][t] += v * xr[t];
                }
            }
            if (k < len) {
                const uint4 ea = e4[16 * k];
                const uint32_t e[4] = {ea.x, ea.y, ea.z, ea.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const T v = tab[e[u] >> 24];
                    const T *xr = xs + (e[u] & 0xFFFFFFu) * TB;
#pragma unroll
                    for (int t = 0; t < TB; ++t) acc[i][u][t] += v * xr[t];
                }
            }
        }
    }
    EpiCoef<T> ec;
    if (EPI) ec = epi_coef(E);
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
        const int q = qa + (int)threadIdx.x + i * BS;
        const bool live = q < nq;
        // with the epilogue a wavefront goes on while its first lane-quad is in
        // range (it reduces over the wavefront), else a lane stops at the end
        if (EPI ? (q - lane >= nq) : !live) continue;
        const int a0 = 4 * (live ? q : 0);
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            if (live) {
                int kk = ds[t];
                for (; kk + 4 <= de[t]; kk += 4) {
                    Q4<T> v[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) v[u] = ld_q4(A.x + (int64_t)A.dn_col[kk + u] * cu64 + a0);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const T w = A.dn_val[kk + u];
#pragma unroll
                        for (int rr = 0; rr < 4; ++rr) acc[i][rr][t] += w * v[u].v[rr];
                    }
                }
                for (; kk < de[t]; ++kk) {
                    const Q4<T> v = ld_q4(A.x + (int64_t)A.dn_col[kk] * cu64 + a0);
                    const T w = A.dn_val[kk];
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) acc[i][rr][t] += w * v.v[rr];
                }
            }
            if (b0 + t < cd) {
                T o[4] = {acc[i][0][t], acc[i][1][t], acc[i][2][t], acc[i][3][t]};
                if (EPI) {
                    double part = 0.0;
                    if (live) {
                        const Q4<T> xv = ld_q4(xb[t] + a0);
                        Q4<T> vp;
                        if (E.vprev) {
                            const T *pv = E.vprev + (int64_t)(b0 + t) * cu64 + a0;
                            vp = A.stream ? ld_q4_nt(pv) : ld_q4(pv);
                        }
#pragma unroll
                        for (int r = 0; r < 4; ++r) o[r] = epi_w(E, ec, o[r], E.vprev ? vp.v[r] : (T)0);
#pragma unroll
                        for (int r = 0; r < 4; ++r) part += (double)o[r] * (double)xv.v[r];
                    }
                    part = quad_wave_sum(part);
                    if (lane == 0) E.gpart[(int64_t)(b0 + t) * E.G + (q >> 6)] = part;
                }
                if (live) {
                    if (EPI && A.stream) st_q4_nt(A.y + (int64_t)(b0 + t) * cu64 + a0, o);
                    else st_q4(A.y + (int64_t)(b0 + t) * cu64 + a0, o);
                }
            }
        }
    }
}

// apart[b] = sum over g of gpart[b][g], g increasing (the columns schedule's order)
__global__ void k_epi_colsum(const double *__restrict__ gpart, int G, int cd, double *__restrict__ apart)
{
    const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (b >= cd) return;
    double sum = 0.0;
    for (int g = 0; g < G; ++g) sum += gpart[(int64_t)b * G + g];
    apart[b] = sum;
}

// ---- one row per lane (count_up % 4 != 0, or unaligned vectors) ------------
// Each lane owns R rows (a, a + BS, ...) at once so the H_dn neighbour reads
// of all R rows are in flight together.  CF: compact entries (else packed
// {column, value} entries, for sectors without the compact format).  EPI: the
// first Lanczos update fused into the store (as in k_kron_quad), each lane
// summing its rows' products in row order and the workgroup combining the
// lanes in a fixed tree, one partial per column.
template <typename T, int TB, int BS, int R, bool CF, bool EPI>
__global__ __launch_bounds__(BS) void k_kron_fused(MvArgs<T> A, const int32_t *__restrict__ sl_off,
                                                   const Pk<T> *__restrict__ ell, const uint32_t *__restrict__ ellc,
                                                   const T *__restrict__ code_v, int ntiles, LzEpi<T> E)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[EPI ? BS : 1];
    T *tab = reinterpret_cast<T *>(smem_raw);       // 256 code values (compact format)
    T *xs = tab + (CF ? 256 : 0);
    const int tile = xcd_tile(ntiles);
    if (tile < 0) return;
    const int cu = A.cu, cd = A.cd;
    const int b0 = tile * TB;
    if (CF)
        for (int i = threadIdx.x; i < 256; i += BS) tab[i] = code_v[i];
    stage_columns<T, TB>(A, xs, b0, BS);
    __syncthreads();
    int ds[TB], de[TB];
    uint32_t dnb[TB];
    T edn[TB];
#pragma unroll
    for (int t = 0; t < TB; ++t) {
        const int b = min(b0 + t, cd - 1);
        ds[t] = A.dn_rp[b];
        de[t] = (b0 + t < cd) ? A.dn_rp[b + 1] : ds[t];
        dnb[t] = A.dn_basis[b];
        edn[t] = A.e_dn[b];
    }
    const int lane = threadIdx.x & 63;
    const int64_t cu64 = cu;
    EpiCoef<T> ec;
    if (EPI) ec = epi_coef(E);
    double part[EPI ? TB : 1] = {};
    for (int a0 = threadIdx.x; a0 < cu; a0 += BS * R) {
        T acc[R][TB];
        int as[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int a = min(a0 + j * BS, cu - 1);
            as[j] = a;
            const uint32_t ua = A.up_basis[a];
            const T eua = A.e_up[a];
            const Vec<T, TB> xa = *reinterpret_cast<const Vec<T, TB> *>(xs + a * TB);
#pragma unroll
            for (int t = 0; t < TB; ++t) acc[j][t] = (diag_u(A, ua & dnb[t]) + eua + edn[t]) * xa.v[t];
            const int s = a >> 6;
            if (CF) up_term_c<T, TB>(acc[j], xs, tab, ellc, sl_off[s] * 64 + lane, sl_off[s + 1] - sl_off[s]);
            else up_term<T, TB>(acc[j], xs, ell, sl_off[s] * 64 + lane, sl_off[s + 1] - sl_off[s]);
        }
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            int k = ds[t];
            for (; k + 4 <= de[t]; k += 4) {
                T y[4][R];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int j = 0; j < R; ++j) y[u][j] = A.x[(int64_t)A.dn_col[k + u] * cu64 + as[j]];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int j = 0; j < R; ++j) acc[j][t] += A.dn_val[k + u] * y[u][j];
            }
            for (; k < de[t]; ++k)
#pragma unroll
                for (int j = 0; j < R; ++j) acc[j][t] += A.dn_val[k] * A.x[(int64_t)A.dn_col[k] * cu64 + as[j]];
        }
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (a0 + j * BS < cu)
#pragma unroll
                for (int t = 0; t < TB; ++t)
                    if (b0 + t < cd) {
                        const int64_t o = (int64_t)(b0 + t) * cu64 + a0 + j * BS;
                        T w = acc[j][t];
                        if (EPI) {
                            w = epi_w(E, ec, w, E.vprev ? E.vprev[o] : (T)0);
                            part[t] += (double)w * (double)xs[(a0 + j * BS) * TB + t];
                        }
                        A.y[o] = w;
                    }
    }
    if (EPI) {
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            red[threadIdx.x] = part[t];
            __syncthreads();
            for (int h = BS / 2; h > 0; h >>= 1) {
                if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
                __syncthreads();
            }
            if (threadIdx.x == 0 && b0 + t < cd) E.apart[b0 + t] = red[0];
            __syncthreads();
        }
    }
}

// ---- fallback: CSR rows, H_up gathered from global memory ----------------
template <typename T, int BS>
__global__ __launch_bounds__(BS) void k_kron_csr(MvArgs<T> A)
{
    const int b = (int)blockIdx.x;
    const int cu = A.cu;
    const T *__restrict__ xb = A.x + (int64_t)b * cu;
    const int ds = A.dn_rp[b], de = A.dn_rp[b + 1];
    const uint32_t dnb = A.dn_basis[b];
    const T edn = A.e_dn[b];
    for (int a = threadIdx.x; a < cu; a += BS) {
        T acc = (diag_u(A, A.up_basis[a] & dnb) + A.e_up[a] + edn) * xb[a];
        for (int k = A.up_rp[a]; k < A.up_rp[a + 1]; ++k) acc += A.up_val[k] * xb[A.up_col[k]];
        dn_term(acc, A, ds, de, A.x + a);
        A.y[(int64_t)b * cu + a] = acc;
    }
}

template <typename T>
__global__ void k_diag(MvArgs<T> A, T *__restrict__ out)
{
    const int64_t n = (int64_t)A.cu * A.cd;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(i % A.cu), b = (int)(i / A.cu);
        out[i] = diag_u(A, A.up_basis[a] & A.dn_basis[b]) + A.e_up[a] + A.e_dn[b];
    }
}

// ========================================================================
// Host side
// ========================================================================

template <typename T>
MvArgs<T> make_args(const hub_sector *s, const void *x, void *y)
{
    const SpinTables &U = s->spin[0];
    const SpinTables &D = s->spin[1];
    MvArgs<T> A;
    A.x = (const T *)x;
    A.y = (T *)y;
    A.cu = (int32_t)U.count;
    A.cd = (int32_t)D.count;
    A.up_rp = U.rp;
    A.up_col = U.col;
    A.dn_rp = D.rp;
    A.dn_col = D.col;
    A.up_basis = U.basis;
    A.dn_basis = D.basis;
    A.uniform = s->uniformU;
    A.umask = s->umask;
    // non-temporal v_prev loads and output stores pay only where a vector is
    // larger than half the 256 MB MALL (4x4 torus FP32 fused product -3 %,
    // ring M=14 (47 MB) +2.6 %)
    A.stream = (double)U.count * (double)D.count * sizeof(T) > 128.0 * 1024 * 1024;
    if constexpr (sizeof(T) == 8) {
        A.up_val = (const T *)U.val64;
        A.dn_val = (const T *)D.val64;
        A.e_up = (const T *)U.e64;
        A.e_dn = (const T *)D.e64;
        A.Us = (const T *)s->d_U64;
    } else {
        A.up_val = (const T *)U.val32;
        A.dn_val = (const T *)D.val32;
        A.e_up = (const T *)U.e32;
        A.e_dn = (const T *)D.e32;
        A.Us = (const T *)s->d_U32;
    }
    A.U = (T)s->U0;
    return A;
}

template <typename T>
const T *code_table(const SpinTables &S)
{
    if constexpr (sizeof(T) == 8) return (const T *)S.code_v64;
    else return (const T *)S.code_v32;
}

template <typename T>
const Pk<T> *ell_of(const SpinTables &U)
{
    if constexpr (sizeof(T) == 8) return (const Pk<T> *)U.ell_pk64;
    else return (const Pk<T> *)U.ell_pk32;
}

// Dynamic LDS beyond 64 KB has to be allowed per kernel (once per process).
template <typename K>
hub_status allow_lds(K kernel, size_t bytes)
{
    static std::mutex mu;
    static std::map<const void *, size_t> done;
    std::lock_guard<std::mutex> lk(mu);
    auto it = done.find((const void *)kernel);
    if (it != done.end() && it->second >= bytes) return HUB_OK;
    HUB_HIP(hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    done[(const void *)kernel] = bytes;
    return HUB_OK;
}

template <typename T>
LzEpi<T> no_epi()
{
    return LzEpi<T>{nullptr, nullptr, nullptr, 0, nullptr, 0, nullptr};
}

// ---- geometry -------------------------------------------------------------

constexpr int kF64 = 0, kF32 = 1;

template <typename T>
constexpr int dix()
{
    return sizeof(T) == 8 ? kF64 : kF32;
}

// A sector whose product can use the 16-byte-access kernels.
bool quad_ok(const hub_sector *s)
{
    return !s->k0 && s->spin[0].ell_c32 && s->spin[1].ell_c32 && (s->spin[0].count % 4) == 0;
}

template <typename T>
bool column_fits(const hub_sector *s, int tb, bool epi)
{
    const int64_t cu = s->spin[0].count;
    const size_t g = (size_t)((cu / 4 + 63) / 64);
    return (size_t)(cu * tb + 256) * sizeof(T) + (epi ? (size_t)tb * g * sizeof(double) : 0) <= s->lds_max;
}

// balanced chunks of at most `maxc` (a multiple of 64) for `n` rows
int balanced_chunk(int64_t n, int64_t maxc)
{
    if (maxc < 64) return 0;
    const int64_t nch = (n + maxc - 1) / maxc;
    const int64_t c = (n + nch - 1) / nch;
    return (int)std::min<int64_t>(maxc, (c + 63) / 64 * 64);
}

// rows per staged chunk of the row-chunked product for TB columns
template <typename T>
int chunked_rows(const hub_sector *s, int tb)
{
    const int64_t maxr = ((int64_t)(s->lds_max / sizeof(T)) - 256) / tb / 64 * 64;
    return balanced_chunk(s->spin[0].count, maxr);
}

// the row-chunked shapes: (TB, QPL) with at most 64 FP32 / 32 FP64 accumulators per lane
template <typename T>
bool chunked_shape_ok(int tb, int qpl)
{
    if (tb != 1 && tb != 2 && tb != 4) return false;
    if (qpl != 4 && qpl != 8) return false;
    return tb * qpl <= (sizeof(T) == 8 ? 8 : 16);
}

// ---- launchers --------------------------------------------------------------

template <typename T, int TB, int BS, bool XC, bool EPI>
hub_status launch_quad_k(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, const LzEpi<T> &E)
{
    const SpinTables &U = s->spin[0];
    const int ntiles = (A.cd + TB - 1) / TB;
    const unsigned grid = XC ? 8u * (unsigned)((ntiles + 7) / 8) : (unsigned)ntiles;
    const size_t lds = (size_t)(A.cu * TB + 256) * sizeof(T) + (EPI ? (size_t)TB * E.G * sizeof(double) : 0);
    if (lds > s->lds_max) {
        set_error("column product: tile does not fit in LDS");
        return HUB_ERR_UNSUPPORTED;
    }
    HUB_TRY(allow_lds(k_kron_quad<T, TB, BS, XC, EPI>, s->lds_max));
    hipLaunchKernelGGL((k_kron_quad<T, TB, BS, XC, EPI>), dim3(grid), dim3(BS), lds, st, A, U.sl_off, U.ell_c32,
                       code_table<T>(U), ntiles, E);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

// column product of shape (tb in 1..3, bs in {512, 1024}, xc); E: fused Lanczos update or NULL
template <typename T>
hub_status launch_quad(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, int tb, int bs, int xc,
                       const LzEpi<T> *E)
{
    const LzEpi<T> ne = no_epi<T>();
#define HUB_QUAD(TBV, BSV, XCV)                                                              \
    if (tb == TBV && bs == BSV && xc == XCV) {                                               \
        if (E) return launch_quad_k<T, TBV, BSV, XCV, true>(s, A, st, *E);                  \
        return launch_quad_k<T, TBV, BSV, XCV, false>(s, A, st, ne);                        \
    }
    HUB_QUAD(1, 512, 0) HUB_QUAD(1, 512, 1) HUB_QUAD(1, 1024, 0) HUB_QUAD(1, 1024, 1)
    HUB_QUAD(2, 512, 0) HUB_QUAD(2, 512, 1) HUB_QUAD(2, 1024, 0) HUB_QUAD(2, 1024, 1)
    HUB_QUAD(3, 512, 0) HUB_QUAD(3, 512, 1) HUB_QUAD(3, 1024, 0) HUB_QUAD(3, 1024, 1)
#undef HUB_QUAD
    set_error("unsupported column product shape");
    return HUB_ERR_UNSUPPORTED;
}

template <typename T, int QPL, int TB, bool EPI>
hub_status launch_chunked_k(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, const ChunkSet &C,
                            const LzEpi<T> &E)
{
    constexpr int BSC = 1024;
    const SpinTables &U = s->spin[0];
    const size_t lds = ((size_t)C.rows * TB + 256) * sizeof(T);
    if (lds > s->lds_max) {
        set_error("row-chunked product: chunk does not fit in LDS");
        return HUB_ERR_UNSUPPORTED;
    }
    const int nq = (int)(A.cu >> 2);
    const int P = (nq + BSC * QPL - 1) / (BSC * QPL);
    const int ntiles = (A.cd + TB - 1) / TB;
    HUB_TRY(allow_lds(k_kron_chunked_parts<T, BSC, QPL, TB, EPI>, s->lds_max));
    const unsigned grid = 8u * (unsigned)P * (unsigned)((ntiles + 7) / 8);
    hipLaunchKernelGGL((k_kron_chunked_parts<T, BSC, QPL, TB, EPI>), dim3(grid), dim3(BSC), lds, st, A, C.off,
                       C.base, C.ell, code_table<T>(U), C.n, C.rows, (int)U.nslices, P, E);
    if (EPI)
        hipLaunchKernelGGL(k_epi_colsum, dim3((unsigned)((A.cd + 255) / 256)), dim3(256), 0, st,
                           (const double *)E.gpart, E.G, A.cd, E.apart);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

// row-chunked product of shape (tb, qpl); E: fused Lanczos update or NULL
template <typename T>
hub_status launch_chunked(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, int tb, int qpl,
                          const ChunkSet &C, const LzEpi<T> *E)
{
    const LzEpi<T> ne = no_epi<T>();
#define HUB_CH(TBV, QV)                                                                  \
    if (tb == TBV && qpl == QV) {                                                        \
        if (E) return launch_chunked_k<T, QV, TBV, true>(s, A, st, C, *E);              \
        return launch_chunked_k<T, QV, TBV, false>(s, A, st, C, ne);                    \
    }
    HUB_CH(1, 4) HUB_CH(1, 8) HUB_CH(2, 4)
    if constexpr (sizeof(T) == 4) {
        HUB_CH(2, 8) HUB_CH(4, 4)
    }
#undef HUB_CH
    set_error("unsupported row-chunked product shape");
    return HUB_ERR_UNSUPPORTED;
}

template <typename T, int TB, int BS, int R, bool EPI>
hub_status launch_rows(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, const LzEpi<T> &E)
{
    const SpinTables &U = s->spin[0];
    const int ntiles = (A.cd + TB - 1) / TB;
    const unsigned grid = 8u * (unsigned)((ntiles + 7) / 8);
    const size_t lim = s->lds_max - (EPI ? (size_t)BS * sizeof(double) : 0);  // beside the static reduction array
    if (U.ell_c32) {
        const size_t lds = (size_t)(A.cu * TB + 256) * sizeof(T);
        HUB_TRY(allow_lds(k_kron_fused<T, TB, BS, R, true, EPI>, lim));
        hipLaunchKernelGGL((k_kron_fused<T, TB, BS, R, true, EPI>), dim3(grid), dim3(BS), lds, st, A, U.sl_off,
                           ell_of<T>(U), U.ell_c32, code_table<T>(U), ntiles, E);
        HUB_HIP(hipGetLastError());
        return HUB_OK;
    }
    const size_t lds = (size_t)A.cu * TB * sizeof(T);
    HUB_TRY(allow_lds(k_kron_fused<T, TB, BS, R, false, EPI>, lim));
    hipLaunchKernelGGL((k_kron_fused<T, TB, BS, R, false, EPI>), dim3(grid), dim3(BS), lds, st, A, U.sl_off,
                       ell_of<T>(U), (const uint32_t *)nullptr, (const T *)nullptr, ntiles, E);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

// one row per lane: two columns per workgroup when they fit in half of the LDS;
// CSR rows when a column does not fit
// One row per lane in the shape the column size allows (two columns per
// workgroup when both fit in half the LDS), else CSR rows; E: the fused Lanczos
// update (its reduction array takes 8 KB of the LDS; no CSR fallback).
template <typename T>
bool rows_fit(const hub_sector *s, bool epi)
{
    const size_t col = (size_t)s->spin[0].count * sizeof(T), extra = 256 * sizeof(T);
    return col + extra <= s->lds_max - (epi ? 1024 * sizeof(double) : 0);
}

template <typename T>
hub_status launch_rows_auto(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, const LzEpi<T> *E = nullptr)
{
    const size_t col = (size_t)A.cu * sizeof(T), extra = 256 * sizeof(T);
    const size_t lim = s->lds_max - (E ? 1024 * sizeof(double) : 0);
    const LzEpi<T> ne = no_epi<T>();
    if (2 * col + extra <= lim / 2)
        return E ? launch_rows<T, 2, 1024, 2, true>(s, A, st, *E) : launch_rows<T, 2, 1024, 2, false>(s, A, st, ne);
    if (col + extra <= lim)
        return E ? launch_rows<T, 1, 1024, 4, true>(s, A, st, *E) : launch_rows<T, 1, 1024, 4, false>(s, A, st, ne);
    if (E) {
        set_error("one-row-per-lane product: a column does not fit in LDS beside the update's reduction");
        return HUB_ERR_UNSUPPORTED;
    }
    hipLaunchKernelGGL((k_kron_csr<T, 512>), dim3((unsigned)A.cd), dim3(512), 0, st, A);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

// Run schedule q; E: the fused Lanczos update (COLUMNS schedules only)
template <typename T>
hub_status launch_sched(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, const Sched &q, const LzEpi<T> *E)
{
    if (E && q.fam == HUB_SCHED_CSR) {
        set_error("the csr schedule has no fused Lanczos update");
        return HUB_ERR_UNSUPPORTED;
    }
    switch (q.fam) {
    case HUB_SCHED_COLUMNS:
        return launch_quad<T>(s, A, st, q.tb, q.bs, q.xc, E);
    case HUB_SCHED_CHUNKED: {
        const ChunkSet *C = nullptr;
        HUB_TRY(chunk_set(s, HUB_SPIN_UP, q.crows > 0 ? q.crows : chunked_rows<T>(s, q.tb), &C, st));
        return launch_chunked<T>(s, A, st, q.tb, q.qpl, *C, E);
    }
    case HUB_SCHED_ROWS:
        return launch_rows_auto<T>(s, A, st, E);
    case HUB_SCHED_CSR:
        hipLaunchKernelGGL((k_kron_csr<T, 512>), dim3((unsigned)A.cd), dim3(512), 0, st, A);
        HUB_HIP(hipGetLastError());
        return HUB_OK;
    default:
        break;
    }
    set_error("product schedule not chosen");
    return HUB_ERR_UNSUPPORTED;
}

// ---- tuner ----------------------------------------------------------------

// Times each candidate launch in two interleaved rounds (one warm-up launch,
// then 5 timed launches, or 2 when one launch takes over 4 ms) and returns the
// index of the fastest (its better round), with its time in ms.
template <typename F>
hub_status time_candidates(hipStream_t st, int n, F launch, int &best, float &best_ms)
{
    hipEvent_t e0, e1;
    HUB_HIP(hipEventCreate(&e0));
    HUB_HIP(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev()
        {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev{e0, e1};
    std::vector<float> ms((size_t)n, 1e30f);
    for (int round = 0; round < 2; ++round)
        for (int c = 0; c < n; ++c) {
            HUB_HIP(hipEventRecord(e0, st));
            HUB_TRY(launch(c));
            HUB_HIP(hipEventRecord(e1, st));
            HUB_HIP(hipEventSynchronize(e1));
            float one = 0.f;
            HUB_HIP(hipEventElapsedTime(&one, e0, e1));
            const int reps = one > 4.0f ? 2 : 5;
            HUB_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < reps; ++r) HUB_TRY(launch(c));
            HUB_HIP(hipEventRecord(e1, st));
            HUB_HIP(hipEventSynchronize(e1));
            HUB_HIP(hipEventElapsedTime(&one, e0, e1));
            ms[(size_t)c] = std::min(ms[(size_t)c], one / (float)reps);
        }
    best = (int)(std::min_element(ms.begin(), ms.end()) - ms.begin());
    best_ms = ms[(size_t)best];
    return HUB_OK;
}

// Candidate schedules of a sector: whole columns in LDS when one fits (1-3
// columns per workgroup, 512 or 1024 lanes, XCD or launch tile order; with the
// fused update, the shapes whose partials also fit), else the row-chunked
// shapes (1, 2 or 4 columns per work item, 4 or 8 lane-quads per lane), with
// or without the fused update.
template <typename T>
std::vector<Sched> candidates(const hub_sector *s, bool epi)
{
    std::vector<Sched> v;
    if (column_fits<T>(s, 1, false)) {
        for (int tb = 1; tb <= 3; ++tb) {
            if (!column_fits<T>(s, tb, epi)) break;
            for (int bs : {512, 1024})
                for (int xc : {0, 1}) {
                    Sched c;
                    c.fam = HUB_SCHED_COLUMNS;
                    c.tb = tb;
                    c.bs = bs;
                    c.xc = xc;
                    v.push_back(c);
                }
        }
        return v;
    }
    for (int tb : {1, 2, 4})
        for (int qpl : {4, 8}) {
            if (!chunked_shape_ok<T>(tb, qpl) || chunked_rows<T>(s, tb) <= 0) continue;
            Sched c;
            c.fam = HUB_SCHED_CHUNKED;
            c.tb = tb;
            c.qpl = qpl;
            c.bs = 1024;
            c.crows = chunked_rows<T>(s, tb);
            v.push_back(c);
        }
    return v;
}

// Tune the product (epi = false) or the product fused with the Lanczos update
// (epi = true, apart: its partials buffer) on the caller's x and y.  The
// epilogue's timing launches read x as v_prev with beta = 0.
template <typename T>
hub_status tune(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, bool epi, double *apart, Sched &out)
{
    double *zero = nullptr;
    struct Buf {
        double *p = nullptr;
        ~Buf() { (void)hipFree(p); }
    } zb;
    LzEpi<T> E = no_epi<T>();
    if (epi) {
        HUB_HIP(hipMalloc((void **)&zero, sizeof(double)));
        zb.p = zero;
        HUB_HIP(hipMemsetAsync(zero, 0, sizeof(double), st));
        E = LzEpi<T>{A.x, zero, apart, (int)(((A.cu >> 2) + 63) / 64), nullptr, 0, apart + A.cd};
    }
    std::vector<Sched> c = candidates<T>(s, epi);
    if (c.empty()) {
        set_error("no product schedule fits this sector");
        return HUB_ERR_UNSUPPORTED;
    }
    int bi = 0;
    float ms = 0.f;
    HUB_TRY(time_candidates(st, (int)c.size(),
                            [&](int k) { return launch_sched<T>(s, A, st, c[(size_t)k], epi ? &E : nullptr); }, bi,
                            ms));
    out = c[(size_t)bi];
    out.ms = ms;
    return HUB_OK;
}

// Tuned schedules are kept per device, dtype and sector structure (dimensions,
// nonzeros; the values of t, U and eps do not change the timing), so sectors of
// the same lattice share one tuning.
struct ShapeKey {
    int device, dtype;
    int64_t cu, cd, nnz_up, nnz_dn;
    int epi;
    bool operator<(const ShapeKey &o) const
    {
        return std::tie(device, dtype, cu, cd, nnz_up, nnz_dn, epi) <
               std::tie(o.device, o.dtype, o.cu, o.cd, o.nnz_up, o.nnz_dn, o.epi);
    }
};
std::mutex g_shape_mu;
std::map<ShapeKey, Sched> g_shapes;

// The schedule of the product (epi = false) or of the product fused with the
// Lanczos update (epi = true) for aligned vectors: forced, cached, shared by a
// sector of the same structure, or tuned now (under the sector's lock: tuning
// launches on the caller's stream and may build chunk tables).
template <typename T>
hub_status schedule_for(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, bool epi, double *apart, Sched &out)
{
    const int di = dix<T>();
    const ShapeKey key{s->device, di, (int64_t)A.cu, (int64_t)A.cd, s->spin[0].nnz, s->spin[1].nnz, epi ? 1 : 0};
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->forced[di]) {
        out = s->sched[di];
        return HUB_OK;
    }
    Sched &q = epi ? s->sched_lz[di] : s->sched[di];
    if (q.fam == 0) {
        std::lock_guard<std::mutex> lk2(g_shape_mu);
        auto it = g_shapes.find(key);
        if (it != g_shapes.end()) q = it->second;
    }
    if (q.fam == 0) {
        Sched t;
        HUB_TRY(tune<T>(s, A, st, epi, apart, t));
        std::lock_guard<std::mutex> lk2(g_shape_mu);
        g_shapes[key] = t;
        q = t;
    }
    out = q;
    return HUB_OK;
}

template <typename T>
hub_status run_kron(const hub_sector *s, const void *x, void *y, hipStream_t st)
{
    MvArgs<T> A = make_args<T>(s, x, y);
    // the 16-byte-access kernels need 16-byte aligned vectors
    const bool aligned16 = (((uintptr_t)x | (uintptr_t)y) & 15u) == 0;
    if (!aligned16 || !quad_ok(s)) {
        bool csr;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            csr = s->forced[dix<T>()] && s->sched[dix<T>()].fam == HUB_SCHED_CSR;
        }
        Sched q;
        q.fam = csr ? HUB_SCHED_CSR : HUB_SCHED_ROWS;
        return launch_sched<T>(s, A, st, q, nullptr);
    }
    Sched q;
    HUB_TRY(schedule_for<T>(s, A, st, false, nullptr, q));
    std::lock_guard<std::mutex> lk(s->mu);  // chunk tables may be built on first use
    return launch_sched<T>(s, A, st, q, nullptr);
}

// Whether the product fused with the first Lanczos update is available: the
// columns schedule with its partials in LDS, the row-chunked schedule, or one
// row per lane (count_up % 4 != 0) when a column fits beside the reduction
// (forced or tuned).
template <typename T>
bool lz_fusable(const hub_sector *s)
{
    if (s->k0) return false;  // the k = 0 block has its own product
    std::lock_guard<std::mutex> lk(s->mu);
    const int di = dix<T>();
    if (s->forced[di]) {
        const Sched &q = s->sched[di];
        if (q.nofuse) return false;
        if (q.fam == HUB_SCHED_COLUMNS) return quad_ok(s) && column_fits<T>(s, q.tb, true);
        if (q.fam == HUB_SCHED_CHUNKED) return quad_ok(s);
        return q.fam == HUB_SCHED_ROWS && rows_fit<T>(s, true);
    }
    if (!quad_ok(s)) return rows_fit<T>(s, true);
    return column_fits<T>(s, 1, true) || (!column_fits<T>(s, 1, false) && chunked_rows<T>(s, 1) > 0);
}

template <typename T>
hub_status run_kron_lz(const hub_sector *s, const void *x, void *w, const void *vprev, const double *beta,
                       const double *beta_prev, int unnorm, double *apart, int64_t *npart, hipStream_t st)
{
    if (!lz_fusable<T>(s)) return HUB_ERR_UNSUPPORTED;
    MvArgs<T> A = make_args<T>(s, x, w);
    Sched q;
    if (quad_ok(s)) {
        HUB_TRY(schedule_for<T>(s, A, st, true, apart, q));
    } else {
        q.fam = HUB_SCHED_ROWS;  // the only fused shape without four-row quads
    }
    const LzEpi<T> E{(const T *)vprev, beta, apart, (int)(((A.cu >> 2) + 63) / 64), beta_prev, unnorm,
                     apart + A.cd};
    *npart = (int64_t)A.cd;
    std::lock_guard<std::mutex> lk(s->mu);
    return launch_sched<T>(s, A, st, q, &E);
}

}  // namespace

hub_status launch_matvec(const hub_sector *s, int dtype, const void *x, void *y, hipStream_t st)
{
    if (dtype == HUB_F64) return run_kron<double>(s, x, y, st);
    return run_kron<float>(s, x, y, st);
}

bool matvec_lz_available(const hub_sector *s, int dtype)
{
    return dtype == HUB_F64 ? lz_fusable<double>(s) : lz_fusable<float>(s);
}

// Partials of the fused product: one per column.
int64_t matvec_lz_partials(const hub_sector *s)
{
    return s->spin[1].count;
}

// Doubles of the fused product's partials buffer: the per-column partials,
// then (row-chunked schedule) one per column and group of 256 rows.
int64_t matvec_lz_workspace(const hub_sector *s)
{
    const int64_t cd = s->spin[1].count, G = ((s->spin[0].count >> 2) + 63) / 64;
    return cd * (1 + G);
}

hub_status launch_matvec_lz(const hub_sector *s, int dtype, const void *x, void *w, const void *vprev,
                            const double *beta, double *apart, int64_t *npart, hipStream_t st,
                            const double *beta_prev, int unnorm)
{
    if (dtype == HUB_F64) return run_kron_lz<double>(s, x, w, vprev, beta, beta_prev, unnorm, apart, npart, st);
    return run_kron_lz<float>(s, x, w, vprev, beta, beta_prev, unnorm, apart, npart, st);
}

hub_status launch_diagonal(const hub_sector *s, int dtype, void *out, hipStream_t st)
{
    const unsigned grid = 4096, block = 256;
    if (dtype == HUB_F64) {
        MvArgs<double> A = make_args<double>(s, nullptr, nullptr);
        hipLaunchKernelGGL(k_diag<double>, dim3(grid), dim3(block), 0, st, A, (double *)out);
    } else {
        MvArgs<float> A = make_args<float>(s, nullptr, nullptr);
        hipLaunchKernelGGL(k_diag<float>, dim3(grid), dim3(block), 0, st, A, (float *)out);
    }
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

int64_t matvec_bytes(const hub_sector *s, int dtype)
{
    const int64_t es = (dtype == HUB_F64) ? 8 : 4;
    int64_t bytes = 2 * s->dim * es;  // read x once, write y once
    const int nsp = s->shared_spin ? 1 : 2;
    for (int sp = 0; sp < nsp; ++sp) {
        const SpinTables &T = s->spin[sp];
        // row pointers, columns, values, basis integers, site sums
        bytes += 4 * (T.count + 1) + T.nnz * (4 + es) + 4 * T.count + es * T.count;
    }
    return bytes;
}

// ---- forced schedules (tests and measurement) --------------------------------

namespace {

template <typename T>
hub_status check_forced(const hub_sector *s, const hub_schedule &h, Sched &q)
{
    q = Sched{};
    q.fam = h.family;
    q.tb = h.tile_cols;
    q.bs = h.block;
    q.xc = h.order;
    q.qpl = h.quads_per_lane;
    q.crows = h.chunk_rows;
    q.nofuse = h.no_fused_update;
    auto bad = [](const char *m) {
        set_error(m);
        return HUB_ERR_INVALID_ARG;
    };
    switch (q.fam) {
    case HUB_SCHED_COLUMNS:
        if (!quad_ok(s)) return bad("columns schedule needs count_up % 4 == 0 and compact entries");
        if (q.tb < 1 || q.tb > 3 || (q.bs != 512 && q.bs != 1024) || (q.xc != 0 && q.xc != 1))
            return bad("columns schedule: tile_cols 1..3, block 512 or 1024, order 0 or 1");
        if (!column_fits<T>(s, q.tb, false)) return bad("columns schedule: the tile does not fit in LDS");
        q.qpl = 0;
        q.crows = 0;
        break;
    case HUB_SCHED_CHUNKED:
        if (!quad_ok(s)) return bad("chunked schedule needs count_up % 4 == 0 and compact entries");
        if (!chunked_shape_ok<T>(q.tb, q.qpl))
            return bad("chunked schedule: tile_cols 1, 2 or 4 and quads_per_lane 4 or 8 "
                       "(tile_cols * quads_per_lane <= 16 in FP32, 8 in FP64)");
        if (q.crows <= 0) q.crows = chunked_rows<T>(s, q.tb);
        if (q.crows <= 0 || q.crows % 4 != 0 || ((size_t)q.crows * q.tb + 256) * sizeof(T) > s->lds_max)
            return bad("chunked schedule: chunk_rows must be a positive multiple of 4 that fits in LDS");
        q.bs = 1024;
        q.xc = 0;
        break;
    case HUB_SCHED_ROWS:
        if (!column_fits<T>(s, 1, false)) return bad("rows schedule: a column does not fit in LDS");
        break;
    case HUB_SCHED_CSR:
        break;
    default:
        return bad("unknown schedule family");
    }
    return HUB_OK;
}

void to_public(const Sched &q, hub_schedule *h)
{
    *h = hub_schedule{};
    h->family = q.fam;
    h->tile_cols = q.tb;
    h->block = q.bs;
    h->order = q.xc;
    h->quads_per_lane = q.qpl;
    h->chunk_rows = q.crows;
    h->no_fused_update = q.nofuse;
    h->ms = q.ms;
}

}  // namespace

hub_status set_schedule(const hub_sector *s, int dtype, const hub_schedule *h)
{
    const int di = dtype == HUB_F64 ? kF64 : kF32;
    if (!h) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->forced[di] = false;
        s->sched[di] = Sched{};
        s->sched_lz[di] = Sched{};
        return HUB_OK;
    }
    Sched q;
    HUB_TRY(dtype == HUB_F64 ? check_forced<double>(s, *h, q) : check_forced<float>(s, *h, q));
    std::lock_guard<std::mutex> lk(s->mu);
    s->forced[di] = true;
    s->sched[di] = q;
    s->sched_lz[di] = q;
    return HUB_OK;
}

hub_status get_schedule(const hub_sector *s, int dtype, int fused, hub_schedule *h)
{
    const int di = dtype == HUB_F64 ? kF64 : kF32;
    std::lock_guard<std::mutex> lk(s->mu);
    to_public(fused && !s->forced[di] ? s->sched_lz[di] : s->sched[di], h);
    return HUB_OK;
}

}  // namespace hub
