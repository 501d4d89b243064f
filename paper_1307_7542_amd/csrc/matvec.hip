// Kronecker-sum product of the sector Hamiltonian (Sec. IV A):
//
//     Y = H_up V + V H_dn^T + D o V,   V, Y: count_up x count_dn, column-major.
//
// H_dn is real symmetric, so column b of V H_dn^T is sum_l H_dn[b, l] V[:, l].
// D(a, b) = U-part(basis_up[a] & basis_dn[b]) + e_up[a] + e_dn[b] is generated
// from the bit patterns (the doubly occupied sites of Sec. III B) and never
// stored.
//
// The two terms want orthogonal access patterns.  In column-major storage the
// H_dn term combines whole neighbouring columns (coalesced, with a row of H_dn
// that is uniform over a workgroup), while the H_up term gathers inside one
// column along a different row of H_up for every lane.  Schedules:
//
//   k_kron_quad (default when count_up % 4 == 0 and a column fits in LDS): one
//             workgroup per TB output columns, the TB input columns staged in
//             LDS for the H_up gathers, the H_dn neighbour columns read through
//             L2 / MALL; each lane owns four consecutive rows (16-byte accesses).
//             The tile shape is timed on the first product and cached; the
//             first Lanczos update can be fused into its epilogue.
//   k_kron_fused: the same schedule with one row per lane (count_up % 4 != 0).
//   k_kron_chunked_parts (a column larger than the LDS): work items of TB
//             columns x a part of the rows; the row chunks of the columns are
//             staged in turn and the output rows stay in registers.
//   two-pass, csr, one-row chunked: kept for measurement and for sectors whose
//             entries do not fit the compact format (csr fallback).
//
// H_up is read from its sliced-ELL copy: lane r of a wavefront owns row
// 64*s + r of slice s and loads entry k from a coalesced address; the default
// entry is {column : 24, code : 8} with the value looked up in a 256-entry
// table in LDS.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
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
    T *y;  // may alias the intermediate of the two-pass product
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
        for (int t = 0; t < TB; ++t) acc[t] += (v0 * x0.v[t] + v1 * x1.v[t]) + (v2 * x2.v[t] + v3 * x3.v[t]);
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
        for (int t = 0; t < TB; ++t) acc[t] += (v0 * x0.v[t] + v1 * x1.v[t]) + (v2 * x2.v[t] + v3 * x3.v[t]);
    }
    for (; k < len; ++k) {
        const uint32_t e0 = ell[o0 + 64 * k];
        const T v0 = tab[e0 >> 24];
        const Vec<T, TB> x0 = *reinterpret_cast<const Vec<T, TB> *>(xs + (e0 & 0xFFFFFFu) * TB);
#pragma unroll
        for (int t = 0; t < TB; ++t) acc[t] += v0 * x0.v[t];
    }
}

// sum_k H_dn[b, k] x[a + col_k * cu] over row b of H_dn (uniform over the wavefront).
template <typename T>
__device__ __forceinline__ T dn_term(const MvArgs<T> &A, int ks, int ke, const T *__restrict__ xa)
{
    const int64_t cu = A.cu;
    T s = (T)0;
    int k = ks;
    for (; k + 4 <= ke; k += 4) {
        const int64_t l0 = A.dn_col[k], l1 = A.dn_col[k + 1], l2 = A.dn_col[k + 2], l3 = A.dn_col[k + 3];
        const T y0 = xa[l0 * cu], y1 = xa[l1 * cu], y2 = xa[l2 * cu], y3 = xa[l3 * cu];
        s += (A.dn_val[k] * y0 + A.dn_val[k + 1] * y1) + (A.dn_val[k + 2] * y2 + A.dn_val[k + 3] * y3);
    }
    for (; k < ke; ++k) s += A.dn_val[k] * xa[(int64_t)A.dn_col[k] * cu];
    return s;
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

// ---- fused, four consecutive rows per lane ------------------------------
// Same schedule and per-element arithmetic order as k_kron_fused, but lane q
// owns rows 4q .. 4q+3 (count_up % 4 == 0): the column staging, the H_dn
// neighbour reads and the stores become 16-byte (FP32) or 2 x 16-byte (FP64)
// accesses, and the four rows' sliced-ELL entries k are four consecutive
// lanes of the slice, read with one 16-byte load.  XC: XCD-contiguous tile
// order (workgroup i on XCD i mod 8 takes the i-th tile of that XCD's range)
// or plain launch order.
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
// (rounded as the separate update kernel does) and the sum of w * x per column:
// each group of 64 lane-quads (256 rows) is summed by one wavefront in a fixed
// order, then the groups of a column in increasing order, so the per-column
// partials do not depend on the tile shape.
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
    double bt = 0.0, sx = 1.0;
    if (EPI) {
        if (E.unnorm) {
            sx = inv_beta(E.beta);
            bt = E.vprev ? *E.beta * inv_beta(E.beta_prev) : 0.0;
        } else if (E.vprev) {
            bt = *E.beta;
        }
    }
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
                    if (E.unnorm) {
                        if (E.vprev) {
                            const Q4<T> &vp = vpq[t];
#pragma unroll
                            for (int r = 0; r < 4; ++r) o[r] = (T)fma(sx, (double)o[r], -(bt * (double)vp.v[r]));
                        } else {
#pragma unroll
                            for (int r = 0; r < 4; ++r) o[r] = (T)(sx * (double)o[r]);
                        }
                    } else if (E.vprev) {
                        const Q4<T> &vp = vpq[t];
#pragma unroll
                        for (int r = 0; r < 4; ++r) o[r] = (T)fma(-bt, (double)vp.v[r], (double)o[r]);
                    }
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

// Row-chunked product with four consecutive rows per lane (count_up and the
// chunk length multiples of 4): the access pattern of k_kron_quad applied to
// the phases of k_kron_chunked.
template <typename T, int BS, bool XC>
__global__ __launch_bounds__(BS) void k_kron_chunked_quad(MvArgs<T> A, const int32_t *__restrict__ ch_off,
                                                          const int64_t *__restrict__ ch_base,
                                                          const uint32_t *__restrict__ ch_ell,
                                                          const T *__restrict__ code_v, int nchunks, int chunk_rows,
                                                          int nslices)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tab = reinterpret_cast<T *>(smem_raw);
    T *xs = tab + 256;
    const int tile = XC ? xcd_tile(A.cd) : ((int)blockIdx.x < A.cd ? (int)blockIdx.x : -1);
    if (tile < 0) return;
    const int cu = A.cu, nq = cu >> 2;
    const int b = tile;
    const int64_t cu64 = cu;
    const T *__restrict__ xb = A.x + (int64_t)b * cu;
    T *yb = A.y + (int64_t)b * cu;
    for (int i = threadIdx.x; i < 256; i += BS) tab[i] = code_v[i];
    const int ds = A.dn_rp[b], de = A.dn_rp[b + 1];
    const uint32_t dnb = A.dn_basis[b];
    const T edn = A.e_dn[b];
    for (int p = 0; p < nchunks; ++p) {
        const int q0 = (p * chunk_rows) >> 2;
        const int q1 = min(nq, q0 + (chunk_rows >> 2));
        __syncthreads();  // previous phase done with xs
        for (int q = q0 + threadIdx.x; q < q1; q += BS) {
            const Q4<T> v = ld_q4(xb + 4 * q);
#pragma unroll
            for (int r = 0; r < 4; ++r) xs[4 * (q - q0) + r] = v.v[r];
        }
        __syncthreads();
        const int32_t *off = ch_off + (int64_t)p * (nslices + 1);
        const uint32_t *ell = ch_ell + ch_base[p];
        for (int q = threadIdx.x; q < nq; q += BS) {
            const int a0 = 4 * q;
            T acc[4];
            if (p == 0) {
                const uint4 ub = *reinterpret_cast<const uint4 *>(A.up_basis + a0);
                const uint32_t uu[4] = {ub.x, ub.y, ub.z, ub.w};
                const Q4<T> eu = ld_q4(A.e_up + a0);
                const Q4<T> xv = ld_q4(xb + a0);
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] = (diag_u(A, uu[r] & dnb) + eu.v[r] + edn) * xv.v[r];
            } else {
                const Q4<T> yv = ld_q4(yb + a0);
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] = yv.v[r];
            }
            const int s = a0 >> 6;
            const uint4 *__restrict__ e4 = reinterpret_cast<const uint4 *>(ell + (int64_t)off[s] * 64 + (a0 & 63));
            const int len = off[s + 1] - off[s];
            int k = 0;
            for (; k + 2 <= len; k += 2) {
                const uint4 ea = e4[16 * k], eb = e4[16 * (k + 1)];
                const uint32_t e[8] = {ea.x, ea.y, ea.z, ea.w, eb.x, eb.y, eb.z, eb.w};
#pragma unroll
                for (int i = 0; i < 8; ++i) acc[i & 3] += tab[e[i] >> 24] * xs[e[i] & 0xFFFFFFu];
            }
            if (k < len) {
                const uint4 ea = e4[16 * k];
                const uint32_t e[4] = {ea.x, ea.y, ea.z, ea.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[i] += tab[e[i] >> 24] * xs[e[i] & 0xFFFFFFu];
            }
            if (p == 0) {
                int kk = ds;
                for (; kk + 4 <= de; kk += 4) {
                    Q4<T> v[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) v[u] = ld_q4(A.x + (int64_t)A.dn_col[kk + u] * cu64 + a0);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const T w = A.dn_val[kk + u];
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[r] += w * v[u].v[r];
                    }
                }
                for (; kk < de; ++kk) {
                    const Q4<T> v = ld_q4(A.x + (int64_t)A.dn_col[kk] * cu64 + a0);
                    const T w = A.dn_val[kk];
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[r] += w * v.v[r];
                }
            }
            st_q4(yb + a0, acc);
        }
    }
}

// Row-chunked product with the output held in registers: work item (tile of TB
// columns, row part j) owns quads [j BS QPL, (j+1) BS QPL) of its columns, QPL
// per lane.  It stages every row chunk of its columns in turn (interleaved,
// element (a, t) at a TB + t) and accumulates the chunk's H_up entries of its
// rows, each entry serving the TB columns; then the H_dn term and one store.
// Per element: diagonal, H_up entries in column order, H_dn entries -- the
// order of k_kron_quad -- and no partial results in memory.  Tiles are
// interleaved over the XCDs (tile = 8 k + xcd), row parts dispatched in turn.
template <typename T, int BS, int QPL, int TB>
__global__ __launch_bounds__(BS) void k_kron_chunked_parts(MvArgs<T> A, const int32_t *__restrict__ ch_off,
                                                           const int64_t *__restrict__ ch_base,
                                                           const uint32_t *__restrict__ ch_ell,
                                                           const T *__restrict__ code_v, int nchunks,
                                                           int chunk_rows, int nslices, int P)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tab = reinterpret_cast<T *>(smem_raw);
    T *xs = tab + 256;
    const int xcd = (int)(blockIdx.x & 7), r = (int)(blockIdx.x >> 3);
    const int cd = A.cd;
    const int ntiles = (cd + TB - 1) / TB;
    // part-major: every tile's first row part, then every tile's second, ... so
    // the neighbour rows the chip reads at a time are one part's (2x9 ladder:
    // FP32 30.6 -> 30.0 ms, FP64 57.8 -> 56.1 ms against the parts of a tile
    // dispatched together)
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
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
        const int q = qa + (int)threadIdx.x + i * BS;
        if (q >= nq) continue;
        const int a0 = 4 * q;
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
                    for (int rr = 0; rr < 4; ++rr) acc[i][rr][t] += w * v[u].v[rr];
                }
            }
            for (; kk < de[t]; ++kk) {
                const Q4<T> v = ld_q4(A.x + (int64_t)A.dn_col[kk] * cu64 + a0);
                const T w = A.dn_val[kk];
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) acc[i][rr][t] += w * v.v[rr];
            }
            if (b0 + t < cd) {
                const T o[4] = {acc[i][0][t], acc[i][1][t], acc[i][2][t], acc[i][3][t]};
                st_q4(A.y + (int64_t)(b0 + t) * cu64 + a0, o);
            }
        }
    }
}

// ---- fused ------------------------------------------------------------
// Each lane owns R rows (a, a + BS, ...) at once so the H_dn neighbour reads
// of all R rows are in flight together.
template <typename T, int TB, int BS, int R, bool CF>
__global__ __launch_bounds__(BS) void k_kron_fused(MvArgs<T> A, const int32_t *__restrict__ sl_off,
                                                   const Pk<T> *__restrict__ ell, const uint32_t *__restrict__ ellc,
                                                   const T *__restrict__ code_v, int ntiles)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
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
                    if (b0 + t < cd) A.y[(int64_t)(b0 + t) * cu64 + a0 + j * BS] = acc[j][t];
    }
}

// ---- row-chunked fused product (columns larger than the LDS) -------------
// One workgroup per output column b.  The column is processed in P row
// chunks: phase p stages V[chunk p, b] in LDS and adds, for every row, the
// H_up entries whose column lies in chunk p; phase 0 also adds the diagonal and
// the H_dn term.  Y[:, b] is written in phase 0 and updated in place by the
// later phases of the same workgroup (the column is still in L2 by then).
template <typename T, int BS, int R>
__global__ __launch_bounds__(BS) void k_kron_chunked(MvArgs<T> A, const int32_t *__restrict__ ch_off,
                                                     const int64_t *__restrict__ ch_base,
                                                     const uint32_t *__restrict__ ch_ell, const T *__restrict__ code_v,
                                                     int nchunks, int chunk_rows, int nslices)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tab = reinterpret_cast<T *>(smem_raw);
    T *xs = tab + 256;
    const int tile = xcd_tile(A.cd);
    if (tile < 0) return;
    const int cu = A.cu;
    const int b = tile;
    const int64_t cu64 = cu;
    const T *__restrict__ xb = A.x + (int64_t)b * cu;
    T *yb = A.y + (int64_t)b * cu;
    for (int i = threadIdx.x; i < 256; i += BS) tab[i] = code_v[i];
    const int ds = A.dn_rp[b], de = A.dn_rp[b + 1];
    const uint32_t dnb = A.dn_basis[b];
    const T edn = A.e_dn[b];
    const int lane = threadIdx.x & 63;
    for (int p = 0; p < nchunks; ++p) {
        const int r0 = p * chunk_rows;
        const int r1 = min(cu, r0 + chunk_rows);
        __syncthreads();  // previous phase done with xs
        for (int i = r0 + threadIdx.x; i < r1; i += BS) xs[i - r0] = xb[i];
        __syncthreads();
        const int32_t *off = ch_off + (int64_t)p * (nslices + 1);
        const uint32_t *ell = ch_ell + ch_base[p];
        for (int a0 = threadIdx.x; a0 < cu; a0 += BS * R) {
            T acc[R][1];
            int as[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int a = min(a0 + j * BS, cu - 1);
                as[j] = a;
                if (p == 0) acc[j][0] = (diag_u(A, A.up_basis[a] & dnb) + A.e_up[a] + edn) * xb[a];
                else acc[j][0] = yb[a];
                const int s = a >> 6;
                up_term_c<T, 1>(acc[j], xs, tab, ell, off[s] * 64 + lane, off[s + 1] - off[s]);
            }
            if (p == 0) {
                int k = ds;
                for (; k + 4 <= de; k += 4) {
                    T y[4][R];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int j = 0; j < R; ++j) y[u][j] = A.x[(int64_t)A.dn_col[k + u] * cu64 + as[j]];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int j = 0; j < R; ++j) acc[j][0] += A.dn_val[k + u] * y[u][j];
                }
                for (; k < de; ++k)
#pragma unroll
                    for (int j = 0; j < R; ++j) acc[j][0] += A.dn_val[k] * A.x[(int64_t)A.dn_col[k] * cu64 + as[j]];
            }
#pragma unroll
            for (int j = 0; j < R; ++j)
                if (a0 + j * BS < cu) yb[a0 + j * BS] = acc[j][0];
        }
    }
}

// ---- two-pass, pass 1: Z = V H_dn^T on XCD-cooperative row tiles --------
// A tile is TA = 128 B / sizeof(T) rows (one cache line per column), so two
// tiles in flight stay well inside one XCD's 4 MB L2 for count_dn ~ 10^4.  A
// wavefront covers 64 / TA output columns of the tile; each group of TA lanes
// walks its own row of H_dn with 8 neighbour reads in flight.
template <typename T, int BS, bool NT>
__global__ __launch_bounds__(BS) void k_kron_dn_tiles(MvArgs<T> A, T *z, int ntiles, int per_xcd)
{
    constexpr int TA = 128 / (int)sizeof(T);
    constexpr int CPW = 64 / TA;                // output columns per wavefront
    constexpr int CPB = (BS / 64) * CPW;        // output columns per workgroup step
    const int64_t cu = A.cu;
    const int cd = A.cd;
    const int xcd = blockIdx.x & 7;
    const int r = blockIdx.x >> 3;  // rank of this workgroup within its XCD
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane / TA, row = lane % TA;
    const int cols_per = (cd + per_xcd - 1) / per_xcd;
    const int c0 = r * cols_per, c1 = min(cd, c0 + cols_per);
    for (int tile = xcd; tile < ntiles; tile += 8) {
        const int a = tile * TA + row;
        const bool live = a < cu;
        const T *__restrict__ xa = A.x + (live ? a : 0);
        for (int b = c0 + wave * CPW + sub; b < c1; b += CPB) {
            const int ks = A.dn_rp[b], ke = A.dn_rp[b + 1];
            T acc = (T)0;
            int k = ks;
            for (; k + 8 <= ke; k += 8) {
                T y[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) y[u] = xa[(int64_t)A.dn_col[k + u] * cu];
#pragma unroll
                for (int u = 0; u < 8; ++u) acc += A.dn_val[k + u] * y[u];
            }
            for (; k < ke; ++k) acc += A.dn_val[k] * xa[(int64_t)A.dn_col[k] * cu];
            if (live) {
                if (NT) __builtin_nontemporal_store(acc, z + (int64_t)b * cu + a);
                else z[(int64_t)b * cu + a] = acc;
            }
        }
    }
}

// Pass 1 in dispatch order: workgroup g takes (row tile, column chunk) with
// the tiles of XCD g mod 8 in increasing order and the chunks of one tile
// consecutive.  Workgroups are dispatched in index order, so the ones resident
// on an XCD at any moment share one or two row tiles (TA rows of every
// column), which stay in that XCD's L2 while the neighbour reads hit them.
template <typename T, int BS, bool NT>
__global__ __launch_bounds__(BS) void k_kron_dn_otiles(MvArgs<T> A, T *z, int ntiles, int nchunks, int chunk_cols)
{
    constexpr int TA = 128 / (int)sizeof(T);
    constexpr int CPW = 64 / TA;
    constexpr int CPB = (BS / 64) * CPW;
    const int64_t cu = A.cu;
    const int cd = A.cd;
    const int xcd = blockIdx.x & 7;
    const int r = blockIdx.x >> 3;
    const int tile = (r / nchunks) * 8 + xcd;
    if (tile >= ntiles) return;
    const int chunk = r - (r / nchunks) * nchunks;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane / TA, row = lane % TA;
    const int c0 = chunk * chunk_cols, c1 = min(cd, c0 + chunk_cols);
    const int a = tile * TA + row;
    const bool live = a < cu;
    const T *__restrict__ xa = A.x + (live ? a : 0);
    for (int b = c0 + wave * CPW + sub; b < c1; b += CPB) {
        const int ks = A.dn_rp[b], ke = A.dn_rp[b + 1];
        T acc = (T)0;
        int k = ks;
        for (; k + 8 <= ke; k += 8) {
            T y[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) y[u] = xa[(int64_t)A.dn_col[k + u] * cu];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += A.dn_val[k + u] * y[u];
        }
        for (; k < ke; ++k) acc += A.dn_val[k] * xa[(int64_t)A.dn_col[k] * cu];
        if (live) {
            if (NT) __builtin_nontemporal_store(acc, z + (int64_t)b * cu + a);
            else z[(int64_t)b * cu + a] = acc;
        }
    }
}

// ---- two-pass, pass 2: Y = Z + H_up V + D o V on LDS column panels --------
template <typename T, int TB, int BS>
__global__ __launch_bounds__(BS) void k_kron_up_panels(MvArgs<T> A, const T *z, const int32_t *__restrict__ sl_off,
                                                       const Pk<T> *__restrict__ ell, int ntiles)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *xs = reinterpret_cast<T *>(smem_raw);
    const int tile = xcd_tile(ntiles);
    if (tile < 0) return;
    const int cu = A.cu, cd = A.cd;
    const int b0 = tile * TB;
    stage_columns<T, TB>(A, xs, b0, BS);
    __syncthreads();
    uint32_t dnb[TB];
    T edn[TB];
#pragma unroll
    for (int t = 0; t < TB; ++t) {
        const int b = min(b0 + t, cd - 1);
        dnb[t] = A.dn_basis[b];
        edn[t] = A.e_dn[b];
    }
    const int lane = threadIdx.x & 63;
    for (int a = threadIdx.x; a < cu; a += BS) {
        const uint32_t ua = A.up_basis[a];
        const T eua = A.e_up[a];
        const Vec<T, TB> xa = *reinterpret_cast<const Vec<T, TB> *>(xs + a * TB);
        T acc[TB];
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            const int b = min(b0 + t, cd - 1);
            acc[t] = z[(int64_t)b * cu + a] + (diag_u(A, ua & dnb[t]) + eua + edn[t]) * xa.v[t];
        }
        const int s = a >> 6;
        up_term<T, TB>(acc, xs, ell, sl_off[s] * 64 + lane, sl_off[s + 1] - sl_off[s]);
#pragma unroll
        for (int t = 0; t < TB; ++t)
            if (b0 + t < cd) A.y[(int64_t)(b0 + t) * cu + a] = acc[t];
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
        acc += dn_term(A, ds, de, A.x + a);
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
const Pk<T> *ell_of(const SpinTables &U)
{
    if constexpr (sizeof(T) == 8) return (const Pk<T> *)U.ell_pk64;
    else return (const Pk<T> *)U.ell_pk32;
}

template <typename K>
hub_status allow_lds(K kernel, size_t bytes)
{
    HUB_HIP(hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return HUB_OK;
}

template <typename T, int TB, int BS, int R = 4>
hub_status launch_fused(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, bool cf)
{
    const SpinTables &U = s->spin[0];
    const int ntiles = (A.cd + TB - 1) / TB;
    const unsigned grid = 8u * (unsigned)((ntiles + 7) / 8);
    if (cf && U.ell_c32) {
        const size_t lds = (size_t)(A.cu * TB + 256) * sizeof(T);
        static std::atomic<bool> attr{false};
        if (!attr) {
            HUB_TRY(allow_lds(k_kron_fused<T, TB, BS, R, true>, s->lds_max));
            attr = true;
        }
        const T *cv;
        if constexpr (sizeof(T) == 8) cv = (const T *)U.code_v64;
        else cv = (const T *)U.code_v32;
        hipLaunchKernelGGL((k_kron_fused<T, TB, BS, R, true>), dim3(grid), dim3(BS), lds, st, A, U.sl_off,
                           ell_of<T>(U), U.ell_c32, cv, ntiles);
        HUB_HIP(hipGetLastError());
        return HUB_OK;
    }
    const size_t lds = (size_t)A.cu * TB * sizeof(T);
    static std::atomic<bool> attr{false};
    if (!attr) {
        HUB_TRY(allow_lds(k_kron_fused<T, TB, BS, R, false>, s->lds_max));
        attr = true;
    }
    hipLaunchKernelGGL((k_kron_fused<T, TB, BS, R, false>), dim3(grid), dim3(BS), lds, st, A, U.sl_off,
                       ell_of<T>(U), (const uint32_t *)nullptr, (const T *)nullptr, ntiles);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

int env_int(const char *name, int dflt)
{
    const char *v = getenv(name);
    return v ? atoi(v) : dflt;
}

template <typename T, int TB, int BS>
hub_status launch_two_pass(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, int occ, int nt)
{
    constexpr int BSD = 256;
    const SpinTables &U = s->spin[0];
    const int ntiles_d = (A.cu + (128 / (int)sizeof(T)) - 1) / (128 / (int)sizeof(T));
    const int per_xcd = (s->cu_count / 8) * occ;
    static const int ordered = env_int("HUB_DN_ORDER", 1);
    static const int chunk_env = env_int("HUB_DN_CH", 256);
    if (ordered) {
        const int chunk_cols = std::max(1, chunk_env);
        const int nchunks = (A.cd + chunk_cols - 1) / chunk_cols;
        const unsigned grid = 8u * (unsigned)((ntiles_d + 7) / 8) * (unsigned)nchunks;
        if (nt)
            hipLaunchKernelGGL((k_kron_dn_otiles<T, BSD, true>), dim3(grid), dim3(BSD), 0, st, A, A.y, ntiles_d,
                               nchunks, chunk_cols);
        else
            hipLaunchKernelGGL((k_kron_dn_otiles<T, BSD, false>), dim3(grid), dim3(BSD), 0, st, A, A.y, ntiles_d,
                               nchunks, chunk_cols);
    } else if (nt)
        hipLaunchKernelGGL((k_kron_dn_tiles<T, BSD, true>), dim3(8 * per_xcd), dim3(BSD), 0, st, A, A.y, ntiles_d,
                           per_xcd);
    else
        hipLaunchKernelGGL((k_kron_dn_tiles<T, BSD, false>), dim3(8 * per_xcd), dim3(BSD), 0, st, A, A.y, ntiles_d,
                           per_xcd);
    const size_t lds = (size_t)A.cu * TB * sizeof(T);
    static std::atomic<bool> attr{false};
    if (!attr) {
        HUB_TRY(allow_lds(k_kron_up_panels<T, TB, BS>, s->lds_max));
        attr = true;
    }
    const int ntiles = (A.cd + TB - 1) / TB;
    const unsigned grid = 8u * (unsigned)((ntiles + 7) / 8);
    hipLaunchKernelGGL((k_kron_up_panels<T, TB, BS>), dim3(grid), dim3(BS), lds, st, A, (const T *)A.y, U.sl_off,
                       ell_of<T>(U), ntiles);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

template <typename T, int TB, int BS, bool XC, bool EPI>
hub_status launch_quad_e(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, const LzEpi<T> &E)
{
    const SpinTables &U = s->spin[0];
    const int ntiles = (A.cd + TB - 1) / TB;
    const unsigned grid = XC ? 8u * (unsigned)((ntiles + 7) / 8) : (unsigned)ntiles;
    // columns (cu % 4 == 0 keeps the FP32 case 8-byte aligned), then the group partials
    const size_t lds = (size_t)(A.cu * TB + 256) * sizeof(T) + (EPI ? (size_t)TB * E.G * sizeof(double) : 0);
    if (lds > s->lds_max) {
        set_error("fused product: tile does not fit in LDS");
        return HUB_ERR_UNSUPPORTED;
    }
    static std::atomic<bool> attr{false};
    if (!attr) {
        HUB_TRY(allow_lds(k_kron_quad<T, TB, BS, XC, EPI>, s->lds_max));
        attr = true;
    }
    const T *cv;
    if constexpr (sizeof(T) == 8) cv = (const T *)U.code_v64;
    else cv = (const T *)U.code_v32;
    hipLaunchKernelGGL((k_kron_quad<T, TB, BS, XC, EPI>), dim3(grid), dim3(BS), lds, st, A, U.sl_off, U.ell_c32, cv,
                       ntiles, E);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

template <typename T, int TB, int BS, bool XC>
hub_status launch_quad_t(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, const LzEpi<T> *E)
{
    if (E) return launch_quad_e<T, TB, BS, XC, true>(s, A, st, *E);
    return launch_quad_e<T, TB, BS, XC, false>(s, A, st, LzEpi<T>{nullptr, nullptr, nullptr, 0, nullptr, 0});
}

// shape code: TB in 1..3, BS in {512, 1024}, XC in {0, 1}; E: fused Lanczos epilogue or NULL
template <typename T>
hub_status launch_quad(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, int tb, int bs, int xc,
                       const LzEpi<T> *E = nullptr)
{
#define HUB_QUAD(TBV, BSV, XCV)                                                                       \
    if (tb == TBV && bs == BSV && xc == XCV) return launch_quad_t<T, TBV, BSV, XCV>(s, A, st, E);
    HUB_QUAD(1, 512, 0) HUB_QUAD(1, 512, 1) HUB_QUAD(1, 1024, 0) HUB_QUAD(1, 1024, 1)
    HUB_QUAD(2, 512, 0) HUB_QUAD(2, 512, 1) HUB_QUAD(2, 1024, 0) HUB_QUAD(2, 1024, 1)
    HUB_QUAD(3, 512, 0) HUB_QUAD(3, 512, 1) HUB_QUAD(3, 1024, 0) HUB_QUAD(3, 1024, 1)
#undef HUB_QUAD
    set_error("untuned product shape");
    return HUB_ERR_UNSUPPORTED;
}

// First product of a dtype on a sector: time every shape whose columns fit in
// the LDS (1 warm-up + 5 timed launches on the caller's x and y; every shape
// computes the same values in the same order) and keep the fastest; a later
// candidate must win by 3 % so that timing noise rarely changes the pick.
// Times every shape that fits, in two interleaved rounds of five launches,
// and keeps the one with the smallest time (each shape's better round).  epi: the shapes are timed as the
// product fused with the first Lanczos update, whose ranking differs from the
// plain product's (on the ring M=14, FP32 with two columns per workgroup:
// 57 vs 55 us plain but 90 vs 75 us fused for 1024 vs 512 lanes); the epilogue
// then reads x as v_prev with beta = 0 and writes its partials to apart
// (count_dn doubles), all overwritten by the caller's own launch.
template <typename T>
hub_status tune_quad(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, QuadShape &out, bool epi,
                     double *apart)
{
    hipEvent_t e0, e1;
    HUB_HIP(hipEventCreate(&e0));
    HUB_HIP(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } ev{e0, e1};
    const int G = (int)(((A.cu >> 2) + 63) / 64);
    double *zero = nullptr;
    struct Buf {
        double *p = nullptr;
        ~Buf() { (void)hipFree(p); }
    } zb;
    LzEpi<T> E{};
    if (epi) {
        HUB_HIP(hipMalloc((void **)&zero, sizeof(double)));
        zb.p = zero;
        HUB_HIP(hipMemsetAsync(zero, 0, sizeof(double), st));
        E = LzEpi<T>{A.x, zero, apart, G, nullptr, 0};
    }
    std::vector<QuadShape> cand;
    for (int tb = 1; tb <= 3; ++tb) {
        const size_t lds = (size_t)(A.cu * tb + 256) * sizeof(T) + (epi ? (size_t)tb * G * sizeof(double) : 0);
        if (lds > s->lds_max) break;
        for (int bs : {512, 1024})
            for (int xc : {0, 1}) {
                QuadShape c;
                c.tb = tb;
                c.bs = bs;
                c.xc = xc;
                c.ms = 1e30f;
                cand.push_back(c);
            }
    }
    if (cand.empty()) {
        set_error("no product shape fits in LDS");
        return HUB_ERR_UNSUPPORTED;
    }
    for (int round = 0; round < 2; ++round)
        for (QuadShape &c : cand) {
            HUB_TRY(launch_quad<T>(s, A, st, c.tb, c.bs, c.xc, epi ? &E : nullptr));
            HUB_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < 5; ++r) HUB_TRY(launch_quad<T>(s, A, st, c.tb, c.bs, c.xc, epi ? &E : nullptr));
            HUB_HIP(hipEventRecord(e1, st));
            HUB_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            HUB_HIP(hipEventElapsedTime(&ms, e0, e1));
            c.ms = std::min(c.ms, ms / 5.0f);
        }
    out = *std::min_element(cand.begin(), cand.end(),
                            [](const QuadShape &a, const QuadShape &b) { return a.ms < b.ms; });
    return HUB_OK;
}

// Tuned shapes are kept per device, dtype and sector structure (dimensions and
// nonzeros; the values of t, U and eps do not change the timing), so sectors
// of the same lattice share one tuning.
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
std::map<ShapeKey, QuadShape> g_shapes;

// Shape of the four-rows-per-lane product: forced by HUB_MATVEC_TB / _BS / _XC,
// else the sector's tuned shape (tuning on first use, shared by sectors of
// the same structure).  epi: the shape of the product fused with the Lanczos
// update, tuned separately (apart: its partials buffer, used while tuning).
template <typename T>
hub_status quad_shape(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, QuadShape &out, bool epi = false,
                      double *apart = nullptr)
{
    const int di = (sizeof(T) == 8) ? 0 : 1;
    const int tb_env = env_int("HUB_MATVEC_TB", 0);
    const int bs_env = env_int("HUB_MATVEC_BS", 0);
    if (tb_env > 0 || bs_env > 0) {
        out.tb = std::min(std::max(tb_env > 0 ? tb_env : 1, 1), 3);
        out.bs = bs_env == 512 ? 512 : 1024;
        out.xc = env_int("HUB_MATVEC_XC", 1) != 0 ? 1 : 0;
        return HUB_OK;
    }
    // the sector's cached shape and the shared table are read and written under
    // one mutex (a sector may serve products on several threads); tuning runs
    // outside it, and two threads that tune at once both store a valid shape
    QuadShape &q = epi ? s->quad_lz[di] : s->quad[di];
    const ShapeKey key{s->device, di, (int64_t)A.cu, (int64_t)A.cd, s->spin[0].nnz, s->spin[1].nnz, epi ? 1 : 0};
    {
        std::lock_guard<std::mutex> lk(g_shape_mu);
        if (q.tb == 0) {
            auto it = g_shapes.find(key);
            if (it != g_shapes.end()) q = it->second;
        }
        if (q.tb != 0) {
            out = q;
            return HUB_OK;
        }
    }
    QuadShape t;
    HUB_TRY(tune_quad<T>(s, A, st, t, epi, apart));
    std::lock_guard<std::mutex> lk(g_shape_mu);
    g_shapes[key] = t;
    q = t;
    out = t;
    return HUB_OK;
}

// Whether the fused product + first Lanczos update is available for the sector.
template <typename T>
bool lz_fusable(const hub_sector *s)
{
    const SpinTables &U = s->spin[0];
    const size_t col_bytes = (size_t)U.count * sizeof(T);
    return !s->k0 && env_int("HUB_MATVEC_IMPL", 2) == 2 && env_int("HUB_MATVEC_QUAD", 1) != 0 &&
           env_int("HUB_ELL_FMT", 1) != 0 && env_int("HUB_LZ_FUSE", 1) != 0 && U.ell_c32 && !s->force_chunked &&
           (U.count % 4) == 0 &&
           col_bytes + 256 * sizeof(T) + (size_t)((U.count / 4 + 63) / 64) * sizeof(double) <= s->lds_max;
}

template <typename T>
hub_status run_kron_lz(const hub_sector *s, const void *x, void *w, const void *vprev, const double *beta,
                       const double *beta_prev, int unnorm, double *apart, int64_t *npart, hipStream_t st)
{
    if (!lz_fusable<T>(s)) return HUB_ERR_UNSUPPORTED;
    MvArgs<T> A = make_args<T>(s, x, w);
    QuadShape q;
    HUB_TRY(quad_shape<T>(s, A, st, q, true, apart));
    const int G = (int)(((A.cu >> 2) + 63) / 64);
    const LzEpi<T> E{(const T *)vprev, beta, apart, G, beta_prev, unnorm};
    *npart = (int64_t)A.cd;
    // the group partials need TB * G doubles of LDS beside the columns: fall back to fewer columns
    for (int tb = q.tb; tb >= 1; --tb) {
        if ((size_t)(A.cu * tb + 256) * sizeof(T) + (size_t)tb * G * sizeof(double) <= s->lds_max)
            return launch_quad<T>(s, A, st, tb, q.bs, q.xc, &E);
    }
    return HUB_ERR_UNSUPPORTED;
}

// Row-chunked product with register-held output rows: TB columns per work
// item (the chunk tables were sized for TB), 4 x 1024 lane-quads per row part.
template <typename T, int TB>
hub_status launch_chunked_parts_t(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, const T *cv)
{
    constexpr int BSC = 1024, QPL = 4;
    const int di = (sizeof(T) == 8) ? 0 : 1;
    const SpinTables &U = s->spin[0];
    const size_t lds = ((size_t)U.chunk_rows[di] * TB + 256) * sizeof(T);
    if (lds > s->lds_max) {
        set_error("row-chunked product: chunk does not fit in LDS");
        return HUB_ERR_UNSUPPORTED;
    }
    const int nq = (int)(A.cu >> 2);
    const int P = (nq + BSC * QPL - 1) / (BSC * QPL);
    const int ntiles = (A.cd + TB - 1) / TB;
    static std::atomic<bool> attr{false};
    if (!attr) {
        HUB_TRY(allow_lds(k_kron_chunked_parts<T, BSC, QPL, TB>, s->lds_max));
        attr = true;
    }
    const unsigned grid = 8u * (unsigned)P * (unsigned)((ntiles + 7) / 8);
    hipLaunchKernelGGL((k_kron_chunked_parts<T, BSC, QPL, TB>), dim3(grid), dim3(BSC), lds, st, A, U.ch_off[di],
                       U.ch_base[di], U.ch_ell[di], cv, U.nchunks[di], U.chunk_rows[di], (int)U.nslices, P);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

template <typename T>
hub_status launch_chunked_parts(const hub_sector *s, const MvArgs<T> &A, hipStream_t st, int tb, const T *cv)
{
    // FP64 with four columns would need more registers than a 1024-lane workgroup has
    if constexpr (sizeof(T) == 4)
        if (tb >= 4) return launch_chunked_parts_t<T, 4>(s, A, st, cv);
    if (tb >= 2) return launch_chunked_parts_t<T, 2>(s, A, st, cv);
    return launch_chunked_parts_t<T, 1>(s, A, st, cv);
}

// Schedule selection.  Environment overrides for measurement: HUB_MATVEC_IMPL
// (1 csr, 2 fused, 3 two-pass), HUB_MATVEC_TB, HUB_MATVEC_BS (512 / 1024),
// HUB_MATVEC_XC (tile order), HUB_MATVEC_QUAD (0: one row per lane),
// HUB_FUSED_R, HUB_ELL_FMT (0 packed, 1 compact), HUB_DN_OCC, HUB_DN_NT.
// Default: the four-rows-per-lane fused kernel when count_up % 4 == 0 (shape
// tuned on the first product of each dtype), else the one-row fused kernel
// with two columns per workgroup when they fit in half of the LDS; the
// row-chunked kernel when a column does not fit in the LDS.
template <typename T>
hub_status run_kron(const hub_sector *s, const void *x, void *y, hipStream_t st)
{
    MvArgs<T> A = make_args<T>(s, x, y);
    const size_t col_bytes = (size_t)A.cu * sizeof(T);
    // read on every call so a variant or shape can be forced for measurement or tests
    const int impl = env_int("HUB_MATVEC_IMPL", 2);
    const int tb_env = env_int("HUB_MATVEC_TB", 0);
    const int bs_env = env_int("HUB_MATVEC_BS", 0);
    const int occ = env_int("HUB_DN_OCC", 4);
    const int nt = env_int("HUB_DN_NT", 1);
    const int rows = env_int("HUB_FUSED_R", 4);
    const bool cf = env_int("HUB_ELL_FMT", 1) != 0;
    // four-rows-per-lane kernels use 16-byte accesses: caller vectors that are
    // not 16-byte aligned take the one-row-per-lane kernels
    const bool aligned16 = (((uintptr_t)x | (uintptr_t)y) & 15u) == 0;
    const bool quad = env_int("HUB_MATVEC_QUAD", 1) != 0 && aligned16;
    const size_t extra = 256 * sizeof(T);
    const size_t half = s->lds_max / 2;
    int tb = tb_env;
    if (tb <= 0) tb = (2 * col_bytes + extra <= half) ? 2 : 1;
    while (tb > 1 && tb * col_bytes + extra > s->lds_max) tb >>= 1;
    const bool fits = col_bytes + extra <= s->lds_max;
    const bool big = bs_env != 512;
    if (impl == 3 && fits) {
        if (tb >= 2)
            return big ? launch_two_pass<T, 2, 1024>(s, A, st, occ, nt) : launch_two_pass<T, 2, 512>(s, A, st, occ, nt);
        return big ? launch_two_pass<T, 1, 1024>(s, A, st, occ, nt) : launch_two_pass<T, 1, 512>(s, A, st, occ, nt);
    }
    const int di = (sizeof(T) == 8) ? 0 : 1;
    const SpinTables &U = s->spin[0];
    if (impl != 1 && (!fits || s->force_chunked) && U.ch_ell[di]) {
        constexpr int BSC = 1024;
        const size_t lds = (size_t)(U.chunk_rows[di] + 256) * sizeof(T);
        static std::atomic<bool> attr{false};
        if (!attr) {
            HUB_TRY(allow_lds(k_kron_chunked<T, BSC, 4>, s->lds_max));
            attr = true;
        }
        const T *cv;
        if constexpr (sizeof(T) == 8) cv = (const T *)U.code_v64;
        else cv = (const T *)U.code_v32;
        const unsigned grid = 8u * (unsigned)((A.cd + 7) / 8);
        const int ctb = U.chunk_tb[di];
        if (quad && (A.cu % 4) == 0 && (U.chunk_rows[di] % 4) == 0 && env_int("HUB_CHUNK_PARTS", 1) != 0) {
            HUB_TRY(launch_chunked_parts<T>(s, A, st, ctb, cv));
        } else if (quad && (A.cu % 4) == 0 && (U.chunk_rows[di] % 4) == 0) {
            // tile order: launch order (all XCDs on nearby columns, so recently read
            // neighbour columns are more often still in the MALL: 2x9 ladder FP32 39.3 -> 37.6 ms)
            // or XCD-contiguous ranges (HUB_CHUNK_XC=1)
            const bool xc = env_int("HUB_CHUNK_XC", 0) != 0;
            static std::atomic<bool> attrq{false};
            if (!attrq) {
                HUB_TRY(allow_lds(k_kron_chunked_quad<T, BSC, true>, s->lds_max));
                HUB_TRY(allow_lds(k_kron_chunked_quad<T, BSC, false>, s->lds_max));
                attrq = true;
            }
            if (xc)
                hipLaunchKernelGGL((k_kron_chunked_quad<T, BSC, true>), dim3(grid), dim3(BSC), lds, st, A,
                                   U.ch_off[di], U.ch_base[di], U.ch_ell[di], cv, U.nchunks[di], U.chunk_rows[di],
                                   (int)U.nslices);
            else
                hipLaunchKernelGGL((k_kron_chunked_quad<T, BSC, false>), dim3(grid), dim3(BSC), lds, st, A,
                                   U.ch_off[di], U.ch_base[di], U.ch_ell[di], cv, U.nchunks[di], U.chunk_rows[di],
                                   (int)U.nslices);
        } else {
            hipLaunchKernelGGL((k_kron_chunked<T, BSC, 4>), dim3(grid), dim3(BSC), lds, st, A, U.ch_off[di],
                               U.ch_base[di], U.ch_ell[di], cv, U.nchunks[di], U.chunk_rows[di], (int)U.nslices);
        }
        HUB_HIP(hipGetLastError());
        return HUB_OK;
    }
    if (impl == 2 && fits && cf && U.ell_c32 && (A.cu % 4) == 0 && quad) {
        QuadShape q;
        HUB_TRY(quad_shape<T>(s, A, st, q));
        return launch_quad<T>(s, A, st, q.tb, q.bs, q.xc);
    }
    if (impl == 2 && fits) {
        if (tb >= 4) return big ? launch_fused<T, 4, 1024, 1>(s, A, st, cf) : launch_fused<T, 4, 512, 1>(s, A, st, cf);
        if (tb >= 2) return big ? launch_fused<T, 2, 1024, 2>(s, A, st, cf) : launch_fused<T, 2, 512, 2>(s, A, st, cf);
        if (rows >= 4) return big ? launch_fused<T, 1, 1024, 4>(s, A, st, cf) : launch_fused<T, 1, 512, 4>(s, A, st, cf);
        return big ? launch_fused<T, 1, 1024, 1>(s, A, st, cf) : launch_fused<T, 1, 512, 1>(s, A, st, cf);
    }
    hipLaunchKernelGGL((k_kron_csr<T, 512>), dim3((unsigned)A.cd), dim3(512), 0, st, A);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
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

int64_t matvec_lz_partials(const hub_sector *s)
{
    return s->spin[1].count;
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
        // row pointers, columns, values, basis integers, site energies
        bytes += 4 * (T.count + 1) + T.nnz * (4 + es) + 4 * T.count + es * T.count;
    }
    return bytes;
}

}  // namespace hub
