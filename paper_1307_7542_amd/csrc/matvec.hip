// Kronecker-sum product of the sector Hamiltonian (Sec. IV A):
//
//     Y = H_up V + V H_dn^T + D o V,   V, Y: count_up x count_dn, column-major.
//
// H_dn is real symmetric, so column b of V H_dn^T is sum_l H_dn[b, l] V[:, l].
// D(a, b) = U-part(basis_up[a] & basis_dn[b]) + e_up[a] + e_dn[b] is generated
// from the bit patterns (the doubly occupied sites of Sec. III B) and never
// stored.
//
// Work decomposition: one workgroup per output column b.  The column V[:, b]
// is staged in LDS once; each lane then owns rows a and forms
//   - the diagonal term from the two occupation integers,
//   - the H_up term by gathering inside the LDS column along row a of H_up,
//   - the H_dn term by reading whole neighbouring columns V[:, l] (coalesced
//     along a; the row of H_dn is the same for the whole workgroup, so its
//     indices and values are scalar loads).
// Columns whose LDS footprint exceeds the per-workgroup limit gather the H_up
// term from global memory (L2) instead.
#include "internal.h"

namespace hub {
namespace {

template <typename T>
struct MvArgs {
    const T *__restrict__ x;
    T *__restrict__ y;
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
    const T *__restrict__ Us;   // per-site U (non-uniform case)
    const int32_t *__restrict__ order;  // column processing order or null
    T U;
    int32_t uniform;
    uint32_t umask;
};

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

template <typename T, bool USE_LDS, int BS>
__global__ __launch_bounds__(BS) void k_kron(MvArgs<T> A)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *xs = reinterpret_cast<T *>(smem_raw);
    const int b = A.order ? A.order[blockIdx.x] : (int)blockIdx.x;
    const int cu = A.cu;
    const T *__restrict__ xb = A.x + (int64_t)b * cu;
    T *__restrict__ yb = A.y + (int64_t)b * cu;
    if (USE_LDS) {
        for (int i = threadIdx.x; i < cu; i += BS) xs[i] = xb[i];
        __syncthreads();
    }
    const int ds = A.dn_rp[b], de = A.dn_rp[b + 1];
    const uint32_t dnb = A.dn_basis[b];
    const T edn = A.e_dn[b];
    for (int a = threadIdx.x; a < cu; a += BS) {
        const T xa = USE_LDS ? xs[a] : xb[a];
        const T d = diag_u(A, A.up_basis[a] & dnb) + A.e_up[a] + edn;
        T acc = d * xa;
        const int us = A.up_rp[a], ue = A.up_rp[a + 1];
        for (int k = us; k < ue; ++k) {
            const int l = A.up_col[k];
            acc += A.up_val[k] * (USE_LDS ? xs[l] : xb[l]);
        }
        for (int k = ds; k < de; ++k) acc += A.dn_val[k] * A.x[(int64_t)A.dn_col[k] * cu + a];
        yb[a] = acc;
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
    A.order = s->col_order;
    A.uniform = s->uniformU;
    A.umask = s->umask;
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
hub_status run_kron(const hub_sector *s, const void *x, void *y, hipStream_t st)
{
    constexpr int BS = 512;
    MvArgs<T> A = make_args<T>(s, x, y);
    const size_t lds = (size_t)A.cu * sizeof(T);
    if (lds <= s->lds_max) {
        static bool attr_set = false;
        if (!attr_set) {
            HUB_HIP(hipFuncSetAttribute((const void *)k_kron<T, true, BS>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)s->lds_max));
            attr_set = true;
        }
        hipLaunchKernelGGL((k_kron<T, true, BS>), dim3((unsigned)A.cd), dim3(BS), lds, st, A);
    } else {
        hipLaunchKernelGGL((k_kron<T, false, BS>), dim3((unsigned)A.cd), dim3(BS), 0, st, A);
    }
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

}  // namespace

hub_status launch_matvec(const hub_sector *s, int dtype, const void *x, void *y, hipStream_t st)
{
    if (dtype == HUB_F64) return run_kron<double>(s, x, y, st);
    return run_kron<float>(s, x, y, st);
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
