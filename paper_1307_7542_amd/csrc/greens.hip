// Zero-temperature one-particle Green's function (Sec. VII A, the second
// equation labelled count8):
//   G_s(p, z) = <psi0| c_ps (z + E0 - H)^-1 c+_ps |psi0> + <psi0| c+_ps (z - E0 + H)^-1 c_ps |psi0>.
// The start vectors c+_ps|psi0> (sector N_s + 1) and c_ps|psi0> (sector N_s - 1)
// come from one gather kernel driven by a per-spin index map: only the spin
// whose particle number changes is remapped, so the scatter of Sec. VII A
// (one loop over the changed spin's basis, the other spin's index carried
// along) becomes a coalesced gather on the destination vector.  The
// resolvents are continued fractions whose coefficients come from the plain
// Lanczos recurrence (Sec. IV) in the destination sector.
//
// Operator ordering: all up creation operators (ascending site) to the left
// of all down ones, as in the basis kets of Sec. II; so c+_p,s picks up
// (-1)^(occupied sites of spin s below p) and, for s = down, a further
// (-1)^(N_up) from passing the up operators.
#include <chrono>
#include <complex>
#include <cstring>
#include <vector>

#include "internal.h"

namespace hub {
namespace {

// rank of an occupation pattern: sum over its set bits b_1 < ... < b_N of C(b_k, k)
__device__ __forceinline__ int64_t op_rank(uint32_t x, const uint64_t *__restrict__ C)
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

// For every state r of the destination spin basis: the source state it comes
// from (or -1) and the sign.  create: dst = c+_p src (dst has p occupied);
// otherwise dst = c_p src (dst has p empty).
__global__ void k_op_map(const uint32_t *__restrict__ dst_basis, int64_t count, int site, int create, int flip,
                         const uint64_t *__restrict__ C, int32_t *__restrict__ map, double *__restrict__ sgn)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint32_t x = dst_basis[i];
    const uint32_t bit = 1u << site;
    const uint32_t below = bit - 1u;
    int32_t src = -1;
    double s = 0.0;
    if (create && (x & bit)) {
        const uint32_t y = x ^ bit;
        src = (int32_t)op_rank(y, C);
        s = (__popc(y & below) & 1) ? -1.0 : 1.0;
    } else if (!create && !(x & bit)) {
        src = (int32_t)op_rank(x | bit, C);
        s = (__popc(x & below) & 1) ? -1.0 : 1.0;
    }
    map[i] = src;
    sgn[i] = flip ? -s : s;
}

// y[a + b cu_dst] = su[a] sd[b] x[mu[a] + md[b] cu_src], zero where a map is -1;
// a NULL map is the identity (the spin whose number does not change).
__global__ __launch_bounds__(256) void k_op_apply(const double *__restrict__ x, double *__restrict__ y,
                                                  int64_t cu_src, int64_t cu_dst, int64_t cd_dst,
                                                  const int32_t *__restrict__ mu, const double *__restrict__ su,
                                                  const int32_t *__restrict__ md, const double *__restrict__ sd)
{
    for (int64_t b = blockIdx.y; b < cd_dst; b += gridDim.y) {
        const int64_t sb = md ? (int64_t)md[b] : b;
        const double fb = md ? sd[b] : 1.0;
        for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < cu_dst;
             a += (int64_t)gridDim.x * blockDim.x) {
            const int64_t sa = mu ? (int64_t)mu[a] : a;
            const double fa = mu ? su[a] : 1.0;
            double v = 0.0;
            if (sa >= 0 && sb >= 0) v = (fa * fb) * x[sa + sb * cu_src];
            y[a + b * cu_dst] = v;
        }
    }
}

hub_status gfail(hub_status c, const std::string &m)
{
    set_error(m);
    return c;
}

struct DevBuf {
    std::vector<void *> p;
    ~DevBuf()
    {
        for (void *q : p) (void)hipFree(q);
    }
    hub_status alloc(void **q, size_t bytes)
    {
        hipError_t e = hipMalloc(q, bytes == 0 ? 1 : bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return gfail(HUB_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        p.push_back(*q);
        return HUB_OK;
    }
};

// <f| (w - H)^-1 |f> = norm2 / (w - a0 - b1^2 / (w - a1 - b2^2 / (... (w - a_{m-1}))))
std::complex<double> cfrac(const double *a, const double *b, int m, double norm2, std::complex<double> w)
{
    if (m <= 0 || norm2 == 0.0) return {0.0, 0.0};
    std::complex<double> d = w - a[m - 1];
    for (int j = m - 2; j >= 0; --j) d = w - a[j] - (b[j + 1] * b[j + 1]) / d;
    return norm2 / d;
}

// Particle-number change of one spin between two sectors of the same lattice.
hub_status check_pair(const hub_sector *src, const hub_sector *dst, int spin, int create)
{
    if (src->M != dst->M) return gfail(HUB_ERR_INVALID_ARG, "sectors of different lattices");
    if (src->k0 || dst->k0) return gfail(HUB_ERR_UNSUPPORTED, "not available for translation (k = 0) sectors");
    const int d = create ? 1 : -1;
    const int other = 1 - spin;
    if (dst->spin[spin].N != src->spin[spin].N + d || dst->spin[other].N != src->spin[other].N)
        return gfail(HUB_ERR_INVALID_ARG, "destination sector must differ by one particle of the given spin");
    if (src->device != dst->device) return gfail(HUB_ERR_INVALID_ARG, "sectors on different devices");
    return HUB_OK;
}

hub_status apply_op(const hub_sector *src, const hub_sector *dst, int site, int spin, int create, const double *x,
                    double *y, hipStream_t st)
{
    DevBuf mem;
    const SpinTables &D = dst->spin[spin];
    int32_t *map = nullptr;
    double *sgn = nullptr;
    HUB_TRY(mem.alloc((void **)&map, sizeof(int32_t) * (size_t)D.count));
    HUB_TRY(mem.alloc((void **)&sgn, sizeof(double) * (size_t)D.count));
    const int flip = (spin == 1) ? (src->spin[0].N & 1) : 0;
    hipLaunchKernelGGL(k_op_map, dim3((unsigned)((D.count + 255) / 256)), dim3(256), 0, st, D.basis, D.count, site,
                       create, flip, (const uint64_t *)src->d_binom, map, sgn);
    const int64_t cu_src = src->spin[0].count, cu_dst = dst->spin[0].count, cd_dst = dst->spin[1].count;
    const unsigned gx = (unsigned)std::min<int64_t>((cu_dst + 255) / 256, 64);
    const unsigned gy = (unsigned)std::min<int64_t>(cd_dst, 65535);
    hipLaunchKernelGGL(k_op_apply, dim3(gx, gy), dim3(256), 0, st, x, y, cu_src, cu_dst, cd_dst,
                       spin == 0 ? (const int32_t *)map : nullptr, spin == 0 ? (const double *)sgn : nullptr,
                       spin == 1 ? (const int32_t *)map : nullptr, spin == 1 ? (const double *)sgn : nullptr);
    HUB_HIP(hipGetLastError());
    // the map buffers are freed on return: finish the kernels first
    HUB_HIP(hipStreamSynchronize(st));
    return HUB_OK;
}

// A sector of the same lattice with the spin's particle number shifted by d.
hub_status shifted_sector(const hub_sector *s, int spin, int d, hub_sector **out)
{
    hub_model m;
    m.n_sites = s->M;
    m.n_bonds = s->nb;
    m.bond_i = s->bi.data();
    m.bond_j = s->bj.data();
    m.t = s->t.data();
    m.U = s->U.data();
    m.eps = s->eps.data();
    const int nu = s->spin[0].N + (spin == 0 ? d : 0);
    const int nd = s->spin[1].N + (spin == 1 ? d : 0);
    HUB_HIP(hipSetDevice(s->device));
    return hub_sector_create(&m, nu, nd, out);
}

struct SectorGuard {
    hub_sector *s = nullptr;
    ~SectorGuard()
    {
        if (s) hub_sector_destroy(s);
    }
};

}  // namespace
}  // namespace hub

using namespace hub;

extern "C" {

hub_status hub_apply_fermion(const hub_sector *src, const hub_sector *dst, int32_t site, int32_t spin, int32_t create,
                             const void *dev_x, void *dev_y, void *stream)
{
    if (!src || !dst || !dev_x || !dev_y) return gfail(HUB_ERR_INVALID_ARG, "NULL argument");
    if (spin != 0 && spin != 1) return gfail(HUB_ERR_INVALID_ARG, "spin must be 0 (up) or 1 (down)");
    if (site < 0 || site >= src->M) return gfail(HUB_ERR_INVALID_ARG, "site out of range");
    HUB_TRY(check_pair(src, dst, spin, create != 0));
    const char *x = (const char *)dev_x, *y = (const char *)dev_y;
    const size_t bx = (size_t)src->dim * 8, by = (size_t)dst->dim * 8;
    if (x < y + by && y < x + bx) return gfail(HUB_ERR_INVALID_ARG, "x and y overlap");
    HUB_HIP(hipSetDevice(src->device));
    return apply_op(src, dst, site, spin, create != 0, (const double *)dev_x, (double *)dev_y, (hipStream_t)stream);
}

hub_status hub_lanczos_coefficients(const hub_sector *sec, const void *dev_f, int32_t max_steps, double *alpha,
                                    double *beta, double *norm2, int32_t *steps, void *stream)
{
    if (!sec || !dev_f || !alpha || !beta || !norm2 || !steps) return gfail(HUB_ERR_INVALID_ARG, "NULL argument");
    if (max_steps < 1) return gfail(HUB_ERR_INVALID_ARG, "max_steps must be positive");
    HUB_HIP(hipSetDevice(sec->device));
    return lanczos_coefficients(sec, (const double *)dev_f, max_steps, alpha, beta, norm2, steps,
                                (hipStream_t)stream);
}

hub_status hub_continued_fraction(const double *alpha, const double *beta, int32_t steps, double norm2, int32_t nz,
                                  const double *w_re, const double *w_im, double *out_re, double *out_im)
{
    if (steps < 0 || nz < 0) return gfail(HUB_ERR_INVALID_ARG, "negative size");
    if (nz > 0 && (!w_re || !w_im || !out_re || !out_im)) return gfail(HUB_ERR_INVALID_ARG, "NULL argument");
    if (steps > 0 && (!alpha || !beta)) return gfail(HUB_ERR_INVALID_ARG, "NULL coefficients");
    for (int i = 0; i < nz; ++i) {
        const std::complex<double> g = cfrac(alpha, beta, steps, norm2, {w_re[i], w_im[i]});
        out_re[i] = g.real();
        out_im[i] = g.imag();
    }
    return HUB_OK;
}

hub_status hub_greens_function(const hub_sector *sec, double e0, const void *dev_psi, int32_t site, int32_t spin,
                               int32_t max_steps, int32_t nz, const double *z_re, const double *z_im, double *g_re,
                               double *g_im, double *coef, hub_gf_info *info, void *stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!sec || !dev_psi) return gfail(HUB_ERR_INVALID_ARG, "NULL argument");
    if (sec->k0) return gfail(HUB_ERR_UNSUPPORTED, "not available for a translation (k = 0) sector");
    if (spin != 0 && spin != 1) return gfail(HUB_ERR_INVALID_ARG, "spin must be 0 (up) or 1 (down)");
    if (site < 0 || site >= sec->M) return gfail(HUB_ERR_INVALID_ARG, "site out of range");
    if (max_steps < 1) return gfail(HUB_ERR_INVALID_ARG, "max_steps must be positive");
    if (nz < 0 || (nz > 0 && (!z_re || !z_im || !g_re || !g_im))) return gfail(HUB_ERR_INVALID_ARG, "bad z arrays");
    HUB_HIP(hipSetDevice(sec->device));
    hipStream_t st = (hipStream_t)stream;
    const int L = max_steps + 1;
    std::vector<double> a[2], b[2];
    double nrm[2] = {0.0, 0.0};
    int32_t m[2] = {0, 0};
    for (int part = 0; part < 2; ++part) {  // 0: particle (c+), 1: hole (c)
        a[part].assign(L, 0.0);
        b[part].assign(L, 0.0);
        const int N = sec->spin[spin].N;
        if ((part == 0 && N >= sec->M) || (part == 1 && N <= 0)) continue;  // empty target sector
        SectorGuard g;
        HUB_TRY(shifted_sector(sec, spin, part == 0 ? 1 : -1, &g.s));
        DevBuf mem;
        double *f = nullptr;
        HUB_TRY(mem.alloc((void **)&f, sizeof(double) * (size_t)g.s->dim));
        HUB_TRY(apply_op(sec, g.s, site, spin, part == 0, (const double *)dev_psi, f, st));
        HUB_TRY(lanczos_coefficients(g.s, f, max_steps, a[part].data(), b[part].data(), &nrm[part], &m[part], st));
    }
    for (int i = 0; i < nz; ++i) {
        const std::complex<double> z(z_re[i], z_im[i]);
        const std::complex<double> gp = cfrac(a[0].data(), b[0].data(), m[0], nrm[0], z + e0);
        const std::complex<double> gh = cfrac(a[1].data(), b[1].data(), m[1], nrm[1], e0 - z);
        const std::complex<double> g = gp - gh;
        g_re[i] = g.real();
        g_im[i] = g.imag();
    }
    if (coef)
        for (int part = 0; part < 2; ++part) {
            std::memcpy(coef + (size_t)(2 * part) * L, a[part].data(), sizeof(double) * L);
            std::memcpy(coef + (size_t)(2 * part + 1) * L, b[part].data(), sizeof(double) * L);
        }
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->steps_particle = m[0];
        info->steps_hole = m[1];
        info->norm2_particle = nrm[0];
        info->norm2_hole = nrm[1];
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return HUB_OK;
}

}  // extern "C"
