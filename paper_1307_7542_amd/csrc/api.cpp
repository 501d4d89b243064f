// C ABI of libhubbard: argument validation, sector construction, host copies,
// and dispatch to the HIP kernels.  No entry point aborts or throws.
#include <cmath>
#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <utility>

#include "internal.h"

namespace hub {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

namespace {

hub_status fail(hub_status code, const std::string &msg)
{
    set_error(msg);
    return code;
}

bool finite_all(const double *p, int n)
{
    if (!p) return true;
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

void free_sector(hub_sector *s)
{
    if (!s) return;
    for (void *p : s->owned) (void)hipFree(p);
    s->owned.clear();
    delete s->k0;
    delete s;
}

template <typename T>
hub_status dalloc(hub_sector *s, T **p, size_t n)
{
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, (n == 0 ? 1 : n) * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(HUB_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    s->owned.push_back(q);
    *p = (T *)q;
    return HUB_OK;
}

hub_status check_sector(const hub_sector *s)
{
    if (!s) return fail(HUB_ERR_INVALID_ARG, "sector is NULL");
    HUB_HIP(hipSetDevice(s->device));
    return HUB_OK;
}

hub_status check_spin(int32_t spin)
{
    if (spin != HUB_SPIN_UP && spin != HUB_SPIN_DN) return fail(HUB_ERR_INVALID_ARG, "spin must be 0 (up) or 1 (down)");
    return HUB_OK;
}

hub_status check_dtype(int32_t dt)
{
    if (dt != HUB_F64 && dt != HUB_F32) return fail(HUB_ERR_INVALID_ARG, "dtype must be HUB_F64 or HUB_F32");
    return HUB_OK;
}

hub_status create(const hub_model *m, int32_t n_up, int32_t n_dn, hub_sector **out)
{
    if (!out) return fail(HUB_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!m) return fail(HUB_ERR_INVALID_ARG, "model is NULL");
    const int M = m->n_sites;
    if (M < 1 || M > kMaxSites) return fail(HUB_ERR_RANGE, "n_sites must be in 1..32");
    if (n_up < 0 || n_up > M || n_dn < 0 || n_dn > M) return fail(HUB_ERR_RANGE, "N_up and N_dn must be in 0..M");
    if (m->n_bonds < 0) return fail(HUB_ERR_INVALID_ARG, "n_bonds < 0");
    if (m->n_bonds > 0 && (!m->bond_i || !m->bond_j || !m->t))
        return fail(HUB_ERR_INVALID_ARG, "bond arrays are NULL");
    if (!finite_all(m->t, m->n_bonds) || !finite_all(m->U, M) || !finite_all(m->eps, M))
        return fail(HUB_ERR_INVALID_ARG, "non-finite t, U or eps");

    hub_sector *s = new (std::nothrow) hub_sector();
    if (!s) return fail(HUB_ERR_OOM, "host allocation failed");
    struct Guard {
        hub_sector *s;
        ~Guard() { free_sector(s); }
    } guard{s};

    s->M = M;
    // canonical bonds: (min, max), repeated pairs merged in input order
    std::map<std::pair<int, int>, int> where;
    for (int b = 0; b < m->n_bonds; ++b) {
        int i = m->bond_i[b], j = m->bond_j[b];
        if (i < 0 || i >= M || j < 0 || j >= M) return fail(HUB_ERR_INVALID_ARG, "bond endpoint out of range");
        if (i == j) return fail(HUB_ERR_INVALID_ARG, "bond with i == j");
        if (i > j) std::swap(i, j);
        auto it = where.find({i, j});
        if (it == where.end()) {
            where[{i, j}] = (int)s->bi.size();
            s->bi.push_back(i);
            s->bj.push_back(j);
            s->t.push_back(m->t[b]);
        } else {
            s->t[it->second] += m->t[b];
        }
    }
    s->nb = (int)s->bi.size();
    if (s->nb > kMaxBonds) return fail(HUB_ERR_RANGE, "more than 512 distinct bonds");
    s->U.assign(M, 0.0);
    s->eps.assign(M, 0.0);
    for (int i = 0; i < M; ++i) {
        if (m->U) s->U[i] = m->U[i];
        if (m->eps) s->eps[i] = m->eps[i];
    }
    s->uniformU = 1;
    s->U0 = s->U[0];
    s->umask = 0;
    for (int i = 0; i < M; ++i) {
        if (s->U[i] != s->U0) s->uniformU = 0;
        if (s->U[i] != 0.0) s->umask |= 1u << i;
    }

    HUB_HIP(hipGetDevice(&s->device));
    int lds = 0, ncu = 0;
    HUB_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, s->device));
    HUB_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, s->device));
    s->lds_max = (size_t)lds;
    s->cu_count = ncu;

    // binomial table C[n][k], n, k <= 32
    uint64_t C[kBinomN * kBinomN] = {};
    for (int nn = 0; nn < kBinomN; ++nn) {
        C[nn * kBinomN] = 1;
        for (int k = 1; k <= nn; ++k) C[nn * kBinomN + k] = C[(nn - 1) * kBinomN + k - 1] + C[(nn - 1) * kBinomN + k];
    }
    HUB_TRY(dalloc(s, &s->d_binom, kBinomN * kBinomN));
    HUB_TRY(dalloc(s, &s->d_bi, s->nb));
    HUB_TRY(dalloc(s, &s->d_bj, s->nb));
    HUB_TRY(dalloc(s, &s->d_t, s->nb));
    HUB_TRY(dalloc(s, &s->d_eps, M));
    HUB_TRY(dalloc(s, &s->d_U64, M));
    HUB_TRY(dalloc(s, &s->d_U32, M));
    std::vector<float> U32(M);
    for (int i = 0; i < M; ++i) U32[i] = (float)s->U[i];
    HUB_HIP(hipMemcpy(s->d_binom, C, sizeof(C), hipMemcpyHostToDevice));
    if (s->nb > 0) {
        HUB_HIP(hipMemcpy(s->d_bi, s->bi.data(), sizeof(int32_t) * s->nb, hipMemcpyHostToDevice));
        HUB_HIP(hipMemcpy(s->d_bj, s->bj.data(), sizeof(int32_t) * s->nb, hipMemcpyHostToDevice));
        HUB_HIP(hipMemcpy(s->d_t, s->t.data(), sizeof(double) * s->nb, hipMemcpyHostToDevice));
    }
    HUB_HIP(hipMemcpy(s->d_eps, s->eps.data(), sizeof(double) * M, hipMemcpyHostToDevice));
    HUB_HIP(hipMemcpy(s->d_U64, s->U.data(), sizeof(double) * M, hipMemcpyHostToDevice));
    HUB_HIP(hipMemcpy(s->d_U32, U32.data(), sizeof(float) * M, hipMemcpyHostToDevice));

    hipStream_t st = nullptr;
    HUB_TRY(build_spin_tables(s, HUB_SPIN_UP, n_up, st));
    if (n_dn == n_up) {
        s->shared_spin = true;
        s->spin[1] = s->spin[0];
    } else {
        HUB_TRY(build_spin_tables(s, HUB_SPIN_DN, n_dn, st));
    }
    const int64_t cu = s->spin[0].count, cd = s->spin[1].count;
    if (cu > INT32_MAX || cd > INT32_MAX) return fail(HUB_ERR_RANGE, "one-spin dimension exceeds 2^31");
    s->dim = cu * cd;
    HUB_HIP(hipDeviceSynchronize());
    guard.s = nullptr;
    *out = s;
    return HUB_OK;
}

}  // namespace
}  // namespace hub

using namespace hub;

extern "C" {

hub_status hub_sector_create(const hub_model *model, int32_t n_up, int32_t n_dn, hub_sector **out)
{
    return create(model, n_up, n_dn, out);
}

void hub_sector_destroy(hub_sector *sec)
{
    if (!sec) return;
    (void)hipSetDevice(sec->device);
    free_sector(sec);
}

hub_status hub_sector_dims(const hub_sector *sec, int64_t *count_up, int64_t *count_dn, int64_t *dim)
{
    if (!sec) return fail(HUB_ERR_INVALID_ARG, "sector is NULL");
    if (count_up) *count_up = sec->spin[0].count;
    if (count_dn) *count_dn = sec->spin[1].count;
    if (dim) *dim = sec->dim;
    return HUB_OK;
}

hub_status hub_sector_bonds(const hub_sector *sec, int32_t *n_bonds, int32_t *bond_i, int32_t *bond_j, double *t)
{
    if (!sec) return fail(HUB_ERR_INVALID_ARG, "sector is NULL");
    if (n_bonds) *n_bonds = sec->nb;
    for (int b = 0; b < sec->nb; ++b) {
        if (bond_i) bond_i[b] = sec->bi[b];
        if (bond_j) bond_j[b] = sec->bj[b];
        if (t) t[b] = sec->t[b];
    }
    return HUB_OK;
}

hub_status hub_basis(const hub_sector *sec, int32_t spin, uint64_t *host_out)
{
    HUB_TRY(check_sector(sec));
    HUB_TRY(check_spin(spin));
    if (!host_out) return fail(HUB_ERR_INVALID_ARG, "host_out is NULL");
    const SpinTables &T = sec->spin[spin];
    std::vector<uint32_t> tmp((size_t)T.count);
    HUB_HIP(hipMemcpy(tmp.data(), T.basis, sizeof(uint32_t) * T.count, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < T.count; ++i) host_out[i] = tmp[i];
    return HUB_OK;
}

hub_status hub_rank(const hub_sector *sec, int32_t spin, const uint64_t *host_x, int64_t n, int64_t *host_out)
{
    HUB_TRY(check_sector(sec));
    HUB_TRY(check_spin(spin));
    if (n < 0) return fail(HUB_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return HUB_OK;
    if (!host_x || !host_out) return fail(HUB_ERR_INVALID_ARG, "NULL array");
    void *dx = nullptr, *dout = nullptr;
    hipError_t e1 = hipMalloc(&dx, sizeof(uint64_t) * n);
    hipError_t e2 = hipMalloc(&dout, sizeof(int64_t) * n);
    hub_status st = HUB_OK;
    if (e1 != hipSuccess || e2 != hipSuccess) {
        (void)hipGetLastError();
        st = fail(HUB_ERR_OOM, "hipMalloc failed in hub_rank");
    }
    if (st == HUB_OK && hipMemcpy(dx, host_x, sizeof(uint64_t) * n, hipMemcpyHostToDevice) != hipSuccess)
        st = fail(HUB_ERR_DEVICE, "copy to device failed");
    if (st == HUB_OK) st = rank_device(sec, spin, (const uint64_t *)dx, n, (int64_t *)dout, nullptr);
    if (st == HUB_OK && hipMemcpy(host_out, dout, sizeof(int64_t) * n, hipMemcpyDeviceToHost) != hipSuccess)
        st = fail(HUB_ERR_DEVICE, "copy to host failed");
    if (dx) (void)hipFree(dx);
    if (dout) (void)hipFree(dout);
    return st;
}

hub_status hub_hopping_nnz(const hub_sector *sec, int32_t spin, int64_t *nnz)
{
    if (!sec) return fail(HUB_ERR_INVALID_ARG, "sector is NULL");
    HUB_TRY(check_spin(spin));
    if (!nnz) return fail(HUB_ERR_INVALID_ARG, "nnz is NULL");
    *nnz = sec->spin[spin].nnz;
    return HUB_OK;
}

hub_status hub_hopping_csr(const hub_sector *sec, int32_t spin, int64_t *row_ptr, int32_t *col, double *val,
                           int32_t *bond_id)
{
    HUB_TRY(check_sector(sec));
    HUB_TRY(check_spin(spin));
    const SpinTables &T = sec->spin[spin];
    if (row_ptr) {
        std::vector<int32_t> rp((size_t)T.count + 1);
        HUB_HIP(hipMemcpy(rp.data(), T.rp, sizeof(int32_t) * (T.count + 1), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i <= T.count; ++i) row_ptr[i] = rp[i];
    }
    if (T.nnz > 0) {
        if (col) HUB_HIP(hipMemcpy(col, T.col, sizeof(int32_t) * T.nnz, hipMemcpyDeviceToHost));
        if (val) HUB_HIP(hipMemcpy(val, T.val64, sizeof(double) * T.nnz, hipMemcpyDeviceToHost));
        if (bond_id) HUB_HIP(hipMemcpy(bond_id, T.bond, sizeof(int32_t) * T.nnz, hipMemcpyDeviceToHost));
    }
    return HUB_OK;
}

hub_status hub_diagonal(const hub_sector *sec, int32_t dtype, void *dev_out, void *stream)
{
    HUB_TRY(check_sector(sec));
    HUB_TRY(check_dtype(dtype));
    if (!dev_out) return fail(HUB_ERR_INVALID_ARG, "dev_out is NULL");
    if (sec->k0) return fail(HUB_ERR_UNSUPPORTED, "not available for a translation (k = 0) sector");
    return launch_diagonal(sec, dtype, dev_out, (hipStream_t)stream);
}

hub_status hub_start_vector(const hub_sector *sec, int32_t dtype, uint64_t seed, int32_t normalize, void *dev_out,
                            void *stream)
{
    HUB_TRY(check_sector(sec));
    HUB_TRY(check_dtype(dtype));
    if (!dev_out) return fail(HUB_ERR_INVALID_ARG, "dev_out is NULL");
    hipStream_t st = (hipStream_t)stream;
    HUB_TRY(launch_start_vector(HUB_F64 == dtype ? HUB_F64 : HUB_F32, seed, dev_out, sec->dim, st));
    HUB_TRY(k0_project(sec, dtype, dev_out, st));
    if (normalize) {
        double *tmp = nullptr;
        const size_t nb = sizeof(double) * (kRedGrid + 4);
        HUB_HIP(hipMalloc((void **)&tmp, nb));
        hub_status r = launch_dot(dtype, dev_out, dev_out, sec->dim, tmp + 4, tmp, 1, st);
        if (r == HUB_OK) r = launch_convert(dtype, dev_out, dtype, dev_out, sec->dim, tmp, 1, st);
        if (r == HUB_OK && hipStreamSynchronize(st) != hipSuccess) r = fail(HUB_ERR_DEVICE, "synchronize failed");
        (void)hipFree(tmp);
        return r;
    }
    return HUB_OK;
}

hub_status hub_start_vector_noalloc(const hub_sector *sec, int32_t dtype, uint64_t seed, int32_t normalize,
                                    void *dev_out, void *stream)
{
    HUB_TRY(check_sector(sec));
    HUB_TRY(check_dtype(dtype));
    if (!dev_out) return fail(HUB_ERR_INVALID_ARG, "dev_out is NULL");
    return start_vector_noalloc(sec, dtype, seed, normalize, dev_out, (hipStream_t)stream);
}

hub_status hub_matvec(const hub_sector *sec, int32_t dtype, const void *dev_x, void *dev_y, void *stream)
{
    HUB_TRY(check_sector(sec));
    HUB_TRY(check_dtype(dtype));
    if (!dev_x || !dev_y) return fail(HUB_ERR_INVALID_ARG, "NULL vector");
    const size_t bytes = (size_t)sec->dim * (dtype == HUB_F64 ? 8 : 4);
    const char *x = (const char *)dev_x, *y = (const char *)dev_y;
    if (x < y + bytes && y < x + bytes) return fail(HUB_ERR_INVALID_ARG, "x and y overlap");
    const uintptr_t es = (dtype == HUB_F64) ? 8 : 4;
    if (((uintptr_t)x | (uintptr_t)y) % es) return fail(HUB_ERR_INVALID_ARG, "x or y not aligned to its element");
    return apply_h(sec, dtype, dev_x, dev_y, (hipStream_t)stream);
}

hub_status hub_set_schedule(hub_sector *sec, int32_t dtype, const hub_schedule *sched)
{
    HUB_TRY(check_sector(sec));
    HUB_TRY(check_dtype(dtype));
    if (sec->k0) return fail(HUB_ERR_UNSUPPORTED, "k = 0 sectors have a product of their own");
    HUB_HIP(hipSetDevice(sec->device));
    return set_schedule(sec, dtype, sched);
}

hub_status hub_get_schedule(const hub_sector *sec, int32_t dtype, int32_t fused, hub_schedule *out)
{
    HUB_TRY(check_sector(sec));
    HUB_TRY(check_dtype(dtype));
    if (!out) return fail(HUB_ERR_INVALID_ARG, "out is NULL");
    return get_schedule(sec, dtype, fused, out);
}

hub_status hub_gram(int32_t dtype, const void *const *dev_q, int32_t m, int64_t n, double *host_g, void *stream)
{
    HUB_TRY(check_dtype(dtype));
    if (m < 0 || n < 0) return fail(HUB_ERR_INVALID_ARG, "negative size");
    if (m == 0) return HUB_OK;
    if (!dev_q || !host_g) return fail(HUB_ERR_INVALID_ARG, "NULL argument");
    for (int i = 0; i < m; ++i)
        if (!dev_q[i]) return fail(HUB_ERR_INVALID_ARG, "NULL vector pointer");
    hipStream_t st = (hipStream_t)stream;
    const int ld = 16 * ((m + 15) / 16);
    void **dq = nullptr;
    double *dG = nullptr;
    struct Free {
        void *a = nullptr, *b = nullptr;
        ~Free()
        {
            (void)hipFree(a);
            (void)hipFree(b);
        }
    } fr;
    HUB_HIP(hipMalloc((void **)&dq, sizeof(void *) * (size_t)m));
    fr.a = dq;
    HUB_HIP(hipMalloc((void **)&dG, sizeof(double) * (size_t)ld * ld));
    fr.b = dG;
    HUB_HIP(hipMemcpyAsync(dq, dev_q, sizeof(void *) * (size_t)m, hipMemcpyHostToDevice, st));
    HUB_TRY(gram_mfma(dtype, (const void *const *)dq, m, n, dG, ld, st));
    std::vector<double> G((size_t)ld * ld);
    HUB_HIP(hipMemcpy(G.data(), dG, sizeof(double) * G.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) host_g[(size_t)i * m + j] = G[(size_t)i * ld + j];
    return HUB_OK;
}

hub_status hub_matvec_bytes(const hub_sector *sec, int32_t dtype, int64_t *bytes)
{
    if (!sec) return fail(HUB_ERR_INVALID_ARG, "sector is NULL");
    HUB_TRY(check_dtype(dtype));
    if (!bytes) return fail(HUB_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = matvec_bytes(sec, dtype);
    return HUB_OK;
}

hub_status hub_ground_state(const hub_sector *sec, const hub_lanczos_opts *opts, double *e0, void *dev_psi,
                            void *stream, hub_lanczos_info *info)
{
    HUB_TRY(check_sector(sec));
    if (!opts) return fail(HUB_ERR_INVALID_ARG, "opts is NULL");
    HUB_TRY(check_dtype(opts->vec_dtype));
    if (opts->reorth < 0 || opts->reorth > 2) return fail(HUB_ERR_INVALID_ARG, "reorth must be 0, 1 or 2");
    if (dev_psi && !(opts->want_vector || opts->refine))
        return fail(HUB_ERR_INVALID_ARG, "dev_psi given but want_vector is 0");
    return ground_state(sec, opts, e0, dev_psi, (hipStream_t)stream, info);
}

hub_status hub_param_bilinear(const hub_sector *sec, const void *dev_g, const void *dev_x, double *dbond, double *dU,
                              double *deps, void *stream)
{
    HUB_TRY(check_sector(sec));
    if (!dev_g || !dev_x) return fail(HUB_ERR_INVALID_ARG, "NULL vector");
    if (sec->k0) return fail(HUB_ERR_UNSUPPORTED, "not available for a translation (k = 0) sector");
    return param_bilinear(sec, (const double *)dev_g, (const double *)dev_x, dbond, dU, deps, (hipStream_t)stream);
}

const char *hub_status_str(hub_status s)
{
    switch (s) {
    case HUB_OK: return "HUB_OK";
    case HUB_ERR_INVALID_ARG: return "HUB_ERR_INVALID_ARG";
    case HUB_ERR_RANGE: return "HUB_ERR_RANGE";
    case HUB_ERR_OOM: return "HUB_ERR_OOM";
    case HUB_ERR_DEVICE: return "HUB_ERR_DEVICE";
    case HUB_ERR_NOT_CONVERGED: return "HUB_ERR_NOT_CONVERGED";
    case HUB_ERR_UNSUPPORTED: return "HUB_ERR_UNSUPPORTED";
    default: return "HUB_ERR_UNKNOWN";
    }
}

const char *hub_last_error(void) { return g_last_error.c_str(); }

const char *hub_version(void) { return "libhubbard 0.1 (gfx950)"; }

}  // extern "C"
