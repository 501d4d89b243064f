// Host driver of the Lanczos ground-state solve (Sec. IV).  The product and all
// vector work run in the HIP kernels of matvec.hip / vec.hip on the caller's
// stream; alpha and beta are formed on the device and reach the host either
// through pinned memory that the step's last kernel writes (plain recurrence)
// or by a copy at the convergence test (full reorthogonalisation, k = 0
// reprojection); the test runs while the GPU computes the next step.  The small
// tridiagonal eigenproblem is solved on the host: the lowest eigenvalue by
// bisection on the Sturm sequence count, its eigenvector by inverse iteration
// with a partially pivoted tridiagonal LU.
#include <algorithm>
#include <chrono>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace hub {
namespace {

// Up to this many per-column partials of alpha, every block of the update
// kernel sums them itself (the 4x4 torus: 11440, a few microseconds per
// launch) instead of a separate single-block launch.
constexpr int64_t kSumInUpdate = 65536;

// Number of eigenvalues of T (diag a, off-diagonal b) smaller than x.
int sturm_count(const double *a, const double *b, int m, double x, double pivmin)
{
    int cnt = 0;
    double q = a[0] - x;
    if (std::fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
    for (int i = 1; i < m; ++i) {
        q = (a[i] - x) - b[i - 1] * b[i - 1] / q;
        if (std::fabs(q) < pivmin) q = -pivmin;
        if (q < 0) ++cnt;
    }
    return cnt;
}

}  // namespace

// Lowest eigenpair of the m x m symmetric tridiagonal matrix; y has unit norm.
double tri_lowest(const double *a, const double *b, int m, std::vector<double> &y)
{
    y.assign(m, 0.0);
    if (m == 1) {
        y[0] = 1.0;
        return a[0];
    }
    double tnorm = 0.0, bmax2 = 0.0;
    double lo = a[0], hi = a[0];
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
        tnorm = std::max(tnorm, std::fabs(a[i]) + r);
        if (i < m - 1) bmax2 = std::max(bmax2, b[i] * b[i]);
    }
    const double pivmin = DBL_MIN * std::max(1.0, bmax2);
    lo -= 2.0 * DBL_EPSILON * tnorm + pivmin;
    hi += 2.0 * DBL_EPSILON * tnorm + pivmin;
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (hi - lo <= 2.0 * DBL_EPSILON * std::max(std::fabs(lo), std::fabs(hi)) + pivmin) break;
        if (sturm_count(a, b, m, mid, pivmin) >= 1) hi = mid;
        else lo = mid;
    }
    const double theta = 0.5 * (lo + hi);

    // Inverse iteration: (T - theta I) z = r with partial pivoting.
    std::vector<double> U0(m), U1(m), U2(m), L(m), r(m, 1.0);
    std::vector<char> sw(m, 0);
    const double tiny = DBL_EPSILON * std::max(tnorm, DBL_MIN);
    double c0 = a[0] - theta, c1 = b[0], c2 = 0.0;
    for (int i = 0; i < m - 1; ++i) {
        const double n0 = b[i], n1 = a[i + 1] - theta, n2 = (i + 1 < m - 1) ? b[i + 1] : 0.0;
        double p0, p1, p2, o0, o1, o2;
        if (std::fabs(n0) > std::fabs(c0)) {
            sw[i] = 1;
            p0 = n0; p1 = n1; p2 = n2;
            o0 = c0; o1 = c1; o2 = c2;
        } else {
            sw[i] = 0;
            p0 = c0; p1 = c1; p2 = c2;
            o0 = n0; o1 = n1; o2 = n2;
        }
        if (p0 == 0.0) p0 = tiny;
        const double f = o0 / p0;
        L[i] = f;
        U0[i] = p0; U1[i] = p1; U2[i] = p2;
        c0 = o1 - f * p1;
        c1 = o2 - f * p2;
        c2 = 0.0;
    }
    U0[m - 1] = (c0 == 0.0) ? tiny : c0;
    U1[m - 1] = 0.0;
    U2[m - 1] = 0.0;
    std::vector<double> z(m);
    for (int pass = 0; pass < 3; ++pass) {
        for (int i = 0; i < m - 1; ++i) {
            if (sw[i]) std::swap(r[i], r[i + 1]);
            r[i + 1] -= L[i] * r[i];
        }
        for (int i = m - 1; i >= 0; --i) {
            double s = r[i];
            if (i + 1 < m) s -= U1[i] * z[i + 1];
            if (i + 2 < m) s -= U2[i] * z[i + 2];
            z[i] = s / U0[i];
        }
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm += z[i] * z[i];
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0) || !std::isfinite(nrm)) {
            for (int i = 0; i < m; ++i) z[i] = (i == 0) ? 1.0 : 0.0;
            nrm = 1.0;
        }
        for (int i = 0; i < m; ++i) r[i] = z[i] / nrm;
    }
    y = r;
    return theta;
}

namespace {

struct DevMem {
    std::vector<void *> ptrs;
    ~DevMem()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
    hub_status alloc(void **p, size_t bytes)
    {
        hipError_t e = hipMalloc(p, bytes == 0 ? 1 : bytes);
        if (e != hipSuccess) {
            set_error(std::string("workspace hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
            (void)hipGetLastError();
            return HUB_ERR_OOM;
        }
        ptrs.push_back(*p);
        return HUB_OK;
    }
};

// HIP events around sampled product launches: every `every`-th product when
// on (an event record between two kernels delays the second by a few
// microseconds, so timing every launch of a short product slows the solve).
struct EventTimer {
    bool on = false;
    int every = 1;
    int seen = 0;
    int timed = 0;
    hipStream_t st = nullptr;
    std::vector<hipEvent_t> ev;
    int used = 0;
    bool sample()
    {
        if (!on) return false;
        const bool t = (seen++ % every) == 0;
        if (t) ++timed;
        return t;
    }
    ~EventTimer()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    hub_status mark()
    {
        if (!on) return HUB_OK;
        if (used == (int)ev.size()) {
            hipEvent_t e;
            HUB_HIP(hipEventCreate(&e));
            ev.push_back(e);
        }
        HUB_HIP(hipEventRecord(ev[used++], st));
        return HUB_OK;
    }
    double total_ms()
    {
        double t = 0.0;
        for (int i = 0; i + 1 < used; i += 2) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) t += ms;
        }
        return t;
    }
};

using clk = std::chrono::steady_clock;

}  // namespace

hub_status ground_state(const hub_sector *s, const hub_lanczos_opts *o, double *e0_out, void *dev_psi,
                        hipStream_t st, hub_lanczos_info *info)
{
    const auto t0 = clk::now();
    const int dt = o->vec_dtype;
    const size_t es = (dt == HUB_F64) ? 8 : 4;
    const int64_t n = s->dim;
    int max_iter = o->max_iter > 0 ? o->max_iter : 400;
    if ((int64_t)max_iter > n) max_iter = (int)n;
    const double tol = o->tol > 0 ? o->tol : (dt == HUB_F64 ? 1e-12 : 1e-7);
    const int check_every = o->check_every > 0 ? o->check_every : 1;
    const bool reorth = o->reorth != 0;          // the Lanczos vectors are stored
    const bool partial_ro = o->reorth == 2;      // Gram-Schmidt only where the omega estimate asks for it
    const bool want_vec = o->want_vector != 0 || o->refine != 0;
    // k = 0 sectors with short-period rows: the vectors live in the consistent
    // subspace; rounding noise outside it is removed from every new vector (the
    // discarded directions carry eigenvalue 0, which may lie below the k = 0 block)
    const bool reproject = s->k0 && s->k0->n_short > 0;

    hub_lanczos_info inf;
    std::memset(&inf, 0, sizeof(inf));
    inf.true_residual = -1.0;
    inf.iters_to_target = -1;
    inf.seconds_to_target = -1.0;
    const bool want_target = o->e0_target_rel > 0.0;
    inf.matvec_bytes = matvec_bytes(s, dt);

    DevMem mem;
    EventTimer tm;
    tm.on = o->time_kernels > 0;
    tm.every = std::max(1, o->time_kernels);
    tm.st = st;

    const int kmax = max_iter + 1;
    // Refuse before allocating anything when the vectors cannot fit in the free
    // device memory: three (plain recurrence) or up to max_iter + 1 stored
    // Lanczos vectors plus the update's (full reorthogonalisation), an FP64 psi
    // when the caller passes none, the refinement's FP64 H psi, and the fused
    // product's partials.
    {
        size_t free_b = 0, total_b = 0;
        HUB_HIP(hipMemGetInfo(&free_b, &total_b));
        const double vec = (double)es * (double)n;
        double need = vec * (reorth ? (double)kmax + 1.0 : 3.0);
        if (want_vec && !dev_psi) need += 8.0 * (double)n;
        if (o->refine) need += 8.0 * (double)n;
        if (matvec_lz_available(s, dt)) need += 8.0 * (double)matvec_lz_workspace(s);
        if (need > (double)free_b) {
            set_error("Lanczos workspace of " + std::to_string(need / 1e9) + " GB exceeds the " +
                      std::to_string((double)free_b / 1e9) + " GB of free device memory" +
                      (reorth ? " (full reorthogonalisation stores up to max_iter + 1 vectors)" : ""));
            return HUB_ERR_OOM;
        }
    }
    double *dscal = nullptr;  // alpha[kmax] beta[kmax+1] misc[16] ycoef[kmax]
    HUB_TRY(mem.alloc((void **)&dscal, sizeof(double) * (size_t)(3 * kmax + 32)));
    double *d_alpha = dscal, *d_beta = dscal + kmax, *d_misc = dscal + 2 * kmax + 1,
           *d_y = dscal + 2 * kmax + 17;
    HUB_HIP(hipMemsetAsync(dscal, 0, sizeof(double) * (size_t)(3 * kmax + 32), st));
    double *partial = nullptr;
    const size_t npart = (size_t)kRedGrid * (size_t)std::max(kmax, 2) + 2 * (size_t)kRedGrid;
    HUB_TRY(mem.alloc((void **)&partial, sizeof(double) * npart));
    void **dQ = nullptr;  // device array of vector pointers
    HUB_TRY(mem.alloc((void **)&dQ, sizeof(void *) * (size_t)kmax));
    double *d_coef = nullptr;  // Gram coefficients against the stored vectors
    HUB_TRY(mem.alloc((void **)&d_coef, sizeof(double) * (size_t)kmax));
    int *d_flag = nullptr;  // skip flag of the second Gram-Schmidt pass; [4..8): partial reorthogonalisation state
    HUB_TRY(mem.alloc((void **)&d_flag, sizeof(int) * 8));
    HUB_HIP(hipMemsetAsync(d_flag, 0, sizeof(int) * 8, st));
    int *d_pro = d_flag + 4;
    double *om[3] = {nullptr, nullptr, nullptr};  // omega_{k-1}, omega_k, omega_{k+1}
    if (partial_ro) {
        double *omb = nullptr;
        HUB_TRY(mem.alloc((void **)&omb, sizeof(double) * 3 * (size_t)(kmax + 2)));
        HUB_HIP(hipMemsetAsync(omb, 0, sizeof(double) * 3 * (size_t)(kmax + 2), st));
        const double one = 1.0;
        for (int i = 0; i < 3; ++i) om[i] = omb + (size_t)i * (kmax + 2);
        HUB_HIP(hipMemcpyAsync(om[1], &one, sizeof(double), hipMemcpyHostToDevice, st));  // omega_{0,0} = 1
        HUB_HIP(hipStreamSynchronize(st));
    }
    // unit roundoff of the stored vectors
    const double eps_store = (dt == HUB_F64) ? DBL_EPSILON / 2 : FLT_EPSILON / 2;

    void *W = nullptr, *Va = nullptr, *Vb = nullptr;
    HUB_TRY(mem.alloc(&W, es * (size_t)n));
    std::vector<void *> Q;  // reorth: every Lanczos vector (append-only, never reallocated)
    Q.reserve((size_t)kmax);
    auto new_q = [&](void **p) -> hub_status {
        HUB_TRY(mem.alloc(p, es * (size_t)n));
        Q.push_back(*p);
        return HUB_OK;
    };
    double *wpart = nullptr;  // reorth: partials of ||w||^2 left by the Gram update
    if (reorth) {
        HUB_TRY(new_q(&Va));
        HUB_TRY(mem.alloc((void **)&wpart, sizeof(double) * (size_t)gram_norm_parts(n)));
    } else {
        HUB_TRY(mem.alloc(&Va, es * (size_t)n));
        HUB_TRY(mem.alloc(&Vb, es * (size_t)n));
    }

    // start vector v0 = x / ||x|| in storage precision
    auto make_start = [&](void *v) -> hub_status {
        if (o->dev_start) {
            HUB_TRY(launch_dot(HUB_F64, o->dev_start, o->dev_start, n, partial, d_misc, 1, st));
            HUB_TRY(launch_convert(HUB_F64, o->dev_start, dt, v, n, d_misc, 1, st));
        } else {
            HUB_TRY(launch_start_vector(dt, o->seed, W, n, st));
            HUB_TRY(k0_project(s, dt, W, st));
            HUB_TRY(launch_dot(dt, W, W, n, partial, d_misc, 1, st));
            HUB_TRY(launch_convert(dt, W, dt, v, n, d_misc, 1, st));
        }
        return HUB_OK;
    };
    auto product = [&](const void *x, void *y) -> hub_status {
        const bool timed = tm.sample();
        if (timed) HUB_TRY(tm.mark());
        HUB_TRY(apply_h(s, dt, x, y, st));
        if (timed) HUB_TRY(tm.mark());
        inf.matvec_count++;
        return HUB_OK;
    };
    // y = H x - beta v_prev and alpha = <y, x>: one fused launch (plus a fixed-order
    // sum of its partials) where the product kernel supports it, else product + update
    const bool fused = matvec_lz_available(s, dt);
    double *apart = nullptr;
    if (fused) HUB_TRY(mem.alloc((void **)&apart, sizeof(double) * (size_t)matvec_lz_workspace(s)));
    if (fused) inf.matvec_bytes += (int64_t)es * n;  // the update's read of v_prev
    // fused: alpha's per-column partials are left in apart[0 .. np_alpha) and
    // summed by the w -= alpha v update (lz_b below); otherwise alpha goes to aout
    int64_t np_alpha = 0;
    auto product_lz = [&](const void *x, void *y, const void *vp, const double *bk, double *aout,
                          const double *bprev = nullptr, int un = 0) -> hub_status {
        if (fused) {
            const bool timed = tm.sample();
            if (timed) HUB_TRY(tm.mark());
            HUB_TRY(launch_matvec_lz(s, dt, x, y, vp, bk, apart, &np_alpha, st, bprev, un));
            if (timed) HUB_TRY(tm.mark());
            inf.matvec_count++;
            return HUB_OK;
        }
        HUB_TRY(product(x, y));
        if (!aout) return launch_lz_a(dt, y, vp, bk, x, n, partial, nullptr, st);
        // partials of alpha beside the ones the update writes; summed inside it
        np_alpha = red_grid(n);
        return launch_lz_a(dt, y, vp, bk, x, n, partial + kRedGrid, nullptr, st);
    };
    // W -= alpha_k v with alpha_k written to *alpha_io (fused: formed from the
    // product's partials, inside the update when they are few); beta^2 partials
    // left in partial[0 .. red_grid(n)), their square-rooted sum in *beta_out if given
    auto lz_b = [&](const void *vv, double *alpha_io, double *beta_out) -> hub_status {
        if (fused && np_alpha <= kSumInUpdate) {
            HUB_TRY(launch_lz_b_sum(dt, W, vv, apart, np_alpha, alpha_io, n, partial, st));
            if (beta_out) HUB_TRY(launch_sum(partial, red_grid(n), beta_out, st, 1));
            return HUB_OK;
        }
        if (!fused) {
            HUB_TRY(launch_lz_b_sum(dt, W, vv, partial + kRedGrid, np_alpha, alpha_io, n, partial, st));
            if (beta_out) HUB_TRY(launch_sum(partial, red_grid(n), beta_out, st, 1));
            return HUB_OK;
        }
        HUB_TRY(launch_sum(apart, np_alpha, alpha_io, st));
        return launch_lz_b(dt, W, vv, alpha_io, n, partial, beta_out, st);
    };

    HUB_TRY(make_start(Va));
    void *v_prev = nullptr, *v = Va, *spare = Vb;
    void *const B0 = Va, *const B1 = Vb, *const B2 = W;  // the three vector buffers

    // Convergence checks run on the host while the GPU computes the next step:
    // at a check step k, alpha_0..alpha_{k-1} and beta_1..beta_k are copied (one
    // asynchronous copy into pinned memory) before step k is enqueued, and the
    // host waits only for that copy.  A step finished after convergence is
    // discarded (its coefficients are never used).
    //
    // On the plain path (no reorthogonalisation, no reprojection) the
    // normalisation kernel of step j itself stores alpha_j and beta_{j+1} into
    // the pinned buffer and then publishes j + 1 in a pinned counter, so a check
    // waits on host memory only: no copy and no event between the kernels.
    double *hpin = nullptr;  // pinned copy of dscal[0 .. 2 kmax + 1)
    int *hflag = nullptr;    // pinned count of published steps
    HUB_HIP(hipHostMalloc((void **)&hpin, sizeof(double) * (size_t)(2 * kmax + 1),
                          hipHostMallocMapped | hipHostMallocCoherent));
    // (kernels still queued on an early error return may write here: drain the stream first)
    struct PinGuard {
        void *p;
        hipStream_t st;
        ~PinGuard()
        {
            if (!p) return;
            (void)hipStreamSynchronize(st);
            (void)hipHostFree(p);
        }
    } pin_guard{hpin, st}, flag_guard{nullptr, st};
    HUB_HIP(hipHostMalloc((void **)&hflag, 64, hipHostMallocMapped | hipHostMallocCoherent));
    flag_guard.p = hflag;
    std::memset(hpin, 0, sizeof(double) * (size_t)(2 * kmax + 1));
    __atomic_store_n(hflag, 0, __ATOMIC_RELEASE);
    double *dpin = nullptr;
    int *dflag = nullptr;
    HUB_HIP(hipHostGetDevicePointer((void **)&dpin, hpin, 0));
    HUB_HIP(hipHostGetDevicePointer((void **)&dflag, hflag, 0));
    const bool publish = !reorth && !reproject;
    // Plain fused path: the vectors stay unnormalised, u_k = beta_k v_k (u_0 = v_0).
    // The product's epilogue and the update scale by 1 / beta_k in FP64, so no
    // normalisation pass is needed; a step is the fused product, the update and a
    // one-block kernel that forms and publishes beta_{k+1}.
    const bool unnorm = fused && publish && matvec_lz_partials(s) <= kSumInUpdate;
    const double *ha = hpin, *hb = hpin + kmax;
    hipEvent_t copied;
    HUB_HIP(hipEventCreateWithFlags(&copied, hipEventDisableTiming));
    struct EvGuard {
        hipEvent_t e;
        ~EvGuard() { (void)hipEventDestroy(e); }
    } ev_guard{copied};
    std::vector<double> y;
    int m_final = 0;
    double theta = 0.0, res = 0.0;
    bool converged = false, breakdown = false;
    double t_e0 = -1.0;
    double tmax = 0.0;

    // m steps done: test the Ritz residual of T_m (host arrays ha, hb)
    auto check = [&](int m) -> bool {
        int mm = m;
        for (int j = 0; j < m; ++j) {
            tmax = std::max(tmax, std::fabs(ha[j]) + 2.0 * std::fabs(hb[j + 1]));
            const double thr = 64.0 * ((dt == HUB_F64) ? DBL_EPSILON : FLT_EPSILON) * std::max(tmax, DBL_MIN);
            if (!(hb[j + 1] > thr)) {
                mm = j + 1;
                breakdown = true;
                break;
            }
        }
        theta = tri_lowest(ha, hb + 1, mm, y);
        res = std::fabs(hb[mm]) * std::fabs(y[mm - 1]);
        if (want_target && inf.iters_to_target < 0 &&
            std::fabs(theta - o->e0_target) <= o->e0_target_rel * std::fabs(o->e0_target)) {
            inf.iters_to_target = mm;
            inf.seconds_to_target = std::chrono::duration<double>(clk::now() - t0).count();
        }
        const double scale = std::fabs(theta) > 0 ? std::fabs(theta) : 1.0;
        m_final = mm;
        if (breakdown || res <= tol * scale) {
            converged = true;
            if (breakdown) res = 0.0;
            t_e0 = std::chrono::duration<double>(clk::now() - t0).count();
            return true;
        }
        return false;
    };
    auto fetch = [&](int k) -> hub_status {  // alpha_0..alpha_{k-1}, beta_0..beta_k
        HUB_HIP(hipMemcpyAsync(hpin, dscal, sizeof(double) * (size_t)(kmax + k + 1), hipMemcpyDeviceToHost, st));
        HUB_HIP(hipEventRecord(copied, st));
        return HUB_OK;
    };
    // publish mode: wait until steps 0 .. k-1 are published (a stream
    // synchronisation after half a second of spinning surfaces device errors)
    auto wait_published = [&](int k) -> hub_status {
        const auto tw = clk::now();
        unsigned spins = 0;
        while (__atomic_load_n(hflag, __ATOMIC_ACQUIRE) < k) {
            if ((++spins & 1023u) == 0 && clk::now() - tw > std::chrono::milliseconds(500)) {
                HUB_HIP(hipStreamSynchronize(st));
                if (__atomic_load_n(hflag, __ATOMIC_ACQUIRE) < k) {
                    set_error("Lanczos: a step's coefficients were not published");
                    return HUB_ERR_DEVICE;
                }
                break;
            }
            __builtin_ia32_pause();
        }
        return HUB_OK;
    };
    for (int k = 0; unnorm && k < max_iter; ++k) {
        const bool check_now = k >= 1 && (k % check_every) == 0;
        const double *bk = k >= 1 ? d_beta + k : nullptr, *bprev = k >= 2 ? d_beta + k - 1 : nullptr;
        HUB_TRY(product_lz(v, W, v_prev, bk, nullptr, bprev, 1));
        HUB_TRY(launch_lz_b_sum(dt, W, v, apart, np_alpha, d_alpha + k, n, partial, st, bk, 1));
        if (check_now) {
            HUB_TRY(wait_published(k));  // step k keeps running meanwhile
            if (check(k)) break;
        }
        if (k + 1 == max_iter) {
            HUB_TRY(launch_sum(partial, red_grid(n), d_beta + k + 1, st, 1));
            HUB_TRY(fetch(k + 1));
            HUB_HIP(hipEventSynchronize(copied));
            check(k + 1);
            break;
        }
        HUB_TRY(launch_beta_pub(partial, n, d_beta + k + 1, st, dpin, dflag, d_alpha + k, k, kmax));
        // W now holds u_{k+1}; the oldest buffer becomes the next output
        void *freed = v_prev ? v_prev : spare;
        if (!v_prev) spare = nullptr;
        v_prev = v;
        v = W;
        W = freed;
    }
    for (int k = 0; !unnorm && k < max_iter; ++k) {
        const bool check_now = k >= 1 && (k % check_every) == 0;
        if (check_now && !publish) HUB_TRY(fetch(k));
        HUB_TRY(product_lz(v, W, v_prev, d_beta + k, d_alpha + k));
        if (reorth) {
            // classical Gram-Schmidt against every stored vector; the second pass
            // runs only when the first removed more than 1 - 1/sqrt(2) of the norm
            HUB_TRY(lz_b(v, d_alpha + k, d_misc + 8));
            HUB_HIP(hipMemcpyAsync(dQ, Q.data(), sizeof(void *) * Q.size(), hipMemcpyHostToDevice, st));
            // partial: the omega estimate decides (on the device) whether this step
            // runs the passes; full: the first pass always runs
            const int *skip1 = nullptr, *skip2 = d_flag;
            if (partial_ro) {
                HUB_TRY(launch_pro_omega(d_alpha, d_beta, d_misc + 8, om[0], om[1], om[2], k, eps_store, d_pro, st));
                skip1 = d_pro + 1;
                skip2 = d_pro + 3;
            }
            // the norms come from the update's partials: after the first pass, and
            // (second pass run or skipped) after the second
            const int nq = gram_norm_parts(n);
            HUB_TRY(launch_gram(dt, (const void *const *)dQ, (int)Q.size(), W, n, partial, d_coef, st, skip1,
                                wpart));
            HUB_TRY(launch_sum(wpart, nq, d_misc + 9, st, 1));
            if (partial_ro) HUB_TRY(launch_pro_flag2(d_misc + 8, d_misc + 9, d_pro, st));
            else HUB_TRY(launch_dgks_flag(d_misc + 8, d_misc + 9, d_flag, st));
            HUB_TRY(launch_gram(dt, (const void *const *)dQ, (int)Q.size(), W, n, partial, d_coef, st, skip2,
                                wpart));
            if (reproject) {
                HUB_TRY(k0_project(s, dt, W, st));
                HUB_TRY(launch_dot(dt, W, W, n, partial, d_beta + k + 1, 1, st));
            } else {
                HUB_TRY(launch_sum(wpart, nq, d_beta + k + 1, st, 1));
                if (partial_ro) HUB_TRY(launch_pro_beta(d_pro, d_misc + 8, d_beta + k + 1, st));
            }
            if (partial_ro) {
                double *o0 = om[0];
                om[0] = om[1];
                om[1] = om[2];
                om[2] = o0;
            }
        } else {
            // beta_{k+1} is formed from the partials by the normalisation below
            // (or here, on the last step); with reprojection, from the projected W
            HUB_TRY(lz_b(v, d_alpha + k, nullptr));
            if (reproject) {
                HUB_TRY(k0_project(s, dt, W, st));
                HUB_TRY(launch_dot(dt, W, W, n, partial, d_beta + k + 1, 1, st));
            }
        }
        const bool beta_pending = publish;
        const bool last = (k + 1 == max_iter);
        if (check_now) {
            // step k keeps running meanwhile
            if (publish) {
                HUB_TRY(wait_published(k));
            } else {
                HUB_HIP(hipEventSynchronize(copied));
            }
            if (check(k)) break;
        }
        if (last) {
            if (beta_pending) HUB_TRY(launch_sum(partial, red_grid(n), d_beta + k + 1, st, 1));
            HUB_TRY(fetch(k + 1));
            HUB_HIP(hipEventSynchronize(copied));
            check(k + 1);
            break;
        }
        // v_{k+1} = w / beta_{k+1}
        void *vn = nullptr;
        if (reorth) {
            HUB_TRY(new_q(&vn));
        } else {
            vn = v_prev ? v_prev : spare;
        }
        if (beta_pending) {
            HUB_TRY(launch_lz_next_sum(dt, W, vn, partial, d_beta + k + 1, n, st, dpin, dflag, d_alpha + k, k, kmax));
        } else {
            HUB_TRY(launch_lz_next(dt, W, vn, d_beta + k + 1, n, st));
        }
        if (!reorth && !v_prev) spare = nullptr;
        v_prev = v;
        v = vn;
    }
    inf.iters = m_final;
    inf.orth_loss = -1.0;
    inf.reorth_steps = 0;
    if (reorth) {
        int ph[8] = {0};
        HUB_HIP(hipMemcpyAsync(ph, d_flag, sizeof(ph), hipMemcpyDeviceToHost, st));
        HUB_HIP(hipStreamSynchronize(st));
        inf.reorth_steps = partial_ro ? ph[6] : m_final;
        // max |Q^T Q - I| over the stored basis, from the FP64 matrix-core Gram
        const int mq = std::min<int>((int)Q.size(), m_final);
        if (o->orth_check && mq > 0 && mq <= 304) {
            const int ld = 16 * ((mq + 15) / 16);
            double *dG = nullptr;
            HUB_TRY(mem.alloc((void **)&dG, sizeof(double) * (size_t)ld * ld));
            HUB_HIP(hipMemcpyAsync(dQ, Q.data(), sizeof(void *) * mq, hipMemcpyHostToDevice, st));
            HUB_TRY(gram_mfma(dt, (const void *const *)dQ, mq, n, dG, ld, st));
            std::vector<double> G((size_t)ld * ld);
            HUB_HIP(hipMemcpy(G.data(), dG, sizeof(double) * G.size(), hipMemcpyDeviceToHost));
            double loss = 0.0;
            for (int i = 0; i < mq; ++i)
                for (int j = 0; j < mq; ++j)
                    loss = std::max(loss, std::fabs(G[(size_t)i * ld + j] - (i == j ? 1.0 : 0.0)));
            inf.orth_loss = loss;
        }
    }
    inf.converged = converged ? 1 : 0;
    inf.breakdown = breakdown ? 1 : 0;
    inf.e0_ritz = theta;
    inf.e0_refined = theta;
    inf.residual = res;
    inf.seconds_to_e0 = t_e0;
    double e0 = theta;

    if (want_vec) {
        const int m = m_final;
        double *psi = (double *)dev_psi;
        if (!psi) HUB_TRY(mem.alloc((void **)&psi, sizeof(double) * (size_t)n));
        HUB_HIP(hipMemcpyAsync(d_y, y.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
        if (reorth) {
            HUB_HIP(hipMemcpyAsync(dQ, Q.data(), sizeof(void *) * Q.size(), hipMemcpyHostToDevice, st));
            HUB_TRY(launch_psi_from_basis(dt, (const void *const *)dQ, m, d_y, psi, n, st));
        } else if (unnorm) {
            // second pass over the same unnormalised recurrence: psi = sum_j (y_j / beta_j) u_j
            W = B2;
            void *u = B0, *up = nullptr, *wb = B1, *sp = B2;
            HUB_TRY(make_start(u));
            HUB_TRY(launch_psi_acc(dt, psi, u, d_y, n, 1, st));
            for (int j = 0; j + 1 < m; ++j) {
                const double *bj = j >= 1 ? d_beta + j : nullptr, *bjp = j >= 2 ? d_beta + j - 1 : nullptr;
                HUB_TRY(product_lz(u, wb, up, bj, nullptr, bjp, 1));
                HUB_TRY(launch_lz_b(dt, wb, u, d_alpha + j, n, partial, nullptr, st, bj));
                HUB_TRY(launch_psi_acc(dt, psi, wb, d_y + j + 1, n, 0, st, d_beta + j + 1));
                void *freed = up ? up : sp;
                if (!up) sp = nullptr;
                up = u;
                u = wb;
                wb = freed;
            }
        } else {
            // second pass over the same recurrence with the stored alpha / beta
            void *a = Va, *b = Vb;
            HUB_TRY(make_start(a));
            HUB_TRY(launch_psi_acc(dt, psi, a, d_y, n, 1, st));
            void *vp = nullptr, *vc = a, *sp = b;
            for (int j = 0; j + 1 < m; ++j) {
                if (fused) {
                    // same two roundings as the first pass: the fused update, then w -= alpha_j v
                    HUB_TRY(product_lz(vc, W, vp, d_beta + j, nullptr));
                    HUB_TRY(launch_lz_b(dt, W, vc, d_alpha + j, n, partial, nullptr, st));
                } else {
                    HUB_TRY(product(vc, W));
                    HUB_TRY(launch_lz_replay(dt, W, vp, d_beta + j, vc, d_alpha + j, n, st));
                }
                if (reproject) HUB_TRY(k0_project(s, dt, W, st));
                void *vn = vp ? vp : sp;
                HUB_TRY(launch_lz_next(dt, W, vn, d_beta + j + 1, n, st));
                vp = vc;
                vc = vn;
                HUB_TRY(launch_psi_acc(dt, psi, vc, d_y + j + 1, n, 0, st));
            }
        }
        HUB_TRY(launch_normalize_sign(psi, n, partial, d_misc, st));
        if (o->refine) {
            double *hpsi = nullptr;
            if (dt == HUB_F64) {
                hpsi = (double *)W;
            } else {
                HUB_TRY(mem.alloc((void **)&hpsi, sizeof(double) * (size_t)n));
            }
            HUB_TRY(apply_h(s, HUB_F64, psi, hpsi, st));
            HUB_TRY(launch_dot(HUB_F64, psi, hpsi, n, partial, d_misc + 4, 0, st));
            HUB_TRY(launch_residual(hpsi, psi, d_misc + 4, n, partial, d_misc + 5, st));
            double h2[2];
            HUB_HIP(hipMemcpyAsync(h2, d_misc + 4, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
            HUB_HIP(hipStreamSynchronize(st));
            inf.e0_refined = h2[0];
            inf.true_residual = h2[1];
            e0 = h2[0];
        }
    }
    HUB_HIP(hipStreamSynchronize(st));
    if (tm.on) {
        inf.matvec_ms = tm.total_ms();
        inf.matvec_timed = tm.timed;
    }
    inf.seconds = std::chrono::duration<double>(clk::now() - t0).count();
    if (e0_out) *e0_out = e0;
    if (info) *info = inf;
    if (!converged) {
        set_error("Lanczos did not converge within max_iter");
        return HUB_ERR_NOT_CONVERGED;
    }
    return HUB_OK;
}

// Continued-fraction coefficients of <f|(w - H)^-1|f> (Sec. VII A): the plain
// FP64 recurrence from v0 = f / |f|, run for min(max_steps, dim) steps or to the
// first breakdown (beta below 64 eps of the running |T| bound, checked every
// 16 steps).  alpha[0..m-1], beta[1..m-1] (beta[0] = 0), norm2 = <f|f>.
hub_status lanczos_coefficients(const hub_sector *s, const double *f, int max_steps, double *alpha, double *beta,
                                double *norm2, int32_t *steps, hipStream_t st)
{
    const int64_t n = s->dim;
    int kmax = max_steps;
    if ((int64_t)kmax > n) kmax = (int)n;
    DevMem mem;
    double *dscal = nullptr;  // alpha[kmax] beta[kmax + 1] norm[2]
    HUB_TRY(mem.alloc((void **)&dscal, sizeof(double) * (size_t)(2 * kmax + 4)));
    HUB_HIP(hipMemsetAsync(dscal, 0, sizeof(double) * (size_t)(2 * kmax + 4), st));
    double *d_alpha = dscal, *d_beta = dscal + kmax, *d_norm = dscal + 2 * kmax + 1;
    double *partial = nullptr;
    HUB_TRY(mem.alloc((void **)&partial, sizeof(double) * (size_t)kRedGrid * 2));
    void *W = nullptr, *Va = nullptr, *Vb = nullptr;
    HUB_TRY(mem.alloc(&W, sizeof(double) * (size_t)n));
    HUB_TRY(mem.alloc(&Va, sizeof(double) * (size_t)n));
    HUB_TRY(mem.alloc(&Vb, sizeof(double) * (size_t)n));
    HUB_TRY(launch_dot(HUB_F64, f, f, n, partial, d_norm, 0, st));
    double nf = 0.0;
    HUB_HIP(hipMemcpyAsync(&nf, d_norm, sizeof(double), hipMemcpyDeviceToHost, st));
    HUB_HIP(hipStreamSynchronize(st));
    *norm2 = nf;
    *steps = 0;
    for (int j = 0; j <= max_steps; ++j) alpha[j] = beta[j] = 0.0;
    if (!(nf > 0.0)) return HUB_OK;
    HUB_TRY(launch_dot(HUB_F64, f, f, n, partial, d_norm + 1, 1, st));
    HUB_TRY(launch_convert(HUB_F64, f, HUB_F64, Va, n, d_norm + 1, 1, st));
    void *v_prev = nullptr, *v = Va, *spare = Vb;
    std::vector<double> ha(kmax), hb(kmax + 1);
    int m = kmax;
    double tmax = 0.0;
    // the product with the first update in its epilogue where available (its
    // per-column partials of alpha summed inside the next kernel), else the
    // product and a separate first update
    const bool fused = matvec_lz_available(s, HUB_F64) && matvec_lz_partials(s) <= kSumInUpdate;
    double *apart = nullptr;
    if (fused) HUB_TRY(mem.alloc((void **)&apart, sizeof(double) * (size_t)matvec_lz_workspace(s)));
    for (int k = 0; k < kmax; ++k) {
        if (fused) {
            int64_t np = 0;
            HUB_TRY(launch_matvec_lz(s, HUB_F64, v, W, v_prev, d_beta + k, apart, &np, st));
            HUB_TRY(launch_lz_b_sum(HUB_F64, W, v, apart, np, d_alpha + k, n, partial, st));
        } else {
            HUB_TRY(apply_h(s, HUB_F64, v, W, st));
            // alpha's partials beside beta's; both summed inside the kernels that use them
            HUB_TRY(launch_lz_a(HUB_F64, W, v_prev, d_beta + k, v, n, partial + kRedGrid, nullptr, st));
            HUB_TRY(launch_lz_b_sum(HUB_F64, W, v, partial + kRedGrid, red_grid(n), d_alpha + k, n, partial, st));
        }
        const bool last = (k + 1 == kmax);
        const bool check_now = (k + 1) % 16 == 0 || last;
        if (check_now) HUB_TRY(launch_sum(partial, red_grid(n), d_beta + k + 1, st, 1));
        if (check_now) {
            const int mm = k + 1;
            HUB_HIP(hipMemcpyAsync(ha.data(), d_alpha, sizeof(double) * mm, hipMemcpyDeviceToHost, st));
            HUB_HIP(hipMemcpyAsync(hb.data(), d_beta, sizeof(double) * (mm + 1), hipMemcpyDeviceToHost, st));
            HUB_HIP(hipStreamSynchronize(st));
            bool brk = false;
            tmax = 0.0;
            for (int j = 0; j < mm; ++j) {
                tmax = std::max(tmax, std::fabs(ha[j]) + 2.0 * std::fabs(hb[j + 1]));
                if (!(hb[j + 1] > 64.0 * DBL_EPSILON * std::max(tmax, DBL_MIN))) {
                    m = j + 1;
                    brk = true;
                    break;
                }
            }
            if (brk) break;
        }
        if (last) break;
        void *vn = v_prev ? v_prev : spare;
        if (check_now) {
            HUB_TRY(launch_lz_next(HUB_F64, W, vn, d_beta + k + 1, n, st));
        } else {
            HUB_TRY(launch_lz_next_sum(HUB_F64, W, vn, partial, d_beta + k + 1, n, st));
        }
        v_prev = v;
        v = vn;
    }
    HUB_HIP(hipMemcpyAsync(ha.data(), d_alpha, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    HUB_HIP(hipMemcpyAsync(hb.data(), d_beta, sizeof(double) * (m + 1), hipMemcpyDeviceToHost, st));
    HUB_HIP(hipStreamSynchronize(st));
    for (int j = 0; j < m; ++j) alpha[j] = ha[j];
    for (int j = 1; j < m; ++j) beta[j] = hb[j];
    *steps = m;
    return HUB_OK;
}

}  // namespace hub
