// Vector kernels of the Lanczos iteration (Sec. IV): start vector, FP64
// reductions, the three-term recurrence updates, Gram-Schmidt against stored
// Lanczos vectors, and the assembly / normalisation of the eigenvector.
//
// Reductions are deterministic: a fixed number of blocks (a function of n
// only) each reduce a contiguous stride pattern into one FP64 partial with an
// LDS tree, and the partials are summed in a fixed order, by a single block or
// by every block of the kernel that needs the total (the same order, so the
// same value).  Repeating a computation therefore reproduces it bit for bit,
// which the two-pass eigenvector assembly relies on.
//
// Vectors of FP32 ("mixed") or FP64 storage; every scalar (alpha, beta, Gram
// coefficients, norms) is FP64 and every update is evaluated in FP64 and
// rounded once to the storage type.
#include <mutex>
#include <vector>

#include "internal.h"

namespace hub {
namespace {

constexpr int RB = kRedBlock;

__device__ __forceinline__ double block_sum(double v, double *s)
{
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = RB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < (unsigned)off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

// 1 / beta for a device beta (NULL: 1, beta <= 0: 0); the scale that turns an
// unnormalised Lanczos vector beta_k v_k back into v_k
__device__ __forceinline__ double inv_beta(const double *b)
{
    if (!b) return 1.0;
    const double v = *b;
    return v > 0.0 ? 1.0 / v : 0.0;
}

__device__ __forceinline__ double splitmix_entry(uint64_t seed, int64_t k)
{
    // SplitMix64 (Steele, Lea & Flood 2014) output for state seed + (k+1) gamma,
    // top 53 bits as a uniform in [0, 1), mapped to [-1, 1).
    uint64_t z = seed + (uint64_t)(k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return -1.0 + 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0));
}

template <typename T>
__global__ void k_start(T *__restrict__ out, int64_t n, uint64_t seed)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (T)splitmix_entry(seed, i);
}

template <typename T>
__global__ __launch_bounds__(RB) void k_dot(const T *__restrict__ x, const T *__restrict__ y, int64_t n,
                                            double *__restrict__ partial)
{
    __shared__ double s[RB];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB)
        acc += (double)x[i] * (double)y[i];
    const double r = block_sum(acc, s);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// Sum of partial[0 .. np) in a fixed order by one block of RB threads.  Every
// block that calls it obtains the same value, so a kernel that needs the total
// of a previous kernel's partials can form it per block instead of waiting for
// a separate single-block launch.
__device__ __forceinline__ double block_total(const double *__restrict__ partial, int np, double *s)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += RB) acc += partial[i];
    return block_sum(acc, s);
}

__global__ __launch_bounds__(RB) void k_final(const double *__restrict__ partial, int np, double *__restrict__ out,
                                              int sqrt_result)
{
    __shared__ double s[RB];
    const double r = block_total(partial, np, s);
    if (threadIdx.x == 0) *out = sqrt_result ? sqrt(r) : r;
}

template <typename Ti, typename To>
__global__ void k_convert(const Ti *__restrict__ x, To *__restrict__ y, int64_t n, const double *__restrict__ sc,
                          int invert)
{
    // invert: divide by the scalar (a unit vector of one entry comes out as exactly +-1)
    const double f = sc ? *sc : 1.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (To)(invert ? (double)x[i] / f : (double)x[i] * f);
}

// w <- w - beta * vprev ; partial alpha = <w, v>
template <typename T>
__global__ __launch_bounds__(RB) void k_lz_a(T *__restrict__ w, const T *__restrict__ vprev,
                                             const double *__restrict__ beta, const T *__restrict__ v, int64_t n,
                                             double *__restrict__ partial)
{
    __shared__ double s[RB];
    const double bt = vprev ? *beta : 0.0;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
        T wi = w[i];
        if (vprev) {
            wi = (T)((double)wi - bt * (double)vprev[i]);
            w[i] = wi;
        }
        acc += (double)wi * (double)v[i];
    }
    const double r = block_sum(acc, s);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// w <- w - alpha * v ; partial beta^2 = <w, w>.  beta_div (may be NULL): v is
// the unnormalised beta_k v_k and the coefficient is alpha / beta_k.
template <typename T>
__global__ __launch_bounds__(RB) void k_lz_b(T *__restrict__ w, const T *__restrict__ v,
                                             const double *__restrict__ alpha, int64_t n,
                                             double *__restrict__ partial, const double *__restrict__ beta_div)
{
    __shared__ double s[RB];
    const double al = beta_div ? *alpha * inv_beta(beta_div) : *alpha;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
        const T wi = (T)((double)w[i] - al * (double)v[i]);
        w[i] = wi;
        acc += (double)wi * (double)wi;
    }
    const double r = block_sum(acc, s);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

template <typename T>
__global__ void k_lz_next(const T *__restrict__ w, T *__restrict__ vnext, const double *__restrict__ beta, int64_t n)
{
    const double bt = *beta;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        vnext[i] = (bt > 0.0) ? (T)((double)w[i] / bt) : (T)0;
}

// Second pass: the same two roundings as k_lz_a followed by k_lz_b.
template <typename T>
__global__ void k_lz_replay(T *__restrict__ w, const T *__restrict__ vprev, const double *__restrict__ beta,
                            const T *__restrict__ v, const double *__restrict__ alpha, int64_t n)
{
    const double bt = vprev ? *beta : 0.0;
    const double al = *alpha;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        T wi = w[i];
        if (vprev) wi = (T)((double)wi - bt * (double)vprev[i]);
        w[i] = (T)((double)wi - al * (double)v[i]);
    }
}

template <typename T>
__global__ void k_psi_acc(double *__restrict__ psi, const T *__restrict__ v, const double *__restrict__ y, int64_t n,
                          int first, const double *__restrict__ div)
{
    const double c = div ? *y * inv_beta(div) : *y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        psi[i] = (first ? 0.0 : psi[i]) + c * (double)v[i];
}

// Gram coefficients c_j = <q_j, w> for the stored vectors, GJ at a time so w
// is read once per group.  Each wavefront reduces its GJ sums with lane
// shuffles (fixed butterfly order), then one barrier combines the wavefronts.
// partial layout: [block][j].  A non-null `skip` pointing at a non-zero flag
// turns the launch into a no-op (second Gram-Schmidt pass not needed).
constexpr int GJ = 16;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Four consecutive elements per lane: 16-byte loads (FP32) or two 16-byte loads (FP64).
template <typename T>
struct E4 {
    T v[4];
};

template <typename T>
__device__ __forceinline__ E4<T> ld_e4(const T *p)
{
    E4<T> r;
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

template <typename T>
__device__ __forceinline__ void st_e4(T *p, const T (&v)[4])
{
    if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        reinterpret_cast<double2 *>(p)[0] = make_double2(v[0], v[1]);
        reinterpret_cast<double2 *>(p)[1] = make_double2(v[2], v[3]);
    }
}

// k_lz_b with alpha = the sum of the product's per-column partials (the value
// k_final would give), written to *alpha_out by block 0.  Lanes take four
// consecutive elements (16-byte aligned vectors), block 0 also the n % 4 tail.
//
// unnorm: v is the unnormalised beta_k v_k (beta_k NULL at the first step) and
// the partials sum to beta_k alpha_k: alpha_k = that sum / beta_k, and the
// update subtracts (alpha_k / beta_k) v, leaving the unnormalised beta_{k+1} v_{k+1}.
template <typename T>
__global__ __launch_bounds__(RB) void k_lz_b_sum(T *__restrict__ w, const T *__restrict__ v,
                                                 const double *__restrict__ apart, int np,
                                                 double *__restrict__ alpha_out, int64_t n,
                                                 double *__restrict__ partial, const double *__restrict__ beta_k,
                                                 int unnorm)
{
    __shared__ double s[RB];
    const double tot = block_total(apart, np, s);
    const double alpha = unnorm ? tot * inv_beta(beta_k) : tot;
    if (blockIdx.x == 0 && threadIdx.x == 0) *alpha_out = alpha;
    const double al = unnorm ? alpha * inv_beta(beta_k) : alpha;
    double acc = 0.0;
    const int64_t n4 = n >> 2;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n4; i += (int64_t)gridDim.x * RB) {
        const E4<T> wv = ld_e4(w + 4 * i), vv = ld_e4(v + 4 * i);
        T o[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            o[r] = (T)((double)wv.v[r] - al * (double)vv.v[r]);
            acc += (double)o[r] * (double)o[r];
        }
        st_e4(w + 4 * i, o);
    }
    if (blockIdx.x == 0)
        for (int64_t i = 4 * n4 + threadIdx.x; i < n; i += RB) {
            const T wi = (T)((double)w[i] - al * (double)v[i]);
            w[i] = wi;
            acc += (double)wi * (double)wi;
        }
    const double r = block_sum(acc, s);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// k_lz_next with beta = sqrt(sum of k_lz_b's partials), written to *beta_out by
// block 0; the same element layout as k_lz_b_sum.  When `pub` is set, block 0
// also publishes alpha_k and beta_{k+1} to host memory and then the step count
// k + 1, so the host can follow the recurrence without a copy or an event.
struct HostPublish {
    double *ab;           // host (device-visible) alpha[0 .. kmax) then beta[0 .. kmax]
    int *step;            // host (device-visible) count of published steps
    const double *alpha;  // device alpha_k
    int k, kmax;
};

template <typename T>
__global__ __launch_bounds__(RB) void k_lz_next_sum(const T *__restrict__ w, T *__restrict__ vnext,
                                                    const double *__restrict__ partial, int np,
                                                    double *__restrict__ beta_out, int64_t n, HostPublish pub)
{
    __shared__ double s[RB];
    const double bt = sqrt(block_total(partial, np, s));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *beta_out = bt;
        if (pub.ab) {
            volatile double *ab = pub.ab;
            ab[pub.k] = *pub.alpha;
            ab[pub.kmax + pub.k + 1] = bt;
            __threadfence_system();
            *(volatile int *)pub.step = pub.k + 1;
        }
    }
    const int64_t n4 = n >> 2;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n4; i += (int64_t)gridDim.x * RB) {
        const E4<T> wv = ld_e4(w + 4 * i);
        T o[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) o[r] = (bt > 0.0) ? (T)((double)wv.v[r] / bt) : (T)0;
        st_e4(vnext + 4 * i, o);
    }
    if (blockIdx.x == 0)
        for (int64_t i = 4 * n4 + threadIdx.x; i < n; i += RB) vnext[i] = (bt > 0.0) ? (T)((double)w[i] / bt) : (T)0;
}

// beta_{k+1} = sqrt(sum of the update's partials) into *beta_out, and the same
// publication to host memory as k_lz_next_sum (one block)
__global__ __launch_bounds__(RB) void k_beta_pub(const double *__restrict__ partial, int np,
                                                 double *__restrict__ beta_out, HostPublish pub)
{
    __shared__ double s[RB];
    const double bt = sqrt(block_total(partial, np, s));
    if (threadIdx.x == 0) {
        *beta_out = bt;
        if (pub.ab) {
            volatile double *ab = pub.ab;
            ab[pub.k] = *pub.alpha;
            ab[pub.kmax + pub.k + 1] = bt;
            __threadfence_system();
            *(volatile int *)pub.step = pub.k + 1;
        }
    }
}

// partial[block * kstride + j] = sum over the block's elements of q_j * w, for
// the k stored vectors in groups of GJ; lanes take four consecutive elements,
// block 0 also the n % 4 tail.  Every vector is a separate allocation (aligned).
template <typename T>
__global__ __launch_bounds__(RB) void k_gram_dot(const T *const *__restrict__ Q, int k, const T *__restrict__ w,
                                                 int64_t n, double *__restrict__ partial, int kstride,
                                                 const int *__restrict__ skip)
{
    if (skip && *skip) return;
    __shared__ double s[RB / 64][GJ];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t n4 = n >> 2;
    const int64_t tail = n - 4 * n4;
    for (int j0 = 0; j0 < k; j0 += GJ) {
        double acc[GJ];
#pragma unroll
        for (int u = 0; u < GJ; ++u) acc[u] = 0.0;
        const int jn = min(GJ, k - j0);
        const T *q[GJ];
#pragma unroll
        for (int u = 0; u < GJ; ++u) q[u] = Q[j0 + (u < jn ? u : 0)];
        for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n4; i += (int64_t)gridDim.x * RB) {
            const E4<T> wv = ld_e4(w + 4 * i);
#pragma unroll
            for (int u = 0; u < GJ; ++u)
                if (u < jn) {
                    const E4<T> qv = ld_e4(q[u] + 4 * i);
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[u] += (double)qv.v[r] * (double)wv.v[r];
                }
        }
        if (blockIdx.x == 0 && threadIdx.x < tail) {
            const int64_t i = 4 * n4 + threadIdx.x;
#pragma unroll
            for (int u = 0; u < GJ; ++u)
                if (u < jn) acc[u] += (double)q[u][i] * (double)w[i];
        }
#pragma unroll
        for (int u = 0; u < GJ; ++u) {
            const double r = wave_sum(acc[u]);
            if (lane == 0) s[wave][u] = r;
        }
        __syncthreads();
        if (threadIdx.x < (unsigned)jn) {
            double r = 0.0;
#pragma unroll
            for (int v = 0; v < RB / 64; ++v) r += s[v][threadIdx.x];
            partial[(int64_t)blockIdx.x * kstride + j0 + threadIdx.x] = r;
        }
        __syncthreads();
    }
}

// One block per coefficient: fixed-order tree over the block partials.
__global__ __launch_bounds__(RB) void k_gram_final(const double *__restrict__ partial, int np, int k, int kstride,
                                                   double *__restrict__ coef, const int *__restrict__ skip)
{
    if (skip && *skip) return;
    __shared__ double s[RB];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < np; b += RB) acc += partial[(int64_t)b * kstride + j];
    const double r = block_sum(acc, s);
    if (threadIdx.x == 0) coef[j] = r;
}

// w <- w - sum_j c_j q_j, evaluated in FP64 per element; lanes take four
// consecutive elements (the n % 4 tail element by element).  npart (or NULL):
// one partial of the new ||w||^2 per block (RB threads), so the norm needs no
// separate pass over w; a skipped launch leaves npart as it was.
template <typename T>
__global__ __launch_bounds__(RB) void k_gram_update(const T *const *__restrict__ Q, int k,
                                                    const double *__restrict__ coef, T *__restrict__ w, int64_t n,
                                                    const int *__restrict__ skip, double *__restrict__ npart)
{
    if (skip && *skip) return;
    __shared__ double s[RB];
    double nacc = 0.0;
    const int64_t n4 = n >> 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int j = 0; j < k; ++j) {
            const double c = coef[j];
            const E4<T> qv = ld_e4(Q[j] + 4 * i);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] += c * (double)qv.v[r];
        }
        const E4<T> wv = ld_e4(w + 4 * i);
        T o[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            o[r] = (T)((double)wv.v[r] - acc[r]);
            nacc += (double)o[r] * (double)o[r];
        }
        st_e4(w + 4 * i, o);
    }
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc += coef[j] * (double)Q[j][i];
        const T o = (T)((double)w[i] - acc);
        w[i] = o;
        nacc += (double)o * (double)o;
    }
    if (!npart) return;
    const double r = block_sum(nacc, s);
    if (threadIdx.x == 0) npart[blockIdx.x] = r;
}

// flag = 1 when the first pass kept more than 1/sqrt(2) of the norm (a second
// classical Gram-Schmidt pass would not change w to working precision).
__global__ void k_dgks_flag(const double *__restrict__ before, const double *__restrict__ after, int *__restrict__ flag)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *flag = (*after > 0.70710678118654752 * *before) ? 1 : 0;
}

// ---- partial reorthogonalisation (Simon, Math. Comp. 42 (1984) 115) ------------
// The rounding errors of the Lanczos step obey a recurrence that estimates
// om_{k+1,j} ~ <v_j, v_{k+1}> from alpha and beta alone:
//   beta_{k+1} om_{k+1,j} = beta_{j+1} om_{k,j+1} + (alpha_j - alpha_k) om_{k,j}
//                         + beta_j om_{k,j-1} - beta_k om_{k-1,j} + theta_{k,j},
// om_{k,k} = 1, with theta_{k,j} = eps (beta_{j+1} + beta_{k+1}) added in the
// direction that increases |om| (an over-estimate of the rounding term).  A
// Gram-Schmidt pass against the stored vectors runs when some |om_{k+1,j}|,
// j < k, reaches sqrt(eps) -- the vectors then stay semi-orthogonal, which keeps
// the Ritz values as accurate as full reorthogonalisation -- and once more at
// the next step, since the recurrence couples two consecutive steps; om_{k+1,.}
// is reset to eps after a pass.  beta_t is ||w|| before any pass.
// state[0]: the pass is forced at this step; state[1]: skip flag of the first
// pass (1 = skip); state[2]: passes run so far; state[3]: skip flag of the second
// pass (set by k_pro_flag2).
__global__ __launch_bounds__(256) void k_pro_omega(const double *__restrict__ alpha, const double *__restrict__ beta,
                                                   const double *__restrict__ beta_t,
                                                   const double *__restrict__ om_prev,
                                                   const double *__restrict__ om_cur, double *__restrict__ om_next,
                                                   int k, double eps, int *__restrict__ state)
{
    __shared__ double smax[256];
    __shared__ int srun;
    const double bk1 = *beta_t, bk = beta[k], ak = alpha[k];
    double mx = 0.0;
    for (int j = (int)threadIdx.x; j < k; j += 256) {
        const double om_j1 = (j + 1 == k) ? 1.0 : om_cur[j + 1];
        const double om_prev_j = (j + 1 == k) ? 1.0 : om_prev[j];
        double t = beta[j + 1] * om_j1 + (alpha[j] - ak) * om_cur[j] - bk * om_prev_j;
        if (j > 0) t += beta[j] * om_cur[j - 1];
        const double th = eps * (beta[j + 1] + bk1);
        t += (t >= 0.0) ? th : -th;
        const double o = bk1 > 0.0 ? t / bk1 : 1.0;
        om_next[j] = o;
        mx = fmax(mx, fabs(o));
    }
    smax[threadIdx.x] = mx;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int forced = state[0];
        const int run = (forced || smax[0] >= sqrt(eps)) ? 1 : 0;
        state[1] = run ? 0 : 1;
        state[0] = (run && !forced) ? 1 : 0;
        state[2] += run;
        om_next[k] = eps;  // local orthogonality after the explicit alpha subtraction
        om_next[k + 1] = 1.0;
        srun = run;
    }
    __syncthreads();
    if (srun)
        for (int j = (int)threadIdx.x; j < k; j += 256) om_next[j] = eps;
}

// second pass of a partial reorthogonalisation step: run only when the first
// ran and kept less than 1/sqrt(2) of the norm (the DGKS test)
__global__ void k_pro_flag2(const double *__restrict__ before, const double *__restrict__ after, int *__restrict__ state)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        state[3] = (state[1] || *after > 0.70710678118654752 * *before) ? 1 : 0;
}

// beta_{k+1}: the norm after the passes, or ||w|| when none ran
__global__ void k_pro_beta(const int *__restrict__ state, const double *__restrict__ beta_t, double *__restrict__ beta)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && state[1]) *beta = *beta_t;
}

template <typename T>
__global__ void k_psi_basis(const T *const *__restrict__ Q, int k, const double *__restrict__ y,
                            double *__restrict__ psi, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc += y[j] * (double)Q[j][i];
        psi[i] = acc;
    }
}

// Per block: max |psi| and its lowest index; then sum of squares.
__global__ __launch_bounds__(RB) void k_absmax(const double *__restrict__ x, int64_t n, double *__restrict__ pv,
                                               int64_t *__restrict__ pi)
{
    __shared__ double sv[RB];
    __shared__ int64_t si[RB];
    double best = -1.0;
    int64_t bi = 0;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
        const double a = fabs(x[i]);
        if (a > best) { best = a; bi = i; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int off = RB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < (unsigned)off) {
            const double a = sv[threadIdx.x + off];
            const int64_t ai = si[threadIdx.x + off];
            if (a > sv[threadIdx.x] || (a == sv[threadIdx.x] && ai < si[threadIdx.x])) {
                sv[threadIdx.x] = a;
                si[threadIdx.x] = ai;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { pv[blockIdx.x] = sv[0]; pi[blockIdx.x] = si[0]; }
}

// scal[0] = sum of squares (already reduced), finds the sign of the entry with
// the largest magnitude and stores scal[1] = sign / norm.
__global__ void k_sign_scale(const double *__restrict__ x, const double *__restrict__ pv,
                             const int64_t *__restrict__ pi, int np, double *__restrict__ scal)
{
    if (threadIdx.x != 0) return;
    double best = -1.0;
    int64_t bi = 0;
    for (int b = 0; b < np; ++b)
        if (pv[b] > best || (pv[b] == best && pi[b] < bi)) { best = pv[b]; bi = pi[b]; }
    const double nrm = sqrt(scal[0]);
    const double sg = (x[bi] < 0.0) ? -1.0 : 1.0;
    scal[1] = (nrm > 0.0) ? sg / nrm : 0.0;
}

__global__ void k_scale_inplace(double *__restrict__ x, int64_t n, const double *__restrict__ f)
{
    const double c = *f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] *= c;
}

__global__ __launch_bounds__(RB) void k_resid(const double *__restrict__ hp, const double *__restrict__ p,
                                              const double *__restrict__ e, int64_t n, double *__restrict__ partial)
{
    __shared__ double s[RB];
    const double E = *e;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
        const double r = hp[i] - E * p[i];
        acc += r * r;
    }
    const double r = block_sum(acc, s);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

inline unsigned ew_grid(int64_t n)
{
    const int64_t g = (n + 255) / 256;
    return (unsigned)(g < 8192 ? (g < 1 ? 1 : g) : 8192);
}

}  // namespace

int gram_norm_parts(int64_t n)
{
    return (int)ew_grid(n);
}

int red_grid(int64_t n)
{
    int64_t g = (n + (int64_t)RB * 4 - 1) / ((int64_t)RB * 4);
    if (g < 1) g = 1;
    if (g > kRedGrid) g = kRedGrid;
    return (int)g;
}

#define HUB_DISPATCH(dtype, KERNEL, ...)                                                            \
    do {                                                                                            \
        if ((dtype) == HUB_F64) hipLaunchKernelGGL(KERNEL<double>, __VA_ARGS__);                    \
        else hipLaunchKernelGGL(KERNEL<float>, __VA_ARGS__);                                       \
    } while (0)

hub_status launch_start_vector(int dtype, uint64_t seed, void *out, int64_t n, hipStream_t st)
{
    if (dtype == HUB_F64)
        hipLaunchKernelGGL(k_start<double>, dim3(ew_grid(n)), dim3(256), 0, st, (double *)out, n, seed);
    else
        hipLaunchKernelGGL(k_start<float>, dim3(ew_grid(n)), dim3(256), 0, st, (float *)out, n, seed);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_dot(int dtype, const void *x, const void *y, int64_t n, double *partial, double *out,
                      int sqrt_result, hipStream_t st)
{
    const int G = red_grid(n);
    if (dtype == HUB_F64)
        hipLaunchKernelGGL(k_dot<double>, dim3(G), dim3(RB), 0, st, (const double *)x, (const double *)y, n,
                           partial);
    else
        hipLaunchKernelGGL(k_dot<float>, dim3(G), dim3(RB), 0, st, (const float *)x, (const float *)y, n, partial);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(RB), 0, st, partial, G, out, sqrt_result);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_convert(int din, const void *x, int dout, void *y, int64_t n, const double *sc, int invert,
                          hipStream_t st)
{
    const dim3 g(ew_grid(n)), b(256);
    if (din == HUB_F64 && dout == HUB_F64)
        hipLaunchKernelGGL((k_convert<double, double>), g, b, 0, st, (const double *)x, (double *)y, n, sc, invert);
    else if (din == HUB_F64 && dout == HUB_F32)
        hipLaunchKernelGGL((k_convert<double, float>), g, b, 0, st, (const double *)x, (float *)y, n, sc, invert);
    else if (din == HUB_F32 && dout == HUB_F64)
        hipLaunchKernelGGL((k_convert<float, double>), g, b, 0, st, (const float *)x, (double *)y, n, sc, invert);
    else
        hipLaunchKernelGGL((k_convert<float, float>), g, b, 0, st, (const float *)x, (float *)y, n, sc, invert);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_sum(const double *partial, int64_t np, double *out, hipStream_t st, int sqrt_result)
{
    hipLaunchKernelGGL(k_final, dim3(1), dim3(RB), 0, st, partial, (int)np, out, sqrt_result);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_lz_a(int dtype, void *w, const void *vprev, const double *beta, const void *v, int64_t n,
                       double *partial, double *alpha_out, hipStream_t st)
{
    const int G = red_grid(n);
    if (dtype == HUB_F64)
        hipLaunchKernelGGL(k_lz_a<double>, dim3(G), dim3(RB), 0, st, (double *)w, (const double *)vprev, beta,
                           (const double *)v, n, partial);
    else
        hipLaunchKernelGGL(k_lz_a<float>, dim3(G), dim3(RB), 0, st, (float *)w, (const float *)vprev, beta,
                           (const float *)v, n, partial);
    if (alpha_out) hipLaunchKernelGGL(k_final, dim3(1), dim3(RB), 0, st, partial, G, alpha_out, 0);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_lz_b(int dtype, void *w, const void *v, const double *alpha, int64_t n, double *partial,
                       double *beta_out, hipStream_t st, const double *beta_div)
{
    const int G = red_grid(n);
    if (dtype == HUB_F64)
        hipLaunchKernelGGL(k_lz_b<double>, dim3(G), dim3(RB), 0, st, (double *)w, (const double *)v, alpha, n,
                           partial, beta_div);
    else
        hipLaunchKernelGGL(k_lz_b<float>, dim3(G), dim3(RB), 0, st, (float *)w, (const float *)v, alpha, n,
                           partial, beta_div);
    if (beta_out) hipLaunchKernelGGL(k_final, dim3(1), dim3(RB), 0, st, partial, G, beta_out, 1);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_lz_b_sum(int dtype, void *w, const void *v, const double *apart, int64_t np, double *alpha_out,
                          int64_t n, double *partial, hipStream_t st, const double *beta_k, int unnorm)
{
    if (((uintptr_t)w | (uintptr_t)v) % 16) {
        set_error("lz_b_sum: vectors must be 16-byte aligned");
        return HUB_ERR_INVALID_ARG;
    }
    const int G = red_grid(n);
    if (dtype == HUB_F64)
        hipLaunchKernelGGL(k_lz_b_sum<double>, dim3(G), dim3(RB), 0, st, (double *)w, (const double *)v, apart,
                           (int)np, alpha_out, n, partial, beta_k, unnorm);
    else
        hipLaunchKernelGGL(k_lz_b_sum<float>, dim3(G), dim3(RB), 0, st, (float *)w, (const float *)v, apart,
                           (int)np, alpha_out, n, partial, beta_k, unnorm);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_lz_next_sum(int dtype, const void *w, void *vnext, const double *partial, double *beta_out,
                              int64_t n, hipStream_t st, double *host_ab, int *host_step, const double *alpha_k,
                              int k, int kmax)
{
    const HostPublish pub{host_ab, host_step, alpha_k, k, kmax};
    if (((uintptr_t)w | (uintptr_t)vnext) % 16) {
        set_error("lz_next_sum: vectors must be 16-byte aligned");
        return HUB_ERR_INVALID_ARG;
    }
    const int G = red_grid(n);
    if (dtype == HUB_F64)
        hipLaunchKernelGGL(k_lz_next_sum<double>, dim3(G), dim3(RB), 0, st, (const double *)w, (double *)vnext,
                           partial, G, beta_out, n, pub);
    else
        hipLaunchKernelGGL(k_lz_next_sum<float>, dim3(G), dim3(RB), 0, st, (const float *)w, (float *)vnext,
                           partial, G, beta_out, n, pub);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_beta_pub(const double *partial, int64_t n, double *beta_out, hipStream_t st, double *host_ab,
                           int *host_step, const double *alpha_k, int k, int kmax)
{
    const HostPublish pub{host_ab, host_step, alpha_k, k, kmax};
    hipLaunchKernelGGL(k_beta_pub, dim3(1), dim3(RB), 0, st, partial, red_grid(n), beta_out, pub);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_lz_next(int dtype, const void *w, void *vnext, const double *beta, int64_t n, hipStream_t st)
{
    if (dtype == HUB_F64)
        hipLaunchKernelGGL(k_lz_next<double>, dim3(ew_grid(n)), dim3(256), 0, st, (const double *)w,
                           (double *)vnext, beta, n);
    else
        hipLaunchKernelGGL(k_lz_next<float>, dim3(ew_grid(n)), dim3(256), 0, st, (const float *)w, (float *)vnext,
                           beta, n);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_lz_replay(int dtype, void *w, const void *vprev, const double *beta, const void *v,
                            const double *alpha, int64_t n, hipStream_t st)
{
    if (dtype == HUB_F64)
        hipLaunchKernelGGL(k_lz_replay<double>, dim3(ew_grid(n)), dim3(256), 0, st, (double *)w,
                           (const double *)vprev, beta, (const double *)v, alpha, n);
    else
        hipLaunchKernelGGL(k_lz_replay<float>, dim3(ew_grid(n)), dim3(256), 0, st, (float *)w,
                           (const float *)vprev, beta, (const float *)v, alpha, n);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_psi_acc(int dtype, double *psi, const void *v, const double *ycoef, int64_t n, int first,
                          hipStream_t st, const double *div)
{
    if (dtype == HUB_F64)
        hipLaunchKernelGGL(k_psi_acc<double>, dim3(ew_grid(n)), dim3(256), 0, st, psi, (const double *)v, ycoef, n,
                           first, div);
    else
        hipLaunchKernelGGL(k_psi_acc<float>, dim3(ew_grid(n)), dim3(256), 0, st, psi, (const float *)v, ycoef, n,
                           first, div);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

// coef must hold k doubles; partial must hold red_grid(n) * kmax doubles with kmax >= k.
hub_status launch_gram(int dtype, const void *const *dQ, int k, void *w, int64_t n, double *partial, double *coef,
                       hipStream_t st, const int *skip, double *npart)
{
    if (k <= 0) {
        if (npart) {
            set_error("gram: norm partials need at least one stored vector");
            return HUB_ERR_INVALID_ARG;
        }
        return HUB_OK;
    }
    const int G = red_grid(n);
    if (dtype == HUB_F64) {
        hipLaunchKernelGGL(k_gram_dot<double>, dim3(G), dim3(RB), 0, st, (const double *const *)dQ, k,
                           (const double *)w, n, partial, k, skip);
    } else {
        hipLaunchKernelGGL(k_gram_dot<float>, dim3(G), dim3(RB), 0, st, (const float *const *)dQ, k,
                           (const float *)w, n, partial, k, skip);
    }
    hipLaunchKernelGGL(k_gram_final, dim3(k), dim3(RB), 0, st, partial, G, k, k, coef, skip);
    if (dtype == HUB_F64)
        hipLaunchKernelGGL(k_gram_update<double>, dim3(ew_grid(n)), dim3(RB), 0, st, (const double *const *)dQ, k,
                           coef, (double *)w, n, skip, npart);
    else
        hipLaunchKernelGGL(k_gram_update<float>, dim3(ew_grid(n)), dim3(RB), 0, st, (const float *const *)dQ, k,
                           coef, (float *)w, n, skip, npart);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_dgks_flag(const double *before, const double *after, int *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_dgks_flag, dim3(1), dim3(64), 0, st, before, after, flag);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_pro_omega(const double *alpha, const double *beta, const double *beta_t, const double *om_prev,
                            const double *om_cur, double *om_next, int k, double eps, int *state, hipStream_t st)
{
    hipLaunchKernelGGL(k_pro_omega, dim3(1), dim3(256), 0, st, alpha, beta, beta_t, om_prev, om_cur, om_next, k, eps,
                       state);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_pro_flag2(const double *before, const double *after, int *state, hipStream_t st)
{
    hipLaunchKernelGGL(k_pro_flag2, dim3(1), dim3(64), 0, st, before, after, state);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_pro_beta(const int *state, const double *beta_t, double *beta, hipStream_t st)
{
    hipLaunchKernelGGL(k_pro_beta, dim3(1), dim3(64), 0, st, state, beta_t, beta);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_psi_from_basis(int dtype, const void *const *dQ, int k, const double *ycoef, double *psi,
                                 int64_t n, hipStream_t st)
{
    if (dtype == HUB_F64)
        hipLaunchKernelGGL(k_psi_basis<double>, dim3(ew_grid(n)), dim3(256), 0, st, (const double *const *)dQ, k,
                           ycoef, psi, n);
    else
        hipLaunchKernelGGL(k_psi_basis<float>, dim3(ew_grid(n)), dim3(256), 0, st, (const float *const *)dQ, k,
                           ycoef, psi, n);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

// scal: 2 doubles of device scratch; partial: red_grid(n) doubles + red_grid(n) int64.
hub_status launch_normalize_sign(double *psi, int64_t n, double *partial, double *scal, hipStream_t st)
{
    const int G = red_grid(n);
    HUB_TRY(launch_dot(HUB_F64, psi, psi, n, partial, scal, 0, st));
    double *pv = partial;
    int64_t *pi = (int64_t *)(partial + kRedGrid);
    hipLaunchKernelGGL(k_absmax, dim3(G), dim3(RB), 0, st, psi, n, pv, pi);
    hipLaunchKernelGGL(k_sign_scale, dim3(1), dim3(64), 0, st, psi, pv, pi, G, scal);
    hipLaunchKernelGGL(k_scale_inplace, dim3(ew_grid(n)), dim3(256), 0, st, psi, n, scal + 1);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

hub_status launch_residual(const double *hpsi, const double *psi, const double *e, int64_t n, double *partial,
                           double *out, hipStream_t st)
{
    const int G = red_grid(n);
    hipLaunchKernelGGL(k_resid, dim3(G), dim3(RB), 0, st, hpsi, psi, e, n, partial);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(RB), 0, st, partial, G, out, 1);
    HUB_HIP(hipGetLastError());
    return HUB_OK;
}

// ---- allocation-free start vector ---------------------------------------------
//
// hub_start_vector_noalloc keeps the partial sums of the norm and the norm
// itself in `scratch` instead of a buffer allocated per call.  Each device
// holds its own copy of the array until the process ends; its address there
// comes from hipGetSymbolAddress (host code never passes the array's name to a
// kernel).  Calls that overlap on one device race on it.

constexpr int kScratchDoubles = kRedGrid + 4;  // the norm, three spare, then the partials
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_scratch_mu;
std::vector<double *> g_scratch_addr;  // per device, looked up on first use

hub_status scratch_on_current_device(double **out)
{
    int dev = 0;
    HUB_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_addr.size() <= dev) g_scratch_addr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_addr[(size_t)dev]) {
        void *p = nullptr;
        HUB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_addr[(size_t)dev] = (double *)p;
    }
    *out = g_scratch_addr[(size_t)dev];
    return HUB_OK;
}

}  // namespace

hub_status start_vector_noalloc(const hub_sector *s, int dtype, uint64_t seed, int normalize, void *out,
                                hipStream_t st)
{
    const int64_t n = s->dim;
    double *sc = nullptr;
    if (normalize) {
        // the partials come from a fixed grid of at most kRedGrid blocks, so any
        // dimension fits; checked anyway so a change of the grid cannot overrun it
        if (red_grid(n) + 4 > kScratchDoubles) {
            set_error("start vector: " + std::to_string(red_grid(n)) + " partial sums exceed the " +
                      std::to_string(kScratchDoubles - 4) + " of the static scratch");
            return HUB_ERR_RANGE;
        }
        HUB_TRY(scratch_on_current_device(&sc));
    }
    HUB_TRY(launch_start_vector(dtype, seed, out, n, st));
    HUB_TRY(k0_project(s, dtype, out, st));
    if (normalize) {
        // every partial and the norm are written before they are read: nothing to clear
        HUB_TRY(launch_dot(dtype, out, out, n, sc + 4, sc, 1, st));
        HUB_TRY(launch_convert(dtype, out, dtype, out, n, sc, 1, st));
    }
    return HUB_OK;
}

}  // namespace hub
