// Internal declarations shared by the libhubbard translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <deque>
#include <mutex>
#include <string>
#include <vector>

#include "hubbard.h"

namespace hub {

constexpr int kMaxSites = 32;
constexpr int kMaxBonds = 512;
constexpr int kBinomN = 33;  // binomial table C[n][k], 0 <= n, k <= 32

void set_error(const std::string &msg);

// Device tables of one spin sector (Sec. II: basis; Sec. IV A: H_sigma in CSR).
struct SpinTables {
    int N = 0;
    int64_t count = 0;     // C(M, N)
    int64_t nnz = 0;       // stored entries of H_sigma
    uint32_t *basis = nullptr;   // [count] ascending occupation integers
    int32_t *rp = nullptr;       // [count + 1] row pointers
    int32_t *col = nullptr;      // [nnz] column (basis index of the hopped state), ascending per row
    double *val64 = nullptr;     // [nnz] -t_b * esign
    float *val32 = nullptr;      // [nnz] FP32 copy of val64 (exact: a negated / rounded t)
    int32_t *bond = nullptr;     // [nnz] canonical bond id of the entry
    double *e64 = nullptr;       // [count] sum_i eps_i n_i (FP64, ascending i)
    float *e32 = nullptr;        // [count] FP32 copy
    int32_t max_row = 0;         // longest row of H_sigma
    // Sliced ELL copy of H_sigma for the product: rows in slices of 64 (one
    // wavefront), each slice padded to its longest row and stored entry-major,
    // so lane r of a wavefront reads entry k of row 64*s + r at
    // 64*sl_off[s] + 64*k + r (padding: column = the row itself, value 0).
    int64_t nslices = 0;
    int32_t *sl_off = nullptr;   // [nslices + 1] slice offsets in units of 64 entries
    int32_t *ell_col = nullptr;  // [64 sl_off[nslices]]
    float *ell_v32 = nullptr;
    double *ell_v64 = nullptr;
    uint2 *ell_pk32 = nullptr;   // packed {column, FP32 value bits}: one 8-byte load per entry
    uint4 *ell_pk64 = nullptr;   // packed {column, 0, FP64 value low, high}: one 16-byte load
    // Compact entries {column : 24 bits, code : 8 bits}, value = code_v[code] with
    // code = 2*bond + (esign < 0) and code 255 = padding (value 0).  Built when
    // count < 2^24 and the sector has at most 127 bonds.
    uint32_t *ell_c32 = nullptr;
    double *code_v64 = nullptr;  // [256]
    float *code_v32 = nullptr;   // [256]
};

// Translation symmetry, k = 0 (Sec. VI), in the layout phi[i + b R] =
// sqrt(P_i) psi(R_i, b): rows are the up representatives R_i (ascending), columns
// every down state b (basis order).  G lowers every bit position by `w`.
struct K0Tables {
    int w = 1;                  // translation step in sites
    int L = 0;                  // group order M / w
    int64_t R = 0;              // up representatives
    int max_q = 0;              // longest down cycle
    int64_t n_orb = 0;          // down cycles
    uint32_t *reps = nullptr;   // [R] up representatives
    int32_t *period = nullptr;  // [R] period P_i (in steps of G)
    double *rep_e64 = nullptr;  // [R] sum_i eps_i n_i of R_i
    float *rep_e32 = nullptr;
    int32_t *hop_rp = nullptr;  // [R + 1] up hops from each representative
    int32_t *hop_row = nullptr; // [nnz] row of the hopped state's representative
    int32_t *hop_s = nullptr;   // [nnz] translation of the hopped state w.r.t. it
    double *hop_c64 = nullptr;  // [nnz] -t esign * phase * sqrt(P_i / P_i')
    float *hop_c32 = nullptr;
    int64_t hop_nnz = 0;
    int32_t *orb_off = nullptr;   // [n_orb + 1] start of each down cycle in orb_cols
    int32_t *orb_cols = nullptr;  // [count_dn] member a of cycle j -> down basis index
    int32_t *orb_sign = nullptr;  // [count_dn] c_a with G^a |D_j> = c_a |member a>
    int32_t *orb_sigma = nullptr; // [n_orb] G^q |D_j> = sigma |D_j>
    int64_t n_short = 0;          // representatives with P_i < L
    int32_t *short_rows = nullptr;   // [n_short]
    int32_t *short_sigma = nullptr;  // [n_short] G^P_i |R_i> = sigma |R_i>
};

// Compact entries of H_sigma split by column chunk (for products whose staged
// data covers one chunk of columns at a time): chunk p holds, for every row,
// the entries whose column lies in [p rows, (p+1) rows) -- a contiguous
// sub-range of the sorted CSR row -- with columns relative to the chunk, in the
// sliced-ELL layout (slice offsets in units of 64 entries).
struct ChunkSet {
    int spin = 0;
    int rows = 0;               // columns per chunk
    int n = 0;                  // chunks
    int32_t *off = nullptr;     // [n * (nslices + 1)]
    int64_t *base = nullptr;    // [n] first entry of chunk p
    uint32_t *ell = nullptr;    // entries {column - p rows : 24, code : 8}
};

// Product schedule (see hub_schedule in hubbard.h): fam 0 = not chosen yet.
struct Sched {
    int fam = 0;
    int tb = 0, bs = 0, xc = 0;  // columns per workgroup, lanes, tile order
    int qpl = 0;                 // row-chunked: lane-quads per lane
    int crows = 0;               // row-chunked: rows per staged chunk
    int nofuse = 0;              // forced: keep the Lanczos update out of the product
    float ms = 0.f;
};

}  // namespace hub

struct hub_sector {
    int device = 0;
    int M = 0;
    int64_t dim = 0;
    // canonical bonds
    int nb = 0;
    std::vector<int32_t> bi, bj;
    std::vector<double> t;
    std::vector<double> U, eps;
    int uniformU = 1;
    double U0 = 0.0;
    uint32_t umask = 0;
    bool shared_spin = false;         // N_up == N_dn: spin[1] aliases spin[0]
    hub::SpinTables spin[2];
    uint64_t *d_binom = nullptr;      // [33 * 33]
    int32_t *d_bi = nullptr, *d_bj = nullptr;
    double *d_t = nullptr;
    double *d_eps = nullptr;          // [M]
    double *d_U64 = nullptr;          // [M] per-site U
    float *d_U32 = nullptr;           // [M]
    size_t lds_max = 65536;           // dynamic LDS a workgroup may request
    int cu_count = 256;
    std::vector<void *> owned;        // every device allocation, freed by destroy
    hub::K0Tables *k0 = nullptr;      // set for a translation-symmetric k = 0 sector
    // Product schedules per dtype (0: FP64, 1: FP32): the tuner's pick for the
    // plain product and for the product fused with the Lanczos update, or one
    // forced through hub_set_schedule; chunk tables built on first use.  The
    // sector is immutable to callers; these caches are guarded by `mu`.
    mutable std::mutex mu;
    mutable hub::Sched sched[2], sched_lz[2];
    mutable bool forced[2] = {false, false};
    mutable std::deque<hub::ChunkSet> chunks;  // stable addresses
};

namespace hub {

// ---- setup (setup.hip) -------------------------------------------------
hub_status build_spin_tables(hub_sector *s, int spin, int N, hipStream_t st);
// rp[0] = 0, rp[k + 1] = len[0] + ... + len[k] (temporaries owned by s)
hub_status scan_lengths(hub_sector *s, const int32_t *len, int64_t n, int32_t *rp, hipStream_t st);
// chunk tables of H_spin with `rows` columns per chunk (built once, then cached)
hub_status chunk_set(const hub_sector *s, int spin, int rows, const ChunkSet **out, hipStream_t st);
hub_status rank_device(const hub_sector *s, int spin, const uint64_t *dx, int64_t n, int64_t *dout,
                       hipStream_t st);

// ---- product (matvec.hip) ----------------------------------------------
hub_status launch_matvec(const hub_sector *s, int dtype, const void *x, void *y, hipStream_t st);
// Product fused with the first Lanczos update: w = H x - beta v_prev (v_prev may
// be NULL) and partial sums of <w, x> in apart (npart values, summed in order
// they give alpha).  unnorm: x and v_prev are the unnormalised vectors
// beta_k v_k and beta_{k-1} v_{k-1} (beta NULL at the first step, beta_prev
// NULL for beta_0 = 1), w = (H x) / beta_k - (beta_k / beta_{k-1}) v_prev and
// the partials sum to beta_k alpha_k.  Available when matvec_lz_available(s, dtype).
bool matvec_lz_available(const hub_sector *s, int dtype);
int64_t matvec_lz_partials(const hub_sector *s);
int64_t matvec_lz_workspace(const hub_sector *s);  // doubles of the apart buffer launch_matvec_lz needs
hub_status launch_matvec_lz(const hub_sector *s, int dtype, const void *x, void *w, const void *vprev,
                            const double *beta, double *apart, int64_t *npart, hipStream_t st,
                            const double *beta_prev = nullptr, int unnorm = 0);
// sum of np partials in a fixed order into *out (one block); sqrt_result: its square root
hub_status launch_sum(const double *partial, int64_t np, double *out, hipStream_t st, int sqrt_result = 0);
hub_status launch_diagonal(const hub_sector *s, int dtype, void *out, hipStream_t st);
int64_t matvec_bytes(const hub_sector *s, int dtype);
// force a product schedule (NULL: back to the tuned one); the schedule in use
// (fused: the one of the product fused with the Lanczos update)
hub_status set_schedule(const hub_sector *s, int dtype, const hub_schedule *h);
hub_status get_schedule(const hub_sector *s, int dtype, int fused, hub_schedule *h);

// ---- vectors (vec.hip) -------------------------------------------------
constexpr int kRedBlock = 256;
constexpr int kRedGrid = 1024;
int red_grid(int64_t n);
hub_status launch_start_vector(int dtype, uint64_t seed, void *out, int64_t n, hipStream_t st);
// hub_start_vector without allocation: the norm's partials in a static device array
hub_status start_vector_noalloc(const hub_sector *s, int dtype, uint64_t seed, int normalize, void *out,
                                hipStream_t st);
// partial FP64 reductions + final: result written to device double *out
hub_status launch_dot(int dtype, const void *x, const void *y, int64_t n, double *partial, double *out,
                      int sqrt_result, hipStream_t st);
hub_status launch_convert(int din, const void *x, int dout, void *y, int64_t n, const double *scale_dev,
                          int invert, hipStream_t st);
// alpha_out NULL: leave the red_grid(n) partials of alpha in partial, no final sum
hub_status launch_lz_a(int dtype, void *w, const void *vprev, const double *beta, const void *v, int64_t n,
                       double *partial, double *alpha_out, hipStream_t st);
// beta_div (may be NULL): v is the unnormalised beta_k v_k, subtract (alpha / beta_k) v
hub_status launch_lz_b(int dtype, void *w, const void *v, const double *alpha, int64_t n, double *partial,
                       double *beta_out, hipStream_t st, const double *beta_div = nullptr);
hub_status launch_lz_next(int dtype, const void *w, void *vnext, const double *beta, int64_t n,
                          hipStream_t st);
// launch_lz_b with alpha formed inside the kernel from np partials (the value
// launch_sum gives, also written to *alpha_out) and beta^2 partials left in
// partial[0 .. red_grid(n)); launch_lz_next with beta formed from those
// partials (written to *beta_out).  host_ab / host_step (device-visible pinned
// host memory, or NULL): also store *alpha_k at host_ab[k] and beta at
// host_ab[kmax + k + 1], then k + 1 at *host_step.
hub_status launch_lz_b_sum(int dtype, void *w, const void *v, const double *apart, int64_t np, double *alpha_out,
                          int64_t n, double *partial, hipStream_t st, const double *beta_k = nullptr,
                          int unnorm = 0);
// beta = sqrt(sum of the red_grid(n) partials) into *beta_out, published like launch_lz_next_sum (one block)
hub_status launch_beta_pub(const double *partial, int64_t n, double *beta_out, hipStream_t st, double *host_ab,
                           int *host_step, const double *alpha_k, int k, int kmax);
hub_status launch_lz_next_sum(int dtype, const void *w, void *vnext, const double *partial, double *beta_out,
                              int64_t n, hipStream_t st, double *host_ab = nullptr, int *host_step = nullptr,
                              const double *alpha_k = nullptr, int k = 0, int kmax = 0);
hub_status launch_lz_replay(int dtype, void *w, const void *vprev, const double *beta, const void *v,
                            const double *alpha, int64_t n, hipStream_t st);
// psi (= 0 if first) += ycoef[0] * v, or ycoef[0] / div[0] * v when div is given
hub_status launch_psi_acc(int dtype, double *psi, const void *v, const double *ycoef, int64_t n, int first,
                          hipStream_t st, const double *div = nullptr);
// classical Gram-Schmidt pass against the k stored vectors (skipped when *skip);
// npart (or NULL): gram_norm_parts(n) partials of the new ||w||^2, left
// unchanged by a skipped pass
hub_status launch_gram(int dtype, const void *const *dQ, int k, void *w, int64_t n, double *partial,
                       double *coef, hipStream_t st, const int *skip, double *npart = nullptr);
int gram_norm_parts(int64_t n);
hub_status launch_dgks_flag(const double *before, const double *after, int *flag, hipStream_t st);
// partial reorthogonalisation: omega recurrence and pass flags (state: int[4], see vec.hip)
hub_status launch_pro_omega(const double *alpha, const double *beta, const double *beta_t, const double *om_prev,
                            const double *om_cur, double *om_next, int k, double eps, int *state, hipStream_t st);
hub_status launch_pro_flag2(const double *before, const double *after, int *state, hipStream_t st);
hub_status launch_pro_beta(const int *state, const double *beta_t, double *beta, hipStream_t st);
// G = Q^T Q (FP64, ld x ld with ld >= 16 ceil(m / 16), both triangles) of m
// device vectors (device pointer array dq) on the FP64 matrix cores; synchronous
hub_status gram_mfma(int dtype, const void *const *dq, int m, int64_t n, double *dG, int ld, hipStream_t st);
hub_status launch_psi_from_basis(int dtype, const void *const *dQ, int k, const double *ycoef, double *psi,
                                 int64_t n, hipStream_t st);
hub_status launch_normalize_sign(double *psi, int64_t n, double *partial, double *scal, hipStream_t st);
hub_status launch_residual(const double *hpsi, const double *psi, const double *e, int64_t n, double *partial,
                           double *out, hipStream_t st);

// ---- adjoint (adjoint.hip) ---------------------------------------------
hub_status param_bilinear(const hub_sector *s, const double *g, const double *x, double *dbond, double *dU,
                          double *deps, hipStream_t st);

// ---- translation symmetry (translation.hip) ------------------------------
// H x for any sector: the k = 0 product for translation sectors, else launch_matvec.
hub_status apply_h(const hub_sector *s, int dtype, const void *x, void *y, hipStream_t st);
// Project a vector of a k = 0 sector onto its consistent subspace (identity otherwise).
hub_status k0_project(const hub_sector *s, int dtype, void *x, hipStream_t st);

// ---- Lanczos (lanczos.cpp) ---------------------------------------------
double tri_lowest(const double *a, const double *b, int m, std::vector<double> &y);
hub_status lanczos_coefficients(const hub_sector *s, const double *f, int max_steps, double *alpha, double *beta,
                                double *norm2, int32_t *steps, hipStream_t st);
hub_status ground_state(const hub_sector *s, const hub_lanczos_opts *o, double *e0_out, void *dev_psi,
                        hipStream_t st, hub_lanczos_info *info);

}  // namespace hub

#define HUB_HIP(call)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) {                                                                 \
            hub::set_error(std::string(#call) + ": " + hipGetErrorString(e_));                  \
            return (e_ == hipErrorOutOfMemory || e_ == hipErrorMemoryAllocation) ? HUB_ERR_OOM \
                                                                                 : HUB_ERR_DEVICE; \
        }                                                                                       \
    } while (0)

#define HUB_TRY(call)                   \
    do {                                \
        hub_status s_ = (call);         \
        if (s_ != HUB_OK) return s_;    \
    } while (0)
