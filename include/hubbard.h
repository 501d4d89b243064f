/*
 * hubbard.h -- C ABI of libhubbard, an MI355X (gfx950) library for exact
 * diagonalisation of the one-band Hubbard model in one (N_up, N_dn) sector.
 *
 * Method: Sharma & Ahsan, "Organization of the Hilbert Space for Exact
 * Diagonalization of Hubbard Model" (arXiv:1307.7542).  The sector Hamiltonian
 * is never assembled.  It is applied as the Kronecker sum of Sec. IV A,
 *
 *     H = I_dn (x) H_up  +  H_dn (x) I_up  +  D,
 *     Y = H_up V + V H_dn^T + D o V,
 *
 * where V is the count_up x count_dn state matrix obtained from a sector vector
 * by the column-major reshape of Sec. IV A (element (a, b) at a + b*count_up,
 * the 0-based form of Eq. (count2)), H_up / H_dn are the one-spin hopping
 * matrices of Sec. IV A, and D is the diagonal (on-site repulsion, Sec. III B,
 * plus on-site energies).
 *
 * Conventions
 *   - Sites are 0-based.  Site i of a one-spin state is bit i of a 32-bit
 *     occupation integer (Sec. II; M <= 32).
 *   - A one-spin basis is the list of occupation integers with N set bits in
 *     ascending order (what Algorithm I of Appendix A produces); the index of a
 *     state is its 0-based position in that list.
 *   - Bond (i, j) with amplitude t contributes -t (c+_i c_j + c+_j c_i) for each
 *     spin (Eq. count1); the matrix element between two one-spin states is
 *     -t * esign, esign = (-1)^(occupied sites strictly between i and j)
 *     (Sec. III A).  Up operators are ordered before down operators (Sec. II),
 *     so no sign couples the two spins and H is exactly the Kronecker sum.
 *   - Vectors passed as device pointers hold count_up * count_dn elements of the
 *     stated dtype, column-major as above.  Element alignment is required;
 *     16-byte alignment (any fresh allocation) lets the product use its
 *     16-byte-access kernels, otherwise it takes slower one-row kernels.  The
 *     caller owns them.
 *
 * Errors: every entry point returns a hub_status; none aborts or throws.
 * hub_last_error() gives a thread-local message for the last failure.
 *
 * Threading: a sector is immutable after creation; concurrent hub_matvec calls
 * on one sector from different streams are safe.  hub_ground_state allocates
 * its own workspace per call.
 */
#ifndef HUBBARD_H
#define HUBBARD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hub_status;
#define HUB_OK 0
#define HUB_ERR_INVALID_ARG 1   /* null pointer, bad bond, non-finite parameter, aliasing */
#define HUB_ERR_RANGE 2         /* M outside 1..32, N outside 0..M, size overflow */
#define HUB_ERR_OOM 3           /* device or host allocation failed */
#define HUB_ERR_DEVICE 4        /* HIP runtime error */
#define HUB_ERR_NOT_CONVERGED 5 /* Lanczos hit max_iter; best estimate still returned */
#define HUB_ERR_UNSUPPORTED 6   /* option combination not supported */

/* Arithmetic type of vectors and of the matrix-vector product. */
#define HUB_F64 0
#define HUB_F32 1

#define HUB_SPIN_UP 0
#define HUB_SPIN_DN 1

/*
 * Model: Eq. (count1) with per-bond amplitudes t_ij, per-site U_i and on-site
 * energies eps_i (Sec. VIII uses U on the impurity only):
 *     H = -sum_b t_b sum_s (c+_{i_b s} c_{j_b s} + h.c.)
 *         + sum_i U_i n_{i up} n_{i dn} + sum_i eps_i (n_{i up} + n_{i dn}).
 * Bonds are canonicalised to (min, max); repeated bonds are merged by adding
 * their t in input order (FP64), keeping the first occurrence's position.
 * All arrays are host memory owned by the caller and copied by create.
 */
typedef struct hub_model {
    int32_t n_sites;       /* M, 1..32 */
    int32_t n_bonds;       /* >= 0 */
    const int32_t *bond_i; /* n_bonds site indices in 0..M-1 */
    const int32_t *bond_j; /* n_bonds site indices, bond_j[b] != bond_i[b] */
    const double *t;       /* n_bonds finite amplitudes */
    const double *U;       /* M finite on-site repulsions (NULL = all zero) */
    const double *eps;     /* M finite on-site energies (NULL = all zero) */
} hub_model;

typedef struct hub_sector hub_sector; /* opaque; lives on the device current at creation */

/*
 * Build the sector (N_up, N_dn) of `model` on the current HIP device (Sec. II,
 * Sec. III, Sec. IV A): both one-spin bases (combinadic unrank, equivalent to
 * Algorithm I), the hopping matrices H_up and H_dn in CSR (combinadic rank of
 * the hopped state, esign of Sec. III A, columns ascending in each row), and the
 * per-state on-site energy sums.  When N_up == N_dn the two spins share one set
 * of tables (Sec. X: identical matrices for S^z = 0).  Synchronous.
 * Errors: RANGE (M, N), INVALID_ARG (bonds, non-finite values, out == NULL),
 * OOM, DEVICE.
 */
hub_status hub_sector_create(const hub_model *model, int32_t n_up, int32_t n_dn, hub_sector **out);

/* Free all device and host memory of the sector.  NULL is a no-op. */
void hub_sector_destroy(hub_sector *sec);

/* count_sigma = C(M, N_sigma) (Eq. count3) and dim = count_up * count_dn. */
hub_status hub_sector_dims(const hub_sector *sec, int64_t *count_up, int64_t *count_dn, int64_t *dim);

/* Number of canonical bonds after merging, and the merged list (host arrays of
 * that length; any pointer may be NULL). */
hub_status hub_sector_bonds(const hub_sector *sec, int32_t *n_bonds, int32_t *bond_i, int32_t *bond_j,
                            double *t);

/* Copy the ascending one-spin basis of `spin` (count_spin entries) to host memory. */
hub_status hub_basis(const hub_sector *sec, int32_t spin, uint64_t *host_out);

/*
 * Rank (0-based basis index) of n arbitrary occupation integers of `spin`,
 * computed on the device by the combinadic sum (equivalent to locating the
 * state in the Algorithm I list).  Integers that are not states of this spin
 * sector (wrong popcount, bits at or above M) give -1.  Host in, host out.
 */
hub_status hub_rank(const hub_sector *sec, int32_t spin, const uint64_t *host_x, int64_t n, int64_t *host_out);

/* Stored entries of H_spin (= 2 |bonds| C(M-2, N-1) for M > 2, 0 < N < M, Sec. IV A). */
hub_status hub_hopping_nnz(const hub_sector *sec, int32_t spin, int64_t *nnz);

/*
 * Copy H_spin (Sec. IV A) in CSR to host memory: row_ptr (count+1), col (nnz,
 * ascending within a row), val (nnz, -t_b * esign), bond_id (nnz, index of the
 * canonical bond that produced the entry).  Any of col/val/bond_id may be NULL.
 */
hub_status hub_hopping_csr(const hub_sector *sec, int32_t spin, int64_t *row_ptr, int32_t *col, double *val,
                           int32_t *bond_id);

/*
 * Write the diagonal D of H (on-site repulsion, Sec. III B, plus on-site
 * energies) as a dim-long device vector of `dtype`.  Asynchronous on `stream`
 * (a hipStream_t, NULL = default stream).  For tests; the matrix-vector
 * product computes D on the fly and never stores it.
 */
hub_status hub_diagonal(const hub_sector *sec, int32_t dtype, void *dev_out, void *stream);

/*
 * Start vector: x_k = -1 + 2 u_k, u_k = (SplitMix64 output for state
 * seed + (k+1) * 0x9E3779B97F4A7C15) >> 11, times 2^-53 (Steele, Lea & Flood
 * 2014, counter-based), k the 0-based column-major index; scaled to unit FP64
 * norm when `normalize` is non-zero.  dim elements of `dtype` on the device.
 */
hub_status hub_start_vector(const hub_sector *sec, int32_t dtype, uint64_t seed, int32_t normalize,
                            void *dev_out, void *stream);

/*
 * hub_start_vector for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same bits as hub_start_vector, with the norm's partial
 * sums kept in a static device array of 1028 doubles (8 KB per device, held
 * until the process ends) instead of a buffer allocated per call, and no
 * synchronisation (asynchronous on `stream`).  The array's size does not depend
 * on the dimension (the norm is summed over a fixed grid of at most 1024
 * blocks); RANGE if that ever failed to hold.  Every call on a device shares
 * the array, so calls that overlap on one device (other streams or threads)
 * race: serialise them.
 */
hub_status hub_start_vector_noalloc(const hub_sector *sec, int32_t dtype, uint64_t seed, int32_t normalize,
                                    void *dev_out, void *stream);

/*
 * y = H x as the Kronecker sum Y = H_up X + X H_dn^T + D o X (Sec. IV A), in
 * `dtype` arithmetic (FP32 accumulates in FP32).  dev_x and dev_y are dim-long
 * device vectors; they must not overlap (INVALID_ARG).  Asynchronous on
 * `stream`, except that the first product of each dtype for a sector
 * structure (lattice and particle numbers) on a device may first time the
 * tile shapes on dev_x / dev_y (several launches, writing dev_y) and wait for
 * them; the chosen shape is kept for the process and does not change the
 * result.
 */
hub_status hub_matvec(const hub_sector *sec, int32_t dtype, const void *dev_x, void *dev_y, void *stream);

/*
 * Product schedule: which kernel applies the Kronecker sum of Sec. IV A and
 * with what tile shape.  Every schedule computes each element of y with the
 * same operations in the same order (diagonal, H_up entries in column order,
 * H_dn entries in column order, one fused multiply-add each), so the choice
 * never changes a result.
 *
 *   HUB_SCHED_COLUMNS  whole columns of V staged in LDS, four rows per lane
 *                      (count_up % 4 == 0);
 *   HUB_SCHED_CHUNKED  columns staged in LDS in chunks of chunk_rows rows, the
 *                      output rows held in registers (columns larger than the
 *                      LDS);
 *   HUB_SCHED_ROWS     one row per lane (count_up % 4 != 0, unaligned vectors);
 *   HUB_SCHED_CSR      CSR rows from global memory (no compact entries).
 *
 * By default the first product of each dtype on a sector structure times the
 * candidate shapes and keeps the fastest (hub_matvec); hub_get_schedule
 * reports it.  hub_set_schedule forces one, for tests and measurement (NULL:
 * back to the tuned one); it returns INVALID_ARG for a shape the sector cannot
 * run.  A forced schedule also applies to the products inside
 * hub_ground_state, whose Lanczos update is fused into the COLUMNS or CHUNKED
 * product unless no_fused_update is set (the fused update forms the same
 * values and partial sums in both, so a solve does not depend on the choice).
 */
#define HUB_SCHED_AUTO 0
#define HUB_SCHED_COLUMNS 1
#define HUB_SCHED_CHUNKED 2
#define HUB_SCHED_ROWS 3
#define HUB_SCHED_CSR 4

typedef struct hub_schedule {
    int32_t family;          /* HUB_SCHED_* (AUTO in hub_get_schedule: not chosen yet) */
    int32_t tile_cols;       /* COLUMNS: 1..3; CHUNKED: 1, 2 or 4 columns per workgroup */
    int32_t block;           /* COLUMNS: 512 or 1024 lanes per workgroup (CHUNKED: 1024) */
    int32_t order;           /* COLUMNS: 1 = XCD-contiguous tiles, 0 = launch order */
    int32_t quads_per_lane;  /* CHUNKED: 4 or 8 (a work item covers 4096 * quads_per_lane rows);
                                tile_cols * quads_per_lane <= 16 (FP32) or 8 (FP64) */
    int32_t chunk_rows;      /* CHUNKED: rows per staged chunk (0 = as many as fit; multiple of 4) */
    int32_t no_fused_update; /* 1: hub_ground_state keeps its Lanczos update out of the product */
    float ms;                /* tuned: time of one product in milliseconds; 0 when forced */
} hub_schedule;

hub_status hub_set_schedule(hub_sector *sec, int32_t dtype, const hub_schedule *sched);
/* fused = 1: the schedule of the product fused with the Lanczos update */
hub_status hub_get_schedule(const hub_sector *sec, int32_t dtype, int32_t fused, hub_schedule *out);

/*
 * Lanczos ground state (Sec. IV; the paper uses the plain three-term
 * recurrence without reorthogonalisation, Sec. V).
 *
 *   vec_dtype = HUB_F64: vectors, products and scalars in FP64.
 *   vec_dtype = HUB_F32: vectors and products in FP32; alpha, beta, the
 *                        reorthogonalisation coefficients, the tridiagonal
 *                        eigenproblem and the optional refinement in FP64.
 *   reorth = 0: plain recurrence; psi by a second pass over the same
 *               recurrence with the stored alpha/beta.
 *   reorth = 1: full classical Gram-Schmidt against all stored Lanczos
 *               vectors, repeated in the same step when the first pass kept
 *               less than 1/sqrt(2) of the norm (needs max_iter vectors of
 *               memory); psi from the stored vectors.
 *   reorth = 2: partial reorthogonalisation (Simon 1984): the same passes, run
 *               only at the steps where the omega recurrence estimates that
 *               some |<v_j, v_{k+1}>| reached sqrt(eps) of the stored precision
 *               (and at the step after), which keeps the basis semi-orthogonal;
 *               vectors stored as for reorth = 1.
 *   refine = 1: with psi promoted to FP64, an FP64 product gives the Rayleigh
 *               quotient (info.e0_refined, returned as *e0) and the true
 *               residual ||H psi - E psi|| (info.true_residual).
 * Convergence: Ritz residual beta_{k+1} |y_k| <= tol |theta| (tested every
 * check_every steps), or an invariant subspace (breakdown).
 * dev_psi: NULL or a dim-long FP64 device vector receiving the unit-norm
 * ground state with its largest-magnitude entry positive (requires
 * want_vector).  dev_start: NULL (use `seed`) or a dim-long FP64 device start
 * vector (normalised internally).  Synchronous with respect to `stream`.
 * Returns NOT_CONVERGED (with the best estimate written) when max_iter is hit,
 * and OOM, before allocating anything, when the vectors it needs (three, or
 * max_iter + 2 with reorth = 1, plus FP64 psi and refinement buffers) exceed
 * the free device memory (hipMemGetInfo).
 */
typedef struct hub_lanczos_opts {
    int32_t max_iter;      /* default 400 when <= 0 */
    double tol;            /* default 1e-12 (F64) / 1e-7 (F32) when <= 0 */
    uint64_t seed;         /* start-vector seed */
    const void *dev_start; /* optional FP64 start vector */
    int32_t vec_dtype;     /* HUB_F64 or HUB_F32 */
    int32_t reorth;        /* 0 plain, 1 full */
    int32_t want_vector;   /* compute psi */
    int32_t refine;        /* FP64 Rayleigh quotient and residual (needs want_vector) */
    int32_t check_every;   /* host convergence test period; default 1 when <= 0 */
    int32_t time_kernels;  /* > 0: HIP events around every time_kernels-th product launch */
    double e0_target;      /* reference energy for seconds_to_target (used when e0_target_rel > 0) */
    double e0_target_rel;  /* record the first check with |theta - e0_target| <= rel |e0_target| */
    int32_t orth_check;    /* reorth > 0: measure max |Q^T Q - I| of the stored basis (info.orth_loss) */
    int32_t batch_no_graph; /* hub_batch_ground_state only: 1 launches every step's kernels eagerly
                               instead of replaying the captured step graphs (same kernels, same order,
                               same results); ignored by hub_ground_state */
} hub_lanczos_opts;

typedef struct hub_lanczos_info {
    int32_t iters;          /* Lanczos steps taken (dimension of T) */
    int32_t converged;      /* 1 if the Ritz residual test or breakdown stopped it */
    int32_t breakdown;      /* 1 if an invariant subspace was found */
    int32_t matvec_count;   /* products of the Lanczos passes (refinement not counted) */
    double e0_ritz;         /* lowest Ritz value at stop */
    double e0_refined;      /* FP64 Rayleigh quotient of psi (refine), else e0_ritz */
    double residual;        /* Ritz residual estimate at stop */
    double true_residual;   /* ||H psi - E psi||_2 in FP64 (refine), else -1 */
    double seconds;         /* wall time of the call */
    double seconds_to_e0;   /* wall time until the Ritz test passed */
    double matvec_ms;       /* summed event time of the timed products (time_kernels) */
    int64_t matvec_bytes;   /* algorithmic bytes of one product: 2 dim s + tables */
    int32_t iters_to_target; /* steps when the lowest Ritz value first met the e0 target (-1: never / unused) */
    double seconds_to_target; /* wall time from entry until then (-1: never / unused) */
    int32_t matvec_timed;   /* products whose time is in matvec_ms */
    int32_t reorth_steps;   /* steps that ran the Gram-Schmidt passes (reorth > 0) */
    double orth_loss;       /* orth_check: max |Q^T Q - I| over the stored basis (hub_gram), else -1 */
} hub_lanczos_info;

hub_status hub_ground_state(const hub_sector *sec, const hub_lanczos_opts *opts, double *e0, void *dev_psi,
                            void *stream, hub_lanczos_info *info);

/*
 * Bilinear forms of the parameter derivatives of H (H is linear in t, U, eps):
 *   dbond[b] = g^T (dH/dt_b) x    (canonical bond b, both spins),
 *   dU[i]    = sum_k n_{i up} n_{i dn}(k) g_k x_k,
 *   deps[i]  = sum_k (n_{i up} + n_{i dn})(k) g_k x_k,
 * for dim-long FP64 device vectors g and x.  With g = x = psi (unit norm) these
 * are the Hellmann-Feynman derivatives of the eigenvalue.  Host outputs of
 * length n_bonds (canonical) and M; any may be NULL.  Synchronous on `stream`.
 */
hub_status hub_param_bilinear(const hub_sector *sec, const void *dev_g, const void *dev_x, double *dbond,
                              double *dU, double *deps, void *stream);

/*
 * Batches of independent sectors, e.g. the impurity problems an exact-
 * diagonalisation DMFT solver diagonalises at every step (Sec. VIII).  One
 * product launch covers every sector of the batch (work items are column tiles
 * of all sectors); batch vectors are the concatenation of the sector vectors in
 * batch order (offsets from hub_batch_offsets).  The sectors are borrowed and
 * must outlive the batch.  The first product of each dtype times a few tile
 * shapes (columns per workgroup, workgroup size) on the batch itself and keeps
 * the fastest.  Errors of hub_batch_create: INVALID_ARG (NULL, count <= 0,
 * sectors on different devices), UNSUPPORTED (a sector whose FP64 up-spin
 * column does not fit in the LDS, or without 4-byte product entries), OOM.
 */
typedef struct hub_batch hub_batch;

hub_status hub_batch_create(const hub_sector *const *sectors, int32_t count, hub_batch **out);
void hub_batch_destroy(hub_batch *batch);

/* offsets[0..count]: start of each sector's slice in a batch vector; offsets[count] = total length. */
hub_status hub_batch_offsets(const hub_batch *batch, int64_t *offsets);

/* y = H x for every sector of the batch, one launch (after tuning).  Device
 * vectors of the total length, no overlap.  Asynchronous on `stream`. */
hub_status hub_batch_matvec(hub_batch *batch, int32_t dtype, const void *dev_x, void *dev_y, void *stream);

typedef struct hub_batch_info {
    int32_t steps;            /* lockstep Lanczos steps executed (max over sectors; includes the
                                 group run while the last convergence test was on the host) */
    int32_t graph_replays;    /* steps executed by replaying a captured step or group graph */
    int32_t rows_per_lane;    /* tuned product: rows each lane has in flight at once */
    int32_t block_size;       /* tuned workgroup size of the product */
    int32_t cols_per_lane;    /* tuned product: columns each lane forms from one H_up entry stream */
    double seconds;           /* wall time of the call */
    double tune_seconds;      /* part of it spent tuning (first call per dtype) */
} hub_batch_info;

/*
 * Lowest eigenvalue of every sector of the batch by the plain Lanczos
 * recurrence (Sec. IV) run in lockstep: per-sector alpha / beta in FP64 on the
 * device, converged sectors masked out, one step (and one group of check_every
 * steps, default 5) captured once as a HIP graph and replayed.  The test after a
 * group runs on the host while the GPU runs the next group, so a sector may
 * step one group past its convergence (those steps are not used).  opts as for
 * hub_ground_state except reorth (must be 0:
 * UNSUPPORTED) and dev_start (must be NULL: UNSUPPORTED); refine without
 * dev_psi is INVALID_ARG.
 * e0[count] receives the Ritz values (or FP64 Rayleigh quotients with refine),
 * iters[count] (may be NULL) the steps per sector.  dev_psi: NULL or an FP64
 * batch vector receiving the unit-norm ground states (sign as in
 * hub_ground_state).  Synchronous.  NOT_CONVERGED if any sector hit max_iter.
 */
hub_status hub_batch_ground_state(hub_batch *batch, const hub_lanczos_opts *opts, double *e0, int32_t *iters,
                                  void *dev_psi, void *stream, hub_batch_info *info);

/*
 * Translation symmetry, k = 0 (Sec. VI).  For a lattice invariant under the
 * cyclic relabelling site i -> i - shift (mod M) (every bond maps to a bond
 * with the same t; U and eps uniform; shift divides M; M / shift <= 32), the
 * sector's k = 0 block.  Translation T lowers every bit position of an
 * occupation integer by `shift`; with shift = 1 this is the convention of
 * Tables V and VI (representative = smallest integer of its cycle, 1001 one
 * translation from 0011).  Vectors of such a sector are laid out as
 * phi[i + b R] = sqrt(P_i) psi(R_i, b): R_i the up-spin representatives in
 * ascending order (hub_k0_layout), P_i their periods, b every down-spin basis
 * state in Algorithm I order, psi the full two-spin amplitude of the k = 0
 * state.  Euclidean products of phi equal the full-space ones.  The sector
 * then works with hub_sector_dims (dim = R * count_dn), hub_start_vector
 * (projected onto k = 0), hub_matvec and hub_ground_state; hub_diagonal,
 * hub_param_bilinear, batches and the Green's-function calls return
 * UNSUPPORTED.  INVALID_ARG if the model is not translation invariant.
 */
hub_status hub_sector_create_k0(const hub_model *model, int32_t n_up, int32_t n_dn, int32_t shift, hub_sector **out);

/* *n_reps = R; reps[R] (may be NULL) the up representatives (ascending),
 * periods[R] (may be NULL) their periods in units of the translation.
 * INVALID_ARG for a sector made without translation symmetry. */
hub_status hub_k0_layout(const hub_sector *sec, int64_t *n_reps, uint64_t *reps, int32_t *periods);

/*
 * Zero-temperature one-particle Green's function (Sec. VII A, the second
 * equation labelled count8):
 *   G_s(p, z) = <psi0| c_ps (z + E0 - H)^-1 c+_ps |psi0> + <psi0| c+_ps (z - E0 + H)^-1 c_ps |psi0>
 * for site p (0-based, bit p of the occupation integers) and spin s (0 up,
 * 1 down), at complex z (e.g. i w_n).  Operator ordering: all up creation
 * operators (ascending site) left of all down ones, as in the kets of Sec. II,
 * so c+_ps carries (-1)^(occupied spin-s sites below p), times (-1)^N_up for
 * s = down.
 */

/* y = c+_{site,spin} x (create != 0, dst has one more spin-`spin` particle) or
 * y = c_{site,spin} x (create == 0, one fewer) between two sectors of the same
 * lattice.  FP64 device vectors (x: src dim, y: dst dim, no overlap); every
 * element of y is written (exact sign flips and copies, zeros elsewhere).
 * INVALID_ARG if the sectors do not differ by exactly that particle or the
 * site / spin is out of range.  Synchronises `stream` before returning. */
hub_status hub_apply_fermion(const hub_sector *src, const hub_sector *dst, int32_t site, int32_t spin, int32_t create,
                             const void *dev_x, void *dev_y, void *stream);

/* Continued-fraction coefficients of <f|(w - H)^-1|f> = norm2 / (w - a0 - b1^2 / (w - a1 - ...)):
 * plain FP64 Lanczos (Sec. IV) from v0 = f / |f| (dev_f: FP64 device vector of
 * the sector, not modified) for min(max_steps, dim) steps or up to the first
 * breakdown.  Host outputs: alpha[0..max_steps] (a0..a_{m-1}, rest 0),
 * beta[0..max_steps] (beta[0] = 0, b1..b_{m-1}, rest 0), *norm2 = <f|f>,
 * *steps = m (0 when f = 0).  Synchronous. */
hub_status hub_lanczos_coefficients(const hub_sector *sec, const void *dev_f, int32_t max_steps, double *alpha,
                                    double *beta, double *norm2, int32_t *steps, void *stream);

/* out[i] = norm2 / (w_i - a0 - b1^2 / (w_i - a1 - ... / (w_i - a_{steps-1}))), complex w
 * as (re, im) arrays; 0 when steps == 0.  Host only. */
hub_status hub_continued_fraction(const double *alpha, const double *beta, int32_t steps, double norm2, int32_t nz,
                                  const double *w_re, const double *w_im, double *out_re, double *out_im);

typedef struct hub_gf_info {
    int32_t steps_particle;   /* Lanczos steps of the c+ part (0 if the N+1 sector is empty) */
    int32_t steps_hole;       /* Lanczos steps of the c part (0 if N = 0) */
    double norm2_particle;    /* <psi0| c c+ |psi0> */
    double norm2_hole;        /* <psi0| c+ c |psi0>; the two add up to <psi0|psi0> */
    double seconds;
} hub_gf_info;

/* G_s(p, z) at nz points from the ground state (e0, dev_psi: FP64 device vector
 * of `sec`, normalised) of `sec`.  Builds the (N_s + 1) and (N_s - 1) sectors
 * of the same lattice internally, applies c+ / c and runs
 * hub_lanczos_coefficients on each (max_steps each).  coef: NULL or
 * 4 * (max_steps + 1) doubles receiving alpha / beta of the particle part,
 * then alpha / beta of the hole part.  Synchronous. */
hub_status hub_greens_function(const hub_sector *sec, double e0, const void *dev_psi, int32_t site, int32_t spin,
                               int32_t max_steps, int32_t nz, const double *z_re, const double *z_im, double *g_re,
                               double *g_im, double *coef, hub_gf_info *info, void *stream);

/*
 * G = Q^T Q in FP64 for m n-long device vectors of `dtype` (their device
 * pointers listed in the host array dev_q): the dense Gram product of the
 * reorthogonalisation check, on the FP64 matrix cores (FP32 vectors are widened
 * exactly, so the products are exact and the sums FP64).  host_g receives the
 * m x m matrix row-major.  Synchronous on `stream`.  UNSUPPORTED for more than
 * 304 (FP64) or 624 (FP32) vectors.
 */
hub_status hub_gram(int32_t dtype, const void *const *dev_q, int32_t m, int64_t n, double *host_g, void *stream);

/* Algorithmic bytes of one product in `dtype`: read x, write y, plus the tables. */
hub_status hub_matvec_bytes(const hub_sector *sec, int32_t dtype, int64_t *bytes);

const char *hub_status_str(hub_status s);
const char *hub_last_error(void);
const char *hub_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HUBBARD_H */
