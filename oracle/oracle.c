/*
 * Plain CPU oracle for the one-band Hubbard sector Hamiltonian.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the GPU library: it works in the two-spin basis of
 * Lin and Gubernatis, I = I_up + 2^M I_dn (Sec. II), and builds the *full*
 * sparse H row by row from the definition of the Hamiltonian, Eq. (count1),
 * generalised to per-bond t_ij, per-site U_i and on-site energies eps_i.
 *
 * Conventions (all stated in Sec. II):
 *   - site i (0-based) of spin up is bit i of I, of spin down bit M+i;
 *   - a basis ket is the product of creation operators in increasing bit order
 *     acting on the vacuum (all up operators first, then all down ones);
 *   - the hopping term -t (c+_a c_b + c+_b c_a) maps a ket with exactly one of
 *     a, b occupied to the ket with that electron moved, times (-1)^(number of
 *     occupied modes strictly between a and b) (Sec. III A, the esign rule);
 *   - the index of the hopped ket is found by binary search over the sorted
 *     two-spin keys (the two-spin path the paper times in Sec. V).
 *
 * Everything is FP64.  Rows are processed in parallel with OpenMP; within a row
 * the arithmetic order is fixed (diagonal, then bonds in list order, spin up
 * before spin down), so results do not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_BONDS 1024

/* ------------------------------------------------------------------------ */
/* Algorithm I (Appendix A): scan every integer from minrange = 2^N - 1 up to
 * maxrange = sum_{i=1..N} 2^(M-i), count its set bits one position at a time,
 * and keep the integers with exactly N of them.  The kept integers come out in
 * ascending order; their 1-based position is the index of Sec. II.  Returns the
 * count; writes the list to `out` when it is not NULL. */
int64_t orc_enumerate(int M, int N, uint64_t *out)
{
    if (M < 0 || M > 32 || N < 0 || N > M) return -1;
    uint64_t minrange = 0, maxrange = 0;
    for (int i = 1; i <= N; ++i) {
        minrange += (uint64_t)1 << (i - 1);
        maxrange += (uint64_t)1 << (M - i);
    }
    int64_t count = 0;
    for (uint64_t v = minrange; v <= maxrange; ++v) {
        int nbit = 0;
        for (int j = 0; j < M; ++j)
            if ((v >> j) & 1u) ++nbit;
        if (nbit == N) {
            if (out) out[count] = v;
            ++count;
        }
    }
    return count;
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* Two-spin keys I = I_up + 2^M I_dn for every pair of one-spin states (Sec. II),
 * sorted ascending.  The position of a key in this list is its basis index. */
int orc_two_spin_keys(int M, const uint64_t *up, int64_t cu, const uint64_t *dn, int64_t cd,
                      uint64_t *keys)
{
    if (M < 1 || 2 * M > 64) return -1;
    int64_t n = 0;
    for (int64_t i = 0; i < cu; ++i)
        for (int64_t j = 0; j < cd; ++j)
            keys[n++] = up[i] + (dn[j] << M);
    qsort(keys, (size_t)n, sizeof(uint64_t), cmp_u64);
    return 0;
}

/* Key source: either an explicit sorted array, or the same sorted sequence
 * produced from the two ascending one-spin lists (key(n) with the down state as
 * the major and the up state as the minor key).  Both give keys in ascending
 * order; the second avoids storing dim keys for very large sectors. */
typedef struct {
    int M;
    const uint64_t *keys;  /* explicit sorted keys, or NULL */
    const uint64_t *up;
    const uint64_t *dn;
    int64_t cu, cd, dim;
} keyset;

static inline uint64_t key_at(const keyset *ks, int64_t n)
{
    if (ks->keys) return ks->keys[n];
    return ks->up[n % ks->cu] + (ks->dn[n / ks->cu] << ks->M);
}

static int64_t find_key(const keyset *ks, uint64_t key)
{
    int64_t lo = 0, hi = ks->dim - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        uint64_t k = key_at(ks, mid);
        if (k == key) return mid;
        if (k < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

typedef struct {
    int M, nb;
    const int32_t *bi, *bj;
    const double *t, *U, *eps;
} model;

/* Diagonal of Eq. (count1) with per-site U and on-site energies:
 * sum_i U_i n_i,up n_i,dn + sum_i eps_i (n_i,up + n_i,dn), one site at a time. */
static double diag_elem(const model *m, uint64_t I)
{
    double d = 0.0;
    for (int i = 0; i < m->M; ++i) {
        int nu = (int)((I >> i) & 1u);
        int nd = (int)((I >> (m->M + i)) & 1u);
        d += m->U[i] * (double)(nu * nd);
        if (m->eps) d += m->eps[i] * (double)(nu + nd);
    }
    return d;
}

/* One hopping term of bond `b`, spin `s` (0 up, 1 down) applied to key I.
 * Returns 1 and the target key and sign when exactly one end is occupied. */
static int hop(const model *m, int b, int s, uint64_t I, uint64_t *J, double *sign)
{
    int p = m->bi[b] + s * m->M;
    int q = m->bj[b] + s * m->M;
    if (p > q) { int tmp = p; p = q; q = tmp; }
    int np = (int)((I >> p) & 1u), nq = (int)((I >> q) & 1u);
    if (np == nq) return 0;
    int between = 0;
    for (int k = p + 1; k < q; ++k)
        if ((I >> k) & 1u) ++between;
    *J = I ^ (((uint64_t)1 << p) | ((uint64_t)1 << q));
    *sign = (between & 1) ? -1.0 : 1.0;
    return 1;
}

typedef struct { int64_t col; double val; } entry;

/* All entries of row `r`: the diagonal, then every hop; sorted by column with
 * equal columns merged (repeated bonds add up).  Returns the entry count. */
static int row_entries(const model *m, const keyset *ks, int64_t r, entry *e, int *bad)
{
    uint64_t I = key_at(ks, r);
    int n = 0;
    e[n].col = r;
    e[n].val = diag_elem(m, I);
    ++n;
    for (int s = 0; s < 2; ++s) {
        for (int b = 0; b < m->nb; ++b) {
            uint64_t J;
            double sg;
            if (!hop(m, b, s, I, &J, &sg)) continue;
            int64_t c = find_key(ks, J);
            if (c < 0) { *bad = 1; continue; }
            e[n].col = c;
            e[n].val = -m->t[b] * sg;
            ++n;
        }
    }
    /* insertion sort by column, stable, then merge equal columns */
    for (int i = 1; i < n; ++i) {
        entry x = e[i];
        int j = i - 1;
        while (j >= 0 && e[j].col > x.col) { e[j + 1] = e[j]; --j; }
        e[j + 1] = x;
    }
    int w = 0;
    for (int i = 0; i < n; ++i) {
        if (w > 0 && e[w - 1].col == e[i].col) e[w - 1].val += e[i].val;
        else e[w++] = e[i];
    }
    return w;
}

static int check_model(const model *m)
{
    if (m->M < 1 || 2 * m->M > 64 || m->nb < 0 || m->nb > ORC_MAX_BONDS) return -1;
    for (int b = 0; b < m->nb; ++b) {
        if (m->bi[b] < 0 || m->bi[b] >= m->M || m->bj[b] < 0 || m->bj[b] >= m->M) return -1;
        if (m->bi[b] == m->bj[b]) return -1;
    }
    return 0;
}

/* Full sparse H in CSR (diagonal included), rows in two-spin key order.
 * Pass 1 (col == NULL): fills row_ptr only.  Pass 2: fills col/val.
 * keys may be NULL, in which case up/dn/cu/cd define the key sequence. */
int orc_build_csr(int M, int nb, const int32_t *bi, const int32_t *bj, const double *t,
                  const double *U, const double *eps,
                  const uint64_t *keys, const uint64_t *up, int64_t cu, const uint64_t *dn, int64_t cd,
                  int64_t *row_ptr, int32_t *col, double *val)
{
    model m = {M, nb, bi, bj, t, U, eps};
    if (check_model(&m)) return -1;
    keyset ks = {M, keys, up, dn, cu, cd, cu * cd};
    int bad = 0;
    if (!col) {
        row_ptr[0] = 0;
        int64_t *len = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ks.dim > 0 ? ks.dim : 1));
        if (!len) return -2;
#pragma omp parallel
        {
            entry e[2 * ORC_MAX_BONDS + 1];
            int lbad = 0;
#pragma omp for schedule(dynamic, 4096)
            for (int64_t r = 0; r < ks.dim; ++r) len[r] = row_entries(&m, &ks, r, e, &lbad);
            if (lbad) {
#pragma omp atomic write
                bad = 1;
            }
        }
        for (int64_t r = 0; r < ks.dim; ++r) row_ptr[r + 1] = row_ptr[r] + len[r];
        free(len);
    } else {
#pragma omp parallel
        {
            entry e[2 * ORC_MAX_BONDS + 1];
            int lbad = 0;
#pragma omp for schedule(dynamic, 4096)
            for (int64_t r = 0; r < ks.dim; ++r) {
                int n = row_entries(&m, &ks, r, e, &lbad);
                int64_t o = row_ptr[r];
                for (int k = 0; k < n; ++k) {
                    col[o + k] = (int32_t)e[k].col;
                    val[o + k] = e[k].val;
                }
            }
            if (lbad) {
#pragma omp atomic write
                bad = 1;
            }
        }
    }
    return bad ? -3 : 0;
}

/* y = H x with the CSR above; each row summed in column order. */
void orc_spmv(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
              const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        double s = 0.0;
        for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) s += val[k] * x[col[k]];
        y[r] = s;
    }
}

/* Start-vector entries x_k = -1 + 2 u_k, u_k = top 53 bits of the SplitMix64
 * output for state seed + (k+1) * 0x9E3779B97F4A7C15, scaled by 2^-53
 * (Steele, Lea & Flood 2014; counter-based use of the published mixer). */
static inline double start_entry(uint64_t seed, int64_t k)
{
    uint64_t z = seed + (uint64_t)(k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    return -1.0 + 2.0 * u;
}

void orc_start_vector(uint64_t seed, int64_t k0, int64_t n, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) out[k] = start_entry(seed, k0 + k);
}

/* Matrix-free rows: y[i] = sum_J H[rows[i], J] x[J] for the listed rows only.
 * x is either a full vector, or NULL, in which case x_J is the (unnormalised)
 * start-vector entry for index J under `seed`. */
int orc_apply_rows(int M, int nb, const int32_t *bi, const int32_t *bj, const double *t,
                   const double *U, const double *eps,
                   const uint64_t *keys, const uint64_t *up, int64_t cu, const uint64_t *dn, int64_t cd,
                   const double *x, uint64_t seed, const int64_t *rows, int64_t nrows, double *y)
{
    model m = {M, nb, bi, bj, t, U, eps};
    if (check_model(&m)) return -1;
    keyset ks = {M, keys, up, dn, cu, cd, cu * cd};
    int bad = 0;
#pragma omp parallel
    {
        entry e[2 * ORC_MAX_BONDS + 1];
        int lbad = 0;
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < nrows; ++i) {
            int n = row_entries(&m, &ks, rows[i], e, &lbad);
            double s = 0.0;
            for (int k = 0; k < n; ++k)
                s += e[k].val * (x ? x[e[k].col] : start_entry(seed, e[k].col));
            y[i] = s;
        }
        if (lbad) {
#pragma omp atomic write
            bad = 1;
        }
    }
    return bad ? -3 : 0;
}

/* Bilinear forms of the parameter derivatives of H (H is linear in t, U, eps):
 *   dbond[b] = g^T (dH/dt_b) x = sum over rows I and hops of bond b of
 *              (-sign) g_I x_J, both spins;
 *   dU[i]    = sum_I n_i,up n_i,dn g_I x_I;
 *   deps[i]  = sum_I (n_i,up + n_i,dn) g_I x_I.
 * With g = x = psi (normalised) these are the Hellmann-Feynman derivatives of
 * the eigenvalue.  Per-row partial sums are accumulated in row order. */
int orc_param_bilinear(int M, int nb, const int32_t *bi, const int32_t *bj,
                       const uint64_t *keys, const uint64_t *up, int64_t cu, const uint64_t *dn, int64_t cd,
                       const double *g, const double *x, double *dbond, double *dU, double *deps)
{
    model m = {M, nb, bi, bj, NULL, NULL, NULL};
    if (check_model(&m)) return -1;
    keyset ks = {M, keys, up, dn, cu, cd, cu * cd};
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    double *acc = (double *)calloc((size_t)nthreads * (size_t)(nb + 2 * M), sizeof(double));
    if (!acc) return -2;
    int bad = 0;
    /* Static row blocks so the per-thread partials are reproducible, then
     * reduced over threads in thread order. */
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *a = acc + (size_t)tid * (size_t)(nb + 2 * M);
        int lbad = 0;
#pragma omp for schedule(static)
        for (int64_t r = 0; r < ks.dim; ++r) {
            uint64_t I = key_at(&ks, r);
            double gx = g[r] * x[r];
            for (int i = 0; i < M; ++i) {
                int nu = (int)((I >> i) & 1u);
                int nd = (int)((I >> (M + i)) & 1u);
                a[nb + i] += (double)(nu * nd) * gx;
                a[nb + M + i] += (double)(nu + nd) * gx;
            }
            for (int s = 0; s < 2; ++s) {
                for (int b = 0; b < nb; ++b) {
                    uint64_t J;
                    double sg;
                    if (!hop(&m, b, s, I, &J, &sg)) continue;
                    int64_t c = find_key(&ks, J);
                    if (c < 0) { lbad = 1; continue; }
                    a[b] += -sg * g[r] * x[c];
                }
            }
        }
        if (lbad) {
#pragma omp atomic write
            bad = 1;
        }
    }
    for (int b = 0; b < nb; ++b) dbond[b] = 0.0;
    for (int i = 0; i < M; ++i) { dU[i] = 0.0; deps[i] = 0.0; }
    for (int th = 0; th < nthreads; ++th) {
        const double *a = acc + (size_t)th * (size_t)(nb + 2 * M);
        for (int b = 0; b < nb; ++b) dbond[b] += a[b];
        for (int i = 0; i < M; ++i) { dU[i] += a[nb + i]; deps[i] += a[nb + M + i]; }
    }
    free(acc);
    return bad ? -3 : 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
