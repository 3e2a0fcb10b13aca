/*
 * CPU oracle: term-by-term row evaluation of a subspace Hamiltonian.
 *
 * Test infrastructure only (not product code).  Plain C with OpenMP over rows.
 *
 * For a row bit-string b_i and every input term, this code forms the column bit-string and
 * the matrix element <b_i|term|b_j> directly from the definitions (no grouping, no ladder
 * integers, no hashing), then finds j by binary search over the sorted subspace keys:
 *
 *  - qubit words (Methods, Qubit Hamiltonians; properties 1-3): the column flips the row at
 *    off-diagonal letters; the element is the product over listed qubits of the 2x2 entries
 *    <b_i[q]|W_q|b_j[q]>, taken from the caller's table of the seven alphabet matrices;
 *  - fermionic products (Methods, Fermionic Hamiltonians): the row form applies the adjoint
 *    operators to b_i in turn, each with the Jordan-Wigner parity sign
 *    (-1)^popcount(bits below the mode).
 *
 * Entry (i, j) is present iff j is in the subspace and at least one term with a nonzero
 * coefficient yields a nonzero element (values may cancel to 0.0); the diagonal entry is
 * always present.  Keys are [N][W] uint64, sorted ascending as big unsigned integers with
 * word W-1 most significant.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXW 64

typedef struct {
    int64_t col;
    int64_t seq; /* term number: equal columns are summed in ascending term order */
    double re, im;
} entry_t;

static int key_cmp(const uint64_t *a, const uint64_t *b, int W) {
    for (int w = W - 1; w >= 0; --w) {
        if (a[w] < b[w]) return -1;
        if (a[w] > b[w]) return 1;
    }
    return 0;
}

static int64_t find_key(const uint64_t *keys, int64_t N, int W, const uint64_t *q) {
    int64_t lo = 0, hi = N;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int c = key_cmp(keys + mid * W, q, W);
        if (c < 0)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo < N && key_cmp(keys + lo * W, q, W) == 0) return lo;
    return -1;
}

static int entry_cmp(const void *a, const void *b) {
    const entry_t *p = (const entry_t *)a, *q = (const entry_t *)b;
    if (p->col != q->col) return (p->col > q->col) - (p->col < q->col);
    return (p->seq > q->seq) - (p->seq < q->seq);
}

static inline int get_bit(const uint64_t *k, int q) { return (int)((k[q >> 6] >> (q & 63)) & 1u); }
static inline void flip_bit(uint64_t *k, int q) { k[q >> 6] ^= (uint64_t)1 << (q & 63); }

static int parity_below(const uint64_t *k, int q) {
    int c = 0;
    for (int w = 0; w < (q >> 6); ++w) c += __builtin_popcountll(k[w]);
    uint64_t part = k[q >> 6] & (((uint64_t)1 << (q & 63)) - 1);
    c += __builtin_popcountll(part);
    return c & 1;
}

/* One row.  Returns the number of distinct entries (diagonal included) written to `out`
 * (capacity T + 1), sorted by column. */
static int64_t eval_row(int W, int64_t N, const uint64_t *keys, int fermionic, int64_t T,
                        const int64_t *term_ptr, const int32_t *op_idx, const uint8_t *op_code,
                        const double *coef, const double *mats, int64_t row, entry_t *out) {
    const uint64_t *b = keys + row * W;
    uint64_t col[MAXW];
    int64_t n = 0;
    out[n].col = row;
    out[n].seq = -1;
    out[n].re = 0.0;
    out[n].im = 0.0;
    n++;
    for (int64_t t = 0; t < T; ++t) {
        double cre = coef[2 * t], cim = coef[2 * t + 1];
        if (cre == 0.0 && cim == 0.0) continue;
        memcpy(col, b, sizeof(uint64_t) * W);
        double fre = 1.0, fim = 0.0;
        int alive = 1;
        if (!fermionic) {
            for (int64_t k = term_ptr[t]; k < term_ptr[t + 1]; ++k) {
                int q = op_idx[k], code = op_code[k];
                int rb = get_bit(b, q);
                int cb = rb ^ (code > 2 ? 1 : 0);
                const double *m = mats + (((code * 2 + rb) * 2 + cb) * 2);
                double are = m[0], aim = m[1];
                if (are == 0.0 && aim == 0.0) {
                    alive = 0;
                    break;
                }
                double nre = fre * are - fim * aim, nim = fre * aim + fim * are;
                fre = nre;
                fim = nim;
                if (code > 2) flip_bit(col, q);
            }
        } else {
            /* <b|op_1...op_m = (op_m^+ ... op_1^+ |b>)^+ : apply op_1^+ first. */
            for (int64_t k = term_ptr[t]; k < term_ptr[t + 1]; ++k) {
                int q = op_idx[k], code = op_code[k];
                int adj_is_creator = (code == 5); /* f^+ is the adjoint of f (code 5) */
                int bit = get_bit(col, q);
                if (adj_is_creator ? bit : !bit) {
                    alive = 0;
                    break;
                }
                if (parity_below(col, q)) fre = -fre;
                flip_bit(col, q);
            }
        }
        if (!alive) continue;
        int64_t j = find_key(keys, N, W, col);
        if (j < 0) continue;
        double vre = cre * fre - cim * fim, vim = cre * fim + cim * fre;
        out[n].col = j;
        out[n].seq = t;
        out[n].re = vre;
        out[n].im = vim;
        n++;
    }
    qsort(out, (size_t)n, sizeof(entry_t), entry_cmp);
    /* merge equal columns (their values are summed in ascending-term order per column) */
    int64_t m = 0;
    for (int64_t a = 0; a < n; ++a) {
        if (m > 0 && out[m - 1].col == out[a].col) {
            out[m - 1].re += out[a].re;
            out[m - 1].im += out[a].im;
        } else {
            out[m++] = out[a];
        }
    }
    return m;
}

int qo_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Rows `rows[0..nrows)`: always writes row_nnz; when row_off != NULL also writes the sorted
 * entries of row r at [row_off[r], row_off[r] + row_nnz[r]). */
int qo_rows(int W, int64_t N, const uint64_t *keys, int fermionic, int64_t T, const int64_t *term_ptr,
            const int32_t *op_idx, const uint8_t *op_code, const double *coef, const double *mats,
            int64_t nrows, const int64_t *rows, int64_t *row_nnz, const int64_t *row_off, int64_t *cols,
            double *vals, int nthreads) {
    if (W < 1 || W > MAXW) return -1;
    int bad = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : qo_max_threads())
    {
        entry_t *buf = (entry_t *)malloc(sizeof(entry_t) * (size_t)(T + 1));
        if (!buf) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t r = 0; r < nrows; ++r) {
                int64_t m = eval_row(W, N, keys, fermionic, T, term_ptr, op_idx, op_code, coef, mats, rows[r], buf);
                row_nnz[r] = m;
                if (row_off) {
                    for (int64_t a = 0; a < m; ++a) {
                        cols[row_off[r] + a] = buf[a].col;
                        vals[2 * (row_off[r] + a)] = buf[a].re;
                        vals[2 * (row_off[r] + a) + 1] = buf[a].im;
                    }
                }
            }
            free(buf);
        }
    }
    return bad ? -2 : 0;
}

/* y[r][v] = sum_j H[rows[r], j] x[j][v] for complex x, y stored as (re, im) pairs. */
int qo_matvec(int W, int64_t N, const uint64_t *keys, int fermionic, int64_t T, const int64_t *term_ptr,
              const int32_t *op_idx, const uint8_t *op_code, const double *coef, const double *mats,
              int64_t nrows, const int64_t *rows, int nvec, const double *x, double *y, int nthreads) {
    if (W < 1 || W > MAXW) return -1;
    int bad = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : qo_max_threads())
    {
        entry_t *buf = (entry_t *)malloc(sizeof(entry_t) * (size_t)(T + 1));
        if (!buf) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t r = 0; r < nrows; ++r) {
                int64_t m = eval_row(W, N, keys, fermionic, T, term_ptr, op_idx, op_code, coef, mats, rows[r], buf);
                for (int v = 0; v < nvec; ++v) {
                    double are = 0.0, aim = 0.0;
                    for (int64_t a = 0; a < m; ++a) {
                        const double *xj = x + 2 * (buf[a].col * nvec + v);
                        are += buf[a].re * xj[0] - buf[a].im * xj[1];
                        aim += buf[a].re * xj[1] + buf[a].im * xj[0];
                    }
                    y[2 * (r * nvec + v)] = are;
                    y[2 * (r * nvec + v) + 1] = aim;
                }
            }
            free(buf);
        }
    }
    return bad ? -2 : 0;
}
