/*
 * CPU oracle for the pJDS sparse matrix-vector product -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may load this
 * code.  It is deliberately plain and slow: every function is the definition it cites,
 * written out with straightforward loops, in binary64, compiled without floating-point
 * contraction (-ffp-contract=off) so that each product and each sum is rounded on its own.
 * It shares no code, header or table with the GPU library.
 *
 * Citations are to Kreutzer et al., "Sparse matrix-vector multiplication on GPGPU
 * clusters: a new storage format and a scalable implementation" (arXiv:1112.5588).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- y = A x, the plain definition ------------------------------------------------
 * The operation every storage format in Sect. 2.1 computes: y_i = sum_k val[k] * x[col[k]]
 * over the stored entries k of row i, taken in stored (CSR) order, one rounding per
 * product and one per sum.  Empty rows give 0. */
void oracle_csr_spmv(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                     const double *val, const double *x, double *y)
{
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            double p = val[k] * x[col[k]];
            s = s + p;
        }
        y[i] = s;
    }
}

/* Same, for single-precision matrix values: each value is widened to binary64 (exactly)
 * and the product is formed in binary64, so the oracle itself adds no single-precision
 * rounding. */
void oracle_csr_spmv_f32val(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                            const float *val, const double *x, double *y)
{
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            double p = (double)val[k] * x[col[k]];
            s = s + p;
        }
        y[i] = s;
    }
}

/* Many right-hand sides: column v of Y is A times column v of X.  X and Y are row-major
 * with k columns (X[c*k + v]).  Written column by column, straight from that definition. */
void oracle_csr_spmmv(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                      const double *val, int32_t k, const double *X, double *Y)
{
    for (int32_t v = 0; v < k; ++v)
        for (int64_t i = 0; i < n_rows; ++i) {
            double s = 0.0;
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                double p = val[e] * X[(int64_t)col[e] * k + v];
                s = s + p;
            }
            Y[i * (int64_t)k + v] = s;
        }
}

/* ---- pJDS construction (Sect. 2.1, "sort" and "pad" steps; Listing 2) ----------------
 *
 * Step "sort": rows are ordered by their number of non-zeros, longest first.  Rows of equal
 * length keep their original relative order (the paper leaves ties open; this order makes
 * the permutation unique).  With a sort window w < n_rows the rows are sorted only inside
 * consecutive windows of w original rows (a window must hold whole blocks, so w is a
 * multiple of the block height).
 *
 * Step "pad": blocks of b_r consecutive sorted rows are padded to the longest row of the
 * block.  The row count is padded to a multiple of b_r with empty rows, which sort last.
 *
 * Storage: entry j of sorted row i lives at
 *   JD layout (Listing 2):  col_start[j] + i, where column j holds every row of every block
 *                           whose longest row exceeds j (needs a global sort, so that those
 *                           blocks come first);
 *   block layout:           block_start[b] + j*b_r + (i mod b_r), b = i / b_r, each block
 *                           stored as its own b_r x M_b column-major tile;
 *   block layout, T lanes:  T consecutive slots per row and step, the sliced ELLR-T idea
 *                           that the outlook (Sect. 4) names: entry j of sorted row i sits in
 *                           step s = j / T of its block, at block_start[b] + s*(b_r*T)
 *                           + (i mod b_r)*T + (j mod T).  A block holds ceil(M_b / T) steps.
 *                           T = 1 is the block layout above.
 * Padding slots hold value 0 and column 0.  The result row i of the permuted product is
 * original row perm[i].
 */

typedef struct { int64_t len; int64_t row; } oracle_key;

static int by_len_desc_then_row(const void *a, const void *b)
{
    const oracle_key *p = (const oracle_key *)a, *q = (const oracle_key *)b;
    if (p->len != q->len) return p->len > q->len ? -1 : 1;
    if (p->row != q->row) return p->row < q->row ? -1 : 1;
    return 0;
}

/* Fills perm[n_rows] (perm[new] = old) and row_len[n_pad] (length of sorted row, 0 for
 * the padding rows).  Returns n_pad, or -1 on invalid arguments. */
int64_t oracle_pjds_sort(int64_t n_rows, const int64_t *row_ptr, int64_t b_r, int64_t window,
                         int32_t *perm, int32_t *row_len)
{
    if (b_r < 1 || n_rows < 0) return -1;
    if (window <= 0 || window >= n_rows) window = n_rows > 0 ? n_rows : 1;
    else if (window % b_r != 0) return -1;
    int64_t n_pad = (n_rows + b_r - 1) / b_r * b_r;
    oracle_key *keys = (oracle_key *)malloc(sizeof(oracle_key) * (size_t)(n_rows > 0 ? n_rows : 1));
    if (!keys) return -1;
    for (int64_t i = 0; i < n_rows; ++i) {
        keys[i].len = row_ptr[i + 1] - row_ptr[i];
        keys[i].row = i;
    }
    for (int64_t w0 = 0; w0 < n_rows; w0 += window) {
        int64_t w1 = w0 + window < n_rows ? w0 + window : n_rows;
        qsort(keys + w0, (size_t)(w1 - w0), sizeof(oracle_key), by_len_desc_then_row);
    }
    for (int64_t i = 0; i < n_rows; ++i) {
        perm[i] = (int32_t)keys[i].row;
        row_len[i] = (int32_t)keys[i].len;
    }
    for (int64_t i = n_rows; i < n_pad; ++i) row_len[i] = 0;
    free(keys);
    return n_pad;
}

/* Longest row of each block: block_max[b] = max over the b_r sorted rows of block b. */
void oracle_pjds_block_max(int64_t n_pad, int64_t b_r, const int32_t *row_len, int64_t *block_max)
{
    for (int64_t b = 0; b < n_pad / b_r; ++b) {
        int64_t m = 0;
        for (int64_t r = 0; r < b_r; ++r)
            if (row_len[b * b_r + r] > m) m = row_len[b * b_r + r];
        block_max[b] = m;
    }
}

/* JD layout offsets (Listing 2's col_start): col_start[0] = 0 and
 * col_start[j+1] = col_start[j] + (number of sorted rows whose block is padded beyond j).
 * n_cols_jd = longest row; col_start has n_cols_jd + 1 entries, the last being the
 * stored-entry count. */
void oracle_pjds_col_start(int64_t n_blocks, int64_t b_r, const int64_t *block_max,
                           int64_t n_cols_jd, int64_t *col_start)
{
    col_start[0] = 0;
    for (int64_t j = 0; j < n_cols_jd; ++j) {
        int64_t height = 0;
        for (int64_t b = 0; b < n_blocks; ++b)
            if (block_max[b] > j) height += b_r;
        col_start[j + 1] = col_start[j] + height;
    }
}

/* Block layout offsets with T lanes per row: block_start[b+1] = block_start[b] +
 * b_r * T * ceil(block_max[b] / T)  (T = 1: b_r * block_max[b]). */
void oracle_pjds_block_start(int64_t n_blocks, int64_t b_r, int64_t lanes, const int64_t *block_max,
                             int64_t *block_start)
{
    block_start[0] = 0;
    for (int64_t b = 0; b < n_blocks; ++b) {
        int64_t steps = (block_max[b] + lanes - 1) / lanes;
        block_start[b + 1] = block_start[b] + b_r * lanes * steps;
    }
}

/* Where entry j of sorted row i is stored (layout 0 = JD, 1 = block with `lanes` lanes). */
static int64_t oracle_slot(int32_t layout, int64_t b_r, int64_t lanes, const int64_t *offsets,
                           int64_t i, int64_t j)
{
    if (layout == 0) return offsets[j] + i;
    return offsets[i / b_r] + (j / lanes) * (b_r * lanes) + (i % b_r) * lanes + j % lanes;
}

/* Fill the stored arrays (nnz_stored entries each).  layout 0 = JD (offsets = col_start),
 * 1 = block (offsets = block_start) with `lanes` lanes per row.  symmetric != 0 renumbers
 * columns into the permuted basis: col_p = invperm[col] (square matrices only). */
void oracle_pjds_fill(int64_t n_rows, int64_t b_r, int64_t lanes, int32_t layout, int32_t symmetric,
                      const int64_t *row_ptr, const int32_t *col, const double *val,
                      const int32_t *perm, const int64_t *offsets, int64_t nnz_stored,
                      int32_t *col_p, double *val_p)
{
    int32_t *invperm = NULL;
    if (symmetric) {
        invperm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_rows > 0 ? n_rows : 1));
        for (int64_t i = 0; i < n_rows; ++i) invperm[perm[i]] = (int32_t)i;
    }
    for (int64_t a = 0; a < nnz_stored; ++a) { col_p[a] = 0; val_p[a] = 0.0; }
    for (int64_t i = 0; i < n_rows; ++i) {
        int64_t src = perm[i];
        int64_t len = row_ptr[src + 1] - row_ptr[src];
        for (int64_t j = 0; j < len; ++j) {
            int64_t a = oracle_slot(layout, b_r, lanes, offsets, i, j);
            int32_t c = col[row_ptr[src] + j];
            col_p[a] = symmetric ? invperm[c] : c;
            val_p[a] = val[row_ptr[src] + j];
        }
    }
    free(invperm);
}

/* y_p = (pJDS matrix) x with the oracle's own arrays, Listing 2 read literally: for sorted
 * row i, sum over j < row_len[i] of val_p * x[col_p] in j order.  Used only to tie the
 * oracle's construction to the plain product. */
void oracle_pjds_spmv(int64_t n_rows, int64_t b_r, int64_t lanes, int32_t layout, const int32_t *row_len,
                      const int64_t *offsets, const int32_t *col_p, const double *val_p,
                      const double *x, double *y_perm)
{
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < row_len[i]; ++j) {
            int64_t a = oracle_slot(layout, b_r, lanes, offsets, i, j);
            double p = val_p[a] * x[col_p[a]];
            s = s + p;
        }
        y_perm[i] = s;
    }
}

/* ---- ELLPACK-R (Sect. 2.1, Listing 1) ----------------------------------------------
 * Rows keep their order; non-zeros are shifted left and the n_pad x max_len rectangle is
 * stored column by column: entry j of row i at j*n_pad + i, n_pad = rows rounded up to a
 * multiple of pad_to.  rowmax[i] = length of row i (0 for padding rows). */
void oracle_ellr_fill(int64_t n_rows, int64_t n_pad, int64_t max_len, const int64_t *row_ptr,
                      const int32_t *col, const double *val, int32_t *rowmax,
                      int32_t *col_e, double *val_e)
{
    for (int64_t a = 0; a < n_pad * max_len; ++a) { col_e[a] = 0; val_e[a] = 0.0; }
    for (int64_t i = 0; i < n_pad; ++i) rowmax[i] = 0;
    for (int64_t i = 0; i < n_rows; ++i) {
        int64_t len = row_ptr[i + 1] - row_ptr[i];
        rowmax[i] = (int32_t)len;
        for (int64_t j = 0; j < len; ++j) {
            col_e[j * n_pad + i] = col[row_ptr[i] + j];
            val_e[j * n_pad + i] = val[row_ptr[i] + j];
        }
    }
}
