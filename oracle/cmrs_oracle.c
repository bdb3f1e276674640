/*
 * CMRS oracle — plain, slow, obviously correct CPU reference.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant with the GPU
 * library: every rule below is restated here from the paper
 * (Koza, Matyka, Szkoda, Miroslaw, "Compressed Multi-Row Storage Format for
 * Sparse Matrices on Graphics Processing Units", arXiv:1203.2946).
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no -ffast-math, no FMA
 * contraction), so every multiply and every add rounds separately in IEEE
 * binary64.
 *
 * Functions (serial except ora_csr_spmv_par; no blocking, no reordering):
 *   ora_csr_spmv       y = A x over CRS, Sec. 2.1 and 2.3
 *   ora_csr_spmv_par   the same product, rows split into nnz-balanced ranges
 *                      over OpenMP threads (CPU-baseline timing only)
 *   ora_csr_absmv      (|A||x|)_i, the scale of the componentwise error bound
 *   ora_csr_to_dense   COO/CRS scatter into a dense array (duplicates add)
 *   ora_dense_matvec   row-major dense matvec (brute force for tiny cases)
 *   ora_csr_to_cmrs    CRS -> CMRS by the definition of Sec. 3, packed words
 *                      of Sec. 4, optional in-strip reorder of Sec. 4 (4th
 *                      optimisation)
 *   ora_cmrs_to_csr    CMRS -> CRS (the inverse conversion of Sec. 3 / 7)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of strips: ceil(rows / height), Sec. 3. */
int32_t ora_num_strips(int32_t rows, int32_t height)
{
    if (height <= 0 || rows < 0) return -1;
    return (int32_t)(((int64_t)rows + height - 1) / height);
}

/* Width of the RowInStrip field packed into the low bits of a column word.
 * Sec. 4 stores RowInStrip in CMRS_BITS = 4 low bits and the column in the
 * remaining 28 (valid for height <= 16).  For larger heights the field must
 * grow to hold height-1, so: bits = max(4, ceil(log2(height))). */
int32_t ora_bits_for_height(int32_t height)
{
    if (height <= 0) return -1;
    int32_t b = 0;
    while ((1 << b) < height) b++;
    return b < 4 ? 4 : b;
}

/* y_i = sum_k Val[k] * x[ColInd[k]] over the CRS row i (Sec. 2.1: y = A x;
 * Sec. 2.3: the row's entries are Val[RowPtr[i] .. RowPtr[i+1]-1]).
 * The sum starts from +0.0 (Algorithm 1 zero-fills its buffer) and adds the
 * products in CRS order, each product and each add rounded separately. */
void ora_csr_spmv(int32_t rows, const int32_t *row_ptr, const int32_t *col_ind,
                  const double *val, const double *x, double *y)
{
    for (int32_t i = 0; i < rows; i++) {
        double s = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; k++) {
            double p = val[k] * x[col_ind[k]];
            s = s + p;
        }
        y[i] = s;
    }
}

/* The same product with the rows cut into nthreads contiguous ranges of
 * about nnz/nthreads entries each (range t starts at the first row whose
 * RowPtr reaches t*nnz/nthreads), one range per OpenMP thread.  Every row is
 * summed exactly as in ora_csr_spmv, so the result is identical bit for bit;
 * only the CPU-baseline timing uses it.  Without -fopenmp it runs serially.
 * Returns the number of threads that ran. */
int32_t ora_csr_spmv_par(int32_t rows, const int32_t *row_ptr, const int32_t *col_ind,
                         const double *val, const double *x, double *y, int32_t nthreads)
{
    if (nthreads < 1) nthreads = 1;
    int32_t used = 1;
    const int64_t nnz = rows > 0 ? (int64_t)row_ptr[rows] : 0;
#pragma omp parallel num_threads(nthreads)
    {
        int32_t t = 0, nt = 1;
#ifdef _OPENMP
        t = (int32_t)omp_get_thread_num();
        nt = (int32_t)omp_get_num_threads();
#pragma omp single
        used = nt;
#endif
        /* first row of range t: lower bound of t*nnz/nt in RowPtr */
        int32_t bounds[2];
        for (int32_t e = 0; e < 2; e++) {
            const int64_t target = nnz * (int64_t)(t + e) / nt;
            int32_t lo = 0, hi = rows;
            while (lo < hi) {
                const int32_t mid = lo + (hi - lo) / 2;
                if ((int64_t)row_ptr[mid] < target) lo = mid + 1; else hi = mid;
            }
            bounds[e] = (t + e == nt) ? rows : lo;
        }
        if (t == 0) bounds[0] = 0;
        for (int32_t i = bounds[0]; i < bounds[1]; i++) {
            double s = 0.0;
            for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; k++) {
                double p = val[k] * x[col_ind[k]];
                s = s + p;
            }
            y[i] = s;
        }
    }
    return used;
}

/* (|A||x|)_i = sum_k |Val[k]| * |x[ColInd[k]]|, the scale in the
 * componentwise error bound |y - y_ref|_i <= c * k_i * u * (|A||x|)_i. */
void ora_csr_absmv(int32_t rows, const int32_t *row_ptr, const int32_t *col_ind,
                   const double *val, const double *x, double *out)
{
    for (int32_t i = 0; i < rows; i++) {
        double s = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; k++)
            s = s + fabs(val[k]) * fabs(x[col_ind[k]]);
        out[i] = s;
    }
}

/* Scatter a CRS matrix into a dense row-major array; repeated (row, col)
 * entries add, as in the COO reading of Sec. 2.3. */
void ora_csr_to_dense(int32_t rows, int32_t cols, const int32_t *row_ptr,
                      const int32_t *col_ind, const double *val, double *dense)
{
    memset(dense, 0, sizeof(double) * (size_t)rows * (size_t)cols);
    for (int32_t i = 0; i < rows; i++)
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; k++)
            dense[(size_t)i * cols + col_ind[k]] += val[k];
}

/* y = A x for a dense row-major A: every column j in order, from +0.0. */
void ora_dense_matvec(int32_t rows, int32_t cols, const double *dense,
                      const double *x, double *y)
{
    for (int32_t i = 0; i < rows; i++) {
        double s = 0.0;
        for (int32_t j = 0; j < cols; j++) {
            double p = dense[(size_t)i * cols + j] * x[j];
            s = s + p;
        }
        y[i] = s;
    }
}

/* One entry of a strip while it is being reordered. */
typedef struct {
    int32_t col;   /* column index                      */
    int32_t ris;   /* RowInStrip = row mod height        */
    int32_t pos;   /* position in CRS order (tie-break)  */
} ora_item;

static int ora_item_cmp(const void *pa, const void *pb)
{
    const ora_item *a = (const ora_item *)pa, *b = (const ora_item *)pb;
    if (a->col != b->col) return a->col < b->col ? -1 : 1;
    if (a->ris != b->ris) return a->ris < b->ris ? -1 : 1;
    return a->pos < b->pos ? -1 : (a->pos > b->pos ? 1 : 0);
}

/* CRS -> CMRS (Sec. 3 and 4).
 *   StripPtr[j] = RowPtr[j*height] for j < strips, StripPtr[strips] = nnz;
 *   RowInStrip[k] = (row of entry k) mod height;
 *   packed word[k] = (ColInd[k] << bits) | RowInStrip[k]   (Sec. 4: the low
 *   CMRS_BITS hold RowInStrip, the upper bits the column).
 * Val is carried unchanged (elem_size bytes per entry, moved bit for bit).
 * With sorted != 0 each strip is reordered by column, ties broken by
 * RowInStrip (the worked h = 2 example of Sec. 4 puts row 2 before row 3 in
 * column 2), exact duplicates kept in CRS order.
 * Returns 0, or -1 on invalid arguments (out-of-range column, bad RowPtr). */
int32_t ora_csr_to_cmrs(int32_t rows, int32_t cols, int32_t nnz,
                        const int32_t *row_ptr, const int32_t *col_ind,
                        const void *val, int32_t elem_size,
                        int32_t height, int32_t bits, int32_t sorted,
                        int32_t *strip_ptr, uint32_t *word, void *val_out)
{
    int32_t strips = ora_num_strips(rows, height);
    if (strips < 0 || bits < 1 || bits > 31) return -1;
    if (row_ptr[0] != 0 || row_ptr[rows] != nnz) return -1;
    for (int32_t j = 0; j < strips; j++) strip_ptr[j] = row_ptr[j * height];
    strip_ptr[strips] = nnz;

    const unsigned char *vin = (const unsigned char *)val;
    unsigned char *vout = (unsigned char *)val_out;
    for (int32_t i = 0; i < rows; i++) {
        if (row_ptr[i + 1] < row_ptr[i]) return -1;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; k++) {
            int32_t c = col_ind[k];
            if (c < 0 || c >= cols) return -1;
            if ((uint64_t)c >= ((uint64_t)1 << (32 - bits))) return -1;
            uint32_t ris = (uint32_t)(i % height);
            word[k] = ((uint32_t)c << bits) | ris;
            memcpy(vout + (size_t)k * elem_size, vin + (size_t)k * elem_size, (size_t)elem_size);
        }
    }
    if (!sorted) return 0;

    /* In-strip reorder: the strip's entries, as (col, RowInStrip, CRS position),
     * sorted; Val and the packed word follow the permutation. */
    int32_t maxlen = 0;
    for (int32_t s = 0; s < strips; s++)
        if (strip_ptr[s + 1] - strip_ptr[s] > maxlen) maxlen = strip_ptr[s + 1] - strip_ptr[s];
    ora_item *items = (ora_item *)malloc(sizeof(ora_item) * (size_t)(maxlen > 0 ? maxlen : 1));
    unsigned char *tmpv = (unsigned char *)malloc((size_t)elem_size * (size_t)(maxlen > 0 ? maxlen : 1));
    uint32_t *tmpw = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(maxlen > 0 ? maxlen : 1));
    if (!items || !tmpv || !tmpw) { free(items); free(tmpv); free(tmpw); return -1; }
    for (int32_t s = 0; s < strips; s++) {
        int32_t a = strip_ptr[s], n = strip_ptr[s + 1] - a;
        for (int32_t t = 0; t < n; t++) {
            items[t].col = (int32_t)(word[a + t] >> bits);
            items[t].ris = (int32_t)(word[a + t] & (((uint32_t)1 << bits) - 1u));
            items[t].pos = t;
        }
        qsort(items, (size_t)n, sizeof(ora_item), ora_item_cmp);
        for (int32_t t = 0; t < n; t++) {
            tmpw[t] = word[a + items[t].pos];
            memcpy(tmpv + (size_t)t * elem_size, vout + (size_t)(a + items[t].pos) * elem_size, (size_t)elem_size);
        }
        memcpy(word + a, tmpw, sizeof(uint32_t) * (size_t)n);
        memcpy(vout + (size_t)a * elem_size, tmpv, (size_t)elem_size * (size_t)n);
    }
    free(items); free(tmpv); free(tmpw);
    return 0;
}

/* CMRS -> CRS (the inverse of Sec. 3).  The row of entry k of strip s is
 * s*height + (word[k] & (2^bits - 1)); the column is word[k] >> bits.
 * RowPtr comes from per-row counts; entries are placed row by row in the
 * order they appear in the CMRS arrays (a stable scatter by row).
 * Returns 0, or -1 when an entry names a row >= rows. */
int32_t ora_cmrs_to_csr(int32_t rows, int32_t nnz, int32_t height, int32_t bits,
                        const int32_t *strip_ptr, const uint32_t *word,
                        const void *val, int32_t elem_size,
                        int32_t *row_ptr, int32_t *col_ind, void *val_out)
{
    int32_t strips = ora_num_strips(rows, height);
    if (strips < 0 || bits < 1 || bits > 31) return -1;
    if (strip_ptr[0] != 0 || strip_ptr[strips] != nnz) return -1;
    uint32_t mask = ((uint32_t)1 << bits) - 1u;
    int32_t *next = (int32_t *)calloc((size_t)rows + 1, sizeof(int32_t));
    if (!next) return -1;
    for (int32_t i = 0; i <= rows; i++) row_ptr[i] = 0;
    for (int32_t s = 0; s < strips; s++) {
        for (int32_t k = strip_ptr[s]; k < strip_ptr[s + 1]; k++) {
            int64_t row = (int64_t)s * height + (int64_t)(word[k] & mask);
            if ((word[k] & mask) >= (uint32_t)height || row >= rows) { free(next); return -1; }
            row_ptr[row + 1] += 1;
        }
    }
    for (int32_t i = 0; i < rows; i++) row_ptr[i + 1] += row_ptr[i];
    for (int32_t i = 0; i < rows; i++) next[i] = row_ptr[i];
    const unsigned char *vin = (const unsigned char *)val;
    unsigned char *vout = (unsigned char *)val_out;
    for (int32_t s = 0; s < strips; s++) {
        for (int32_t k = strip_ptr[s]; k < strip_ptr[s + 1]; k++) {
            int32_t row = s * height + (int32_t)(word[k] & mask);
            int32_t p = next[row]++;
            col_ind[p] = (int32_t)(word[k] >> bits);
            memcpy(vout + (size_t)p * elem_size, vin + (size_t)k * elem_size, (size_t)elem_size);
        }
    }
    free(next);
    return 0;
}
