/* Exercise the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (TEST INFRASTRUCTURE ONLY; compiled and run by tests/test_oracle_sanitize.py
 * with gcc on the host).  Random small CSR matrices, including empty rows,
 * rows == 0, nnz == 0 and heights 1..32, go through CSR -> CMRS (unsorted and
 * sorted), CMRS -> CSR and the CSR product; the round trip must reproduce the
 * input, and invalid input must be rejected.  Exit status 0 = all good. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int32_t ora_num_strips(int32_t rows, int32_t height);
int32_t ora_bits_for_height(int32_t height);
void ora_csr_spmv(int32_t rows, const int32_t *row_ptr, const int32_t *col_ind, const double *val,
                  const double *x, double *y);
void ora_csr_absmv(int32_t rows, const int32_t *row_ptr, const int32_t *col_ind, const double *val,
                   const double *x, double *y);
int32_t ora_csr_to_cmrs(int32_t rows, int32_t cols, int32_t nnz, const int32_t *row_ptr, const int32_t *col_ind,
                        const void *val, int32_t elem_size, int32_t height, int32_t bits, int32_t sorted,
                        int32_t *strip_ptr, uint32_t *word, void *val_out);
int32_t ora_cmrs_to_csr(int32_t rows, int32_t nnz, int32_t height, int32_t bits, const int32_t *strip_ptr,
                        const uint32_t *word, const void *val, int32_t elem_size, int32_t *row_ptr,
                        int32_t *col_ind, void *val_out);

static uint64_t state = 88172645463325252ull;
static uint32_t rnd(void) {  /* xorshift64 */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (uint32_t)(state >> 16);
}

static int one_case(int rows, int cols, int max_row, int height) {
    /* Row lengths up to max_row, columns strictly ascending inside [0, cols). */
    int32_t *rp = malloc(sizeof(int32_t) * (size_t)(rows + 1));
    int32_t *ci = malloc(sizeof(int32_t) * ((size_t)rows * (size_t)(max_row + 1) + 1));
    double *v = malloc(sizeof(double) * ((size_t)rows * (size_t)(max_row + 1) + 1));
    int nnz = 0;
    rp[0] = 0;
    for (int i = 0; i < rows; i++) {
        int want = max_row ? (int)(rnd() % (uint32_t)(max_row + 1)) : 0;
        int c = (int)(rnd() % 3u);
        for (int t = 0; t < want && c < cols; t++) {
            ci[nnz] = c;
            v[nnz] = (double)(int)(rnd() % 9u) - 4.0;
            nnz++;
            c += 1 + (int)(rnd() % 3u);
        }
        rp[i + 1] = nnz;
    }
    double *x = malloc(sizeof(double) * (size_t)cols), *y = malloc(sizeof(double) * (size_t)(rows + 1));
    for (int j = 0; j < cols; j++) x[j] = (double)(int)(rnd() % 5u) - 2.0;
    ora_csr_spmv(rows, rp, ci, v, x, y);
    ora_csr_absmv(rows, rp, ci, v, x, y);
    int strips = ora_num_strips(rows, height), bits = ora_bits_for_height(height);
    int32_t *sp = malloc(sizeof(int32_t) * (size_t)(strips + 1));
    uint32_t *w = malloc(sizeof(uint32_t) * (size_t)(nnz + 1));
    double *vo = malloc(sizeof(double) * (size_t)(nnz + 1));
    int32_t *rp2 = malloc(sizeof(int32_t) * (size_t)(rows + 1));
    int32_t *ci2 = malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    double *v2 = malloc(sizeof(double) * (size_t)(nnz + 1));
    int bad = 0;
    for (int sorted = 0; sorted < 2; sorted++) {
        if (ora_csr_to_cmrs(rows, cols, nnz, rp, ci, v, 8, height, bits, sorted, sp, w, vo) != 0) bad = 1;
        if (ora_cmrs_to_csr(rows, nnz, height, bits, sp, w, vo, 8, rp2, ci2, v2) != 0) bad = 1;
        if (memcmp(rp, rp2, sizeof(int32_t) * (size_t)(rows + 1)) != 0) bad = 1;
        /* Unsorted: exact round trip.  Sorted: rows come back column-sorted,
         * which the ascending input already is (duplicates keep their order). */
        if (nnz && memcmp(ci, ci2, sizeof(int32_t) * (size_t)nnz) != 0) bad = 1;
        if (nnz && memcmp(v, v2, sizeof(double) * (size_t)nnz) != 0) bad = 1;
    }
    if (nnz > 0) {  /* an out-of-range column must be rejected */
        int32_t keep = ci[0];
        ci[0] = cols;
        if (ora_csr_to_cmrs(rows, cols, nnz, rp, ci, v, 8, height, bits, 1, sp, w, vo) != -1) bad = 1;
        ci[0] = keep;
    }
    free(rp); free(ci); free(v); free(x); free(y); free(sp); free(w); free(vo); free(rp2); free(ci2); free(v2);
    return bad;
}

int main(void) {
    static const int heights[] = {1, 2, 3, 4, 5, 8, 16, 17, 31, 32};
    int bad = 0, cases = 0;
    for (int t = 0; t < 400; t++) {
        int rows = (int)(rnd() % 300u), cols = 1 + (int)(rnd() % 200u), max_row = (int)(rnd() % 40u);
        if (t % 50 == 0) rows = 0;
        if (t % 37 == 0) max_row = 0;
        int h = heights[t % 10];
        bad |= one_case(rows, cols, max_row, h);
        cases++;
    }
    printf("%d cases, %s\n", cases, bad ? "FAILED" : "ok");
    return bad;
}
