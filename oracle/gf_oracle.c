/*
 * Test infrastructure: the plain CPU oracle for echelonisation over GF(p).
 *
 * Only the test suite, the smoke check and the benchmark's cpu_baseline leg
 * may load this file's library.  The GPU library never links, includes or
 * calls it, and it calls nothing of the GPU library.
 *
 * What it computes (the problem statement of the paper, Section 2.2,
 * Remark 2.3 and Eq. (1), applied to the whole matrix as in Eq. (2)):
 * for A in F_p^{m x n} of rank r it returns the pivot columns gamma, the
 * selected rows rho (both ascending, |gamma| = |rho| = r), the reduced row
 * echelon form E (r x n, pivots equal to +1) and an invertible T (m x m)
 * with T * A = [E ; 0].  Rows of T are ordered: first the r pivot rows in
 * increasing pivot column, then the m - r non-selected rows in increasing
 * original index.
 *
 * The pivot rule is the paper's (Section 1): the pivot of a row is its
 * first non-zero entry, rows are taken in their original order, and no
 * other pivot search is done.  So row i is selected exactly when it is not
 * in the span of rows 0..i-1.
 *
 * Method: plain Gauss-Jordan on the augmented matrix W = [A | I_m], one row
 * at a time, keeping every pivot row fully reduced against all others.
 * Cost Theta(m * r * (n + m)) field operations.  No blocking, no reordering
 * and no shared code with the GPU path.  Field inverses come from Fermat's
 * little theorem a^(p-2), recomputed on every use (no tables).
 *
 * Entries are canonical residues in [0, p) stored one per byte, row-major.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORACLE_OK = 0, ORACLE_E_FIELD = 1, ORACLE_E_RANGE = 2, ORACLE_E_NOMEM = 3, ORACLE_E_ARG = 4 };

static int is_prime_u32(uint32_t p) {
    if (p < 2) return 0;
    for (uint32_t d = 2; d * d <= p; ++d)
        if (p % d == 0) return 0;
    return 1;
}

/* a^e mod p by square-and-multiply */
static uint32_t pow_mod(uint32_t a, uint32_t e, uint32_t p) {
    uint32_t r = 1 % p, b = a % p;
    while (e) {
        if (e & 1u) r = (r * b) % p;
        b = (b * b) % p;
        e >>= 1;
    }
    return r;
}

/* multiplicative inverse of a != 0 in GF(p), Fermat: a^(p-2) */
static uint32_t inv_mod(uint32_t a, uint32_t p) { return pow_mod(a, p - 2, p); }

/* dst <- dst + g * src (mod p) over len entries */
static void row_axpy(uint8_t* dst, const uint8_t* src, uint32_t g, uint32_t p, int64_t len) {
    for (int64_t k = 0; k < len; ++k)
        dst[k] = (uint8_t)((dst[k] + g * (uint32_t)src[k]) % p);
}

/* dst <- s * dst (mod p) */
static void row_scale(uint8_t* dst, uint32_t s, uint32_t p, int64_t len) {
    for (int64_t k = 0; k < len; ++k)
        dst[k] = (uint8_t)((s * (uint32_t)dst[k]) % p);
}

int oracle_check_field(uint32_t p) { return (p <= 251 && is_prime_u32(p)) ? ORACLE_OK : ORACLE_E_FIELD; }

/*
 * A: m x n, leading dimension lda (bytes).  Outputs (caller-allocated):
 *   rank_out  : r
 *   pivcols   : int64[min(m,n)], first r entries = gamma ascending
 *   selrows   : int64[min(m,n)], first r entries = rho ascending
 *   E         : m x n bytes (ld n); rows 0..r-1 hold the RREF, the rest zero
 *   T         : m x m bytes (ld m); row order as described in the header
 */
int oracle_echelon(const uint8_t* A, int64_t m, int64_t n, int64_t lda, uint32_t p,
                   int64_t* rank_out, int64_t* pivcols, int64_t* selrows,
                   uint8_t* E, uint8_t* T) {
    if (m < 0 || n < 0 || (m > 0 && n > 0 && lda < n)) return ORACLE_E_ARG;
    if (oracle_check_field(p) != ORACLE_OK) return ORACLE_E_FIELD;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            if (A[i * lda + j] >= p) return ORACLE_E_RANGE;

    const int64_t w = n + m;            /* width of the augmented row [A | I] */
    uint8_t* W = (uint8_t*)calloc((size_t)(m > 0 ? m : 1) * (size_t)(w > 0 ? w : 1), 1);
    int64_t* piv_col = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1)); /* pivot column of pivot t */
    int64_t* piv_row = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1)); /* row index of pivot t   */
    uint8_t* is_sel = (uint8_t*)calloc((size_t)(m > 0 ? m : 1), 1);
    if (!W || !piv_col || !piv_row || !is_sel) {
        free(W); free(piv_col); free(piv_row); free(is_sel);
        return ORACLE_E_NOMEM;
    }
    for (int64_t i = 0; i < m; ++i) {
        memcpy(W + i * w, A + i * lda, (size_t)n);
        W[i * w + n + i] = 1;
    }

    int64_t r = 0;
    for (int64_t i = 0; i < m; ++i) {
        uint8_t* row = W + i * w;
        /* reduce row i by every existing pivot row */
        for (int64_t t = 0; t < r; ++t) {
            uint32_t f = row[piv_col[t]];
            if (f) row_axpy(row, W + piv_row[t] * w, p - f, p, w);
        }
        /* first non-zero among the A columns */
        int64_t c = -1;
        for (int64_t j = 0; j < n; ++j)
            if (row[j]) { c = j; break; }
        if (c < 0) continue;                       /* not selected */
        row_scale(row, inv_mod(row[c], p), p, w);  /* pivot becomes 1 */
        /* keep earlier pivot rows reduced: clear column c in them */
        for (int64_t t = 0; t < r; ++t) {
            uint8_t* s = W + piv_row[t] * w;
            uint32_t g = s[c];
            if (g) row_axpy(s, row, p - g, p, w);
        }
        piv_col[r] = c;
        piv_row[r] = i;
        is_sel[i] = 1;
        ++r;
    }

    /* order pivots by column (insertion sort keeps it plain) */
    for (int64_t a = 1; a < r; ++a) {
        int64_t c = piv_col[a], rr = piv_row[a], b = a - 1;
        while (b >= 0 && piv_col[b] > c) { piv_col[b + 1] = piv_col[b]; piv_row[b + 1] = piv_row[b]; --b; }
        piv_col[b + 1] = c; piv_row[b + 1] = rr;
    }

    if (E) memset(E, 0, (size_t)(m * n));
    if (T) memset(T, 0, (size_t)(m * m));
    for (int64_t t = 0; t < r; ++t) {
        const uint8_t* row = W + piv_row[t] * w;
        if (E) memcpy(E + t * n, row, (size_t)n);
        if (T) memcpy(T + t * m, row + n, (size_t)m);
    }
    int64_t q = r;
    for (int64_t i = 0; i < m; ++i) {
        if (is_sel[i]) continue;
        if (T) memcpy(T + q * m, W + i * w + n, (size_t)m);
        ++q;
    }
    int64_t s = 0;
    for (int64_t i = 0; i < m; ++i)
        if (is_sel[i]) selrows[s++] = i;
    for (int64_t t = 0; t < r; ++t) pivcols[t] = piv_col[t];
    *rank_out = r;

    free(W); free(piv_col); free(piv_row); free(is_sel);
    return ORACLE_OK;
}

/* plain (A + B*C) mod p, A: a x d, B: a x b, C: b x d, all row-major dense (the MAD job, Section 4.1) */
int oracle_mad(const uint8_t* A, const uint8_t* B, const uint8_t* C, uint8_t* out,
               int64_t a, int64_t b, int64_t d, uint32_t p) {
    if (oracle_check_field(p) != ORACLE_OK) return ORACLE_E_FIELD;
    for (int64_t i = 0; i < a; ++i)
        for (int64_t j = 0; j < d; ++j) {
            uint64_t acc = A ? A[i * d + j] : 0;
            for (int64_t k = 0; k < b; ++k) acc += (uint64_t)B[i * b + k] * C[k * d + j];
            out[i * d + j] = (uint8_t)(acc % p);
        }
    return ORACLE_OK;
}

/*
 * GF(2) with rows packed in 64-bit words (bit b of word w = column 64 w + b):
 * the same plain Gauss-Jordan on [A | I_m] as oracle_echelon with p = 2, where
 * a row operation is a word-wise XOR and every non-zero pivot is already 1.
 *   A        : m rows of ldw words (ldw >= ceil(n / 64)); bits past column
 *              n - 1 must be zero
 *   pivcols, selrows : as oracle_echelon
 *   E        : r rows of ceil(n / 64) words (the RREF, packed)
 *   T        : m rows of ceil(m / 64) words (rows ordered as oracle_echelon's)
 */
int oracle_echelon_gf2(const uint64_t* A, int64_t m, int64_t n, int64_t ldw,
                       int64_t* rank_out, int64_t* pivcols, int64_t* selrows,
                       uint64_t* E, uint64_t* T) {
    const int64_t wn = (n + 63) / 64, wm = (m + 63) / 64, w = wn + wm;   /* words of [A | I] */
    if (m < 0 || n < 0 || (m > 0 && n > 0 && ldw < wn)) return ORACLE_E_ARG;
    for (int64_t i = 0; i < m && n % 64; ++i)
        if (A[i * ldw + n / 64] >> (n % 64)) return ORACLE_E_RANGE;
    uint64_t* W = (uint64_t*)calloc((size_t)(m > 0 ? m : 1) * (size_t)(w > 0 ? w : 1), sizeof(uint64_t));
    int64_t* piv_col = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int64_t* piv_row = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    uint8_t* is_sel = (uint8_t*)calloc((size_t)(m > 0 ? m : 1), 1);
    if (!W || !piv_col || !piv_row || !is_sel) {
        free(W); free(piv_col); free(piv_row); free(is_sel);
        return ORACLE_E_NOMEM;
    }
    /* the identity part starts at word wn: bit i of that part is column n + i
       of [A | I] in the unpacked picture */
    for (int64_t i = 0; i < m; ++i) {
        memcpy(W + i * w, A + i * ldw, sizeof(uint64_t) * (size_t)wn);
        W[i * w + wn + i / 64] |= 1ull << (i % 64);
    }
    int64_t r = 0;
    for (int64_t i = 0; i < m; ++i) {
        uint64_t* row = W + i * w;
        /* reduce row i by every existing pivot row */
        for (int64_t t = 0; t < r; ++t)
            if ((row[piv_col[t] / 64] >> (piv_col[t] % 64)) & 1u) {
                const uint64_t* s = W + piv_row[t] * w;
                for (int64_t k = 0; k < w; ++k) row[k] ^= s[k];
            }
        /* first non-zero among the A columns */
        int64_t c = -1;
        for (int64_t j = 0; j < n; ++j)
            if ((row[j / 64] >> (j % 64)) & 1u) { c = j; break; }
        if (c < 0) continue;                       /* not selected */
        /* keep earlier pivot rows reduced: clear column c in them */
        for (int64_t t = 0; t < r; ++t) {
            uint64_t* s = W + piv_row[t] * w;
            if ((s[c / 64] >> (c % 64)) & 1u)
                for (int64_t k = 0; k < w; ++k) s[k] ^= row[k];
        }
        piv_col[r] = c;
        piv_row[r] = i;
        is_sel[i] = 1;
        ++r;
    }
    /* order the pivots by column: exchange neighbours until sorted */
    for (int64_t a = 1; a < r; ++a)
        for (int64_t b = a; b > 0 && piv_col[b - 1] > piv_col[b]; --b) {
            int64_t tc = piv_col[b], tr = piv_row[b];
            piv_col[b] = piv_col[b - 1]; piv_row[b] = piv_row[b - 1];
            piv_col[b - 1] = tc; piv_row[b - 1] = tr;
        }
    for (int64_t t = 0; t < r; ++t) {
        const uint64_t* row = W + piv_row[t] * w;
        if (E) memcpy(E + t * wn, row, sizeof(uint64_t) * (size_t)wn);
        if (T) memcpy(T + t * wm, row + wn, sizeof(uint64_t) * (size_t)wm);
    }
    int64_t q = r;
    for (int64_t i = 0; i < m; ++i) {
        if (is_sel[i]) continue;
        if (T) memcpy(T + q * wm, W + i * w + wn, sizeof(uint64_t) * (size_t)wm);
        ++q;
    }
    int64_t s = 0;
    for (int64_t i = 0; i < m; ++i)
        if (is_sel[i]) selrows[s++] = i;
    for (int64_t t = 0; t < r; ++t) pivcols[t] = piv_col[t];
    *rank_out = r;
    free(W); free(piv_col); free(piv_row); free(is_sel);
    return ORACLE_OK;
}

/* plain (C + A * B) over GF(2) on packed rows: A m x k (lda words), B k x n
   (ldb words), C and out m x n (ldc words); bit j of row i of the product is
   the parity of the k terms A[i][t] B[t][j] (the MAD job over GF(2)) */
int oracle_mad_gf2(const uint64_t* C, const uint64_t* A, const uint64_t* B, uint64_t* out,
                   int64_t m, int64_t k, int64_t n, int64_t lda, int64_t ldb, int64_t ldc) {
    const int64_t wn = (n + 63) / 64;
    for (int64_t i = 0; i < m; ++i) {
        uint64_t* o = out + i * ldc;
        for (int64_t w = 0; w < wn; ++w) o[w] = C ? C[i * ldc + w] : 0u;
        for (int64_t t = 0; t < k; ++t)
            if ((A[i * lda + t / 64] >> (t % 64)) & 1u)
                for (int64_t w = 0; w < wn; ++w) o[w] ^= B[t * ldb + w];
    }
    return ORACLE_OK;
}
