/*
 * CPU oracle for Toeplitz-hash privacy amplification.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header or table with the GPU
 * library.
 *
 * What it computes (paper, Sec. 2.1 and 2.2): a compression function
 * g: {0,1}^n -> {0,1}^m given by an m x n Toeplitz matrix T over GF(2),
 * built from its first row and first column, i.e. from n+m-1 random bits s.
 * Reading used throughout (the paper fixes only "first row and first
 * column"): T[i][j] = s[i - j + n - 1] for 0 <= i < m, 0 <= j < n, so row 0 is
 * s[n-1], s[n-2], ..., s[0] and column 0 is s[n-1], ..., s[n+m-2].  The
 * output is y = T x over GF(2): y_i = XOR_j (T[i][j] AND x_j).
 *
 * Bit layout: little-endian packed uint64, bit k lives in word k >> 6 at
 * position k & 63.  Padding bits of key and seed are ignored; padding bits
 * of the output are written as zero.
 *
 * Method (the plain definition, no transform): substituting t = n-1-j,
 *   y_i = XOR_{t<n} s[i+t] AND xr[t],   xr[t] = x[n-1-t],
 * so y_i is the parity of popcount(window(s, i, n) AND xr).  The key is
 * reversed once; every output bit is then n/64 word ANDs folded by XOR.
 * Precomputing the 64 bit-shifted copies of s makes each window a run of
 * aligned words.  Cost: m * ceil(n/64) word operations.
 *
 * The modified Toeplitz matrix of Sec. 2.2, Eq. (2)-(3) is also provided:
 * S = [I_m | V], V an m x (n-m) Toeplitz matrix, y = x[0:m] XOR V x[m:n].
 * Reading of the garbled printed indices: V is described by n-1 bits v with
 * V[i][j] = v[i - j + (n-m) - 1]; the identity block takes the first m key
 * bits (Eq. (3)), the Toeplitz block the remaining n-m bits.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 3

static inline uint64_t words_for(uint64_t bits) { return (bits + 63) >> 6; }

static inline int get_bit(const uint64_t *w, uint64_t k) {
    return (int)((w[k >> 6] >> (k & 63)) & 1u);
}

/* Bits [a, a+64) of the bit string w (length `len` bits; bits >= len read
 * as zero) as one word. */
static uint64_t read_word_at(const uint64_t *w, uint64_t len, uint64_t a) {
    if (a >= len) return 0;
    uint64_t wi = a >> 6, sh = a & 63, nwords = words_for(len);
    uint64_t lo = w[wi] >> sh;
    uint64_t hi = 0;
    if (sh && wi + 1 < nwords) hi = w[wi + 1] << (64 - sh);
    uint64_t v = lo | hi;
    uint64_t valid = len - a;
    if (valid < 64) v &= (((uint64_t)1 << valid) - 1);
    return v;
}

/* xr[t] = x[n-1-t] for t < n, packed, tail zero. */
static uint64_t *reverse_key(const uint64_t *key, uint64_t n) {
    uint64_t nw = words_for(n);
    uint64_t *xr = (uint64_t *)calloc(nw ? nw : 1, sizeof(uint64_t));
    if (!xr) return NULL;
    for (uint64_t t = 0; t < n; ++t)
        if (get_bit(key, n - 1 - t)) xr[t >> 6] |= (uint64_t)1 << (t & 63);
    return xr;
}

static void set_threads(int threads) {
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Plain Toeplitz hash, all m outputs.  key: ceil(n/64) words, seed:
 * ceil((n+m-1)/64) words, out: ceil(m/64) words (fully overwritten).
 */
int oracle_toeplitz_hash(const uint64_t *key, uint64_t n, const uint64_t *seed,
                         uint64_t m, uint64_t *out, int threads) {
    if (!key || !seed || !out || n == 0 || m == 0 || m > n) return OR_EINVAL;
    set_threads(threads);
    const uint64_t slen = n + m - 1;
    const uint64_t nw = words_for(n);
    const uint64_t ow = words_for(m);
    /* shifted[a][k] = bits [64k + a, 64k + a + 64) of s; the window for
     * output i starts at word i>>6 of copy i&63. */
    const uint64_t sw = words_for(slen) + 1;
    uint64_t *shifted = (uint64_t *)malloc(64 * sw * sizeof(uint64_t));
    uint64_t *xr = reverse_key(key, n);
    if (!shifted || !xr) { free(shifted); free(xr); return OR_ENOMEM; }
#pragma omp parallel for schedule(static)
    for (int a = 0; a < 64; ++a)
        for (uint64_t k = 0; k < sw; ++k)
            shifted[(uint64_t)a * sw + k] = read_word_at(seed, slen, 64 * k + (uint64_t)a);

#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t ow_i = 0; ow_i < (int64_t)ow; ++ow_i) {
        uint64_t word = 0;
        for (int b = 0; b < 64; ++b) {
            uint64_t i = (uint64_t)ow_i * 64 + (uint64_t)b;
            if (i >= m) break;
            const uint64_t *win = shifted + (uint64_t)(i & 63) * sw + (i >> 6);
            uint64_t acc = 0;
            for (uint64_t k = 0; k < nw; ++k) acc ^= win[k] & xr[k];
            word |= (uint64_t)(__builtin_popcountll(acc) & 1) << b;
        }
        out[ow_i] = word;
    }
    free(shifted);
    free(xr);
    return OR_OK;
}

/*
 * Selected output bits of the plain Toeplitz hash, one at a time, without
 * the shifted copies: for each requested index i < m, bits[k] = y_i.  Cost
 * per bit ceil(n/64) word operations, so large blocks can be sampled.
 */
int oracle_toeplitz_bits(const uint64_t *key, uint64_t n, const uint64_t *seed,
                         uint64_t m, const uint64_t *idx, uint64_t count,
                         uint8_t *bits, int threads) {
    if (!key || !seed || !bits || (count && !idx) || n == 0 || m == 0 || m > n)
        return OR_EINVAL;
    for (uint64_t k = 0; k < count; ++k)
        if (idx[k] >= m) return OR_EINVAL;
    set_threads(threads);
    const uint64_t slen = n + m - 1;
    const uint64_t nw = words_for(n);
    uint64_t *xr = reverse_key(key, n);
    if (!xr) return OR_ENOMEM;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < (int64_t)count; ++k) {
        uint64_t i = idx[k];
        uint64_t acc = 0;
        for (uint64_t w = 0; w < nw; ++w)
            acc ^= read_word_at(seed, slen, i + 64 * w) & xr[w];
        bits[k] = (uint8_t)(__builtin_popcountll(acc) & 1);
    }
    free(xr);
    return OR_OK;
}

/*
 * Modified Toeplitz hash (Sec. 2.2 Eq. (2), Sec. 2.3 Eq. (3)):
 *   y = x[0:m] XOR V x[m:n],  V[i][j] = v[i - j + (n-m) - 1],
 * with v the n-1 description bits.  Requires 1 <= m < n.
 * key: ceil(n/64) words, vbits: ceil((n-1)/64) words, out: ceil(m/64).
 */
int oracle_modified_toeplitz_hash(const uint64_t *key, uint64_t n,
                                  const uint64_t *vbits, uint64_t m,
                                  uint64_t *out, int threads) {
    if (!key || !vbits || !out || n < 2 || m == 0 || m >= n) return OR_EINVAL;
    const uint64_t nt = n - m; /* width of V */
    const uint64_t ow = words_for(m);
    /* The Toeplitz part is the plain hash of x[m:n] with n' = n-m, m' = m,
     * whose description length n'+m'-1 = n-1. */
    uint64_t *tail = (uint64_t *)calloc(words_for(nt) ? words_for(nt) : 1, sizeof(uint64_t));
    if (!tail) return OR_ENOMEM;
    for (uint64_t j = 0; j < nt; ++j)
        if (get_bit(key, m + j)) tail[j >> 6] |= (uint64_t)1 << (j & 63);
    int rc;
    if (m <= nt) {
        rc = oracle_toeplitz_hash(tail, nt, vbits, m, out, threads);
    } else {
        /* m > n-m: the plain routine requires m' <= n'; evaluate the rows
         * one by one instead. */
        uint64_t *idx = (uint64_t *)malloc(m * sizeof(uint64_t));
        uint8_t *b = (uint8_t *)malloc(m);
        rc = (idx && b) ? OR_OK : OR_ENOMEM;
        if (rc == OR_OK) {
            const uint64_t nw = words_for(nt);
            uint64_t *xr = reverse_key(tail, nt);
            if (!xr) rc = OR_ENOMEM;
            else {
                const uint64_t vlen = n - 1;
                set_threads(threads);
#pragma omp parallel for schedule(dynamic, 16)
                for (int64_t i = 0; i < (int64_t)m; ++i) {
                    uint64_t acc = 0;
                    for (uint64_t w = 0; w < nw; ++w)
                        acc ^= read_word_at(vbits, vlen, (uint64_t)i + 64 * w) & xr[w];
                    b[i] = (uint8_t)(__builtin_popcountll(acc) & 1);
                }
                free(xr);
                memset(out, 0, ow * sizeof(uint64_t));
                for (uint64_t i = 0; i < m; ++i)
                    if (b[i]) out[i >> 6] |= (uint64_t)1 << (i & 63);
            }
        }
        free(idx);
        free(b);
    }
    free(tail);
    if (rc != OR_OK) return rc;
    for (uint64_t i = 0; i < m; ++i)
        if (get_bit(key, i)) out[i >> 6] ^= (uint64_t)1 << (i & 63);
    if (m & 63) out[ow - 1] &= (((uint64_t)1 << (m & 63)) - 1);
    return OR_OK;
}
