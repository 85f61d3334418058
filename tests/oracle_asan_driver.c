/* Host driver for the oracle under AddressSanitizer and UndefinedBehavior-
 * Sanitizer: exact-size heap buffers (so a read or write past any array is
 * reported), every entry point, sizes around the word boundaries, padding
 * bits set to garbage, and a per-bit cross-check of the full hash against
 * the single-bit sampler and of the modified hash against its definition
 * y_i = x_i XOR sum_j v[i - j + (n-m) - 1] x[m+j], bit by bit.
 * Exit status 0 when every check agrees; the sanitizers abort on a fault. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_toeplitz_hash(const uint64_t *key, uint64_t n, const uint64_t *seed, uint64_t m, uint64_t *out,
                         int threads);
int oracle_toeplitz_bits(const uint64_t *key, uint64_t n, const uint64_t *seed, uint64_t m, const uint64_t *idx,
                         uint64_t count, uint8_t *bits, int threads);
int oracle_modified_toeplitz_hash(const uint64_t *key, uint64_t n, const uint64_t *vbits, uint64_t m, uint64_t *out,
                                  int threads);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint64_t next(void) { /* xorshift64* */
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return state * 0x2545F4914F6CDD1Dull;
}
static uint64_t words(uint64_t bits) { return (bits + 63) / 64; }
static uint64_t *random_bits(uint64_t bits) {
    uint64_t *w = malloc(words(bits) * 8 + (bits == 0));
    for (uint64_t i = 0; i < words(bits); ++i) w[i] = next(); /* padding bits left as garbage */
    return w;
}
static int bit(const uint64_t *w, uint64_t k) { return (int)((w[k / 64] >> (k % 64)) & 1); }

int main(void) {
    const uint64_t sizes[][2] = {{1, 1},     {2, 1},    {63, 1},    {64, 64},    {65, 1},   {65, 65},
                                 {127, 64},  {128, 65}, {129, 100}, {1000, 1},   {1000, 999}, {1000, 1000},
                                 {4097, 700}, {8191, 4096}, {20000, 5000}};
    int failures = 0;
    for (size_t t = 0; t < sizeof(sizes) / sizeof(sizes[0]); ++t) {
        const uint64_t n = sizes[t][0], m = sizes[t][1];
        uint64_t *key = random_bits(n), *seed = random_bits(n + m - 1);
        uint64_t *out = malloc(words(m) * 8);
        memset(out, 0xA5, words(m) * 8);
        if (oracle_toeplitz_hash(key, n, seed, m, out, 1 + (int)(t % 3)) != 0) ++failures;
        uint64_t *idx = malloc(m * 8);
        uint8_t *bits = malloc(m);
        for (uint64_t i = 0; i < m; ++i) idx[i] = i;
        if (oracle_toeplitz_bits(key, n, seed, m, idx, m, bits, 2) != 0) ++failures;
        for (uint64_t i = 0; i < m; ++i)
            if (bits[i] != bit(out, i)) {
                ++failures;
                break;
            }
        if (m % 64 && (out[words(m) - 1] >> (m % 64)) != 0) ++failures; /* tail bits written as 0 */
        if (m < n) {
            uint64_t *v = random_bits(n - 1);
            uint64_t *mo = malloc(words(m) * 8);
            if (oracle_modified_toeplitz_hash(key, n, v, m, mo, 2) != 0) ++failures;
            /* definition, bit by bit: y_i = x_i XOR sum_j V[i][j] x[m+j],
             * V[i][j] = v[i - j + (n-m) - 1], 0 <= j < n-m */
            const uint64_t nt = n - m;
            for (uint64_t i = 0; i < m; ++i) {
                int acc = bit(key, i);
                for (uint64_t j = 0; j < nt; ++j) acc ^= bit(v, i - j + nt - 1) & bit(key, m + j);
                if (bit(mo, i) != acc) {
                    ++failures;
                    break;
                }
            }
            free(v);
            free(mo);
        }
        free(key);
        free(seed);
        free(out);
        free(idx);
        free(bits);
    }
    printf("{\"cases\": %zu, \"failures\": %d}\n", sizeof(sizes) / sizeof(sizes[0]), failures);
    return failures != 0;
}
