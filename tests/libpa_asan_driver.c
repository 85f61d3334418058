/* Host driver for libpa's host code under AddressSanitizer, on a machine
 * with or without a GPU: only entry points that do not launch kernels.
 *   - status strings, version, transform and final-key lengths;
 *   - the planner over every supported length and every (log2 R, W) split;
 *   - the tuning table: set, get, save and load, including malformed files;
 *   - argument validation of the hash entry points (errors before any
 *     device work);
 *   - the serving scheduler with the simulated executor, with seeds
 *     registered, requests submitted and cancelled from several threads.
 * Exit status 0 when every expectation holds; the sanitizer aborts on a
 * fault. */
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pa.h"

static int failures = 0;
#define EXPECT(c)                                                        \
    do {                                                                 \
        if (!(c)) {                                                      \
            ++failures;                                                  \
            fprintf(stderr, "line %d: expectation failed: %s\n", __LINE__, #c); \
        }                                                                \
    } while (0)

static pa_server_t server;
static uint32_t seed_ids[4];

static void *submitter(void *arg) {
    const int t = (int)(intptr_t)arg;
    uint64_t tickets[64];
    int nt = 0;
    for (int i = 0; i < 64; ++i) {
        const uint64_t n = 100000 + (uint64_t)((t * 7919 + i * 104729) % 900000);
        const uint64_t m = n / (2 + (uint64_t)(i % 5));
        uint64_t ticket = 0;
        pa_status s = pa_server_submit(server, seed_ids[(t + i) % 4], (const uint64_t *)0x200000, n, m,
                                       (uint64_t *)0x300000, &ticket);
        if (s == PA_OK) tickets[nt++] = ticket;
        else EXPECT(s == PA_ERR_BUSY);
        if (i % 9 == 0 && nt > 0) {
            s = pa_server_cancel(server, tickets[nt - 1]);
            EXPECT(s == PA_OK || s == PA_ERR_BUSY || s == PA_ERR_INVALID_ARG);
        }
    }
    for (int i = 0; i < nt; ++i) {
        pa_status s = pa_server_wait(server, tickets[i], NULL);
        EXPECT(s == PA_OK || s == PA_ERR_CANCELLED);
    }
    return NULL;
}

/* registers seeds 4..7 while the submitters run, and serves a few requests
 * on each as soon as it exists */
static void *registrar(void *arg) {
    (void)arg;
    for (int i = 4; i < 8; ++i) {
        uint32_t id = 0;
        EXPECT(pa_server_register_seed(server, (const uint64_t *)0x100000, 20000000, &id) == PA_OK);
        uint64_t tickets[8];
        int nt = 0;
        for (int k = 0; k < 8; ++k) {
            uint64_t ticket = 0;
            const uint64_t n = 200000 + 50000 * (uint64_t)k;
            pa_status s = pa_server_submit(server, id, (const uint64_t *)0x200000, n, n / 4, (uint64_t *)0x300000,
                                           &ticket);
            if (s == PA_OK) tickets[nt++] = ticket;
            else EXPECT(s == PA_ERR_BUSY);
        }
        for (int k = 0; k < nt; ++k) EXPECT(pa_server_wait(server, tickets[k], NULL) == PA_OK);
    }
    return NULL;
}

int main(int argc, char **argv) {
    const char *tmpdir = argc > 1 ? argv[1] : "/tmp";
    char path[4096];

    EXPECT(pa_version() && strlen(pa_version()) > 0);
    for (int s = 0; s <= 16; ++s) EXPECT(pa_status_string((pa_status)s) != NULL);
    EXPECT(pa_final_key_length(1000, 100, 50) == 850);
    EXPECT(pa_final_key_length(100, 100, 50) == 0);
    for (uint64_t n = 1; n < 40000000; n = n * 3 + 7)
        for (uint64_t m = 1; m <= n; m = m * 5 + 1) (void)pa_transform_len(n, m);
    EXPECT(pa_transform_len(0, 1) == 0);

    /* the planner over every supported length and split */
    int described = 0;
    for (int k = 7; k <= 20; ++k)
        for (int j = 0; j <= 3; ++j) {
            uint64_t L = (1ull << k);
            for (int i = 0; i < j; ++i) L *= 3;
            if (L < 4096 || L > 27ull * (1ull << 20)) continue;
            for (uint32_t lg = 0; lg <= 12; ++lg)
                for (uint32_t w = 0; w <= 64; w = w ? w * 2 : 8) {
                    pa_plan_info info;
                    memset(&info, 0, sizeof(info));
                    if (pa_plan_describe(L, lg, w, &info) == PA_OK) {
                        ++described;
                        EXPECT(info.transform_len == L);
                        EXPECT((uint64_t)info.rows * info.cols == L);
                    }
                }
        }
    EXPECT(described > 100);
    pa_plan_info info;
    EXPECT(pa_plan_describe(4097, 0, 0, &info) != PA_OK);

    /* the tuning table and its file format */
    const uint64_t L = pa_transform_len(1000000, 250000);
    pa_tune_geometry g = {8, 32, 0, 0}, h;
    EXPECT(pa_tune_set_geometry(L, 0, &g) == PA_OK);
    EXPECT(pa_tune_get_geometry(L, 0, &h) == PA_OK && h.log2_rows == 8 && h.tile_width == 32);
    g.tile_width = 3;
    EXPECT(pa_tune_set_geometry(L, 0, &g) != PA_OK);
    snprintf(path, sizeof(path), "%s/tune_ok.txt", tmpdir);
    EXPECT(pa_tune_save(path) == PA_OK);
    EXPECT(pa_tune_load(path) == PA_OK);
    const char *bad[] = {"1572864 0 8\n", "1572864 0 8 32 0 0 gfx950 extra\n", "x 0 8 32\n", "1572864 0 8 -32\n",
                         "4097 0 8 32\n", "1572864 0 30 32\n", "# only a comment\n\n", "1572864 0 8 32 0 0 gfx000\n",
                         "99999999999999999999999 0 8 32\n"};
    for (size_t i = 0; i < sizeof(bad) / sizeof(bad[0]); ++i) {
        snprintf(path, sizeof(path), "%s/tune_bad%zu.txt", tmpdir, i);
        FILE *f = fopen(path, "w");
        if (!f) return 3;
        fputs(bad[i], f);
        fclose(f);
        (void)pa_tune_load(path); /* accepted or rejected, never a fault */
    }
    EXPECT(pa_tune_load("/nonexistent/dir/file") != PA_OK);
    g.tile_width = 0;
    g.log2_rows = 0;
    EXPECT(pa_tune_set_geometry(L, 0, &g) == PA_OK);

    /* argument validation before any device work */
    uint64_t out[4];
    EXPECT(pa_toeplitz_hash(NULL, 100, (const uint64_t *)0x1000, 10, out, NULL) == PA_ERR_INVALID_ARG);
    EXPECT(pa_toeplitz_hash((const uint64_t *)0x1000, 100, (const uint64_t *)0x2000, 101, out, NULL) ==
           PA_ERR_INVALID_ARG);
    EXPECT(pa_toeplitz_hash((const uint64_t *)0x1000, 0, (const uint64_t *)0x2000, 0, out, NULL) ==
           PA_ERR_INVALID_ARG);
    EXPECT(pa_toeplitz_hash_batched(NULL, 3, NULL) == PA_ERR_INVALID_ARG);
    pa_block blk[2];
    memset(blk, 0, sizeof(blk));
    EXPECT(pa_toeplitz_hash_batched(blk, 2, NULL) == PA_ERR_INVALID_ARG);
    EXPECT(pa_modified_toeplitz_hash((const uint64_t *)0x1000, 100, (const uint64_t *)0x2000, 100, out, NULL) ==
           PA_ERR_INVALID_ARG);
    EXPECT(pa_toeplitz_hash_noalloc((const uint64_t *)0x1000, 100, NULL, 10, out, NULL) == PA_ERR_INVALID_ARG);
    EXPECT(pa_server_create(NULL, NULL) == PA_ERR_INVALID_ARG);

    /* serving scheduler, simulated executor */
    pa_server_config cfg;
    memset(&cfg, 0, sizeof(cfg));
    cfg.hbm_budget_bytes = 96ull << 20;
    cfg.max_inflight = 5;
    cfg.max_queue = 4096;
    cfg.streams = 3;
    cfg.executor = PA_EXEC_SIMULATED;
    cfg.sim_bits_per_us = 5e5;
    EXPECT(pa_server_create(&cfg, &server) == PA_OK);
    for (int i = 0; i < 4; ++i)
        EXPECT(pa_server_register_seed(server, (const uint64_t *)0x100000, 20000000, &seed_ids[i]) == PA_OK);
    pthread_t th[5];
    for (int t = 0; t < 4; ++t) pthread_create(&th[t], NULL, submitter, (void *)(intptr_t)t);
    pthread_create(&th[4], NULL, registrar, NULL);
    for (int t = 0; t < 5; ++t) pthread_join(th[t], NULL);
    (void)pa_server_drain(server);
    pa_server_stats st;
    EXPECT(pa_server_stats_get(server, &st) == PA_OK);
    EXPECT(st.completed + st.cancelled >= st.submitted - st.rejected - st.failed);
    EXPECT(st.peak_bytes_in_flight <= st.budget_bytes);
    EXPECT(pa_server_destroy(server) == PA_OK);

    printf("{\"described\": %d, \"failures\": %d}\n", described, failures);
    return failures != 0;
}
