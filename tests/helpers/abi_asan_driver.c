/* The public C ABI under AddressSanitizer and UndefinedBehaviorSanitizer
 * (host code only: the library is built with -Xarch_host -fsanitize=...;
 * device code is not instrumented).
 * Plain stepping of 2 realizations (40 periods, then a shortened last period)
 * and an engine serving three requests of different lengths, every result
 * against the oracle.  Build with build_abi_asan_driver.sh, run on a GPU with
 * ASAN_OPTIONS=detect_leaks=0 (the HIP runtime keeps allocations until exit);
 * exits non-zero on a mismatch, and the sanitizer aborts on a report. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "rdos.h"
#include "oracle.h"

static int vid(int n, int i, int j, int k) { return i + (n + 1) * (j + (n + 1) * k); }
static uint32_t lcg = 12345u;
static int rnd(int m) { lcg = lcg * 1664525u + 1013904223u; return (int)((lcg >> 8) % (uint32_t)m); }

static const double D[3] = {1e-12, 1e-12, 0.5e-12};
static const int32_t RN[2] = {2, 1}, RIDS[4] = {0, 1, 2, 0}, PN[2] = {1, 2}, PIDS[6] = {2, 0, 0, 0, 1, 0};
static const double K[2] = {3e8, 400.0};

#define CK(x) do { rdos_status st__ = (x); if (st__ != RDOS_OK) { printf("FAIL %s -> %d\n", #x, st__); return 1; } } while (0)

static rdos_sim *make(int nv, const double *xyz, int T, const int32_t *tv, uint64_t seed, int Rz, int32_t *init)
{
    rdos_sim *s = NULL;
    if (rdos_create(&s, 0, seed, Rz) != RDOS_OK) return NULL;
    rdos_set_mesh(s, nv, xyz, T, tv);
    int32_t id;
    for (int m = 0; m < 3; ++m) rdos_add_species(s, D[m], &id);
    rdos_add_reaction(s, 2, (const int32_t[]){0, 1}, 1, (const int32_t[]){2}, K[0], &id);
    rdos_add_reaction(s, 1, (const int32_t[]){2}, 2, (const int32_t[]){0, 1}, K[1], &id);
    double tau;
    if (rdos_finalize(s, 1.0, &tau) != RDOS_OK) { printf("finalize: %s\n", rdos_last_error(s)); return NULL; }
    for (int r = 0; r < Rz; ++r)
        for (int m = 0; m < 3; ++m) rdos_set_counts(s, r, m, init + ((size_t)r * 3 + m) * T);
    return s;
}

static int compare(rdos_sim *s, int Rz, int nv, const double *xyz, int T, const int32_t *tv, uint64_t seed,
                   const int32_t *init, int64_t steps, double t_end, const char *what)
{
    int32_t *got = malloc(sizeof(int32_t) * T), *want = malloc(sizeof(int32_t) * T);
    char err[256];
    int bad = 0;
    for (int r = 0; r < Rz; ++r) {
        orc_sim *o = orc_create(nv, xyz, T, tv, 3, D, 2, RN, RIDS, PN, PIDS, K, 1.0, seed, r, err);
        if (!o) { printf("oracle: %s\n", err); return 1; }
        for (int m = 0; m < 3; ++m) orc_set_counts(o, m, init + ((size_t)r * 3 + m) * T);
        orc_run_steps(o, steps);
        if (t_end > 0) orc_run_until(o, t_end);
        for (int m = 0; m < 3; ++m) {
            orc_get_counts(o, m, want);
            if (rdos_get_counts(s, r, m, got) != RDOS_OK) { printf("get_counts: %s\n", rdos_last_error(s)); return 1; }
            if (memcmp(got, want, sizeof(int32_t) * T)) { printf("%s: realization %d species %d differs\n", what, r, m); bad = 1; }
        }
        orc_destroy(o);
    }
    free(got); free(want);
    if (!bad) printf("%s: identical to the oracle\n", what);
    return bad;
}

int main(void)
{
    const int n = 6; const double a = 0.2e-6;
    int nv = (n + 1) * (n + 1) * (n + 1), T = 6 * n * n * n;
    double *xyz = malloc(sizeof(double) * 3 * nv);
    int32_t *tv = malloc(sizeof(int32_t) * 4 * T);
    for (int k = 0; k <= n; ++k) for (int j = 0; j <= n; ++j) for (int i = 0; i <= n; ++i) {
        int v = vid(n, i, j, k); xyz[3*v] = i * a; xyz[3*v+1] = j * a; xyz[3*v+2] = k * a; }
    static const int perm[6][3] = {{0,1,2},{0,2,1},{1,0,2},{1,2,0},{2,0,1},{2,1,0}};
    int t = 0;
    for (int k = 0; k < n; ++k) for (int j = 0; j < n; ++j) for (int i = 0; i < n; ++i)
        for (int p = 0; p < 6; ++p) {
            int c[3] = {i, j, k};
            tv[4*t] = vid(n, c[0], c[1], c[2]);
            for (int q = 0; q < 3; ++q) { c[perm[p][q]] += 1; tv[4*t+1+q] = vid(n, c[0], c[1], c[2]); }
            ++t;
        }
    int bad = 0;
    /* plain: 2 realizations, 40 periods, then to a time that shortens the last period */
    int32_t *init = malloc(sizeof(int32_t) * 2 * 3 * T);
    for (int q = 0; q < 2 * 3 * T; ++q) init[q] = rnd(3) == 0 ? rnd(20) : 0;
    rdos_sim *s = make(nv, xyz, T, tv, 5, 2, init);
    if (!s) return 1;
    CK(rdos_step(s, 40));
    double t_now; int64_t k_now;
    CK(rdos_get_time(s, &t_now, &k_now));
    CK(rdos_run_until(s, t_now * 1.37));
    bad |= compare(s, 2, nv, xyz, T, tv, 5, init, 40, t_now * 1.37, "plain");
    rdos_destroy(s);
    /* engine: three requests of different lengths */
    rdos_engine *e = NULL;
    CK(rdos_engine_create(&e, 0, 0));
    rdos_sim *sims[3]; uint64_t tk[3]; int64_t len[3] = {24, 40, 56};
    int32_t *inits[3];
    for (int i = 0; i < 3; ++i) {
        inits[i] = malloc(sizeof(int32_t) * 3 * T);
        for (int q = 0; q < 3 * T; ++q) inits[i][q] = rnd(4) == 0 ? rnd(30) : 0;
        sims[i] = make(nv, xyz, T, tv, 100 + i, 1, inits[i]);
        if (!sims[i]) return 1;
        CK(rdos_engine_submit(e, sims[i], len[i], 1.0, &tk[i]));
    }
    CK(rdos_engine_drain(e));
    for (int i = 0; i < 3; ++i) {
        int done = 0; double lat = 0;
        CK(rdos_engine_poll(e, tk[i], &done, &lat));
        rdos_sim *back = NULL;
        CK(rdos_engine_release(e, tk[i], &back));
        char what[32]; snprintf(what, sizeof what, "engine request %d", i);
        bad |= compare(back, 1, nv, xyz, T, tv, 100 + i, inits[i], len[i], 0.0, what);
        rdos_destroy(back);
        free(inits[i]);
    }
    rdos_engine_destroy(e);
    free(init); free(xyz); free(tv);
    printf(bad ? "MISMATCH\n" : "ALL OK\n");
    return bad;
}
