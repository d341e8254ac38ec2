#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
/* Runs the oracle on a 4^3 Kuhn lattice (6 tets per cell, one per axis
 * permutation) with A + B <-> C and a production of A, in both transfer
 * forms (split thresholds 10 and 4) and across a shortened last period,
 * so that a sanitized build exercises the SSA, both split methods and both
 * transfer forms.  Prints
 * the totals; exits non-zero if creation fails. */
static int vid(int n, int i, int j, int k) { return i + (n + 1) * (j + (n + 1) * k); }
int main(void)
{
    const int n = 4; const double a = 0.2e-6;
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
            for (int s = 0; s < 3; ++s) { c[perm[p][s]] += 1; tv[4*t+1+s] = vid(n, c[0], c[1], c[2]); }
            ++t;
        }
    double D[3] = {1e-12, 1e-12, 0.5e-12};
    int32_t rn[3] = {2, 1, 0}, rids[6] = {0, 1, 2, 0, 0, 0}, pn[3] = {1, 2, 1}, pids[9] = {2, 0, 0, 0, 1, 0, 0, 0, 0};
    double kk[3] = {3e8, 400.0, 1e-3};
    char err[256];
    for (int form = 0; form < 2; ++form) {
        orc_sim *s = orc_create(nv, xyz, T, tv, 3, D, 3, rn, rids, pn, pids, kk, 1.0, 7, 0, err);
        if (!s) { printf("create failed: %s\n", err); return 1; }
        orc_set_transfer_form(s, form);
        orc_set_split_threshold(s, form ? 4 : 10);
        int32_t *c = malloc(sizeof(int32_t) * T);
        for (int sp = 0; sp < 3; ++sp) { for (int q = 0; q < T; ++q) c[q] = (q * 7 + sp * 3) % 40; orc_set_counts(s, sp, c); }
        orc_run_steps(s, 200);
        orc_run_until(s, 0.2);
        long tot[3] = {0, 0, 0};
        for (int sp = 0; sp < 3; ++sp) { orc_get_counts(s, sp, c); for (int q = 0; q < T; ++q) tot[sp] += c[q]; }
        printf("form %d: A %ld B %ld C %ld\n", form, tot[0], tot[1], tot[2]);
        free(c); orc_destroy(s);
    }
    free(xyz); free(tv);
    return 0;
}
