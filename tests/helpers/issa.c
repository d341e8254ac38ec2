/*
 * Exact spatial SSA (the "ISSA" the paper compares against, Sec. I and
 * Sec. III.D): Gillespie's direct method over every diffusion channel
 * (molecule of species m in tet t leaving through face f at rate D_m r_tf)
 * and every reaction channel (reaction r in tet t), with no operator
 * splitting.  Test infrastructure: it checks the operator-split oracle in law
 * on tiny meshes.  Own random numbers (SplitMix64), unrelated to Philox.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t sm_next(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static double sm_u(uint64_t *s) /* (0, 1) */
{
    return ((double)(sm_next(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

/*
 * T tets, S species, R reactions.
 *   nbr[T*4], drate[S*T*4] per-molecule rate through each face (1/s)
 *   rn[R], rid[R*2], pn[R], pid[R*3], c[R*T] propensity constants per tet
 *   counts[S*T] initial, overwritten with the final state
 *   n_samples sample times (ascending), out[n_samples*S*T]
 */
void issa_run(int T, int S, int R, const int32_t *nbr, const double *drate, const int32_t *rn,
              const int32_t *rid, const int32_t *pn, const int32_t *pid, const double *c,
              int32_t *counts, int n_samples, const double *times, uint64_t seed, int32_t *out)
{
    uint64_t st = seed * 0x2545F4914F6CDD1DULL + 12345;
    double *dtot = (double *)malloc(sizeof(double) * (size_t)S * T); /* per-molecule leave rate */
    for (int m = 0; m < S; ++m)
        for (int t = 0; t < T; ++t) {
            double s = 0.0;
            for (int f = 0; f < 4; ++f) s += drate[((size_t)m * T + t) * 4 + f];
            dtot[(size_t)m * T + t] = s;
        }
    double now = 0.0;
    int next = 0;
    double *a = (double *)malloc(sizeof(double) * ((size_t)S * T + (size_t)R * T + 1));
    while (next < n_samples) {
        double a0 = 0.0;
        size_t nd = (size_t)S * T;
        for (size_t i = 0; i < nd; ++i) {
            a[i] = counts[i] * dtot[i];
            a0 += a[i];
        }
        for (int r = 0; r < R; ++r)
            for (int t = 0; t < T; ++t) {
                double h;
                if (rn[r] == 0) h = 1.0;
                else if (rn[r] == 1) h = counts[(size_t)rid[2 * r] * T + t];
                else if (rid[2 * r] == rid[2 * r + 1]) {
                    double x = counts[(size_t)rid[2 * r] * T + t];
                    h = x * (x - 1.0);
                } else h = (double)counts[(size_t)rid[2 * r] * T + t] * counts[(size_t)rid[2 * r + 1] * T + t];
                a[nd + (size_t)r * T + t] = c[(size_t)r * T + t] * h;
                a0 += a[nd + (size_t)r * T + t];
            }
        double dt = a0 > 0 ? -log(sm_u(&st)) / a0 : INFINITY;
        while (next < n_samples && now + dt >= times[next]) {
            memcpy(out + (size_t)next * S * T, counts, sizeof(int32_t) * (size_t)S * T);
            ++next;
        }
        if (next >= n_samples) break;
        now += dt;
        double x = sm_u(&st) * a0, cum = 0.0;
        size_t total = nd + (size_t)R * T, ch = total - 1;
        for (size_t i = 0; i < total; ++i) {
            cum += a[i];
            if (x < cum && a[i] > 0) {
                ch = i;
                break;
            }
        }
        while (a[ch] <= 0 && ch > 0) --ch;
        if (ch < nd) { /* diffusion: pick the face */
            int m = (int)(ch / T), t = (int)(ch % T);
            double y = sm_u(&st) * dtot[ch], cf = 0.0;
            int face = -1;
            for (int f = 0; f < 4; ++f) {
                double rr = drate[((size_t)m * T + t) * 4 + f];
                cf += rr;
                if (y < cf && rr > 0) {
                    face = f;
                    break;
                }
            }
            if (face < 0)
                for (int f = 3; f >= 0; --f)
                    if (drate[((size_t)m * T + t) * 4 + f] > 0) {
                        face = f;
                        break;
                    }
            counts[(size_t)m * T + t] -= 1;
            counts[(size_t)m * T + nbr[4 * t + face]] += 1;
        } else {
            size_t q = ch - nd;
            int r = (int)(q / T), t = (int)(q % T);
            for (int i = 0; i < rn[r]; ++i) counts[(size_t)rid[2 * r + i] * T + t] -= 1;
            for (int i = 0; i < pn[r]; ++i) counts[(size_t)pid[3 * r + i] * T + t] += 1;
        }
    }
    free(a);
    free(dtot);
}
