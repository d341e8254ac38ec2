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

/*
 * The same exact process with the direct method organised by tet: the total
 * rate of each tet sits in a binary sum tree, an event picks its tet by
 * descending the tree and its channel inside the tet, and only the tets an
 * event changed are re-summed (O(log T) per event).  The tree is rebuilt
 * from scratch every 2^20 events so that rounding in the partial sums cannot
 * accumulate.  Same arguments as issa_run.
 */
static double tet_rate(int t, int T, int S, int R, const int32_t *counts, const double *dtot, const int32_t *rn,
                       const int32_t *rid, const double *c)
{
    double s = 0.0;
    for (int m = 0; m < S; ++m) s += counts[(size_t)m * T + t] * dtot[(size_t)m * T + t];
    for (int r = 0; r < R; ++r) {
        double h;
        if (rn[r] == 0) h = 1.0;
        else if (rn[r] == 1) h = counts[(size_t)rid[2 * r] * T + t];
        else if (rid[2 * r] == rid[2 * r + 1]) {
            double x = counts[(size_t)rid[2 * r] * T + t];
            h = x * (x - 1.0);
        } else h = (double)counts[(size_t)rid[2 * r] * T + t] * counts[(size_t)rid[2 * r + 1] * T + t];
        s += c[(size_t)r * T + t] * h;
    }
    return s;
}

void issa_tree_run(int T, int S, int R, const int32_t *nbr, const double *drate, const int32_t *rn,
                   const int32_t *rid, const int32_t *pn, const int32_t *pid, const double *c, int32_t *counts,
                   int n_samples, const double *times, uint64_t seed, int32_t *out)
{
    uint64_t st = seed * 0x2545F4914F6CDD1DULL + 777;
    size_t P = 1;
    while (P < (size_t)T) P <<= 1;
    double *tree = (double *)calloc(2 * P, sizeof(double)); /* leaves at [P, P + T) */
    double *dtot = (double *)malloc(sizeof(double) * (size_t)S * T);
    for (int m = 0; m < S; ++m)
        for (int t = 0; t < T; ++t) {
            double s = 0.0;
            for (int f = 0; f < 4; ++f) s += drate[((size_t)m * T + t) * 4 + f];
            dtot[(size_t)m * T + t] = s;
        }
    double now = 0.0;
    int next = 0;
    uint64_t events = 0;
    for (;;) {
        if ((events & ((1u << 20) - 1)) == 0) { /* rebuild */
            for (int t = 0; t < T; ++t) tree[P + t] = tet_rate(t, T, S, R, counts, dtot, rn, rid, c);
            for (size_t i = P - 1; i >= 1; --i) tree[i] = tree[2 * i] + tree[2 * i + 1];
        }
        const double a0 = tree[1];
        double dt = a0 > 0 ? -log(sm_u(&st)) / a0 : INFINITY;
        while (next < n_samples && now + dt >= times[next]) {
            memcpy(out + (size_t)next * S * T, counts, sizeof(int32_t) * (size_t)S * T);
            ++next;
        }
        if (next >= n_samples) break;
        now += dt;
        /* the tet: descend the tree */
        double x = sm_u(&st) * a0;
        size_t i = 1;
        while (i < P) {
            if (x < tree[2 * i] || tree[2 * i + 1] <= 0.0) i = 2 * i;
            else {
                x -= tree[2 * i];
                i = 2 * i + 1;
            }
        }
        int t = (int)(i - P);
        if (t >= T || tree[i] <= 0.0) { /* rounding at the right edge: the last tet with a rate */
            t = T - 1;
            while (t > 0 && tree[P + t] <= 0.0) --t;
        }
        /* the channel inside the tet */
        double y = sm_u(&st) * tree[P + t], cum = 0.0;
        int m_sel = -1, f_sel = -1, r_sel = -1;
        for (int m = 0; m < S && m_sel < 0; ++m)
            for (int f = 0; f < 4; ++f) {
                const double rr = counts[(size_t)m * T + t] * drate[((size_t)m * T + t) * 4 + f];
                cum += rr;
                if (y < cum && rr > 0) {
                    m_sel = m;
                    f_sel = f;
                    break;
                }
            }
        if (m_sel < 0)
            for (int r = 0; r < R; ++r) {
                double h;
                if (rn[r] == 0) h = 1.0;
                else if (rn[r] == 1) h = counts[(size_t)rid[2 * r] * T + t];
                else if (rid[2 * r] == rid[2 * r + 1]) {
                    double xx = counts[(size_t)rid[2 * r] * T + t];
                    h = xx * (xx - 1.0);
                } else h = (double)counts[(size_t)rid[2 * r] * T + t] * counts[(size_t)rid[2 * r + 1] * T + t];
                const double rr = c[(size_t)r * T + t] * h;
                cum += rr;
                if (y < cum && rr > 0) {
                    r_sel = r;
                    break;
                }
                if (rr > 0) r_sel = r; /* fall back to the last channel with a rate */
            }
        int touched[2] = {t, -1};
        if (m_sel >= 0) {
            const int u = nbr[4 * t + f_sel];
            counts[(size_t)m_sel * T + t] -= 1;
            counts[(size_t)m_sel * T + u] += 1;
            touched[1] = u;
        } else if (r_sel >= 0) {
            for (int k = 0; k < rn[r_sel]; ++k) counts[(size_t)rid[2 * r_sel + k] * T + t] -= 1;
            for (int k = 0; k < pn[r_sel]; ++k) counts[(size_t)pid[3 * r_sel + k] * T + t] += 1;
        }
        for (int k = 0; k < 2; ++k) {
            if (touched[k] < 0) continue;
            size_t j = P + (size_t)touched[k];
            tree[j] = tet_rate(touched[k], T, S, R, counts, dtot, rn, rid, c);
            for (j >>= 1; j >= 1; j >>= 1) tree[j] = tree[2 * j] + tree[2 * j + 1];
        }
        ++events;
    }
    free(tree);
    free(dtot);
}
