/*
 * Reference oracle: operator-split stochastic reaction-diffusion on
 * tetrahedral meshes, after Hepburn, Chen & De Schutter (arXiv:1512.03126).
 *
 * TEST INFRASTRUCTURE ONLY -- see oracle.h.  Plain single-threaded C, FP64
 * throughout, built with -ffp-contract=off and no fast-math so that every
 * floating-point expression below is evaluated exactly as written.
 *
 * What it computes, in the paper's order (Algorithm 1, Sec. II.C):
 *   precompute tau = min over tets and diffusing species of 1/d     (Sec. II.A)
 *   per period:  Step 1  align the period to t_end
 *                Step 2  SSA of each tet's reactions up to the last reaction
 *                        before the period ends; on every reaction update the
 *                        occupancy of its reactants and products
 *                Step 3  per diffusing species: mean occupancy Nbar (eq. 2),
 *                        n = binomial(Nbar, zeta) (eq. 3), multinomial split
 *                        over the face neighbours (Sec. II.B)
 *                Step 4  advance time
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - local rate d and weights: finite-volume form, d = D * sum_f A_f/(V delta_f),
 *     w_f proportional to A_f/delta_f; boundary faces carry no flux.
 *   - SSA per tet, independently (diffusion is frozen inside the period).
 *   - non-integer Nbar: stochastic rounding floor(Nbar) + Bernoulli(frac).
 *   - n is clamped to the count present at the end of the SSA.
 *   - transfers are applied synchronously after every tet has drawn.
 *   - binomial: BINV (Kachitvichyanukul & Schmeiser 1988) when n*p < 10,
 *     BTRD (Hoermann 1993) otherwise, reflected for p > 1/2.
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11), key (seed,
 *     realization), counter (draw block, stream, tet, step).
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NA 6.02214076e23          /* Avogadro constant, 1/mol (SI 2019) */
#define ORC_SPLIT_ONE_BY_ONE 10       /* Sec. II.B: below this n, move molecules one by one */
#define ORC_SSA_STREAM 0x80000000u    /* RNG stream id of the reaction SSA */
#define ORC_MAX_SPECIES 64

struct orc_sim {
    int32_t T, S, R;
    int32_t *nbr;        /* [T][4] neighbour across face f (opposite local vertex f), -1 = boundary */
    double *area;        /* [T][4] face areas, m^2 */
    double *w;           /* [T][4] direction weights, sum 1 over interior faces */
    double *g;           /* [T]    sum_f A_f/(V delta_f), 1/m^2; local rate d = D g */
    double *nav;         /* [T]    N_A * volume in litres */
    double *vol;         /* [T]    m^3 */
    double *D;           /* [S] */
    int32_t *rn, *rid, *pn, *pid;  /* reactions: counts and ids */
    double *k;           /* [R] */
    double tau;
    uint32_t key[2];
    int32_t *cnt;        /* [S][T] molecule counts at a period boundary */
    int64_t step;        /* period index k: keys the random streams */
    int64_t anchor_step; /* time(k) = anchor_t + (k - anchor_step) * tau */
    double anchor_t;
    int first_order;     /* 1: n from the count at the end of the period, not Nbar */
    int split_threshold; /* below this n the split goes molecule by molecule */
    int transfer_form;   /* 0: binomial n then split (eq. 3); 1: one split scaled by zeta */
    double tau_scale;
    uint32_t *allowed;   /* [T] bit r: reaction r may fire in the tet (NULL: everywhere) */
    /* per-step scratch */
    int32_t *nend;       /* [S][T] */
    int32_t *out;        /* [T][S][4] molecules sent across each face */
};

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies, with a   */
/* Weyl-sequence key schedule between rounds.                                */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* A uniform double in [0,1) on the 2^-53 grid from two 32-bit words:
 * the top 27 bits of a and the top 26 bits of b. */
static double u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

typedef struct {
    uint32_t key[2];
    uint32_t stream, tet, step;
    uint32_t j;          /* next draw index in this stream */
} orc_rng;

static void rng_init(orc_rng *r, uint64_t seed, int32_t realization, uint32_t stream,
                     uint32_t tet, uint32_t step, uint32_t j)
{
    r->key[0] = (uint32_t)seed;
    r->key[1] = (uint32_t)(seed >> 32) ^ (uint32_t)realization;
    r->stream = stream;
    r->tet = tet;
    r->step = step;
    r->j = j;
}

/* Draw j uses Philox block j/2: words (0,1) when j is even, (2,3) when odd. */
static double next_u(orc_rng *r)
{
    uint32_t ctr[4] = {r->j >> 1, r->stream, r->tet, r->step};
    uint32_t o[4];
    orc_philox4x32_10(ctr, r->key, o);
    double u = (r->j & 1u) ? u53(o[2], o[3]) : u53(o[0], o[1]);
    r->j += 1u;
    return u;
}

double orc_uniform(uint64_t seed, int32_t realization, uint32_t stream, uint32_t tet,
                   uint32_t step, uint32_t j)
{
    orc_rng r;
    rng_init(&r, seed, realization, stream, tet, step, j);
    return next_u(&r);
}

/* ------------------------------------------------------------------------- */
/* Natural logarithm from IEEE basic operations only (Cody & Waite style      */
/* reduction): x = 2^e m with m in [sqrt(1/2), sqrt(2)), f = m - 1,           */
/* s = f/(2+f), ln m = 2 atanh(s) = f - s (f - 2R), R = sum_{i>=1} s^{2i}/(2i+1) */
/* truncated after i = 11 (|s| <= 0.1716, so the tail is below 2^-60).        */
/* ln 2 is split into a 32-bit head (exact when multiplied by e) and a tail.  */
/* ------------------------------------------------------------------------- */
static const double ORC_LN2_HI = 0x1.62e42fee00000p-1;  /* ln 2 with the low 21 mantissa bits cleared */
static const double ORC_LN2_LO = 0x1.a39ef35793c76p-33; /* ln 2 - ORC_LN2_HI, rounded */
static const double ORC_SQRT2 = 0x1.6a09e667f3bcdp+0;   /* sqrt 2, rounded */

double orc_ln(double x)
{
    uint64_t bits;
    memcpy(&bits, &x, sizeof bits);
    int e = (int)((bits >> 52) & 0x7ff);
    if (e == 0) { /* subnormal: scale into the normal range first */
        x = x * 18014398509481984.0; /* 2^54 */
        memcpy(&bits, &x, sizeof bits);
        e = (int)((bits >> 52) & 0x7ff) - 54;
    }
    e -= 1023;
    bits = (bits & 0x000fffffffffffffULL) | 0x3ff0000000000000ULL;
    double m;
    memcpy(&m, &bits, sizeof m);
    if (m > ORC_SQRT2) {
        m = m * 0.5;
        e += 1;
    }
    double f = m - 1.0;
    double s = f / (2.0 + f);
    double z = s * s;
    double R = z * (1.0 / 3.0 + z * (1.0 / 5.0 + z * (1.0 / 7.0 + z * (1.0 / 9.0 +
               z * (1.0 / 11.0 + z * (1.0 / 13.0 + z * (1.0 / 15.0 + z * (1.0 / 17.0 +
               z * (1.0 / 19.0 + z * (1.0 / 21.0 + z * (1.0 / 23.0)))))))))));
    double lnm = f - s * (f - 2.0 * R);
    double de = (double)e;
    return de * ORC_LN2_HI + (lnm + de * ORC_LN2_LO);
}

/* ------------------------------------------------------------------------- */
/* Binomial sampler.  Sec. II.A: n = binomial(N, zeta) drawn with "a standard */
/* binomial function".  Exact-in-law algorithms are used:                     */
/*   p > 1/2        -> n - Binomial(n, 1-p)                                  */
/*   n p < 10       -> BINV inversion (Kachitvichyanukul & Schmeiser 1988)    */
/*   otherwise      -> BTRD transformed rejection with decomposition          */
/*                     (Hoermann 1993, J. Stat. Comput. Simul. 46:101-110)    */
/* ------------------------------------------------------------------------- */

/* q^n by square-and-multiply over the bits of n, low bit first. */
static double pow_int(double q, int64_t n)
{
    double result = 1.0, base = q;
    while (n > 0) {
        if (n & 1) result = result * base;
        n >>= 1;
        if (n > 0) base = base * base;
    }
    return result;
}

static int64_t binv(int64_t n, double p, orc_rng *g)
{
    double q = 1.0 - p;
    double s = p / q;
    double a = (double)(n + 1) * s;
    double r0 = pow_int(q, n);      /* P(X = 0) */
    for (;;) {
        double u = next_u(g);
        int64_t x = 0;
        double pr = r0;
        int ok = 1;
        while (u > pr) {
            u = u - pr;
            x += 1;
            if (x > n) { ok = 0; break; }   /* rounding left mass over: redraw */
            pr = pr * (a / (double)x - s);  /* P(x)/P(x-1) = ((n+1)/x - 1) p/q */
        }
        if (ok) return x;
    }
}

/* Stirling-series error fc(k) = ln k! - [(k+1/2) ln(k+1) - (k+1) + ln(2 pi)/2]:
 * exact values for k < 10, three-term series beyond. */
static const double ORC_FC[10] = {
    0x1.4c071bcda0a5bp-4, 0x1.52a9b923ea649p-5, 0x1.c579a268d80b3p-6,
    0x1.54a2662fd78a9p-6, 0x1.10b4e513fcbedp-6, 0x1.c6b167bebdf36p-7,
    0x1.85d4d612e4a86p-7, 0x1.552805e7b3076p-7, 0x1.2f4871b12ab64p-7,
    0x1.10f9d4c0743a7p-7,
};

static double fc(int64_t k)
{
    if (k < 10) return ORC_FC[k];
    double ikp1 = 1.0 / (double)(k + 1);
    double ik2 = ikp1 * ikp1;
    return (1.0 / 12.0 - (1.0 / 360.0 - (1.0 / 1260.0) * ik2) * ik2) * ikp1;
}

static int64_t btrd(int64_t n, double p, orc_rng *g)
{
    /* set-up (p <= 1/2, n p >= 10) */
    double nd = (double)n;
    double q = 1.0 - p;
    double m = floor((nd + 1.0) * p);          /* mode */
    double r = p / q;
    double nr = (nd + 1.0) * r;
    double npq = (nd * p) * q;
    double sq = sqrt(npq);
    double b = 1.15 + 2.53 * sq;
    double a = (-0.0873 + 0.0248 * b) + 0.01 * p;
    double c = nd * p + 0.5;
    double alpha = (2.83 + 5.1 / b) * sq;
    double vr = 0.92 - 4.2 / b;
    double urvr = 0.86 * vr;

    for (;;) {
        /* 1: the inner box accepts immediately */
        double v = next_u(g);
        double u;
        if (v <= urvr) {
            u = v / vr - 0.43;
            double kd = floor(((2.0 * a) / (0.5 - fabs(u)) + b) * u + c);
            if (kd < 0.0 || kd > nd) continue;   /* cannot happen for n p >= 10 */
            return (int64_t)kd;
        }
        /* 2: a point (u, v) of the hat outside the box */
        if (v >= vr) {
            u = next_u(g) - 0.5;
        } else {
            u = v / vr - 0.93;
            u = (u < 0.0 ? -0.5 : 0.5) - u;
            v = next_u(g) * vr;
        }
        /* 3.0 */
        double us = 0.5 - fabs(u);
        double kd = floor(((2.0 * a) / us + b) * u + c);
        if (kd < 0.0 || kd > nd) continue;
        v = v * alpha / (a / (us * us) + b);
        double km = fabs(kd - m);
        if (km <= 15.0) {
            /* 3.2: f(k)/f(m) by the recursion f(i)/f(i-1) = nr/i - r */
            double f = 1.0;
            if (m < kd) {
                double i = m;
                do {
                    i += 1.0;
                    f = f * (nr / i - r);
                } while (i != kd);
            } else if (m > kd) {
                double i = kd;
                do {
                    i += 1.0;
                    v = v * (nr / i - r);
                } while (i != m);
            }
            if (v <= f) return (int64_t)kd;
            continue;
        }
        /* 3.3: squeeze on log scale */
        v = orc_ln(v);
        double rho = (km / npq) * (((km / 3.0 + 0.625) * km + 1.0 / 6.0) / npq + 0.5);
        double t = -(km * km) / (2.0 * npq);
        if (v < t - rho) return (int64_t)kd;
        if (v > t + rho) continue;
        /* 3.4-3.5: final test with the Stirling corrections */
        double nm = nd - m + 1.0;
        double h = (m + 0.5) * orc_ln((m + 1.0) / (r * nm)) + fc((int64_t)m) + fc(n - (int64_t)m);
        double nk = nd - kd + 1.0;
        if (v <= h + (nd + 1.0) * orc_ln(nm / nk) + (kd + 0.5) * orc_ln(nk * r / (kd + 1.0))
                      - fc((int64_t)kd) - fc(n - (int64_t)kd))
            return (int64_t)kd;
    }
}

static int64_t binomial(int64_t n, double p, orc_rng *g)
{
    if (n <= 0 || p <= 0.0) return 0;
    if (p >= 1.0) return n;
    if (p > 0.5) return n - binomial(n, 1.0 - p, g);
    if ((double)n * p < 10.0) return binv(n, p, g);
    return btrd(n, p, g);
}

int64_t orc_binomial(int64_t n, double p, uint64_t seed, int32_t realization,
                     uint32_t stream, uint32_t tet, uint32_t step, uint32_t *j)
{
    orc_rng r;
    rng_init(&r, seed, realization, stream, tet, step, *j);
    int64_t x = binomial(n, p, &r);
    *j = r.j;
    return x;
}

/* ------------------------------------------------------------------------- */
/* Multinomial split of n departing molecules over the interior faces        */
/* (Sec. II.B).  Below 10 molecules each one picks a face by a categorical    */
/* draw; otherwise n_i = binomial(n - sum_{j<i} n_j, w_i / (1 - sum_{j<i} w_j)) */
/* face by face, the last interior face taking the remainder (p = 1).        */
/* ------------------------------------------------------------------------- */
static void split(int64_t n, const double *w, const int32_t *nbr, int threshold, orc_rng *g, int64_t out[4])
{
    out[0] = out[1] = out[2] = out[3] = 0;
    if (n <= 0) return;
    int faces[4], nf = 0;
    for (int f = 0; f < 4; ++f)
        if (nbr[f] >= 0) faces[nf++] = f;
    if (nf == 0) return;
    if (nf == 1) {
        out[faces[0]] = n;
        return;
    }
    if (n < threshold) {
        for (int64_t i = 0; i < n; ++i) {
            double U = next_u(g);
            int chosen = faces[nf - 1];
            double c = 0.0;
            for (int q = 0; q < nf - 1; ++q) {
                c = c + w[faces[q]];
                if (U < c) {
                    chosen = faces[q];
                    break;
                }
            }
            out[chosen] += 1;
        }
        return;
    }
    int64_t rem = n;
    double S = 0.0;
    for (int q = 0; q < nf; ++q) {
        int f = faces[q];
        if (q == nf - 1) {
            out[f] = rem;
            break;
        }
        double p = w[f] / (1.0 - S);
        if (p > 1.0) p = 1.0;
        int64_t nfc = binomial(rem, p, g);
        out[f] = nfc;
        rem -= nfc;
        S = S + w[f];
        if (rem == 0) break;
    }
}

/* ------------------------------------------------------------------------- */
/* The alternative stated at the end of Sec. II.B: the whole population N    */
/* split at once over the directions with weights zeta w_i, the molecules    */
/* that draw no direction (probability 1 - zeta) staying.  Below the          */
/* threshold one categorical draw per molecule (directions in face order,    */
/* "stay" last); otherwise sequential binomials with                          */
/* p_i = zeta w_i / (1 - sum_{j<i} zeta w_j), "stay" taking the rest.  The    */
/* molecules that leave are Binomial(N, zeta) and, given their number,        */
/* multinomial over w: the law of Steps 3.2-3.3.  Returns how many leave.     */
/* ------------------------------------------------------------------------- */
static int64_t split_scaled(int64_t N, double zeta, const double *w, const int32_t *nbr, int threshold, orc_rng *g,
                            int64_t out[4])
{
    out[0] = out[1] = out[2] = out[3] = 0;
    if (N <= 0) return 0;
    int faces[4], nf = 0;
    for (int f = 0; f < 4; ++f)
        if (nbr[f] >= 0) faces[nf++] = f;
    if (nf == 0) return 0;
    int64_t moved = 0;
    if (N < threshold) {
        for (int64_t i = 0; i < N; ++i) {
            double U = next_u(g);
            double c = 0.0;
            for (int q = 0; q < nf; ++q) {
                c = c + zeta * w[faces[q]];
                if (U < c) {
                    out[faces[q]] += 1;
                    moved += 1;
                    break;
                }
            }
        }
        return moved;
    }
    int64_t rem = N;
    double Sz = 0.0;
    for (int q = 0; q < nf; ++q) {
        int f = faces[q];
        double p = (zeta * w[f]) / (1.0 - Sz);
        if (p > 1.0) p = 1.0;
        int64_t nfc = binomial(rem, p, g);
        out[f] = nfc;
        moved += nfc;
        rem -= nfc;
        Sz = Sz + zeta * w[f];
        if (rem == 0) break;
    }
    return moved;
}

uint32_t orc_split(int64_t n, const double *w, const int32_t *nbr, uint64_t seed,
                   int32_t realization, uint32_t stream, uint32_t tet, uint32_t step,
                   uint32_t j, int64_t *out)
{
    orc_rng r;
    rng_init(&r, seed, realization, stream, tet, step, j);
    split(n, w, nbr, ORC_SPLIT_ONE_BY_ONE, &r, out);
    return r.j;
}

/* ------------------------------------------------------------------------- */
/* Geometry and set-up (Sec. II.A, Algorithm 1 "precompute tau").            */
/* ------------------------------------------------------------------------- */
static void sub3(const double *a, const double *b, double *o)
{
    o[0] = a[0] - b[0];
    o[1] = a[1] - b[1];
    o[2] = a[2] - b[2];
}
static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b)
{
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}
static double norm3(const double *a)
{
    return sqrt((a[0] * a[0] + a[1] * a[1]) + a[2] * a[2]);
}

typedef struct {
    int32_t v[3];
    int32_t tet, face;
} orc_face;

static int face_cmp(const void *pa, const void *pb)
{
    const orc_face *a = (const orc_face *)pa, *b = (const orc_face *)pb;
    for (int i = 0; i < 3; ++i) {
        if (a->v[i] != b->v[i]) return a->v[i] < b->v[i] ? -1 : 1;
    }
    if (a->tet != b->tet) return a->tet < b->tet ? -1 : 1;
    return a->face - b->face;
}

static void sort3(int32_t *v)
{
    int32_t t;
    if (v[0] > v[1]) { t = v[0]; v[0] = v[1]; v[1] = t; }
    if (v[1] > v[2]) { t = v[1]; v[1] = v[2]; v[2] = t; }
    if (v[0] > v[1]) { t = v[0]; v[0] = v[1]; v[1] = t; }
}

static void set_err(char *err, const char *msg)
{
    if (err) snprintf(err, 256, "%s", msg);
}

/* Cells are tetrahedra (nv = 4, volume diffusion) or triangles (nv = 3,     */
/* surface diffusion, the transfer between surface triangles of Sec. III.A). */
/* A triangle is the 2D subvolume: its "faces" are its edges (edge e         */
/* opposite local vertex e), r_e = L_e / (A delta_e) with L_e the edge        */
/* length, A the area and delta_e the distance between barycentres, and the  */
/* unit of amount is N_A A (mol per m^2) instead of N_A V.  Slot 3 of a       */
/* triangle is always a boundary.                                             */
static orc_sim *create_cells(int nv, int32_t n_verts, const double *xyz, int32_t n_tets,
                             const int32_t *tet_verts, int32_t n_species, const double *D,
                             int32_t n_reac, const int32_t *reac_n, const int32_t *reac_ids,
                             const int32_t *prod_n, const int32_t *prod_ids, const double *k,
                             double tau_scale, uint64_t seed, int32_t realization, char *err)
{
    if (n_verts < nv || n_tets < 1 || n_species < 1 || n_species > ORC_MAX_SPECIES || n_reac < 0) {
        set_err(err, "bad sizes");
        return NULL;
    }
    if (!(tau_scale > 0.0 && tau_scale <= 1.0)) {
        set_err(err, "tau_scale must be in (0,1]");
        return NULL;
    }
    for (int64_t i = 0; i < (int64_t)nv * n_tets; ++i) {
        if (tet_verts[i] < 0 || tet_verts[i] >= n_verts) {
            set_err(err, "vertex id out of range");
            return NULL;
        }
    }
    for (int r = 0; r < n_reac; ++r) {
        if (reac_n[r] < 0 || reac_n[r] > 2 || prod_n[r] < 0 || prod_n[r] > 3 || !(k[r] >= 0.0)) {
            set_err(err, "bad reaction");
            return NULL;
        }
        for (int i = 0; i < reac_n[r]; ++i)
            if (reac_ids[2 * r + i] < 0 || reac_ids[2 * r + i] >= n_species) {
                set_err(err, "bad reactant id");
                return NULL;
            }
        for (int i = 0; i < prod_n[r]; ++i)
            if (prod_ids[3 * r + i] < 0 || prod_ids[3 * r + i] >= n_species) {
                set_err(err, "bad product id");
                return NULL;
            }
    }

    orc_sim *s = (orc_sim *)calloc(1, sizeof *s);
    int32_t T = n_tets, S = n_species, R = n_reac;
    s->T = T;
    s->S = S;
    s->R = R;
    s->nbr = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)T);
    s->area = (double *)malloc(sizeof(double) * 4 * (size_t)T);
    s->w = (double *)malloc(sizeof(double) * 4 * (size_t)T);
    s->g = (double *)malloc(sizeof(double) * (size_t)T);
    s->nav = (double *)malloc(sizeof(double) * (size_t)T);
    s->vol = (double *)malloc(sizeof(double) * (size_t)T);
    s->D = (double *)malloc(sizeof(double) * (size_t)S);
    s->rn = (int32_t *)malloc(sizeof(int32_t) * (size_t)(R + 1));
    s->rid = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(R + 1));
    s->pn = (int32_t *)malloc(sizeof(int32_t) * (size_t)(R + 1));
    s->pid = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(R + 1));
    s->k = (double *)malloc(sizeof(double) * (size_t)(R + 1));
    s->cnt = (int32_t *)calloc((size_t)S * T, sizeof(int32_t));
    s->nend = (int32_t *)calloc((size_t)S * T, sizeof(int32_t));
    s->out = (int32_t *)calloc((size_t)T * S * 4, sizeof(int32_t));
    memcpy(s->D, D, sizeof(double) * (size_t)S);
    for (int r = 0; r < R; ++r) {
        s->rn[r] = reac_n[r];
        s->pn[r] = prod_n[r];
        s->rid[2 * r] = reac_ids[2 * r];
        s->rid[2 * r + 1] = reac_ids[2 * r + 1];
        for (int i = 0; i < 3; ++i) s->pid[3 * r + i] = prod_ids[3 * r + i];
        s->k[r] = k[r];
    }
    s->key[0] = (uint32_t)seed;
    s->key[1] = (uint32_t)(seed >> 32) ^ (uint32_t)realization;

    /* volumes, barycentres, face areas; face f is opposite local vertex f */
    double *bc = (double *)malloc(sizeof(double) * 3 * (size_t)T);
    for (int32_t t = 0; t < T && nv == 3; ++t) {
        /* triangle: area, barycentre, edge lengths (edge e opposite vertex e) */
        const double *P[3];
        for (int v = 0; v < 3; ++v) P[v] = xyz + 3 * (size_t)tet_verts[3 * (size_t)t + v];
        double e1[3], e2[3], cr[3];
        sub3(P[1], P[0], e1);
        sub3(P[2], P[0], e2);
        cross3(e1, e2, cr);
        double A = 0.5 * norm3(cr);
        if (!(A > 0.0)) {
            set_err(err, "degenerate triangle");
            free(bc);
            orc_destroy(s);
            return NULL;
        }
        s->vol[t] = A;
        s->nav[t] = ORC_NA * A;
        for (int d = 0; d < 3; ++d) bc[3 * (size_t)t + d] = ((P[0][d] + P[1][d]) + P[2][d]) / 3.0;
        for (int f = 0; f < 3; ++f) {
            const double *Q[2];
            int qi = 0;
            for (int v = 0; v < 3; ++v)
                if (v != f) Q[qi++] = P[v];
            double dd[3];
            sub3(Q[1], Q[0], dd);
            s->area[4 * (size_t)t + f] = norm3(dd);
        }
        s->area[4 * (size_t)t + 3] = 0.0;
    }
    for (int32_t t = 0; t < T && nv == 4; ++t) {
        const double *P[4];
        for (int v = 0; v < 4; ++v) P[v] = xyz + 3 * (size_t)tet_verts[4 * (size_t)t + v];
        double e1[3], e2[3], e3[3], cr[3];
        sub3(P[1], P[0], e1);
        sub3(P[2], P[0], e2);
        sub3(P[3], P[0], e3);
        cross3(e1, e2, cr);
        double vol = fabs(dot3(cr, e3)) / 6.0;
        if (!(vol > 0.0)) {
            set_err(err, "degenerate tetrahedron");
            free(bc);
            orc_destroy(s);
            return NULL;
        }
        s->vol[t] = vol;
        s->nav[t] = ORC_NA * (vol * 1000.0);
        for (int d = 0; d < 3; ++d)
            bc[3 * (size_t)t + d] = ((P[0][d] + P[1][d]) + (P[2][d] + P[3][d])) * 0.25;
        for (int f = 0; f < 4; ++f) {
            const double *Q[3];
            int qi = 0;
            for (int v = 0; v < 4; ++v)
                if (v != f) Q[qi++] = P[v];
            double a1[3], a2[3], ac[3];
            sub3(Q[1], Q[0], a1);
            sub3(Q[2], Q[0], a2);
            cross3(a1, a2, ac);
            s->area[4 * (size_t)t + f] = 0.5 * norm3(ac);
        }
    }

    /* face matching: sort all faces by their sorted vertices (a triangle's */
    /* edges carry -1 as third vertex) */
    orc_face *faces = (orc_face *)malloc(sizeof(orc_face) * (size_t)nv * (size_t)T);
    for (int32_t t = 0; t < T; ++t) {
        for (int f = 0; f < 4; ++f) s->nbr[4 * (size_t)t + f] = -1;
        for (int f = 0; f < nv; ++f) {
            orc_face *F = &faces[(size_t)nv * t + f];
            int qi = 0;
            F->v[2] = -1;
            for (int v = 0; v < nv; ++v)
                if (v != f) F->v[qi++] = tet_verts[(size_t)nv * t + v];
            sort3(F->v);
            F->tet = t;
            F->face = f;
        }
    }
    qsort(faces, (size_t)nv * T, sizeof(orc_face), face_cmp);
    size_t nF = (size_t)nv * T;
    for (size_t i = 0; i < nF;) {
        size_t jn = i + 1;
        while (jn < nF && memcmp(faces[jn].v, faces[i].v, sizeof faces[i].v) == 0) ++jn;
        size_t mult = jn - i;
        if (mult > 2 || (mult == 2 && faces[i].tet == faces[i + 1].tet)) {
            set_err(err, nv == 4 ? "face shared by more than two tetrahedra (or repeated in one)"
                                 : "edge shared by more than two triangles (or repeated in one)");
            free(faces);
            free(bc);
            orc_destroy(s);
            return NULL;
        }
        if (mult == 2) {
            s->nbr[4 * (size_t)faces[i].tet + faces[i].face] = faces[i + 1].tet;
            s->nbr[4 * (size_t)faces[i + 1].tet + faces[i + 1].face] = faces[i].tet;
        }
        i = jn;
    }
    free(faces);

    /* r_f = A_f / (V delta_f), g = sum r_f, w_f = r_f / g */
    for (int32_t t = 0; t < T; ++t) {
        double r[4];
        for (int f = 0; f < 4; ++f) {
            int32_t u = s->nbr[4 * (size_t)t + f];
            if (u < 0) {
                r[f] = 0.0;
                continue;
            }
            double d[3];
            sub3(bc + 3 * (size_t)u, bc + 3 * (size_t)t, d);
            double delta = norm3(d);
            r[f] = s->area[4 * (size_t)t + f] / (s->vol[t] * delta);
        }
        double gt = ((r[0] + r[1]) + r[2]) + r[3];
        s->g[t] = gt;
        for (int f = 0; f < 4; ++f) s->w[4 * (size_t)t + f] = gt > 0.0 ? r[f] / gt : 0.0;
    }
    free(bc);

    /* tau = tau_scale * min over tets and diffusing species of 1/(D_m g_t) */
    double best = INFINITY;
    for (int m = 0; m < S; ++m) {
        if (!(D[m] > 0.0)) continue;
        for (int32_t t = 0; t < T; ++t) {
            if (!(s->g[t] > 0.0)) continue;
            double inv = 1.0 / (D[m] * s->g[t]);
            if (inv < best) best = inv;
        }
    }
    if (!(best < INFINITY)) {
        set_err(err, "no diffusing species on a connected cell: tau undefined");
        orc_destroy(s);
        return NULL;
    }
    s->tau = tau_scale * best;
    s->tau_scale = tau_scale;
    s->split_threshold = ORC_SPLIT_ONE_BY_ONE;
    s->step = 0;
    s->anchor_step = 0;
    s->anchor_t = 0.0;
    return s;
}

orc_sim *orc_create(int32_t n_verts, const double *xyz, int32_t n_tets, const int32_t *tet_verts,
                    int32_t n_species, const double *D, int32_t n_reac, const int32_t *reac_n,
                    const int32_t *reac_ids, const int32_t *prod_n, const int32_t *prod_ids, const double *k,
                    double tau_scale, uint64_t seed, int32_t realization, char *err)
{
    return create_cells(4, n_verts, xyz, n_tets, tet_verts, n_species, D, n_reac, reac_n, reac_ids, prod_n,
                        prod_ids, k, tau_scale, seed, realization, err);
}

orc_sim *orc_create_surface(int32_t n_verts, const double *xyz, int32_t n_tris, const int32_t *tri_verts,
                            int32_t n_species, const double *D, int32_t n_reac, const int32_t *reac_n,
                            const int32_t *reac_ids, const int32_t *prod_n, const int32_t *prod_ids,
                            const double *k, double tau_scale, uint64_t seed, int32_t realization, char *err)
{
    return create_cells(3, n_verts, xyz, n_tris, tri_verts, n_species, D, n_reac, reac_n, reac_ids, prod_n,
                        prod_ids, k, tau_scale, seed, realization, err);
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->nbr);
    free(s->area);
    free(s->w);
    free(s->g);
    free(s->nav);
    free(s->vol);
    free(s->D);
    free(s->rn);
    free(s->rid);
    free(s->pn);
    free(s->pid);
    free(s->k);
    free(s->cnt);
    free(s->nend);
    free(s->out);
    free(s->allowed);
    free(s);
}

double orc_tau(const orc_sim *s) { return s->tau; }

/* The paper's comparison method of Sec. III.B (Fig. 7): the diffusive
 * transfer uses the count at the end of the period instead of Nbar. */
void orc_set_first_order(orc_sim *s, int on) { s->first_order = on ? 1 : 0; }

/* Sec. II.B: the split switches from one-by-one to the multinomial function
 * at this n (10 in the paper's implementation); any threshold >= 1 gives the
 * same law, only the draws differ. */
void orc_set_split_threshold(orc_sim *s, int threshold) { s->split_threshold = threshold < 1 ? 1 : threshold; }
void orc_set_transfer_form(orc_sim *s, int form) { s->transfer_form = form == 1 ? 1 : 0; }

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Sec. II.A: ignoring the k tet-species with the largest local rates raises
 * tau; there zeta would exceed 1 and is held at 1.  tau becomes tau_scale
 * times the (k+1)-th smallest 1/(D_m g_t).  Returns the new tau. */
double orc_set_tau_outliers(orc_sim *s, int32_t k)
{
    size_t cnt = 0;
    double *v = (double *)malloc(sizeof(double) * (size_t)s->T * (size_t)s->S);
    for (int m = 0; m < s->S; ++m) {
        if (!(s->D[m] > 0.0)) continue;
        for (int32_t t = 0; t < s->T; ++t)
            if (s->g[t] > 0.0) v[cnt++] = 1.0 / (s->D[m] * s->g[t]);
    }
    qsort(v, cnt, sizeof(double), cmp_double);
    size_t idx = k < 0 ? 0 : (size_t)k;
    if (idx >= cnt) idx = cnt - 1;
    s->tau = s->tau_scale * v[idx];
    free(v);
    return s->tau;
}

/* Restricts reaction r to the listed tets (a localized reaction, e.g. the
 * influx at the ends of the tube of Sec. III.B). */
void orc_set_reaction_region(orc_sim *s, int32_t r, int32_t n, const int32_t *tets)
{
    if (!s->allowed) {
        s->allowed = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)s->T);
        for (int32_t t = 0; t < s->T; ++t) s->allowed[t] = 0xFFFFFFFFu;
    }
    for (int32_t t = 0; t < s->T; ++t) s->allowed[t] &= ~(1u << r);
    for (int32_t i = 0; i < n; ++i) s->allowed[tets[i]] |= 1u << r;
}

void orc_geometry(const orc_sim *s, int32_t *nbr, double *w, double *g, double *nav, double *vol,
                  double *area)
{
    size_t T = (size_t)s->T;
    if (nbr) memcpy(nbr, s->nbr, sizeof(int32_t) * 4 * T);
    if (w) memcpy(w, s->w, sizeof(double) * 4 * T);
    if (g) memcpy(g, s->g, sizeof(double) * T);
    if (nav) memcpy(nav, s->nav, sizeof(double) * T);
    if (vol) memcpy(vol, s->vol, sizeof(double) * T);
    if (area) memcpy(area, s->area, sizeof(double) * 4 * T);
}

void orc_set_counts(orc_sim *s, int32_t species, const int32_t *counts)
{
    memcpy(s->cnt + (size_t)species * s->T, counts, sizeof(int32_t) * (size_t)s->T);
}

void orc_get_counts(const orc_sim *s, int32_t species, int32_t *counts)
{
    memcpy(counts, s->cnt + (size_t)species * s->T, sizeof(int32_t) * (size_t)s->T);
}

void orc_set_state(orc_sim *s, int64_t step_index, double t)
{
    s->step = step_index;
    s->anchor_step = step_index;
    s->anchor_t = t;
}

static double time_of(const orc_sim *s, int64_t k)
{
    return s->anchor_t + (double)(k - s->anchor_step) * s->tau;
}

void orc_get_time(const orc_sim *s, double *t, int64_t *step_index)
{
    if (t) *t = time_of(s, s->step);
    if (step_index) *step_index = s->step;
}

/* ------------------------------------------------------------------------- */
/* One period (Algorithm 1, Steps 2-3, then synchronous application).        */
/* ------------------------------------------------------------------------- */

/* the stream of one (stream id, tet, period) of this simulation, at draw 0 */
static void rng_sim(orc_rng *r, const orc_sim *s, uint32_t stream, uint32_t tet, uint32_t step)
{
    r->key[0] = s->key[0];
    r->key[1] = s->key[1];
    r->stream = stream;
    r->tet = tet;
    r->step = step;
    r->j = 0;
}

/* propensity constant c_r of reaction r in tet t (mass action, SI units) */
static double rate_const(const orc_sim *s, int r, int32_t t)
{
    if (s->rn[r] == 0) return s->k[r] * s->nav[t];   /* M/s -> molecules/s */
    if (s->rn[r] == 1) return s->k[r];               /* 1/s */
    return s->k[r] / s->nav[t];                      /* 1/(M s) -> 1/s per pair */
}

/* number of distinct reactant combinations h_r */
static double combos(const orc_sim *s, int r, const int64_t *N)
{
    if (s->rn[r] == 0) return 1.0;
    int32_t a = s->rid[2 * r];
    if (s->rn[r] == 1) return (double)N[a];
    int32_t b = s->rid[2 * r + 1];
    if (a == b) return (double)N[a] * (double)(N[a] - 1);
    return (double)N[a] * (double)N[b];
}

static int involves(const orc_sim *s, int r, int m)
{
    for (int i = 0; i < s->rn[r]; ++i)
        if (s->rid[2 * r + i] == m) return 1;
    for (int i = 0; i < s->pn[r]; ++i)
        if (s->pid[3 * r + i] == m) return 1;
    return 0;
}

void orc_step(orc_sim *s, double tau_k, double *nbar_out, int32_t *n_out)
{
    const int32_t T = s->T, S = s->S, R = s->R;
    const uint32_t step32 = (uint32_t)s->step;
    int64_t N[ORC_MAX_SPECIES];
    double occ[ORC_MAX_SPECIES], tl[ORC_MAX_SPECIES];
    int touched[ORC_MAX_SPECIES];
    double a[64 + 1];
    double *av = R > 64 ? (double *)malloc(sizeof(double) * (size_t)R) : a;

    for (int32_t t = 0; t < T; ++t) {
        for (int m = 0; m < S; ++m) {
            N[m] = s->cnt[(size_t)m * T + t];
            occ[m] = 0.0;
            tl[m] = 0.0;
            touched[m] = 0;
        }

        /* Step 2: Gillespie direct method inside this tet over [0, tau_k);
         * the event that would land at or beyond tau_k is discarded. */
        orc_rng rs;
        rng_sim(&rs, s, ORC_SSA_STREAM, (uint32_t)t, step32);
        double now = 0.0;
        for (;;) {
            double a0 = 0.0;
            for (int r = 0; r < R; ++r) {
                av[r] = (s->allowed && !((s->allowed[t] >> r) & 1u)) ? 0.0 : rate_const(s, r, t) * combos(s, r, N);
                a0 = a0 + av[r];
            }
            if (!(a0 > 0.0)) break;
            double U = 1.0 - next_u(&rs);          /* in (0, 1] */
            double dt = -orc_ln(U) / a0;
            if (now + dt >= tau_k) break;
            now = now + dt;
            double x = next_u(&rs) * a0;
            int chosen = -1;
            double cum = 0.0;
            for (int r = 0; r < R; ++r) {
                cum = cum + av[r];
                if (x < cum) {
                    chosen = r;
                    break;
                }
            }
            if (chosen < 0) { /* x rounded up to a0: the last reaction that can fire */
                for (int r = R - 1; r >= 0; --r)
                    if (av[r] > 0.0) {
                        chosen = r;
                        break;
                    }
            }
            /* Step 2.1: occupancy of every reactant and product */
            for (int m = 0; m < S; ++m) {
                if (!involves(s, chosen, m)) continue;
                occ[m] = occ[m] + (double)N[m] * (now - tl[m]);
                tl[m] = now;
                touched[m] = 1;
            }
            for (int i = 0; i < s->rn[chosen]; ++i) N[s->rid[2 * chosen + i]] -= 1;
            for (int i = 0; i < s->pn[chosen]; ++i) N[s->pid[3 * chosen + i]] += 1;
        }

        /* Step 3: diffusion of each diffusing species at the end of the period */
        for (int m = 0; m < S; ++m) {
            int32_t *o = s->out + ((size_t)t * S + m) * 4;
            o[0] = o[1] = o[2] = o[3] = 0;
            double nbar = (touched[m] && !s->first_order)
                              ? (occ[m] + (double)N[m] * (tau_k - tl[m])) / tau_k
                              : (double)N[m];
            int64_t n = 0;
            if (s->D[m] > 0.0) {
                orc_rng rd;
                rng_sim(&rd, s, (uint32_t)m, (uint32_t)t, step32);
                /* Step 3.1: Nbar to an integer population by stochastic rounding */
                int64_t Ni = (int64_t)floor(nbar);
                double fr = nbar - (double)Ni;
                if (fr > 0.0 && next_u(&rd) < fr) Ni += 1;
                /* Step 3.2: n = binomial(Nbar, zeta), zeta = tau_k d = tau_k D g */
                double zeta = (tau_k * s->D[m]) * s->g[t];
                if (zeta > 1.0) zeta = 1.0;
                int64_t nf[4];
                if (s->transfer_form == 1) {
                    /* one multinomial over the directions scaled by zeta; more
                       than the molecules present leave: the present ones are
                       split as in Step 3.3 (the same law as min(., N)) */
                    n = split_scaled(Ni, zeta, s->w + 4 * (size_t)t, s->nbr + 4 * (size_t)t, s->split_threshold,
                                     &rd, nf);
                    if (n > N[m]) {
                        n = N[m];
                        split(n, s->w + 4 * (size_t)t, s->nbr + 4 * (size_t)t, s->split_threshold, &rd, nf);
                    }
                } else {
                    n = binomial(Ni, zeta, &rd);
                    if (n > N[m]) n = N[m];
                    /* Step 3.3: multinomial split over the face neighbours */
                    split(n, s->w + 4 * (size_t)t, s->nbr + 4 * (size_t)t, s->split_threshold, &rd, nf);
                }
                for (int f = 0; f < 4; ++f) o[f] = (int32_t)nf[f];
                N[m] -= n;
            }
            if (nbar_out) nbar_out[(size_t)m * T + t] = nbar;
            if (n_out) n_out[(size_t)m * T + t] = (int32_t)n;
            s->nend[(size_t)m * T + t] = (int32_t)N[m];
        }
    }

    /* all transfers applied together, after every tet has drawn */
    memcpy(s->cnt, s->nend, sizeof(int32_t) * (size_t)S * T);
    for (int32_t t = 0; t < T; ++t)
        for (int m = 0; m < S; ++m)
            for (int f = 0; f < 4; ++f) {
                int32_t c = s->out[((size_t)t * S + m) * 4 + f];
                if (c) s->cnt[(size_t)m * T + s->nbr[4 * (size_t)t + f]] += c;
            }
    if (av != a) free(av);
    s->step += 1;
}

void orc_run_steps(orc_sim *s, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) orc_step(s, s->tau, NULL, NULL);
}

/* Algorithm 1, Step 1: the last period is shortened to end at t_end. */
void orc_run_until(orc_sim *s, double t_end)
{
    for (;;) {
        double t = time_of(s, s->step);
        if (t >= t_end) return;
        if (t + s->tau > t_end) {
            orc_step(s, t_end - t, NULL, NULL);
            s->anchor_step = s->step;
            s->anchor_t = t_end;
            return;
        }
        orc_step(s, s->tau, NULL, NULL);
    }
}

void orc_split_many_threshold(int64_t n, const double *w, const int32_t *nbr, uint64_t seed, int32_t count,
                              int32_t threshold, int64_t *out);

/* ------------------------------------------------------------------------- */
/* Batch helpers for the statistical tests: sample i uses the stream          */
/* (seed, realization 0, stream 0, tet i, step 0) from draw 0.               */
/* ------------------------------------------------------------------------- */
void orc_binomial_many(int64_t n, double p, uint64_t seed, int32_t count, int64_t *out)
{
    for (int32_t i = 0; i < count; ++i) {
        orc_rng r;
        rng_init(&r, seed, 0, 0u, (uint32_t)i, 0u, 0u);
        out[i] = binomial(n, p, &r);
    }
}

void orc_split_many(int64_t n, const double *w, const int32_t *nbr, uint64_t seed, int32_t count,
                    int64_t *out)
{
    orc_split_many_threshold(n, w, nbr, seed, count, ORC_SPLIT_ONE_BY_ONE, out);
}

void orc_split_scaled_many(int64_t n, double zeta, const double *w, const int32_t *nbr, uint64_t seed,
                           int32_t count, int32_t threshold, int64_t *out)
{
    for (int32_t i = 0; i < count; ++i) {
        orc_rng r;
        rng_init(&r, seed, 0, 0u, (uint32_t)i, 0u, 0u);
        (void)split_scaled(n, zeta, w, nbr, threshold < 1 ? 1 : threshold, &r, out + 4 * (size_t)i);
    }
}

void orc_split_many_threshold(int64_t n, const double *w, const int32_t *nbr, uint64_t seed, int32_t count,
                              int32_t threshold, int64_t *out)
{
    for (int32_t i = 0; i < count; ++i) {
        orc_rng r;
        rng_init(&r, seed, 0, 0u, (uint32_t)i, 0u, 0u);
        split(n, w, nbr, threshold < 1 ? 1 : threshold, &r, out + 4 * (size_t)i);
    }
}
