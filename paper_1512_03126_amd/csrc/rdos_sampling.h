// Device-side random numbers and samplers of the diffusion and reaction steps.
//
// Every floating-point expression here is evaluated exactly as written
// (the library is built with -ffp-contract=off and no fast-math), so a CPU
// program that follows the same definitions in the same order reproduces
// every draw bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#pragma clang fp contract(off)

namespace rdos {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of the
// 4x32 S-box with multipliers 0xD2511F53 / 0xCD9E8D57 and a Weyl key
// schedule (0x9E3779B9, 0xBB67AE85).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 x, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo0 = 0xD2511F53u * x.x;
        const uint32_t hi0 = __umulhi(0xD2511F53u, x.x);
        const uint32_t lo1 = 0xCD9E8D57u * x.z;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, x.z);
        x = make_uint4(hi1 ^ x.y ^ k0, lo1, hi0 ^ x.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return x;
}

// One counter-based stream: counter (draw block, stream id, tet, period),
// key (k0, k1).  Draw j takes the block j/2 and, within it, words (x, y)
// for even j or (z, w) for odd j, mapped to a 53-bit uniform in [0, 1).
// Draws are taken in order, so a new block is generated exactly at even j.
struct Stream {
    uint32_t k0, k1, id, tet, period;
    uint32_t j;
    uint4 words;

    __device__ __forceinline__ Stream(uint32_t key0, uint32_t key1, uint32_t stream_id,
                                      uint32_t tet_id, uint32_t period_id)
        : k0(key0), k1(key1), id(stream_id), tet(tet_id), period(period_id), j(0),
          words(make_uint4(0, 0, 0, 0))
    {
    }

    __device__ __forceinline__ double uniform()
    {
        if (!(j & 1u)) words = philox4x32_10(make_uint4(j >> 1, id, tet, period), k0, k1);
        const uint32_t hi = (j & 1u) ? words.z : words.x;
        const uint32_t lo = (j & 1u) ? words.w : words.y;
        ++j;
        return ((double)(hi >> 5) * 67108864.0 + (double)(lo >> 6)) * 0x1p-53;
    }
};

// ---------------------------------------------------------------------------
// Natural logarithm from add/sub/mul/div only (no hardware transcendental):
// reduce x = 2^e m with m in [sqrt(1/2), sqrt(2)); with f = m - 1 and
// s = f / (2 + f), ln m = 2 atanh s = f - s (f - 2 R(s^2)) where
// R(z) = z/3 + z^2/5 + ... + z^11/23 (Horner); add e ln 2 with ln 2 split into
// a head whose products with e are exact and a rounded tail.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double log_basic(double x)
{
    constexpr double kLn2Head = 0x1.62e42fee00000p-1;
    constexpr double kLn2Tail = 0x1.a39ef35793c76p-33;
    constexpr double kSqrt2 = 0x1.6a09e667f3bcdp+0;
    uint64_t bits = (uint64_t)__double_as_longlong(x);
    int e = (int)((bits >> 52) & 0x7ffu);
    if (e == 0) {  // subnormal input
        x = x * 0x1p54;
        bits = (uint64_t)__double_as_longlong(x);
        e = (int)((bits >> 52) & 0x7ffu) - 54;
    }
    e -= 1023;
    double m = __longlong_as_double((long long)((bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull));
    if (m > kSqrt2) {
        m = m * 0.5;
        e += 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    const double R =
        z * (1.0 / 3.0 + z * (1.0 / 5.0 + z * (1.0 / 7.0 + z * (1.0 / 9.0 + z * (1.0 / 11.0 +
        z * (1.0 / 13.0 + z * (1.0 / 15.0 + z * (1.0 / 17.0 + z * (1.0 / 19.0 + z * (1.0 / 21.0 +
        z * (1.0 / 23.0)))))))))));
    const double lnm = f - s * (f - 2.0 * R);
    const double de = (double)e;
    return de * kLn2Head + (lnm + de * kLn2Tail);
}

// ---------------------------------------------------------------------------
// Binomial(n, p), exact in law:
//   BINV  sequential inversion from P(0) = q^n (Kachitvichyanukul &
//         Schmeiser, 1988) when n p < 10,
//   BTRD  transformed rejection with decomposition (Hoermann, 1993)
//         otherwise;
// p > 1/2 is sampled as n - Binomial(n, 1 - p).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double pow_by_squaring(double q, int32_t n)
{
    double acc = 1.0;
    double sq = q;
    while (n > 0) {
        if (n & 1) acc = acc * sq;
        n >>= 1;
        if (n > 0) sq = sq * sq;
    }
    return acc;
}

__device__ inline int32_t binomial_inversion(int32_t n, double p, Stream &rng)
{
    const double q = 1.0 - p;
    const double odds = p / q;
    const double np1_odds = (double)(n + 1) * odds;
    const double p_zero = pow_by_squaring(q, n);
    for (;;) {
        double u = rng.uniform();
        double pk = p_zero;
        int32_t x = 0;
        bool restart = false;
        while (u > pk) {
            u = u - pk;
            ++x;
            if (x > n) {
                restart = true;
                break;
            }
            pk = pk * (np1_odds / (double)x - odds);
        }
        if (!restart) return x;
    }
}

// Stirling-series remainder ln k! - ((k + 1/2) ln(k + 1) - (k + 1) + ln(2 pi)/2):
// correctly rounded values for k <= 9, the series 1/12 - 1/360 + 1/1260 in
// 1/(k+1) beyond.
__constant__ const double kStirlingExact[10] = {
    0x1.4c071bcda0a5bp-4, 0x1.52a9b923ea649p-5, 0x1.c579a268d80b3p-6, 0x1.54a2662fd78a9p-6,
    0x1.10b4e513fcbedp-6, 0x1.c6b167bebdf36p-7, 0x1.85d4d612e4a86p-7, 0x1.552805e7b3076p-7,
    0x1.2f4871b12ab64p-7, 0x1.10f9d4c0743a7p-7,
};

__device__ __forceinline__ double stirling_tail(int32_t k)
{
    if (k < 10) return kStirlingExact[k];
    const double v = 1.0 / (double)(k + 1);
    const double v2 = v * v;
    return (1.0 / 12.0 - (1.0 / 360.0 - (1.0 / 1260.0) * v2) * v2) * v;
}

// The set-up values are recomputed on every pass of the rejection loop
// instead of being held across it: `carry` is +0 after a rejected pass (0
// times a finite uniform), so p + carry == p and every value is bit for bit
// the same, but the compiler cannot hoist them out of the loop, which keeps
// them out of the registers the callers need.  Most draws take one pass.
__device__ inline int32_t binomial_btrd(int32_t n, double p_in, Stream &rng)
{
    const double nd = (double)n;
    double carry = 0.0;
    for (;;) {
        const double p = p_in + carry;
        const double q = 1.0 - p;
        const double npq = (nd * p) * q;
        const double spq = sqrt(npq);
        const double b = 1.15 + 2.53 * spq;
        const double a = (-0.0873 + 0.0248 * b) + 0.01 * p;
        const double c = nd * p + 0.5;
        const double vr = 0.92 - 4.2 / b;
        const double urvr = 0.86 * vr;
        double v = rng.uniform();
        carry = 0.0 * v;
        double u;
        if (v <= urvr) {  // inside the box: accept at once
            u = v / vr - 0.43;
            const double kd = floor(((2.0 * a) / (0.5 - fabs(u)) + b) * u + c);
            if (kd < 0.0 || kd > nd) continue;
            return (int32_t)kd;
        }
        if (v >= vr) {
            u = rng.uniform() - 0.5;
        } else {
            u = v / vr - 0.93;
            u = (u < 0.0 ? -0.5 : 0.5) - u;
            v = rng.uniform() * vr;
        }
        const double us = 0.5 - fabs(u);
        const double kd = floor(((2.0 * a) / us + b) * u + c);
        if (kd < 0.0 || kd > nd) continue;
        const double alpha = (2.83 + 5.1 / b) * spq;
        v = v * alpha / (a / (us * us) + b);
        const double mode = floor((nd + 1.0) * p);
        const double r = p / q;
        const double km = fabs(kd - mode);
        if (km <= 15.0) {
            // ratio f(k)/f(mode) by the recurrence f(i)/f(i-1) = nr/i - r
            const double nr = (nd + 1.0) * r;
            double f = 1.0;
            if (mode < kd) {
                double i = mode;
                do {
                    i += 1.0;
                    f = f * (nr / i - r);
                } while (i != kd);
            } else if (mode > kd) {
                double i = kd;
                do {
                    i += 1.0;
                    v = v * (nr / i - r);
                } while (i != mode);
            }
            if (v <= f) return (int32_t)kd;
            continue;
        }
        v = log_basic(v);
        const double rho = (km / npq) * (((km / 3.0 + 0.625) * km + 1.0 / 6.0) / npq + 0.5);
        const double t = -(km * km) / (2.0 * npq);
        if (v < t - rho) return (int32_t)kd;
        if (v > t + rho) continue;
        const int32_t m_i = (int32_t)mode, k_i = (int32_t)kd;
        const double nm = nd - mode + 1.0;
        const double h = (mode + 0.5) * log_basic((mode + 1.0) / (r * nm)) + stirling_tail(m_i) +
                         stirling_tail(n - m_i);
        const double nk = nd - kd + 1.0;
        if (v <= h + (nd + 1.0) * log_basic(nm / nk) + (kd + 0.5) * log_basic(nk * r / (kd + 1.0)) -
                     stirling_tail(k_i) - stirling_tail(n - k_i))
            return k_i;
    }
}

__device__ inline int32_t binomial(int32_t n, double p, Stream &rng)
{
    if (n <= 0 || p <= 0.0) return 0;
    if (p >= 1.0) return n;
    const bool reflect = p > 0.5;
    const double pp = reflect ? 1.0 - p : p;
    const int32_t x = ((double)n * pp < 10.0) ? binomial_inversion(n, pp, rng) : binomial_btrd(n, pp, rng);
    return reflect ? n - x : x;
}

// ---------------------------------------------------------------------------
// Multinomial split of n leaving molecules over the interior faces
// (Sec. II.B).  n < threshold (10 in the paper): one categorical draw per
// molecule against the running sum of the weights (the last interior face
// closes the interval); otherwise
// n_i = Binomial(n - sum_{j<i} n_j, w_i / (1 - sum_{j<i} w_j)) face by face,
// the last interior face taking what is left.
// ---------------------------------------------------------------------------
__device__ inline void split_over_faces(int32_t n, const int32_t nbr[4], const double w[4], int32_t threshold,
                                        Stream &rng, int32_t out[4])
{
    out[0] = out[1] = out[2] = out[3] = 0;
    if (n <= 0) return;
    int last = -1, interior = 0;
#pragma unroll
    for (int f = 0; f < 4; ++f)
        if (nbr[f] >= 0) {
            last = f;
            ++interior;
        }
    if (interior == 0) return;
    if (interior == 1) {
#pragma unroll
        for (int f = 0; f < 4; ++f)
            if (f == last) out[f] = n;
        return;
    }
    if (n < threshold) {
        for (int32_t i = 0; i < n; ++i) {
            const double u = rng.uniform();
            double edge = 0.0;
            int dest = last;
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                if (f < last && nbr[f] >= 0 && dest == last) {
                    edge = edge + w[f];
                    if (u < edge) dest = f;
                }
            }
#pragma unroll
            for (int f = 0; f < 4; ++f)
                if (f == dest) out[f] += 1;
        }
        return;
    }
    int32_t left = n;
    double taken = 0.0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        if (nbr[f] < 0 || left == 0) continue;
        if (f == last) {
            out[f] = left;
            left = 0;
            continue;
        }
        double pf = w[f] / (1.0 - taken);
        if (pf > 1.0) pf = 1.0;
        const int32_t nf = binomial(left, pf, rng);
        out[f] = nf;
        left -= nf;
        taken = taken + w[f];
    }
}

// ---------------------------------------------------------------------------
// The same split with both transfer forms in one body (the kernel instance
// that serves simulations using the second form calls it; the first form
// alone uses split_over_faces above, which needs fewer registers).
// n_i = Binomial(n - sum_{j<i} n_j, z w_i / (1 - sum_{j<i} z w_j)) face by
// face, or one categorical draw per molecule below the threshold:
//  * Step 3.3 (scaled = false, z = 1): n molecules all leave; the last
//    interior face closes the interval / takes what is left (a single
//    interior face takes everything without a draw);
//  * the alternative at the end of Sec. II.B (scaled = true, z = zeta): the
//    whole population, weights zeta w_i, and a molecule that draws no face
//    stays (probability 1 - zeta).
// 1.0 * w == w exactly, so the first form is bit-identical to the plain
// weights.  Returns the molecules that leave.
// ---------------------------------------------------------------------------
__device__ inline int32_t split_faces(int32_t n, const int32_t nbr[4], const double w[4], double z, bool scaled,
                                      int32_t threshold, Stream &rng, int32_t out[4])
{
    out[0] = out[1] = out[2] = out[3] = 0;
    if (n <= 0) return 0;
    int last = -1, interior = 0;
#pragma unroll
    for (int f = 0; f < 4; ++f)
        if (nbr[f] >= 0) {
            last = f;
            ++interior;
        }
    if (interior == 0) return 0;
    if (!scaled && interior == 1) {
#pragma unroll
        for (int f = 0; f < 4; ++f)
            if (f == last) out[f] = n;
        return n;
    }
    const int open = scaled ? -1 : last;  // where a molecule goes when no face's interval holds its draw
    int32_t moved = 0;
    if (n < threshold) {
        for (int32_t i = 0; i < n; ++i) {
            const double u = rng.uniform();
            double edge = 0.0;
            int dest = open;
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                if (nbr[f] >= 0 && (scaled || f < last) && dest == open) {
                    edge = edge + z * w[f];
                    if (u < edge) dest = f;
                }
            }
#pragma unroll
            for (int f = 0; f < 4; ++f)
                if (f == dest) out[f] += 1;
            moved += dest >= 0 ? 1 : 0;
        }
        return moved;
    }
    int32_t left = n;
    double taken = 0.0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        if (nbr[f] < 0 || left == 0) continue;
        if (!scaled && f == last) {
            out[f] = left;
            moved += left;
            left = 0;
            continue;
        }
        double pf = (z * w[f]) / (1.0 - taken);
        if (pf > 1.0) pf = 1.0;
        const int32_t nf = binomial(left, pf, rng);
        out[f] = nf;
        moved += nf;
        left -= nf;
        taken = taken + z * w[f];
    }
    return moved;
}

}  // namespace rdos
