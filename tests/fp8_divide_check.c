/* Check of the FP8 encoder's divide on the CPU.
 *
 * The vector image gather divides a value v by an FP8 channel scale s as
 *   r = RN(1/s), q0 = RN(v r), e = RN(s * -q0 + v) (exact), q = RN(e r + q0)
 * (Markstein's correction), keeping q0 when |q0| > 2^120, q0 is not finite
 * or q0 is zero (the correction would turn -0 into +0).
 * This program compares q with the correctly rounded quotient RN(v / s),
 * taken as the binary64 quotient rounded to binary32 (innocuous double
 * rounding: 53 >= 2 * 24 + 2), on every binary32 v (or every stride-th bit
 * pattern) and a set of scales: fixed ones (powers of two, significands of
 * all ones, the scales of typical amax values) and random ones with
 * exponents in [-60, 60].  It judges what decides the E4M3 code: equal bits
 * where |RN(v/s)| is in [2^-12, 2^9]; below that, |q| < 2^-11 with the same
 * sign (the code is a signed zero); above, |q| > 448 with the same sign (the
 * code saturates).  NaN v are skipped (NaN stays NaN on both sides).  With
 * a stride, the special values below are checked as well.
 *
 * usage: fp8_divide_check STRIDE N_RANDOM SEED   (exit status 0: no mismatch)
 * The full check: STRIDE 1 (all 2^32 patterns), N_RANDOM 8, SEED 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static float from_bits(uint32_t u)
{
    float f;
    memcpy(&f, &u, 4);
    return f;
}

static uint32_t to_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

static float corrected_quotient(float v, float s, float r)
{
    const float q0 = v * r;
    if (!(fabsf(q0) <= 0x1p120f) || q0 == 0.0f) return q0;
    const float e = fmaf(-q0, s, v);
#ifdef DROP_CORRECTION  /* a planted mistake, for the test that the check fails it */
    return q0 + 0.0f * e;
#endif
    return fmaf(e, r, q0);
}

/* Whether the corrected quotient gives v / s's E4M3 code (NaN v: yes). */
static int agrees(float v, float s, float r)
{
    if (v != v) return 1;
    const float want = (float)((double)v / (double)s);
    const float got = corrected_quotient(v, s, r);
    const float a = fabsf(want);
    if (got != got) return 0;
    if (a >= 0x1p-12f && a <= 0x1p9f) return to_bits(got) == to_bits(want);
    if (a < 0x1p-12f) return fabsf(got) < 0x1p-11f && signbit(got) == signbit(want);
    return fabsf(got) > 448.0f && signbit(got) == signbit(want);
}

/* Patterns every run checks with both signs, whatever the stride: zero, the
 * least subnormal, the largest subnormal, the least normal, one, the largest
 * finite value, infinity. */
static const uint32_t special[] = {0x00000000u, 0x00000001u, 0x007fffffu, 0x00800000u,
                                   0x3f800000u, 0x7f7fffffu, 0x7f800000u};

static uint64_t splitmix(uint64_t* x)
{
    uint64_t z = (*x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

int main(int argc, char** argv)
{
    if (argc != 4) {
        fprintf(stderr, "usage: %s STRIDE N_RANDOM SEED\n", argv[0]);
        return 2;
    }
    const long long stride = atoll(argv[1]);
    const int n_random = atoi(argv[2]);
    uint64_t seed = strtoull(argv[3], NULL, 10);
    if (stride < 1 || n_random < 0 || n_random > 4096) return 2;
    static const float fixed[] = {1.0f, 0.5f, 2.0f, 3.0f, 1.5f, 1.0f / 448.0f, 0.1f, 7.0f / 448.0f, 1e-6f,
                                  1000.0f / 448.0f, 0x1p-60f, 0x1p60f, 0x1.fffffep-1f, 0x1.fffffep+0f,
                                  0x1.000002p+0f, 0x1.fffffep-60f, 0x1.fffffep+59f, 0x1.000002p-60f};
    const int n_fixed = (int)(sizeof fixed / sizeof fixed[0]);
    long long bad_total = 0;
    for (int k = 0; k < n_fixed + n_random; k++) {
        float s;
        if (k < n_fixed) {
            s = fixed[k];
        } else {
            const uint64_t z = splitmix(&seed);
            const int ex = (int)(z % 121) - 60;
            s = from_bits(((uint32_t)(ex + 127) << 23) | (uint32_t)((z >> 32) & 0x7fffff));
        }
        const float r = (float)(1.0 / (double)s);
        long long bad = 0;
#pragma omp parallel for reduction(+ : bad) schedule(static)
        for (long long i = 0; i < (1LL << 32); i += stride) bad += !agrees(from_bits((uint32_t)i), s, r);
        for (int j = 0; j < (int)(sizeof special / sizeof special[0]); j++) {
            bad += !agrees(from_bits(special[j]), s, r);
            bad += !agrees(from_bits(special[j] | 0x80000000u), s, r);
        }
        printf("scale %a: %lld mismatches\n", s, bad);
        fflush(stdout);
        bad_total += bad;
    }
    printf("%d scales, stride %lld: %lld mismatches\n", n_fixed + n_random, stride, bad_total);
    return bad_total != 0;
}
