/*
 * Counter-based random numbers for the thermal field of the oracle.
 * TEST INFRASTRUCTURE ONLY (see sllg_oracle.h).
 *
 * The paper draws its Gaussian numbers with a Mersenne Twister and the
 * Ziggurat method (section "Langevin Dynamics").  Any generator of
 * independent standard normals realises the same Langevin dynamics; here
 * the generator is Philox4x32-10 (Salmon et al., SC'11), a function of a
 * 128-bit counter and a 64-bit key, so every (site, step) pair owns its own
 * numbers and the GPU can regenerate them without storing them.  Uniform
 * words are turned into normals with the Box-Muller transform.
 */
#include <math.h>
#include <stdint.h>

#include "sllg_oracle.h"

/* Round multipliers and key increments of Philox4x32 as published in SC'11. */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

/* One Philox round on the four counter words x with key k.  The two
 * 32x32->64 products give a high and a low word each; the new words are
 * (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, lo(M0*x0)). */
static void philox_round(uint32_t x[4], const uint32_t k[2])
{
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x[0];
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x[1] ^ k[0];
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x[3] ^ k[1];
    uint32_t y3 = lo0;
    x[0] = y0;
    x[1] = y1;
    x[2] = y2;
    x[3] = y3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {            /* the key is bumped between rounds */
            k[0] += PHILOX_W0;
            k[1] += PHILOX_W1;
        }
        philox_round(x, k);
    }
    out[0] = x[0];
    out[1] = x[1];
    out[2] = x[2];
    out[3] = x[3];
}

void orc_philox_batch(int64_t count, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    for (int64_t c = 0; c < count; ++c)
        orc_philox4x32_10(ctr + 4 * c, key + 2 * c, out + 4 * c);
}

void orc_gaussian3(uint64_t seed, uint64_t step, uint64_t site, uint32_t purpose, double g[3])
{
    const double two_pow_m32 = 1.0 / 4294967296.0;
    const double two_pi = 6.283185307179586;
    uint32_t ctr[4] = {(uint32_t)site, (uint32_t)step, (uint32_t)(step >> 32), purpose};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);

    /* Uniforms: (r + 1) / 2^32 lies in (0, 1] so its logarithm is finite;
     * r / 2^32 lies in [0, 1). */
    double u1 = ((double)r[0] + 1.0) * two_pow_m32;
    double u2 = (double)r[1] * two_pow_m32;
    double u3 = ((double)r[2] + 1.0) * two_pow_m32;
    double u4 = (double)r[3] * two_pow_m32;

    /* Box-Muller: radius sqrt(-2 ln u), angle 2 pi u'. */
    double rho1 = sqrt(-2.0 * log(u1));
    double rho2 = sqrt(-2.0 * log(u3));
    g[0] = rho1 * cos(two_pi * u2);
    g[1] = rho1 * sin(two_pi * u2);
    g[2] = rho2 * cos(two_pi * u4);
}

void orc_gaussian3_batch(uint64_t seed, uint64_t step, int64_t count, const uint64_t *sites,
                         uint32_t purpose, double *g)
{
    for (int64_t c = 0; c < count; ++c)
        orc_gaussian3(seed, step, sites[c], purpose, g + 3 * c);
}
