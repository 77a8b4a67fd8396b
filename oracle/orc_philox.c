/*
 * orc_philox.c -- Philox4x32-10 counter-based generator and the 16-bit uniform mapping.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper only says that the fluid may be run stochastically and that the bead noise
 * obeys fluctuation-dissipation (Sec. 1.1).  Both the oracle and the GPU library draw every
 * random number from Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), written here from that published definition: each
 * round multiplies counter words 0 and 2 by the two Philox multipliers, swaps the halves and
 * mixes in the key, and the key is advanced by the two Weyl increments between rounds.
 * Because the generator is a pure function of (counter, key), the oracle and the GPU draw
 * identical noise without sharing any code.
 */
#include "oracle.h"

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k[0] += PHILOX_W0; k[1] += PHILOX_W1; }
        philox_round(c, k);
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* h in [0, 65535] -> (2h + 1 - 2^16) / 2^17, the 2^16 midpoints of equal bins of (-1/2, 1/2).
 * Exact in binary floating point; mean 0, variance (1 - 2^-32)/12.                         */
double orc_uniform16(uint32_t h)
{
    return ((double)(2.0 * (double)(h & 0xFFFFu)) + 1.0 - 65536.0) / 131072.0;
}
