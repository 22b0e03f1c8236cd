/*
 * CPU reference of the serving workload's motion in C.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests to replay, at full size, the
 * motion the device applies to a resident simulation, so that its counts can
 * be checked against the matching oracle.  It shares no code with the GPU
 * path and follows the same published definition as walk.py (whose numpy
 * version pins this one bit for bit):
 *
 *   generator  Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
 *              numbers: as easy as 1, 2, 3", SC 2011): ten rounds on four
 *              32-bit counter words under a two-word key; a round takes the
 *              full 64-bit products of words 0 and 2 with 0xD2511F53 and
 *              0xCD9E8D57 and returns (hi(w2 * M1) ^ w1 ^ k0, lo(w2 * M1),
 *              hi(w0 * M0) ^ w3 ^ k1, lo(w0 * M0)); the key then grows by
 *              (0x9E3779B9, 0xBB67AE85);
 *   z          the twelve output words of the draws at counters (region,
 *              axis, step, j), j = 0, 1, 2, under key (seed mod 2^32,
 *              seed >> 32), each shifted right by 8 and summed as integers,
 *              converted to float32, times 2^-24, minus 6;
 *   step       lo <- lo + sigma * z, hi <- lo + side, float32 with one
 *              rounding per operation (built with -ffp-contract=off).
 */
#include <stdint.h>

static void philox4x32_10(uint32_t w[4], uint32_t k0, uint32_t k1)
{
    for (int round = 0; round < 10; ++round) {
        const uint64_t a = (uint64_t)0xD2511F53u * w[0];
        const uint64_t b = (uint64_t)0xCD9E8D57u * w[2];
        const uint32_t out0 = (uint32_t)(b >> 32) ^ w[1] ^ k0;
        const uint32_t out2 = (uint32_t)(a >> 32) ^ w[3] ^ k1;
        w[0] = out0;
        w[1] = (uint32_t)b;
        w[2] = out2;
        w[3] = (uint32_t)a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

static float normal_z(uint32_t region, uint32_t axis, uint32_t step, uint64_t seed)
{
    uint32_t sum = 0;
    for (uint32_t j = 0; j < 3; ++j) {
        uint32_t w[4] = {region, axis, step, j};
        philox4x32_10(w, (uint32_t)seed, (uint32_t)(seed >> 32));
        for (int i = 0; i < 4; ++i) sum += w[i] >> 8;
    }
    const float s = (float)sum;
    const float scaled = s * 5.9604644775390625e-08f; /* 2^-24 */
    return scaled - 6.0f;
}

/* One step of rows lo / hi (float32 [rows][d], in place) whose first row is
 * region region0. */
void walk_oracle_step(float *lo, float *hi, int64_t rows, int d, uint32_t region0, float side,
                      float sigma, uint64_t seed, uint32_t step)
{
    for (int64_t r = 0; r < rows; ++r) {
        for (int k = 0; k < d; ++k) {
            const float z = normal_z(region0 + (uint32_t)r, (uint32_t)k, step, seed);
            const float delta = sigma * z;
            const float moved = lo[r * d + k] + delta;
            lo[r * d + k] = moved;
            hi[r * d + k] = moved + side;
        }
    }
}
