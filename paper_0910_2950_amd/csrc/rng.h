// Counter-based random numbers for the Markov chain: Philox4x32-10 of Salmon,
// Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC11, 2011), written from its published definition: ten rounds, each two
// 32x32 -> 64-bit products of counter words 0 and 2 with the multipliers
// 0xD2511F53 and 0xCD9E8D57, the high halves XORed with the other two counter
// words and the key; the key is advanced by the Weyl constants 0x9E3779B9,
// 0xBB67AE85 before every round but the first.  Used on the host (the
// Metropolis draw) and on the device (momenta and pseudofermion noise).
//
// Stream layout of one chain (key = the 64-bit seed split in two words):
//   counter (4 l + j, traj, 0, 0)   momenta of link l = mu V + i (lexicographic
//                                   site i), components 2j, 2j+1, j = 0..3
//   counter (12 k + e, traj, 1 | 2, 0)  noise eta1 | eta2 of even site k,
//                                   spin-colour component e = 3 spin + colour
//   counter (0, traj, 3, 0)         the Metropolis uniform of trajectory traj
// Each counter gives two uniforms (52 bits each, from words 0,1 and 2,3) and
// one Box-Muller pair; eta components are (z0 + i z1) / sqrt(2).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace fgi {

enum RngStream { RNG_MOM = 0, RNG_ETA1 = 1, RNG_ETA2 = 2, RNG_METROPOLIS = 3 };

__host__ __device__ inline void philox4x32_10(const uint32_t ctr[4], uint32_t k0, uint32_t k1, uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// uniform in (0, 1) from 52 bits of two words: (m + 1/2) 2^-52, exact in double
__host__ __device__ inline double uniform52(uint32_t a, uint32_t b) {
    const uint64_t m = ((uint64_t)a << 20) | (b >> 12);
    return ((double)m + 0.5) * 0x1p-52;
}

// standard normal pair (Box-Muller) of one counter
__host__ __device__ inline void gauss_pair(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                                           double& z0, double& z1) {
    const uint32_t ctr[4] = {c0, c1, c2, 0u};
    uint32_t x[4];
    philox4x32_10(ctr, k0, k1, x);
    const double r = sqrt(-2.0 * log(uniform52(x[0], x[1])));
    const double ph = 6.283185307179586 * uniform52(x[2], x[3]);
    z0 = r * cos(ph);
    z1 = r * sin(ph);
}

}  // namespace fgi
