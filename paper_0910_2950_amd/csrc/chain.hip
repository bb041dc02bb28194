// Heatbath draws of an HMC Markov chain on the device: Gaussian momenta and
// pseudofermion noise of trajectory `traj` from the counter-based generator of
// rng.h, written straight into the internal layouts.  Every value depends only
// on (seed, traj, field index), so a chain resumed at any trajectory draws
// exactly what an uninterrupted one would.
#include "fgi.h"
#include "fgi_internal.h"
#include "rng.h"

namespace fgi {

static inline int nblocks(long n, int bs) { return (int)((n + bs - 1) / bs); }

// momenta: one thread per link (mu, parity, s), lexicographic link index
// l = mu V + i fixes the counters; components 2j, 2j+1 from counter 4 l + j
__global__ void k_refresh_mom(Geom g, uint32_t k0, uint32_t k1, uint32_t traj, double* __restrict__ P) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * g.V) return;
    const int s = t % g.Vh, r = t / g.Vh, p = r & 1, mu = r >> 1;
    const Coord c = cb_coords(g, p, s);
    const uint32_t i = (uint32_t)(c.c[0] + g.L[0] * (c.c[1] + g.L[1] * (c.c[2] + g.L[2] * c.c[3])));
    const uint32_t l = (uint32_t)mu * (uint32_t)g.V + i;
    double* o = P + (size_t)(r * 8) * g.Vh + s;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        double z0, z1;
        gauss_pair(k0, k1, 4u * l + (uint32_t)j, traj, RNG_MOM, z0, z1);
        o[(size_t)(2 * j) * g.Vh] = z0;
        o[(size_t)(2 * j + 1) * g.Vh] = z1;
    }
}

// noise of the even sites: entry s of the internal even field is the s-th even
// site in lexicographic order; Re, Im ~ N(0, 1/2)
__global__ void k_refresh_eta(Geom g, uint32_t k0, uint32_t k1, uint32_t traj, uint32_t stream, d2* __restrict__ eta) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.Vh) return;
#pragma unroll 4
    for (int e = 0; e < 12; e++) {
        double z0, z1;
        gauss_pair(k0, k1, 12u * (uint32_t)s + (uint32_t)e, traj, stream, z0, z1);
        eta[(size_t)e * g.Vh + s] = d2{z0 * 0.7071067811865476, z1 * 0.7071067811865476};
    }
}

void refresh_momenta(Ctx& c, const Geom& g, uint64_t seed, uint32_t traj, double* P) {
    if (16L * g.V >= (1L << 32)) throw Error(FGI_EINVAL, "lattice too large for the momentum counters");
    hipLaunchKernelGGL(k_refresh_mom, dim3(nblocks(4L * g.V, 256)), dim3(256), 0, c.stream, g, (uint32_t)seed,
                       (uint32_t)(seed >> 32), traj, P);
    FGI_LAUNCH_CHECK();
}

void refresh_noise(Ctx& c, const Geom& g, uint64_t seed, uint32_t traj, int stream, d2* eta) {
    hipLaunchKernelGGL(k_refresh_eta, dim3(nblocks(g.Vh, 256)), dim3(256), 0, c.stream, g, (uint32_t)seed,
                       (uint32_t)(seed >> 32), traj, (uint32_t)stream, eta);
    FGI_LAUNCH_CHECK();
}

double metropolis_uniform(uint64_t seed, uint32_t traj) {
    const uint32_t ctr[4] = {0u, traj, (uint32_t)RNG_METROPOLIS, 0u};
    uint32_t x[4];
    philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), x);
    return uniform52(x[0], x[1]);
}

void philox_host(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    philox4x32_10(ctr, key[0], key[1], out);
}

}  // namespace fgi
