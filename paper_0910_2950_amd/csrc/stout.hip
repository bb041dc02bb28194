// Stout smearing of the links the fermion operator sees (Morningstar and
// Peardon, Phys. Rev. D 69 (2004) 054501), and the back-propagation of a
// force on the smeared links to the thin links.
//
// One level, on every link l = (mu, x):
//   C_l = rho sum_{nu != mu} [U_nu(x) U_mu(x+nu) U_nu(x+mu)^+ + U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu)]
//   Omega_l = C_l U_l^+,  A_l = TA(Omega_l),  U'_l = exp(A_l) U_l.
// Forces are su(3) fields with the pairing <X, Y> = -2 Re Tr(X Y) (the sum of
// component products).  Given the force G' on the smeared links, the force on
// the input links is the adjoint of the level's tangent map (dU_l = xi_l U_l
// -> dU'_l = xi'_l U'_l):
//   G_l = E^+ G'_l E - TA(Gamma_l Omega_l) + (staple terms),  E = exp(A_l),
//   Gamma_l = int_0^1 exp(-s A_l) G'_l exp(s A_l) ds
//           = sum_k (-1)^k ad_A^k(G'_l) / (k+1)!,
// and with M_l = rho U_l^+ Gamma_l every link k on a staple S = L f R of some
// C_l adds TA(U_k R M_l L) when f = U_k and -TA(R M_l L U_k^+) when f = U_k^+.
// The staple terms are gathered per receiving link (18 staple positions hold
// a given link), so every thread writes only its own link.
#include "fgi_internal.h"

namespace fgi {

static const int BS = 256;
static inline int nblocks(long n, int bs) { return (int)((n + bs - 1) / bs); }

namespace {

__device__ __forceinline__ int cparity(const Coord& y) { return (y.c[0] + y.c[1] + y.c[2] + y.c[3]) & 1; }

// (an indexed store: here the compiler's per-thread LDS copy of y is the
// cheaper home; with selects these kernels spill hundreds of bytes a lane)
__device__ __forceinline__ Coord shifted(const Geom& g, Coord y, int d, int k) {
    int v = y.c[d] + k;
    v = v < 0 ? v + g.L[d] : (v >= g.L[d] ? v - g.L[d] : v);
    y.c[d] = v;
    return y;
}

__device__ __forceinline__ M3<double> ld(const Geom& g, const d2* U, int d, const Coord& y) {
    return gauge_load(U, d, cparity(y), cb_index(g, y), g.Vh);
}

// C_l / rho: the six staples of link (mu, x)
__device__ __forceinline__ M3<double> staples(const Geom& g, const d2* __restrict__ U, const Coord& x, int mu) {
    M3<double> C = m3_zero<double>();
    const Coord xm = shifted(g, x, mu, 1);
#pragma unroll 1
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        const Coord xn = shifted(g, x, nu, 1), xmn = shifted(g, x, nu, -1), xpm_mn = shifted(g, xm, nu, -1);
        // U_nu(x) U_mu(x+nu) U_nu(x+mu)^+
        m3_acc(C, m3_mul_nd(m3_mul(ld(g, U, nu, x), ld(g, U, mu, xn)), ld(g, U, nu, xm)));
        // U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu)
        m3_acc(C, m3_mul(m3_mul_dn(ld(g, U, nu, xmn), ld(g, U, mu, xmn)), ld(g, U, nu, xpm_mn)));
    }
    return C;
}

__device__ __forceinline__ M3<double> ta_matrix(const M3<double>& W) {
    double x[8];
    ta_components(W, x);
    return alg_matrix(x);
}

__device__ __forceinline__ void link_of(const Geom& g, int t, int& mu, int& p, int& s, Coord& x) {
    s = t % g.Vh;
    const int r = t / g.Vh;
    p = r & 1;
    mu = r >> 1;
    x = cb_coords(g, p, s);
}

}  // namespace

// U' = exp(TA(C U^+)) U on link t
__device__ __forceinline__ void stout_level_body(const Geom& g, double rho, const d2* __restrict__ U,
                                                 d2* __restrict__ Up, int t) {
    if (t >= 4 * g.V) return;
    int mu, p, s;
    Coord x;
    link_of(g, t, mu, p, s, x);
    const M3<double> u = gauge_load(U, mu, p, s, g.Vh);
    M3<double> C = staples(g, U, x, mu);
    m3_scale(C, rho);
    const M3<double> E = su3_exp(ta_matrix(m3_mul_nd(C, u)));
    gauge_store(Up, mu, p, s, g.Vh, m3_mul(E, u));
}

__global__ void __launch_bounds__(256) k_stout_level(Geom g, double rho, const d2* __restrict__ U,
                                                    d2* __restrict__ Up) {
    stout_level_body(g, rho, U, Up, blockIdx.x * blockDim.x + threadIdx.x);
}

// batched chains (links of chain c from 9 * link0, 256 links per block)
__global__ void __launch_bounds__(256) k_stout_level_b(const ChainDesc* __restrict__ cd, int nc, double rho,
                                                      const d2* __restrict__ U, d2* __restrict__ Up) {
    const int c = find_chain(cd, nc, blockIdx.x, GRID_4V);
    const ChainDesc& d = cd[c];
    stout_level_body(d.g, rho, U + 9 * d.link0, Up + 9 * d.link0,
                     (blockIdx.x - d.blk0[GRID_4V]) * blockDim.x + threadIdx.x);
}

// Per link: part = E^+ G' E - TA(Gamma Omega) (components), M = rho U^+ Gamma
__device__ __forceinline__ void stout_gamma_body(const Geom& g, double rho, const d2* __restrict__ U,
                                                 const double* __restrict__ Gp, double* __restrict__ part,
                                                 d2* __restrict__ Mout, int t) {
    if (t >= 4 * g.V) return;
    int mu, p, s;
    Coord x;
    link_of(g, t, mu, p, s, x);
    const M3<double> u = gauge_load(U, mu, p, s, g.Vh);
    M3<double> C = staples(g, U, x, mu);
    m3_scale(C, rho);
    const M3<double> Om = m3_mul_nd(C, u);
    const M3<double> A = ta_matrix(Om);
    const M3<double> E = su3_exp(A);
    double gx[8];
    mom_load(Gp, mu, p, s, g.Vh, gx);
    const M3<double> G = alg_matrix(gx);
    // Gamma = sum_k (-1)^k ad_A^k(G) / (k+1)!, summed until a term drops below
    // 1e-18 of the sum (|ad_A| <= 2 |A|, |A| <= 6 rho)
    M3<double> term = G, Gam = G;
    double gmax = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) gmax = fmax(gmax, fabs(G.e[i][j].re) + fabs(G.e[i][j].im));
#pragma unroll 1
    for (int k = 1; k <= 48; k++) {
        M3<double> a = m3_mul(A, term), b = m3_mul(term, A);
        double tmax = 0.0;
        const double f = -1.0 / (k + 1);
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                term.e[i][j] = f * (a.e[i][j] - b.e[i][j]);
                tmax = fmax(tmax, fabs(term.e[i][j].re) + fabs(term.e[i][j].im));
            }
        m3_acc(Gam, term);
        if (tmax <= 1e-18 * gmax) break;
    }
    double x1[8], x2[8];
    ta_components(m3_mul(m3_mul_dn(E, G), E), x1);
    ta_components(m3_mul(Gam, Om), x2);
#pragma unroll
    for (int a = 0; a < 8; a++) x1[a] -= x2[a];
    mom_store(part, mu, p, s, g.Vh, x1);
    M3<double> M = m3_mul_dn(u, Gam);
    m3_scale(M, rho);
    gauge_store(Mout, mu, p, s, g.Vh, M);
}

__global__ void __launch_bounds__(256) k_stout_gamma(Geom g, double rho, const d2* __restrict__ U,
                                                    const double* __restrict__ Gp, double* __restrict__ part,
                                                    d2* __restrict__ Mout) {
    stout_gamma_body(g, rho, U, Gp, part, Mout, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void __launch_bounds__(256) k_stout_gamma_b(const ChainDesc* __restrict__ cd, int nc, double rho,
                                                      const d2* __restrict__ U, const double* __restrict__ Gp,
                                                      double* __restrict__ part, d2* __restrict__ Mout) {
    const int c = find_chain(cd, nc, blockIdx.x, GRID_4V);
    const ChainDesc& d = cd[c];
    stout_gamma_body(d.g, rho, U + 9 * d.link0, Gp + 8 * d.link0, part + 8 * d.link0, Mout + 9 * d.link0,
                     (blockIdx.x - d.blk0[GRID_4V]) * blockDim.x + threadIdx.x);
}

// G_k = part_k + the 18 staple terms of link k = (d, y) (coef, accumulate into G)
__device__ __forceinline__ void stout_gather_body(const Geom& g, const d2* __restrict__ U, const d2* __restrict__ M,
                                                  const double* __restrict__ part, double* __restrict__ G,
                                                  double coef, int accumulate, int t) {
    if (t >= 4 * g.V) return;
    int d, p, s;
    Coord y;
    link_of(g, t, d, p, s, y);
    const M3<double> uk = gauge_load(U, d, p, s, g.Vh);
    const Coord yd = shifted(g, y, d, 1);
    M3<double> fw = m3_zero<double>();  // sum of R M L over forward positions: adds TA(U_k (.))
    M3<double> bw = m3_zero<double>();  // sum of R M L over backward positions: adds -TA((.) U_k^+)
#pragma unroll 1
    for (int e = 0; e < 4; e++) {
        if (e == d) continue;
        const Coord ype = shifted(g, y, e, 1), yme = shifted(g, y, e, -1);
        // link k the middle (parallel) link of the upper staple of (d, y-e):
        //   L = U_e(y-e), R = U_e(y-e+d)^+
        m3_acc(fw, m3_mul(m3_mul_dn(ld(g, U, e, shifted(g, yme, d, 1)), ld(g, M, d, yme)), ld(g, U, e, yme)));
        // ... of the lower staple of (d, y+e): L = U_e(y)^+, R = U_e(y+d)
        m3_acc(fw, m3_mul_nd(m3_mul(ld(g, U, e, yd), ld(g, M, d, ype)), ld(g, U, e, y)));
        // first link of the upper staple of (e, y): L = 1, R = U_e(y+d) U_d(y+e)^+
        m3_acc(fw, m3_mul(m3_mul_nd(ld(g, U, e, yd), ld(g, U, d, ype)), ld(g, M, e, y)));
        // last link of the lower staple of (e, y+d-e): L = U_d(y-e)^+ U_e(y-e), R = 1
        m3_acc(fw, m3_mul(ld(g, M, e, shifted(g, yd, e, -1)), m3_mul_dn(ld(g, U, d, yme), ld(g, U, e, yme))));
        // last link (backward) of the upper staple of (e, y-e): L = U_d(y-e) U_e(y-e+d), R = 1
        m3_acc(bw, m3_mul(ld(g, M, e, yme), m3_mul(ld(g, U, d, yme), ld(g, U, e, shifted(g, yme, d, 1)))));
        // first link (backward) of the lower staple of (e, y+d): L = 1, R = U_e(y) U_d(y+e)
        m3_acc(bw, m3_mul(m3_mul(ld(g, U, e, y), ld(g, U, d, ype)), ld(g, M, e, yd)));
    }
    double x1[8], x2[8], x0[8];
    ta_components(m3_mul(uk, fw), x1);
    ta_components(m3_mul_nd(bw, uk), x2);
    mom_load(part, d, p, s, g.Vh, x0);
    double* o = G + (size_t)((d * 2 + p) * 8) * g.Vh + s;
#pragma unroll
    for (int a = 0; a < 8; a++) {
        const double v = coef * (x0[a] + x1[a] - x2[a]);
        o[(size_t)a * g.Vh] = accumulate ? o[(size_t)a * g.Vh] + v : v;
    }
}

__global__ void __launch_bounds__(256) k_stout_gather(Geom g, const d2* __restrict__ U, const d2* __restrict__ M,
                                                     const double* __restrict__ part, double* __restrict__ G,
                                                     double coef, int accumulate) {
    stout_gather_body(g, U, M, part, G, coef, accumulate, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void __launch_bounds__(256) k_stout_gather_b(const ChainDesc* __restrict__ cd, int nc,
                                                       const d2* __restrict__ U, const d2* __restrict__ M,
                                                       const double* __restrict__ part, double* __restrict__ G,
                                                       double coef, int accumulate) {
    const int c = find_chain(cd, nc, blockIdx.x, GRID_4V);
    const ChainDesc& d = cd[c];
    stout_gather_body(d.g, U + 9 * d.link0, M + 9 * d.link0, part + 8 * d.link0, G + 8 * d.link0, coef, accumulate,
                      (blockIdx.x - d.blk0[GRID_4V]) * blockDim.x + threadIdx.x);
}

const d2* stout_smear(Ctx& c, const Geom& g, double rho, int n, const d2* U, d2* levels) {
    const size_t sz = (size_t)4 * 9 * g.V;
    const d2* in = U;
    for (int k = 0; k < n; k++) {
        d2* out = levels + k * sz;
        hipLaunchKernelGGL(k_stout_level, dim3(nblocks(4L * g.V, BS)), dim3(BS), 0, c.stream, g, rho, in, out);
        FGI_LAUNCH_CHECK();
        in = out;
    }
    return in;
}

void stout_backprop(Ctx& c, const Geom& g, double rho, int n, const d2* U, const d2* levels, const double* Fs,
                    double* F, double coef, int accumulate) {
    const size_t sz = (size_t)4 * 9 * g.V;
    const size_t mb = sizeof(double) * 8 * 4 * (size_t)g.V;
    double* ga = (double*)c.stout_ga.get(mb);
    double* gb = (double*)c.stout_gb.get(mb);
    double* part = (double*)c.stout_part.get(mb);
    d2* M = (d2*)c.stout_M.get(sizeof(d2) * sz);
    const double* Gin = Fs;
    for (int k = n - 1; k >= 0; k--) {
        const d2* Uk = k == 0 ? U : levels + (k - 1) * sz;
        hipLaunchKernelGGL(k_stout_gamma, dim3(nblocks(4L * g.V, BS)), dim3(BS), 0, c.stream, g, rho, Uk, Gin, part,
                           M);
        FGI_LAUNCH_CHECK();
        double* Gout = k == 0 ? F : ((n - 1 - k) % 2 == 0 ? ga : gb);
        hipLaunchKernelGGL(k_stout_gather, dim3(nblocks(4L * g.V, BS)), dim3(BS), 0, c.stream, g, Uk, M, part, Gout,
                           k == 0 ? coef : 1.0, k == 0 ? accumulate : 0);
        FGI_LAUNCH_CHECK();
        Gin = Gout;
    }
}

const d2* stout_smear_b(Ctx& c, const Batch& B, double rho, int n, const d2* U, d2* levels) {
    const size_t sz = (size_t)9 * B.links;
    const d2* in = U;
    for (int k = 0; k < n; k++) {
        d2* out = levels + k * sz;
        hipLaunchKernelGGL(k_stout_level_b, dim3(B.nblk[GRID_4V]), dim3(BS), 0, c.stream, B.cd, B.nc, rho, in, out);
        FGI_LAUNCH_CHECK();
        in = out;
    }
    return in;
}

void stout_backprop_b(Ctx& c, const Batch& B, double rho, int n, const d2* U, const d2* levels, const double* Fs,
                      double* F, double coef, int accumulate) {
    const size_t sz = (size_t)9 * B.links;
    const size_t mb = sizeof(double) * 8 * (size_t)B.links;
    double* ga = (double*)c.stout_ga.get(mb);
    double* gb = (double*)c.stout_gb.get(mb);
    double* part = (double*)c.stout_part.get(mb);
    d2* M = (d2*)c.stout_M.get(sizeof(d2) * sz);
    const double* Gin = Fs;
    for (int k = n - 1; k >= 0; k--) {
        const d2* Uk = k == 0 ? U : levels + (k - 1) * sz;
        hipLaunchKernelGGL(k_stout_gamma_b, dim3(B.nblk[GRID_4V]), dim3(BS), 0, c.stream, B.cd, B.nc, rho, Uk, Gin,
                           part, M);
        FGI_LAUNCH_CHECK();
        double* Gout = k == 0 ? F : ((n - 1 - k) % 2 == 0 ? ga : gb);
        hipLaunchKernelGGL(k_stout_gather_b, dim3(B.nblk[GRID_4V]), dim3(BS), 0, c.stream, B.cd, B.nc, Uk, M, part,
                           Gout, k == 0 ? coef : 1.0, k == 0 ? accumulate : 0);
        FGI_LAUNCH_CHECK();
        Gin = Gout;
    }
}

}  // namespace fgi
