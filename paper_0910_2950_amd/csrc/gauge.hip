// Gauge-side kernels: layout conversion, Hamiltonian densities, the Wilson
// gauge (staple) force and its tangent (the force gradient along a field),
// the exact su(3) link update and reunitarisation.  FP64 throughout.
#include "fgi_coord.h"
#include "fgi_internal.h"

namespace fgi {

static inline int nblocks(long n, int bs) { return (int)((n + bs - 1) / bs); }
static const int BS = 256;

// lexicographic index of checkerboard site (p, s)
__device__ __forceinline__ int lex_index(const Geom& g, int p, int s) {
    Coord c = cb_coords(g, p, s);
    return c.c[0] + g.L[0] * (c.c[1] + g.L[1] * (c.c[2] + g.L[2] * c.c[3]));
}

// ---------------------------------------------------------------- layout ---
__device__ __forceinline__ void pack_gauge_body(const Geom& g, const d2* __restrict__ user, d2* __restrict__ U,
                                                int to_internal, int t) {
    if (t >= 4 * g.V) return;
    int s = t % g.Vh, r = t / g.Vh, p = r & 1, mu = r >> 1;
    int i = lex_index(g, p, s);
    d2* in = U + (size_t)((mu * 2 + p) * 9) * g.Vh + s;
    const size_t ub = ((size_t)mu * g.V + i) * 9;
    if (to_internal) {
#pragma unroll
        for (int k = 0; k < 9; k++) in[(size_t)k * g.Vh] = user[ub + k];
    } else {
#pragma unroll
        for (int k = 0; k < 9; k++) ((d2*)user)[ub + k] = in[(size_t)k * g.Vh];
    }
}

__global__ void k_pack_gauge(Geom g, const d2* __restrict__ user, d2* __restrict__ U, int to_internal) {
    pack_gauge_body(g, user, U, to_internal, blockIdx.x * blockDim.x + threadIdx.x);
}

__device__ __forceinline__ void pack_mom_body(const Geom& g, const double* __restrict__ user, double* __restrict__ P,
                                              int to_internal, int t) {
    if (t >= 4 * g.V) return;
    int s = t % g.Vh, r = t / g.Vh, p = r & 1, mu = r >> 1;
    int i = lex_index(g, p, s);
    double* in = P + (size_t)((mu * 2 + p) * 8) * g.Vh + s;
    const size_t ub = ((size_t)mu * g.V + i) * 8;
    if (to_internal) {
#pragma unroll
        for (int a = 0; a < 8; a++) in[(size_t)a * g.Vh] = user[ub + a];
    } else {
#pragma unroll
        for (int a = 0; a < 8; a++) ((double*)user)[ub + a] = in[(size_t)a * g.Vh];
    }
}

__global__ void k_pack_mom(Geom g, const double* __restrict__ user, double* __restrict__ P, int to_internal) {
    pack_mom_body(g, user, P, to_internal, blockIdx.x * blockDim.x + threadIdx.x);
}

// user even spinor: entry k (= checkerboard index of the k-th even site) holds [4][3] complex
__device__ __forceinline__ void pack_even_body(const Geom& g, const d2* __restrict__ user, d2* __restrict__ X,
                                               int to_internal, int s) {
    if (s >= g.Vh) return;
    if (to_internal) {
#pragma unroll
        for (int k = 0; k < 12; k++) X[(size_t)k * g.Vh + s] = user[(size_t)s * 12 + k];
    } else {
#pragma unroll
        for (int k = 0; k < 12; k++) ((d2*)user)[(size_t)s * 12 + k] = X[(size_t)k * g.Vh + s];
    }
}

__global__ void k_pack_even(Geom g, const d2* __restrict__ user, d2* __restrict__ X, int to_internal) {
    pack_even_body(g, user, X, to_internal, blockIdx.x * blockDim.x + threadIdx.x);
}

// batched: field 0 links, 1 momenta, 2 even spinor (the chain's user pointer)
__global__ void k_pack_b(const ChainDesc* __restrict__ cd, int nc, void* internal, int field, int to_internal) {
    const int kind = field == 2 ? GRID_VH : GRID_4V;
    const int c = find_chain(cd, nc, blockIdx.x, kind);
    const ChainDesc& d = cd[c];
    const int t = (blockIdx.x - d.blk0[kind]) * blockDim.x + threadIdx.x;
    if (field == 0) pack_gauge_body(d.g, (const d2*)d.user_U, (d2*)internal + 9 * d.link0, to_internal, t);
    else if (field == 1) pack_mom_body(d.g, (const double*)d.user_P, (double*)internal + 8 * d.link0, to_internal, t);
    else pack_even_body(d.g, (const d2*)d.user_eta, (d2*)internal + 12 * d.site0, to_internal, t);
}

void pack_gauge(Ctx& c, const Geom& g, const void* user, d2* U) {
    hipLaunchKernelGGL(k_pack_gauge, dim3(nblocks(4L * g.V, BS)), dim3(BS), 0, c.stream, g, (const d2*)user, U, 1);
    FGI_LAUNCH_CHECK();
}
void unpack_gauge(Ctx& c, const Geom& g, const d2* U, void* user) {
    hipLaunchKernelGGL(k_pack_gauge, dim3(nblocks(4L * g.V, BS)), dim3(BS), 0, c.stream, g, (const d2*)user, (d2*)U, 0);
    FGI_LAUNCH_CHECK();
}
void pack_mom(Ctx& c, const Geom& g, const double* user, double* P) {
    hipLaunchKernelGGL(k_pack_mom, dim3(nblocks(4L * g.V, BS)), dim3(BS), 0, c.stream, g, user, P, 1);
    FGI_LAUNCH_CHECK();
}
void unpack_mom(Ctx& c, const Geom& g, const double* P, double* user) {
    hipLaunchKernelGGL(k_pack_mom, dim3(nblocks(4L * g.V, BS)), dim3(BS), 0, c.stream, g, (const double*)user, (double*)P, 0);
    FGI_LAUNCH_CHECK();
}
void pack_even_spinor(Ctx& c, const Geom& g, const void* user, d2* X) {
    hipLaunchKernelGGL(k_pack_even, dim3(nblocks(g.Vh, BS)), dim3(BS), 0, c.stream, g, (const d2*)user, X, 1);
    FGI_LAUNCH_CHECK();
}
void unpack_even_spinor(Ctx& c, const Geom& g, const d2* X, void* user) {
    hipLaunchKernelGGL(k_pack_even, dim3(nblocks(g.Vh, BS)), dim3(BS), 0, c.stream, g, (const d2*)user, (d2*)X, 0);
    FGI_LAUNCH_CHECK();
}

// sloppy copies of the FP64 master gauge field
__device__ __forceinline__ void make_sloppy_body(const Geom& g, const d2* __restrict__ U, void* __restrict__ out,
                                                 int prec, int recon, int t) {
    if (t >= 4 * g.V) return;
    int s = t % g.Vh, r = t / g.Vh;  // r = mu * 2 + p
    const d2* in = U + (size_t)(r * 9) * g.Vh + s;
    cx<double> e[9];
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const d2 v = in[(size_t)k * g.Vh];
        e[k] = {v.x, v.y};
    }
    store_sloppy_link(out, prec, recon, r, s, g.Vh, e);
}

__global__ void k_make_sloppy(Geom g, const d2* __restrict__ U, void* __restrict__ out, int prec, int recon) {
    make_sloppy_body(g, U, out, prec, recon, blockIdx.x * blockDim.x + threadIdx.x);
}

// byte offset of a chain's sloppy links in the concatenated sloppy field
__device__ __forceinline__ size_t sloppy_byte_off(const ChainDesc& d, int prec, int recon) {
    return (size_t)d.link0 * sloppy_link_bytes(prec, recon);
}

__global__ void k_make_sloppy_b(const ChainDesc* __restrict__ cd, int nc, const d2* __restrict__ U,
                                void* __restrict__ out, int prec, int recon) {
    const int c = find_chain(cd, nc, blockIdx.x, GRID_4V);
    const ChainDesc& d = cd[c];
    make_sloppy_body(d.g, U + 9 * d.link0, (char*)out + sloppy_byte_off(d, prec, recon), prec, recon,
                     (blockIdx.x - d.blk0[GRID_4V]) * blockDim.x + threadIdx.x);
}

void make_sloppy(Ctx& c, const Geom& g, const d2* U, void* sloppy, int prec, int recon) {
    hipLaunchKernelGGL(k_make_sloppy, dim3(nblocks(4L * g.V, BS)), dim3(BS), 0, c.stream, g, U, sloppy, prec, recon);
    FGI_LAUNCH_CHECK();
}

// ----------------------------------------------------------- densities ---
// h(x) = beta sum_{mu<nu} (1 - ReTr[U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+]/3)
//        + 1/2 sum_mu |p_mu(x)|^2
__device__ __forceinline__ void ham_density_body(const Geom& g, double beta, const d2* __restrict__ U,
                                                 const double* __restrict__ P, double* __restrict__ h, int t) {
    if (t >= g.V) return;
    int p = t / g.Vh, s = t % g.Vh;
    Coord c = cb_coords(g, p, s);
    double acc = 0.0;
#pragma unroll 1
    for (int mu = 0; mu < (U ? 4 : 0); mu++) {
        M3<double> umu = gauge_load(U, mu, p, s, g.Vh);
        int smu = cb_neighbour(g, c, mu, +1);
#pragma unroll 1
        for (int nu = mu + 1; nu < 4; nu++) {
            int snu = cb_neighbour(g, c, nu, +1);
            M3<double> a = m3_mul(umu, gauge_load(U, nu, 1 - p, smu, g.Vh));
            M3<double> b = m3_mul(gauge_load(U, nu, p, s, g.Vh), gauge_load(U, mu, 1 - p, snu, g.Vh));
            double tr = 0.0;
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) tr += a.e[i][j].re * b.e[i][j].re + a.e[i][j].im * b.e[i][j].im;
            acc += 1.0 - tr / 3.0;
        }
    }
    acc *= beta;
    if (P) {
        double kin = 0.0;
        for (int mu = 0; mu < 4; mu++) {
            double x[8];
            mom_load(P, mu, p, s, g.Vh, x);
#pragma unroll
            for (int a = 0; a < 8; a++) kin += x[a] * x[a];
        }
        acc += 0.5 * kin;
    }
    h[t] = acc;
}

__global__ void __launch_bounds__(256) k_ham_density(Geom g, double beta, const d2* __restrict__ U, const double* __restrict__ P,
                              double* __restrict__ h) {
    ham_density_body(g, beta, U, P, h, blockIdx.x * blockDim.x + threadIdx.x);
}

// bscale multiplies each chain's beta (1 - 8 c1 for the plaquettes of the improved action)
__global__ void __launch_bounds__(256) k_ham_density_b(const ChainDesc* __restrict__ cd, int nc, const d2* __restrict__ U,
                                const double* __restrict__ P, double* __restrict__ h, double bscale) {
    const int c = find_chain(cd, nc, blockIdx.x, GRID_V);
    const ChainDesc& d = cd[c];
    ham_density_body(d.g, d.beta * bscale, U ? U + 9 * d.link0 : nullptr, P ? P + 8 * d.link0 : nullptr, h + d.vol0,
                     (blockIdx.x - d.blk0[GRID_V]) * blockDim.x + threadIdx.x);
}

void rect_density_add(Ctx& c, const Geom& g, double bc1, const d2* U, double* h);

void ham_density(Ctx& c, const Geom& g, double beta, const d2* U, const double* P, double* h, double c1) {
    hipLaunchKernelGGL(k_ham_density, dim3(nblocks(g.V, BS)), dim3(BS), 0, c.stream, g, beta * (1.0 - 8.0 * c1), U,
                       P, h);
    FGI_LAUNCH_CHECK();
    if (c1 != 0.0 && U) rect_density_add(c, g, beta * c1, U, h);
}

__global__ void k_diff_partials(int n, const double* __restrict__ h1, const double* __restrict__ h0,
                                double* __restrict__ partial) {
    __shared__ double lds[16];
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    double v[1] = {0.0};
    if (t < n) v[0] = h0 ? h1[t] - h0[t] : h1[t];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

// partial[blk0 + b] = sum over chain-local block b of (h1 - h0) on the chain's V sites
__global__ void k_diff_partials_b(const ChainDesc* __restrict__ cd, int nc, const double* __restrict__ h1,
                                  const double* __restrict__ h0, double* __restrict__ partial) {
    __shared__ double lds[16];
    const int c = find_chain(cd, nc, blockIdx.x, GRID_V);
    const ChainDesc& d = cd[c];
    const int t = (blockIdx.x - d.blk0[GRID_V]) * blockDim.x + threadIdx.x;
    double v[1] = {0.0};
    if (t < d.g.V) v[0] = h0 ? h1[d.vol0 + t] - h0[d.vol0 + t] : h1[d.vol0 + t];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

// out[c] = fixed-order sum of chain c's partials (one block per chain)
__global__ void k_final_sum_b(const ChainDesc* __restrict__ cd, const double* __restrict__ partial, int kind,
                              double* __restrict__ out) {
    __shared__ double lds[16];
    const ChainDesc& d = cd[blockIdx.x];
    double s = sum_partials(partial + d.blk0[kind], d.nblk[kind], lds);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

int diff_partials(Ctx& c, int n, const double* h1, const double* h0, double* partial) {
    int nb = nblocks(n, BS);
    hipLaunchKernelGGL(k_diff_partials, dim3(nb), dim3(BS), 0, c.stream, n, h1, h0, partial);
    FGI_LAUNCH_CHECK();
    return nb;
}

__global__ void k_final_sum(const double* __restrict__ partial, int n, double* __restrict__ out) {
    __shared__ double lds[16];
    double s = sum_partials(partial, n, lds);
    if (threadIdx.x == 0) *out = s;
}

void final_sum(Ctx& c, const double* partial, int n, double* out) {
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(BS), 0, c.stream, partial, n, out);
    FGI_LAUNCH_CHECK();
}

// ------------------------------------------------------------- force -----
// Staple sum A_mu(x) = sum_{nu != mu} [U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
//                                     + U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)];
// the part of S_G holding U_mu(x) is -beta/3 ReTr(U_mu(x) A_mu(x)), so
// F_mu(x) = -e S = -(beta/6) TA(U_mu(x) A_mu(x)).
// one link U_mu(x); MU known at compile time (every block of the force
// launch holds links of one direction, so the switch below does not diverge)
template <int MU>
__device__ __forceinline__ void gauge_force_link(const Geom& g, double beta, const d2* __restrict__ U,
                                                 double* __restrict__ F, double coef, int accumulate, int s, int p,
                                                 int r) {
    const Coord c = cb_coords(g, p, s);
    const int s_pmu = cb_neighbour(g, c, MU, +1);
    const Coord cpm = cb_shift(g, c, MU, +1);
    M3<double> A = m3_zero<double>();
#pragma unroll 1
    for (int nu = 0; nu < 4; nu++) {
        if (nu == MU) continue;
        int s_pnu = cb_neighbour(g, c, nu, +1);
        int s_mnu = cb_neighbour(g, c, nu, -1);
        int s_pmu_mnu = cb_neighbour(g, cpm, nu, -1);
        // upper: U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
        M3<double> up = m3_mul_nd(m3_mul_nd(gauge_load(U, nu, 1 - p, s_pmu, g.Vh), gauge_load(U, MU, 1 - p, s_pnu, g.Vh)),
                                  gauge_load(U, nu, p, s, g.Vh));
        m3_acc(A, up);
        // lower: (U_mu(x-nu) U_nu(x+mu-nu))^+ U_nu(x-nu)
        M3<double> ed = m3_mul(gauge_load(U, MU, 1 - p, s_mnu, g.Vh), gauge_load(U, nu, p, s_pmu_mnu, g.Vh));
        m3_acc(A, m3_mul_dn(ed, gauge_load(U, nu, 1 - p, s_mnu, g.Vh)));
    }
    M3<double> W = m3_mul(gauge_load(U, MU, p, s, g.Vh), A);
    double x[8];
    ta_components(W, x);
    double* o = F + (size_t)(r * 8) * g.Vh + s;
    double f = -beta / 6.0 * coef;
#pragma unroll
    for (int a = 0; a < 8; a++) {
        double v = f * x[a];
        o[(size_t)a * g.Vh] = accumulate ? o[(size_t)a * g.Vh] + v : v;
    }
}

__device__ __forceinline__ void gauge_force_body(const Geom& g, double beta, const d2* __restrict__ U,
                                                 double* __restrict__ F, double coef, int accumulate, int t) {
    if (t >= 4 * g.V) return;
    int s = t % g.Vh, r = t / g.Vh, p = r & 1, mu = r >> 1;
    switch (mu) {
    case 0: gauge_force_link<0>(g, beta, U, F, coef, accumulate, s, p, r); break;
    case 1: gauge_force_link<1>(g, beta, U, F, coef, accumulate, s, p, r); break;
    case 2: gauge_force_link<2>(g, beta, U, F, coef, accumulate, s, p, r); break;
    default: gauge_force_link<3>(g, beta, U, F, coef, accumulate, s, p, r); break;
    }
}

__global__ void __launch_bounds__(256) k_gauge_force(Geom g, double beta, const d2* __restrict__ U,
                                                    double* __restrict__ F, double coef, int accumulate, int xcd) {
    gauge_force_body(g, beta, U, F, coef, accumulate, slab_thread(g.Vh, 8, xcd));
}

__global__ void __launch_bounds__(256) k_gauge_force_b(const ChainDesc* __restrict__ cd, int nc,
                                                      const d2* __restrict__ U, double* __restrict__ F, double coef,
                                                      int accumulate) {
    const int c = find_chain(cd, nc, blockIdx.x, GRID_4V);
    const ChainDesc& d = cd[c];
    gauge_force_body(d.g, d.beta, U + 9 * d.link0, F + 8 * d.link0, coef, accumulate,
                     (blockIdx.x - d.blk0[GRID_4V]) * blockDim.x + threadIdx.x);
}

void rect_force(Ctx& c, const Geom& g, double beta, double c1, const d2* U, double* F, double coef);

void gauge_force(Ctx& c, const Geom& g, double beta, const d2* U, double* F, double coef, int accumulate, double c1) {
    hipLaunchKernelGGL(k_gauge_force, dim3(slab_blocks(g.Vh, 8, BS, c.ds_xcd)), dim3(BS), 0, c.stream, g, beta, U, F,
                       coef * (1.0 - 8.0 * c1), accumulate, c.ds_xcd);
    FGI_LAUNCH_CHECK();
    if (c1 != 0.0) rect_force(c, g, beta, c1, U, F, coef);
}

// Tangent of the gauge force along a field of su(3) elements V:
// d/dt F_G(exp(tV) U) at t = 0.  Each link moves as dU = V U, dU^+ = -U^+ V;
// the product rule is applied factor by factor to U_mu(x) A_mu(x).
__device__ __forceinline__ M3<double> valg(const double* Vd, int mu, int p, int s, int Vh) {
    double x[8];
    mom_load(Vd, mu, p, s, Vh, x);
    return alg_matrix(x);
}

// mode 0: J = coef * d/dt F_G(exp(tV) U)
// mode 1: J = coef * (Hessian of S_G in the chart exp(omega) U at omega = 0) V
//         = coef * (-J_V[F_G] + [V, F_G] / 2)   (per link commutator)
__global__ void __launch_bounds__(256) k_gauge_tangent(Geom g, double beta, const d2* __restrict__ U,
                                                      const double* __restrict__ Vd, double* __restrict__ J,
                                                      double coef, int accumulate, int mode, int xcd) {
    int t = slab_thread(g.Vh, 8, xcd);
    if (t >= 4 * g.V) return;
    int s = t % g.Vh, r = t / g.Vh, p = r & 1, mu = r >> 1;
    Coord c = cb_coords(g, p, s);
    // indexed coordinates here (cb_neighbour_ix): with selects this kernel
    // spills more and runs 3 % slower than with the compiler's LDS copy
    int s_pmu = cb_neighbour_ix(g, c, mu, +1);
    Coord cpm = c;
    cpm.c[mu] = (c.c[mu] + 1) % g.L[mu];
    M3<double> A = m3_zero<double>(), dA = m3_zero<double>();
#pragma unroll 1
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        int s_pnu = cb_neighbour_ix(g, c, nu, +1);
        int s_mnu = cb_neighbour_ix(g, c, nu, -1);
        int s_pmu_mnu = cb_neighbour_ix(g, cpm, nu, -1);
        {   // upper staple a b^+ c^+
            M3<double> a = gauge_load(U, nu, 1 - p, s_pmu, g.Vh);
            M3<double> b = gauge_load(U, mu, 1 - p, s_pnu, g.Vh);
            M3<double> cc = gauge_load(U, nu, p, s, g.Vh);
            M3<double> da = m3_mul(valg(Vd, nu, 1 - p, s_pmu, g.Vh), a);
            M3<double> db = m3_mul(valg(Vd, mu, 1 - p, s_pnu, g.Vh), b);
            M3<double> dc = m3_mul(valg(Vd, nu, p, s, g.Vh), cc);
            M3<double> bc = m3_mul_nd(m3_dag(b), cc);  // b^+ c^+
            m3_acc(A, m3_mul(a, bc));
            m3_acc(dA, m3_mul(da, bc));
            m3_acc(dA, m3_mul_nd(m3_mul_nd(a, db), cc));
            m3_acc(dA, m3_mul_nd(m3_mul_nd(a, b), dc));
        }
        {   // lower staple d^+ e^+ f
            M3<double> d = gauge_load(U, nu, p, s_pmu_mnu, g.Vh);
            M3<double> e = gauge_load(U, mu, 1 - p, s_mnu, g.Vh);
            M3<double> f = gauge_load(U, nu, 1 - p, s_mnu, g.Vh);
            M3<double> dd = m3_mul(valg(Vd, nu, p, s_pmu_mnu, g.Vh), d);
            M3<double> de = m3_mul(valg(Vd, mu, 1 - p, s_mnu, g.Vh), e);
            M3<double> df = m3_mul(valg(Vd, nu, 1 - p, s_mnu, g.Vh), f);
            M3<double> ed = m3_mul(e, d);  // (d^+ e^+)^+
            m3_acc(A, m3_mul_dn(ed, f));
            m3_acc(dA, m3_mul_dn(m3_mul(e, dd), f));
            m3_acc(dA, m3_mul_dn(m3_mul(de, d), f));
            m3_acc(dA, m3_mul_dn(ed, df));
        }
    }
    M3<double> u = gauge_load(U, mu, p, s, g.Vh);
    M3<double> vl = valg(Vd, mu, p, s, g.Vh);
    M3<double> du = m3_mul(vl, u);
    M3<double> dW = m3_mul(du, A);
    m3_acc(dW, m3_mul(u, dA));
    double x[8];
    ta_components(dW, x);
    double* o = J + (size_t)(r * 8) * g.Vh + s;
    const double f = -beta / 6.0;
    if (mode == 1) {
        // F = f TA(U A) as a matrix; [V, F] components
        double fx[8];
        ta_components(m3_mul(u, A), fx);
#pragma unroll
        for (int a = 0; a < 8; a++) fx[a] *= f;
        M3<double> Fm = alg_matrix(fx);
        M3<double> C = m3_mul(vl, Fm);
        M3<double> D = m3_mul(Fm, vl);
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) C.e[i][j] = C.e[i][j] - D.e[i][j];
        double cx8[8];
        ta_components(C, cx8);
#pragma unroll
        for (int a = 0; a < 8; a++) x[a] = -f * x[a] + 0.5 * cx8[a];
    } else {
#pragma unroll
        for (int a = 0; a < 8; a++) x[a] = f * x[a];
    }
#pragma unroll
    for (int a = 0; a < 8; a++) {
        double v = coef * x[a];
        o[(size_t)a * g.Vh] = accumulate ? o[(size_t)a * g.Vh] + v : v;
    }
}

void rect_tangent(Ctx& c, const Geom& g, double beta, double c1, const d2* U, const double* Vd, double* J,
                  double coef, int mode);

void gauge_force_tangent(Ctx& c, const Geom& g, double beta, const d2* U, const double* Vd, double* J, double coef,
                         int accumulate, int mode, double c1) {
    hipLaunchKernelGGL(k_gauge_tangent, dim3(slab_blocks(g.Vh, 8, BS, c.ds_xcd)), dim3(BS), 0, c.stream, g, beta, U,
                       Vd, J, coef * (1.0 - 8.0 * c1), accumulate, mode, c.ds_xcd);
    FGI_LAUNCH_CHECK();
    if (c1 != 0.0) rect_tangent(c, g, beta, c1, U, Vd, J, coef, mode);
}

// ------------------------------------------------- rectangle (2x1) terms ---
// Improved gauge action
//   S_G = beta sum_x [c0 sum_{mu<nu} (1 - ReTr P_{mu nu}(x)/3) + c1 sum_{mu!=nu} (1 - ReTr R_{mu nu}(x)/3)],
// c0 = 1 - 8 c1, R_{mu nu}(x) the rectangle two links along mu and one along nu
// (c1 = -1/12: tree-level Symanzik, Luscher and Weisz 1985; c1 = -0.331:
// Iwasaki).  Everything is linear in (c0, c1): the plaquette kernels above run
// with their coefficient scaled by c0 and the kernels below add the c1 part.

// The 18 rectangle staples of link (mu, x) are the 5-link paths from x + mu
// back to x that close a 2x1 rectangle through U_mu(x); per nu != mu, six
// shapes, written as steps (+-1: along +-mu, +-2: along +-nu):
//   two long along mu, +nu side, U_mu(x) the first or the second mu link;
//   the same on the -nu side; two long along nu on the +nu and -nu sides.
__constant__ int RECT_SHAPES[6][5] = {{1, 2, -1, -1, -2}, {2, -1, -1, -2, 1}, {1, -2, -1, -1, 2},
                                      {-2, -1, -1, 2, 1},  {2, 2, -1, -2, -2}, {-2, -2, -1, 2, 2}};

// One factor of a path walked from y: a step along +d multiplies U_d(y) and
// moves to y + d; a step along -d moves to y - d and multiplies U_d(y)^+.
// With TAN, dl is the derivative of the factor along V (V U, or -U^+ V).
template <bool TAN>
__device__ __forceinline__ M3<double> path_factor(const Geom& g, const d2* __restrict__ U,
                                                  const double* __restrict__ Vd, Coord& y, int d, int fwd,
                                                  M3<double>& dl) {
    if (!fwd) coord_step(g, y, d, 0);
    const int par = coord_parity(y), s = cb_index(g, y);
    const M3<double> u = gauge_load(U, d, par, s, g.Vh);
    if (TAN) {
        const M3<double> v = valg(Vd, d, par, s, g.Vh);
        if (fwd) {
            dl = m3_mul(v, u);
        } else {
            dl = m3_mul_dn(u, v);
            m3_scale(dl, -1.0);
        }
    }
    if (fwd) coord_step(g, y, d, 1);
    return fwd ? u : m3_dag(u);
}

// A = sum of the 18 rectangle staples of link (mu, x); with TAN, dA = its
// derivative along V by the product rule, factor by factor.
template <bool TAN>
__device__ __forceinline__ void rect_staples(const Geom& g, const d2* __restrict__ U, const double* __restrict__ Vd,
                                             const Coord& c, int mu, M3<double>& A, M3<double>& dA) {
    A = m3_zero<double>();
    if (TAN) dA = m3_zero<double>();
#pragma unroll 1
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
#pragma unroll 1
        for (int k = 0; k < 6; k++) {
            Coord y = c;
            coord_step(g, y, mu, 1);
            M3<double> P, D, dl;
#pragma unroll 1
            for (int j = 0; j < 5; j++) {
                const int st = RECT_SHAPES[k][j];
                const int d = (st == 1 || st == -1) ? mu : nu;
                const M3<double> f = path_factor<TAN>(g, U, Vd, y, d, st > 0, dl);
                if (j == 0) {
                    P = f;
                    if (TAN) D = dl;
                } else {
                    if (TAN) {
                        D = m3_mul(D, f);
                        m3_acc(D, m3_mul(P, dl));
                    }
                    P = m3_mul(P, f);
                }
            }
            m3_acc(A, P);
            if (TAN) m3_acc(dA, D);
        }
    }
}

// h(x) += bc1 sum_{mu != nu} (1 - ReTr R_{mu nu}(x) / 3), with
// ReTr R = ReTr(a b^+), a = U_mu(x) U_mu(x+mu) U_nu(x+2mu), b = U_nu(x) U_mu(x+nu) U_mu(x+mu+nu)
__device__ __forceinline__ void rect_density_body(const Geom& g, double bc1, const d2* __restrict__ U,
                                                  double* __restrict__ h, int t) {
    if (t >= g.V) return;
    const int p = t / g.Vh, s = t % g.Vh;
    const Coord c = cb_coords(g, p, s);
    double acc = 0.0;
#pragma unroll 1
    for (int mu = 0; mu < 4; mu++) {
        Coord xm = c;
        coord_step(g, xm, mu, 1);
        Coord x2m = xm;
        coord_step(g, x2m, mu, 1);
        const M3<double> aa = m3_mul(gauge_load(U, mu, p, s, g.Vh), link_at(g, U, mu, xm));
#pragma unroll 1
        for (int nu = 0; nu < 4; nu++) {
            if (nu == mu) continue;
            Coord xn = c, xmn = xm;
            coord_step(g, xn, nu, 1);
            coord_step(g, xmn, nu, 1);
            const M3<double> a = m3_mul(aa, link_at(g, U, nu, x2m));
            const M3<double> b = m3_mul(m3_mul(gauge_load(U, nu, p, s, g.Vh), link_at(g, U, mu, xn)),
                                        link_at(g, U, mu, xmn));
            double tr = 0.0;
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) tr += a.e[i][j].re * b.e[i][j].re + a.e[i][j].im * b.e[i][j].im;
            acc += 1.0 - tr / 3.0;
        }
    }
    h[t] += bc1 * acc;
}

__global__ void __launch_bounds__(256) k_rect_density(Geom g, double bc1, const d2* __restrict__ U,
                                                     double* __restrict__ h) {
    rect_density_body(g, bc1, U, h, blockIdx.x * blockDim.x + threadIdx.x);
}

// batched chains: chain c adds its beta * c1 times its rectangle sum
__global__ void __launch_bounds__(256) k_rect_density_b(const ChainDesc* __restrict__ cd, int nc, double c1,
                                                       const d2* __restrict__ U, double* __restrict__ h) {
    const int c = find_chain(cd, nc, blockIdx.x, GRID_V);
    const ChainDesc& d = cd[c];
    rect_density_body(d.g, d.beta * c1, U + 9 * d.link0, h + d.vol0,
                      (blockIdx.x - d.blk0[GRID_V]) * blockDim.x + threadIdx.x);
}

void rect_density_add(Ctx& c, const Geom& g, double bc1, const d2* U, double* h) {
    hipLaunchKernelGGL(k_rect_density, dim3(nblocks(g.V, BS)), dim3(BS), 0, c.stream, g, bc1, U, h);
    FGI_LAUNCH_CHECK();
}

// The six shapes per nu pair up on their first step from x + mu (+mu, +nu,
// -nu): A gathers F (R_a + R_b) with F the shared first factor and R_a, R_b
// the four-link remainders, 21 products per nu in place of 24. Loops stay
// rolled, one link load and one product per step, so only four 3x3 matrices
// (A, R, the running product, the factor) are live.
__constant__ int RECT_PAIRS[3][9] = {{1, 2, -1, -1, -2, -2, -1, -1, 2},
                                     {2, -1, -1, -2, 1, 2, -1, -2, -2},
                                     {-2, -1, -1, 2, 1, -2, -1, 2, 2}};

__device__ __forceinline__ M3<double> rect_staples_paired(const Geom& g, const d2* __restrict__ U, const Coord& c,
                                                          int mu) {
    M3<double> A = m3_zero<double>(), dl;
#pragma unroll 1
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
#pragma unroll 1
        for (int k = 0; k < 3; k++) {
            Coord y0 = c;
            coord_step(g, y0, mu, 1);
            const int st0 = RECT_PAIRS[k][0];
            Coord y1 = y0;
            coord_step(g, y1, (st0 == 1 || st0 == -1) ? mu : nu, st0 > 0);
            M3<double> R;
#pragma unroll 1
            for (int h = 0; h < 2; h++) {
                Coord y = y1;
                const int* st = RECT_PAIRS[k] + 1 + 4 * h;
                M3<double> P = path_factor<false>(g, U, nullptr, y, (st[0] == 1 || st[0] == -1) ? mu : nu, st[0] > 0, dl);
#pragma unroll 1
                for (int j = 1; j < 4; j++) {
                    const int d = (st[j] == 1 || st[j] == -1) ? mu : nu;
                    P = m3_mul(P, path_factor<false>(g, U, nullptr, y, d, st[j] > 0, dl));
                }
                if (h == 0) R = P;
                else m3_acc(R, P);
            }
            m3_acc(A, m3_mul(path_factor<false>(g, U, nullptr, y0, (st0 == 1 || st0 == -1) ? mu : nu, st0 > 0, dl), R));
        }
    }
    return A;
}

// F_mu(x) += f TA(U_mu(x) A^R_mu(x)), f = -beta c1 coef / 6
__device__ __forceinline__ void rect_force_body(const Geom& g, double f, const d2* __restrict__ U,
                                                double* __restrict__ F, int t) {
    if (t >= 4 * g.V) return;
    const int s = t % g.Vh, r = t / g.Vh, p = r & 1, mu = r >> 1;
    const Coord c = cb_coords(g, p, s);
    const M3<double> A = rect_staples_paired(g, U, c, mu);
    const M3<double> W = m3_mul(gauge_load(U, mu, p, s, g.Vh), A);
    double x[8];
    ta_components(W, x);
    double* o = F + (size_t)(r * 8) * g.Vh + s;
#pragma unroll
    for (int a = 0; a < 8; a++) o[(size_t)a * g.Vh] += f * x[a];
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_rect_force(Geom g, double f, const d2* __restrict__ U,
                                                   double* __restrict__ F, int xcd) {
    rect_force_body(g, f, U, F, slab_thread(g.Vh, 8, xcd));
}

// batched chains: f = -beta_c c1 coef / 6 per chain
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_rect_force_b(const ChainDesc* __restrict__ cd, int nc, double c1, double coef,
                                                     const d2* __restrict__ U, double* __restrict__ F) {
    const int c = find_chain(cd, nc, blockIdx.x, GRID_4V);
    const ChainDesc& d = cd[c];
    rect_force_body(d.g, -d.beta * c1 * coef / 6.0, U + 9 * d.link0, F + 8 * d.link0,
                    (blockIdx.x - d.blk0[GRID_4V]) * blockDim.x + threadIdx.x);
}

void rect_force(Ctx& c, const Geom& g, double beta, double c1, const d2* U, double* F, double coef) {
    hipLaunchKernelGGL(k_rect_force, dim3(slab_blocks(g.Vh, 8, BS, c.ds_xcd)), dim3(BS), 0, c.stream, g,
                       -beta * c1 * coef / 6.0, U, F, c.ds_xcd);
    FGI_LAUNCH_CHECK();
}

// J += coef * (mode 0: J_V[F_R]; mode 1: -J_V[F_R] + [V, F_R] / 2) for the
// rectangle part F_R = -(beta c1 / 6) TA(U A^R) of the force
__global__ void __launch_bounds__(256) k_rect_tangent(Geom g, double bc1, const d2* __restrict__ U,
                                                     const double* __restrict__ Vd, double* __restrict__ J,
                                                     double coef, int mode, int xcd) {
    const int t = slab_thread(g.Vh, 8, xcd);
    if (t >= 4 * g.V) return;
    const int s = t % g.Vh, r = t / g.Vh, p = r & 1, mu = r >> 1;
    const Coord c = cb_coords(g, p, s);
    M3<double> A, dA;
    rect_staples<true>(g, U, Vd, c, mu, A, dA);
    const M3<double> u = gauge_load(U, mu, p, s, g.Vh);
    const M3<double> vl = valg(Vd, mu, p, s, g.Vh);
    M3<double> dW = m3_mul(m3_mul(vl, u), A);
    m3_acc(dW, m3_mul(u, dA));
    double x[8];
    ta_components(dW, x);
    const double f = -bc1 / 6.0;
    if (mode == 1) {
        double fx[8];
        ta_components(m3_mul(u, A), fx);
#pragma unroll
        for (int a = 0; a < 8; a++) fx[a] *= f;
        const M3<double> Fm = alg_matrix(fx);
        M3<double> C = m3_mul(vl, Fm);
        const M3<double> D = m3_mul(Fm, vl);
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) C.e[i][j] = C.e[i][j] - D.e[i][j];
        double cx8[8];
        ta_components(C, cx8);
#pragma unroll
        for (int a = 0; a < 8; a++) x[a] = -f * x[a] + 0.5 * cx8[a];
    } else {
#pragma unroll
        for (int a = 0; a < 8; a++) x[a] = f * x[a];
    }
    double* o = J + (size_t)(r * 8) * g.Vh + s;
#pragma unroll
    for (int a = 0; a < 8; a++) o[(size_t)a * g.Vh] += coef * x[a];
}

void rect_tangent(Ctx& c, const Geom& g, double beta, double c1, const d2* U, const double* Vd, double* J,
                  double coef, int mode) {
    hipLaunchKernelGGL(k_rect_tangent, dim3(slab_blocks(g.Vh, 8, BS, c.ds_xcd)), dim3(BS), 0, c.stream, g,
                       beta * c1, U, Vd, J, coef, mode, c.ds_xcd);
    FGI_LAUNCH_CHECK();
}

// ------------------------------------------------------------ updates ----
__device__ __forceinline__ void link_update_body(const Geom& g, double h, const double* __restrict__ X,
                                                 const d2* __restrict__ src, d2* __restrict__ dst,
                                                 void* __restrict__ sloppy, int prec, int recon, int t) {
    if (t >= 4 * g.V) return;
    int s = t % g.Vh, r = t / g.Vh, p = r & 1, mu = r >> 1;
    double x[8];
    mom_load(X, mu, p, s, g.Vh, x);
#pragma unroll
    for (int a = 0; a < 8; a++) x[a] *= h;
    M3<double> E = su3_exp(alg_matrix(x));
    M3<double> u = m3_mul(E, gauge_load(src, mu, p, s, g.Vh));
    gauge_store(dst, mu, p, s, g.Vh, u);
    if (sloppy) {
        cx<double> e[9];
#pragma unroll
        for (int k = 0; k < 9; k++) e[k] = u.e[k / 3][k % 3];
        store_sloppy_link(sloppy, prec, recon, r, s, g.Vh, e);
    }
}

__global__ void __launch_bounds__(256) k_link_update(Geom g, double h, const double* __restrict__ X, const d2* __restrict__ src,
                              d2* __restrict__ dst, void* __restrict__ sloppy, int prec, int recon) {
    link_update_body(g, h, X, src, dst, sloppy, prec, recon, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void __launch_bounds__(256) k_link_update_b(const ChainDesc* __restrict__ cd, int nc, double h, const double* __restrict__ X,
                                const d2* __restrict__ src, d2* __restrict__ dst, void* __restrict__ sloppy, int prec,
                                int recon) {
    const int c = find_chain(cd, nc, blockIdx.x, GRID_4V);
    const ChainDesc& d = cd[c];
    link_update_body(d.g, h, X + 8 * d.link0, src + 9 * d.link0, dst + 9 * d.link0,
                     sloppy ? (char*)sloppy + sloppy_byte_off(d, prec, recon) : nullptr, prec, recon,
                     (blockIdx.x - d.blk0[GRID_4V]) * blockDim.x + threadIdx.x);
}

void link_update(Ctx& c, const Geom& g, double h, const double* X, const d2* src, d2* dst, void* sloppy, int prec,
                 int recon) {
    hipLaunchKernelGGL(k_link_update, dim3(nblocks(4L * g.V, BS)), dim3(BS), 0, c.stream, g, h, X, src, dst, sloppy,
                       prec, recon);
    FGI_LAUNCH_CHECK();
}

// W_l = V_l U_l: the derivative of exp(t V_l) U_l at t = 0.  The hopping term
// is linear in each link and its adjoint, and d(U^+) = (V U)^+, so the
// hopping term on W is the derivative of D along V (Section 4, e_j acting
// on the fermion kernel).
__global__ void k_tangent_links(Geom g, const double* __restrict__ Vd, const d2* __restrict__ U,
                                d2* __restrict__ W) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * g.V) return;
    int s = t % g.Vh, r = t / g.Vh, p = r & 1, mu = r >> 1;
    double x[8];
    mom_load(Vd, mu, p, s, g.Vh, x);
    gauge_store(W, mu, p, s, g.Vh, m3_mul(alg_matrix(x), gauge_load(U, mu, p, s, g.Vh)));
}

void tangent_links(Ctx& c, const Geom& g, const double* Vd, const d2* U, d2* W) {
    hipLaunchKernelGGL(k_tangent_links, dim3(nblocks(4L * g.V, BS)), dim3(BS), 0, c.stream, g, Vd, U, W);
    FGI_LAUNCH_CHECK();
}

__global__ void k_axpy(long n, double a, const double* __restrict__ x, double* __restrict__ y) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] += a * x[t];
}

void mom_axpy(Ctx& c, const Geom& g, double a, const double* x, double* y) {
    long n = 4L * 2 * 8 * g.Vh;
    hipLaunchKernelGGL(k_axpy, dim3(nblocks(n, BS)), dim3(BS), 0, c.stream, n, a, x, y);
    FGI_LAUNCH_CHECK();
}

__global__ void k_dot_partials(long n, const double* __restrict__ x, const double* __restrict__ y,
                               double* __restrict__ partial) {
    __shared__ double lds[16];
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double v[1] = {t < n ? x[t] * y[t] : 0.0};
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

int dot_partials(Ctx& c, long n, const double* x, const double* y, double* partial) {
    int nb = nblocks(n, BS);
    hipLaunchKernelGGL(k_dot_partials, dim3(nb), dim3(BS), 0, c.stream, n, x, y, partial);
    FGI_LAUNCH_CHECK();
    return nb;
}

__global__ void k_zero_d(size_t n, double* __restrict__ p) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0;
}

void zero_doubles(Ctx& c, double* p, size_t n) {
    hipLaunchKernelGGL(k_zero_d, dim3(nblocks((long)n, BS)), dim3(BS), 0, c.stream, n, p);
    FGI_LAUNCH_CHECK();
}

// Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1)
__device__ __forceinline__ void reunitarize_body(const Geom& g, d2* __restrict__ U, int t) {
    if (t >= 4 * g.V) return;
    int s = t % g.Vh, r = t / g.Vh, p = r & 1, mu = r >> 1;
    M3<double> u = gauge_load(U, mu, p, s, g.Vh);
    double n0 = 0;
    for (int j = 0; j < 3; j++) n0 += u.e[0][j].re * u.e[0][j].re + u.e[0][j].im * u.e[0][j].im;
    n0 = 1.0 / sqrt(n0);
    for (int j = 0; j < 3; j++) u.e[0][j] = n0 * u.e[0][j];
    cx<double> d = {0, 0};
    for (int j = 0; j < 3; j++) d = d + cmul(u.e[0][j], u.e[1][j]);
    for (int j = 0; j < 3; j++) u.e[1][j] = u.e[1][j] - d * u.e[0][j];
    double n1 = 0;
    for (int j = 0; j < 3; j++) n1 += u.e[1][j].re * u.e[1][j].re + u.e[1][j].im * u.e[1][j].im;
    n1 = 1.0 / sqrt(n1);
    for (int j = 0; j < 3; j++) u.e[1][j] = n1 * u.e[1][j];
    recon_row2(u);
    gauge_store(U, mu, p, s, g.Vh, u);
}

__global__ void k_reunitarize(Geom g, d2* __restrict__ U) {
    reunitarize_body(g, U, blockIdx.x * blockDim.x + threadIdx.x);
}

void reunitarize(Ctx& c, const Geom& g, d2* U) {
    hipLaunchKernelGGL(k_reunitarize, dim3(nblocks(4L * g.V, BS)), dim3(BS), 0, c.stream, g, U);
    FGI_LAUNCH_CHECK();
}

__global__ void __launch_bounds__(256) k_exp_batch(int n, const double* __restrict__ p, double h, d2* __restrict__ out) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double x[8];
    for (int a = 0; a < 8; a++) x[a] = h * p[(size_t)t * 8 + a];
    M3<double> E = su3_exp(alg_matrix(x));
    for (int k = 0; k < 9; k++) out[(size_t)t * 9 + k] = d2{E.e[k / 3][k % 3].re, E.e[k / 3][k % 3].im};
}

void exp_su3_batch(Ctx& c, int n, const double* p, double h, void* out) {
    hipLaunchKernelGGL(k_exp_batch, dim3(nblocks(n, BS)), dim3(BS), 0, c.stream, n, p, h, (d2*)out);
    FGI_LAUNCH_CHECK();
}

// ------------------------------------------------------ batched launchers ---
void pack_b(Ctx& c, const Batch& B, void* internal, int field, int to_internal) {
    int nb = field == 2 ? B.nblk[GRID_VH] : B.nblk[GRID_4V];
    hipLaunchKernelGGL(k_pack_b, dim3(nb), dim3(BS), 0, c.stream, B.cd, B.nc, internal, field, to_internal);
    FGI_LAUNCH_CHECK();
}

void make_sloppy_b(Ctx& c, const Batch& B, const d2* U, void* sloppy, int prec, int recon) {
    hipLaunchKernelGGL(k_make_sloppy_b, dim3(B.nblk[GRID_4V]), dim3(BS), 0, c.stream, B.cd, B.nc, U, sloppy, prec, recon);
    FGI_LAUNCH_CHECK();
}

void ham_density_b(Ctx& c, const Batch& B, const d2* U, const double* P, double* h, double c1) {
    hipLaunchKernelGGL(k_ham_density_b, dim3(B.nblk[GRID_V]), dim3(BS), 0, c.stream, B.cd, B.nc, U, P, h,
                       1.0 - 8.0 * c1);
    FGI_LAUNCH_CHECK();
    if (c1 != 0.0 && U) {
        hipLaunchKernelGGL(k_rect_density_b, dim3(B.nblk[GRID_V]), dim3(BS), 0, c.stream, B.cd, B.nc, c1, U, h);
        FGI_LAUNCH_CHECK();
    }
}

void diff_sums_b(Ctx& c, const Batch& B, const double* h1, const double* h0, double* partial, double* out) {
    hipLaunchKernelGGL(k_diff_partials_b, dim3(B.nblk[GRID_V]), dim3(BS), 0, c.stream, B.cd, B.nc, h1, h0, partial);
    FGI_LAUNCH_CHECK();
    final_sums_b(c, B, partial, GRID_V, out);
}

void final_sums_b(Ctx& c, const Batch& B, const double* partial, int kind, double* out) {
    hipLaunchKernelGGL(k_final_sum_b, dim3(B.nc), dim3(BS), 0, c.stream, B.cd, partial, kind, out);
    FGI_LAUNCH_CHECK();
}

void gauge_force_b(Ctx& c, const Batch& B, const d2* U, double* F, double coef, int accumulate, double c1) {
    hipLaunchKernelGGL(k_gauge_force_b, dim3(B.nblk[GRID_4V]), dim3(BS), 0, c.stream, B.cd, B.nc, U, F,
                       coef * (1.0 - 8.0 * c1), accumulate);
    FGI_LAUNCH_CHECK();
    if (c1 != 0.0) {
        hipLaunchKernelGGL(k_rect_force_b, dim3(B.nblk[GRID_4V]), dim3(BS), 0, c.stream, B.cd, B.nc, c1, coef, U, F);
        FGI_LAUNCH_CHECK();
    }
}

void link_update_b(Ctx& c, const Batch& B, double h, const double* X, const d2* src, d2* dst, void* sloppy, int prec,
                   int recon) {
    hipLaunchKernelGGL(k_link_update_b, dim3(B.nblk[GRID_4V]), dim3(BS), 0, c.stream, B.cd, B.nc, h, X, src, dst, sloppy,
                       prec, recon);
    FGI_LAUNCH_CHECK();
}

}  // namespace fgi
