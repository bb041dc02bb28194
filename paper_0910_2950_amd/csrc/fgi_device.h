// Device-side building blocks of the force-gradient HMC library for gfx950:
// lattice geometry on the even/odd checkerboard, the structure-of-arrays field
// layouts, SU(3)/su(3) algebra, Wilson spin projectors, storage precisions and
// deterministic wave64 block reductions.
//
// Internal layouts (all per parity p in {0 even, 1 odd}, checkerboard index s
// in [0, Vh), Vh = V/2; a "chunk" is one 16- or 8-byte vector, consecutive s
// consecutive in memory so a wave's 64 lanes read one contiguous span):
//   gauge FP64        double2 [4 mu][2 p][9 elem][Vh]      (row-major 3x3)
//   gauge FP32 / 18   float2  [4][2][9][Vh]
//   gauge FP32 / 12   float4  [4][2][3][Vh]    rows 0,1 (row 2 rebuilt)
//   gauge FP16 / 12   half4   [4][2][3][Vh]    rows 0,1
//   momentum / force  double  [4][2][8][Vh]    su(3) components p_a
//   spinor FP64       double2 [12][Vh]         (spin*3 + colour)
//   spinor FP32       float4  [6][Vh]          two complex per chunk
//   spinor FP16       half8   [3][Vh] + float norm[Vh]   (values / norm)
// The site with checkerboard index s and parity p is the lexicographic site
// i = 2 s + ((y + z + t + p) & 1), i = x + Lx (y + Ly (z + Lz t)).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace fgi {

// --------------------------------------------------------------------------
// geometry
// --------------------------------------------------------------------------
struct Geom {
    int L[4];   // extents x, y, z, t (all even)
    int Lxh;    // L[0] / 2
    int V, Vh;  // volume, half volume
};

struct Coord { int c[4]; };

__device__ __forceinline__ Coord cb_coords(const Geom& g, int p, int s) {
    Coord r;
    int xh = s % g.Lxh;
    int q = s / g.Lxh;
    r.c[1] = q % g.L[1]; q /= g.L[1];
    r.c[2] = q % g.L[2];
    r.c[3] = q / g.L[2];
    r.c[0] = 2 * xh + ((r.c[1] + r.c[2] + r.c[3] + p) & 1);
    return r;
}

__device__ __forceinline__ int cb_index(const Geom& g, const Coord& c) {
    int i = c.c[0] + g.L[0] * (c.c[1] + g.L[1] * (c.c[2] + g.L[2] * c.c[3]));
    return i >> 1;
}

// checkerboard index of the neighbour x +/- mu (it has the other parity)
// a[d] read and written by selects: indexing a small array with a run-time d
// makes the compiler keep a per-thread copy of it in LDS (or scratch); with d
// known at compile time the selects fold to the plain access.
__device__ __forceinline__ int sel4(const int a[4], int d) {
    return d == 0 ? a[0] : (d == 1 ? a[1] : (d == 2 ? a[2] : a[3]));
}
__device__ __forceinline__ void put4(int a[4], int d, int v) {
    a[0] = d == 0 ? v : a[0];
    a[1] = d == 1 ? v : a[1];
    a[2] = d == 2 ? v : a[2];
    a[3] = d == 3 ? v : a[3];
}

// c moved by dir (+1 or -1) along mu, periodically
__device__ __forceinline__ Coord cb_shift(const Geom& g, Coord c, int mu, int dir) {
    const int L = sel4(g.L, mu);
    int v = sel4(c.c, mu) + dir;
    v = v < 0 ? v + L : (v >= L ? v - L : v);
    put4(c.c, mu, v);
    return c;
}

__device__ __forceinline__ int cb_neighbour(const Geom& g, Coord c, int mu, int dir) {
    return cb_index(g, cb_shift(g, c, mu, dir));
}

// the same with indexed accesses, for the few kernels where the compiler's
// per-thread LDS copy of c costs less than the registers the selects need
__device__ __forceinline__ int cb_neighbour_ix(const Geom& g, Coord c, int mu, int dir) {
    int v = c.c[mu] + dir;
    v = v < 0 ? v + g.L[mu] : (v >= g.L[mu] ? v - g.L[mu] : v);
    c.c[mu] = v;
    return cb_index(g, c);
}

// XCD-aware block order: the hardware hands consecutive workgroups to the 8
// XCDs round-robin; remap so each XCD walks one contiguous slab of sites and
// neighbour reads stay in its own L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int nx = 8;
    int q = nb / nx, r = nb % nx;
    int x = b % nx, k = b / nx;
    return x * q + (x < r ? x : r) + k;
}

// Thread index of a launch over nt arrays of Vh sites ([type][s], type =
// mu * 2 + parity for links, the parity for sites), blocks of blockDim.x.
// xcd = 0: linear.  xcd = 1: the nt blocks of each group of blockDim.x sites
// are adjacent and every XCD owns a contiguous range of groups (xcd_block),
// so the neighbour links and vectors a block reads were mostly fetched into
// its own XCD's L2 by the blocks beside it.  Past the end: nt * Vh.
__device__ __forceinline__ int slab_thread(int Vh, int nt, int xcd) {
    if (!xcd) return blockIdx.x * blockDim.x + threadIdx.x;
    const int B = xcd_block(blockIdx.x, gridDim.x);
    const int s = (B / nt) * blockDim.x + threadIdx.x;
    return s < Vh ? (B % nt) * Vh + s : nt * Vh;
}

// --------------------------------------------------------------------------
// batched chains: independent lattices stored one after another in every
// field; a kernel launched over all of them finds its chain from its block.
// --------------------------------------------------------------------------
// GRID_VH, GRID_V, GRID_4V: blocks of 256 even sites, sites or links;
// GRID_DS: even sites in blocks of the Dslash block size (a tuned schedule)
enum GridKind { GRID_VH = 0, GRID_V = 1, GRID_4V = 2, GRID_DS = 3 };

struct ChainDesc {
    Geom g;
    long site0;     // sum of Vh of the chains before (spinor offsets)
    long vol0;      // sum of V (per-site densities)
    long link0;     // sum of 4V (link / momentum offsets)
    double beta, kappa;
    int blk0[4];    // first block of the chain in each grid kind
    int nblk[4];    // its number of blocks there
    const void* user_U;   // user-layout buffers (pack / unpack)
    void* user_P;
    const void* user_eta;
};

// chain owning global block `blk` of a grid of the given kind (binary search)
__device__ __forceinline__ int find_chain(const ChainDesc* cd, int nchains, int blk, int kind) {
    int lo = 0, hi = nchains - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (cd[mid].blk0[kind] <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// element offsets of one chain's part of a concatenated field
__device__ __forceinline__ size_t gauge_chunk_off(const ChainDesc& c, int prec, int recon) {
    return (prec == 0 || recon == 18) ? 9 * (size_t)c.link0 : 3 * (size_t)c.link0;
}
__device__ __forceinline__ size_t spinor_chunk_off(const ChainDesc& c, int prec) {
    return prec == 0 ? 12 * (size_t)c.site0 : (prec == 1 ? 6 * (size_t)c.site0 : 3 * (size_t)c.site0);
}

// --------------------------------------------------------------------------
// complex numbers and 3x3 matrices, templated on the real type
// --------------------------------------------------------------------------
template <typename R> struct cx { R re, im; };

template <typename R> __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R> __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> __device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
// a0 b0 + a1 b1 + a2 b2 and conj(a0) b0 + conj(a1) b1 + conj(a2) b2, each
// component one chain of fused multiply-adds (a row or column of a link times
// a colour vector)
template <typename R>
__device__ __forceinline__ cx<R> cdot3(cx<R> a0, cx<R> b0, cx<R> a1, cx<R> b1, cx<R> a2, cx<R> b2) {
    R re = a0.re * b0.re;
    re = fma(-a0.im, b0.im, re);
    re = fma(a1.re, b1.re, re);
    re = fma(-a1.im, b1.im, re);
    re = fma(a2.re, b2.re, re);
    re = fma(-a2.im, b2.im, re);
    R im = a0.re * b0.im;
    im = fma(a0.im, b0.re, im);
    im = fma(a1.re, b1.im, im);
    im = fma(a1.im, b1.re, im);
    im = fma(a2.re, b2.im, im);
    im = fma(a2.im, b2.re, im);
    return {re, im};
}
template <typename R>
__device__ __forceinline__ cx<R> cdot3c(cx<R> a0, cx<R> b0, cx<R> a1, cx<R> b1, cx<R> a2, cx<R> b2) {
    R re = a0.re * b0.re;
    re = fma(a0.im, b0.im, re);
    re = fma(a1.re, b1.re, re);
    re = fma(a1.im, b1.im, re);
    re = fma(a2.re, b2.re, re);
    re = fma(a2.im, b2.im, re);
    R im = a0.re * b0.im;
    im = fma(-a0.im, b0.re, im);
    im = fma(a1.re, b1.im, im);
    im = fma(-a1.im, b1.re, im);
    im = fma(a2.re, b2.im, im);
    im = fma(-a2.im, b2.re, im);
    return {re, im};
}
// conj(a b - c d) as two FMA chains
template <typename R> __device__ __forceinline__ cx<R> conj_cross(cx<R> a, cx<R> b, cx<R> c, cx<R> d) {
    R re = a.re * b.re;
    re = fma(-a.im, b.im, re);
    re = fma(-c.re, d.re, re);
    re = fma(c.im, d.im, re);
    R im = -a.re * b.im;
    im = fma(-a.im, b.re, im);
    im = fma(c.re, d.im, im);
    im = fma(c.im, d.re, im);
    return {re, im};
}
// y + w z with one fused multiply-add per component
template <typename R> __device__ __forceinline__ cx<R> axpy(R w, cx<R> z, cx<R> y) {
    return {fma(w, z.re, y.re), fma(w, z.im, y.im)};
}
template <typename R> __device__ __forceinline__ cx<R> times_i(cx<R> a) { return {-a.im, a.re}; }
template <typename R> __device__ __forceinline__ cx<R> times_mi(cx<R> a) { return {a.im, -a.re}; }
// a * conj(b)
template <typename R> __device__ __forceinline__ cx<R> mulc(cx<R> a, cx<R> b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// conj(a) * b
template <typename R> __device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

template <typename R> struct M3 { cx<R> e[3][3]; };

template <typename R> __device__ __forceinline__ M3<R> m3_zero() {
    M3<R> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) r.e[i][j] = {R(0), R(0)};
    return r;
}

template <typename R> __device__ __forceinline__ M3<R> m3_mul(const M3<R>& a, const M3<R>& b) {
    M3<R> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) r.e[i][j] = a.e[i][0] * b.e[0][j] + a.e[i][1] * b.e[1][j] + a.e[i][2] * b.e[2][j];
    return r;
}

// a * b^+
template <typename R> __device__ __forceinline__ M3<R> m3_mul_nd(const M3<R>& a, const M3<R>& b) {
    M3<R> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            r.e[i][j] = mulc(a.e[i][0], b.e[j][0]) + mulc(a.e[i][1], b.e[j][1]) + mulc(a.e[i][2], b.e[j][2]);
    return r;
}

// a^+ * b
template <typename R> __device__ __forceinline__ M3<R> m3_mul_dn(const M3<R>& a, const M3<R>& b) {
    M3<R> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            r.e[i][j] = cmul(a.e[0][i], b.e[0][j]) + cmul(a.e[1][i], b.e[1][j]) + cmul(a.e[2][i], b.e[2][j]);
    return r;
}

template <typename R> __device__ __forceinline__ M3<R> m3_dag(const M3<R>& a) {
    M3<R> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) r.e[i][j] = conj(a.e[j][i]);
    return r;
}

template <typename R> __device__ __forceinline__ void m3_acc(M3<R>& a, const M3<R>& b) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) a.e[i][j] = a.e[i][j] + b.e[i][j];
}

template <typename R> __device__ __forceinline__ void m3_scale(M3<R>& a, R s) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) a.e[i][j] = s * a.e[i][j];
}

// --------------------------------------------------------------------------
// su(3) <-> components.  Basis T^a = i lambda^a / 2 (Gell-Mann lambda),
// Tr(T^a T^b) = -delta_ab / 2; X = sum_a x_a T^a; x_a = -2 Tr(T^a X).
// Written out element by element.
// --------------------------------------------------------------------------
__device__ __forceinline__ M3<double> alg_matrix(const double x[8]) {
    const double r3 = 0.57735026918962576451;  // 1/sqrt(3)
    M3<double> X;
    // diagonal: i/2 (x3 + x8/sqrt3), i/2 (-x3 + x8/sqrt3), i/2 (-2 x8/sqrt3)
    X.e[0][0] = {0.0, 0.5 * (x[2] + r3 * x[7])};
    X.e[1][1] = {0.0, 0.5 * (-x[2] + r3 * x[7])};
    X.e[2][2] = {0.0, -r3 * x[7]};
    // (0,1): i/2 (x1 - i x2) = (x2/2, x1/2); (1,0): i/2 (x1 + i x2) = (-x2/2, x1/2)
    X.e[0][1] = {0.5 * x[1], 0.5 * x[0]};
    X.e[1][0] = {-0.5 * x[1], 0.5 * x[0]};
    X.e[0][2] = {0.5 * x[4], 0.5 * x[3]};
    X.e[2][0] = {-0.5 * x[4], 0.5 * x[3]};
    X.e[1][2] = {0.5 * x[6], 0.5 * x[5]};
    X.e[2][1] = {-0.5 * x[6], 0.5 * x[5]};
    return X;
}

// components of the traceless anti-Hermitian part TA(W) = (W - W^+)/2 - Tr(W - W^+)/6,
// i.e. x_a = -2 Tr(T^a TA(W)) = Im-parts combined as below.
template <typename R> __device__ __forceinline__ void ta_components(const M3<R>& W, R x[8]) {
    const R r3 = R(0.57735026918962576451);
    // A = (W - W^+)/2: A01 = (W01 - conj W10)/2 etc.; A has diagonal i*Im(W_kk)
    // -2 Tr(T^a A) for the off-diagonal generators:
    //   a=1: Im(W01 + W10)          a=2: Re(W01 - W10)
    //   a=4: Im(W02 + W20)          a=5: Re(W02 - W20)
    //   a=6: Im(W12 + W21)          a=7: Re(W12 - W21)
    //   a=3: Im(W00) - Im(W11)      a=8: (Im W00 + Im W11 - 2 Im W22)/sqrt3
    x[0] = W.e[0][1].im + W.e[1][0].im;
    x[1] = W.e[0][1].re - W.e[1][0].re;
    x[2] = W.e[0][0].im - W.e[1][1].im;
    x[3] = W.e[0][2].im + W.e[2][0].im;
    x[4] = W.e[0][2].re - W.e[2][0].re;
    x[5] = W.e[1][2].im + W.e[2][1].im;
    x[6] = W.e[1][2].re - W.e[2][1].re;
    x[7] = r3 * (W.e[0][0].im + W.e[1][1].im - R(2) * W.e[2][2].im);
}

// --------------------------------------------------------------------------
// su(3) exponential: exp(X) for traceless anti-Hermitian X, by the
// Cayley-Hamilton closed form of Morningstar and Peardon (Phys. Rev. D 69
// (2004) 054501): with Q = -i X Hermitian traceless, exp(iQ) = f0 + f1 Q + f2 Q^2,
// where f_j follow from c0 = det Q, c1 = Tr Q^2 / 2.  Negative c0 is mapped
// to positive c0 with f_j(-c0) = (-1)^j conj(f_j(c0)).  Tiny Q uses a Taylor
// series instead (the closed form divides by a quantity of order c1).
// --------------------------------------------------------------------------
__device__ inline M3<double> su3_exp(const M3<double>& X) {
    M3<double> Q;  // Q = -i X
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) Q.e[i][j] = times_mi(X.e[i][j]);
    M3<double> Q2 = m3_mul(Q, Q);
    double c1 = 0.5 * (Q2.e[0][0].re + Q2.e[1][1].re + Q2.e[2][2].re);
    M3<double> r;
    if (c1 < 1e-6) {
        // exp(X) = sum_k X^k / k!, |X|^2 ~ 2 c1 < 2e-6: 9 terms leave < 1e-30
        M3<double> term, sum;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                term.e[i][j] = {i == j ? 1.0 : 0.0, 0.0};
                sum.e[i][j] = term.e[i][j];
            }
        for (int k = 1; k <= 9; k++) {
            term = m3_mul(term, X);
            m3_scale(term, 1.0 / k);
            m3_acc(sum, term);
        }
        return sum;
    }
    // c0 = det Q = Tr Q^3 / 3 (real for Hermitian traceless Q)
    M3<double> Q3 = m3_mul(Q2, Q);
    double c0 = (Q3.e[0][0].re + Q3.e[1][1].re + Q3.e[2][2].re) / 3.0;
    bool neg = c0 < 0;
    c0 = fabs(c0);
    double c0max = 2.0 * pow(c1 / 3.0, 1.5);
    double ratio = c0 / c0max;
    ratio = ratio > 1.0 ? 1.0 : ratio;
    double theta = acos(ratio);
    double u = sqrt(c1 / 3.0) * cos(theta / 3.0);
    double w = sqrt(c1) * sin(theta / 3.0);
    double u2 = u * u, w2 = w * w;
    double xi0 = (fabs(w) < 0.05) ? 1.0 - w2 / 6.0 * (1.0 - w2 / 20.0 * (1.0 - w2 / 42.0 * (1.0 - w2 / 72.0)))
                                  : sin(w) / w;
    double cw = cos(w);
    double s2u, c2u, su, cu;
    sincos(2.0 * u, &s2u, &c2u);
    sincos(u, &su, &cu);
    cx<double> e2iu = {c2u, s2u};
    cx<double> emiu = {cu, -su};
    // h0 = (u^2 - w^2) e^{2iu} + e^{-iu} (8 u^2 cos w + 2 i u (3u^2 + w^2) xi0)
    cx<double> h0 = (u2 - w2) * e2iu + emiu * mk(8.0 * u2 * cw, 2.0 * u * (3.0 * u2 + w2) * xi0);
    // h1 = 2u e^{2iu} - e^{-iu} (2u cos w - i (3u^2 - w^2) xi0)
    cx<double> h1 = (2.0 * u) * e2iu - emiu * mk(2.0 * u * cw, -(3.0 * u2 - w2) * xi0);
    // h2 = e^{2iu} - e^{-iu} (cos w + 3 i u xi0)
    cx<double> h2 = e2iu - emiu * mk(cw, 3.0 * u * xi0);
    double den = 1.0 / (9.0 * u2 - w2);
    cx<double> f0 = den * h0, f1 = den * h1, f2 = den * h2;
    if (neg) {
        f0 = conj(f0);
        f1 = -conj(f1);
        f2 = conj(f2);
    }
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<double> v = f1 * Q.e[i][j] + f2 * Q2.e[i][j];
            if (i == j) v = v + f0;
            r.e[i][j] = v;
        }
    return r;
}

// --------------------------------------------------------------------------
// Wilson spin projectors in the DeGrand-Rossi basis (gamma_1..4 for x,y,z,t).
// proj<MU, SIGN> returns the two independent spin components h0, h1 of
// (1 + SIGN gamma_MU) psi; recon<MU, SIGN> rebuilds the full 4-spinor (as an
// accumulation) from h0, h1 (already multiplied by a link).
//   (1 - g1): h = (p0 - i p3, p1 - i p2), full = (h0, h1,  i h1,  i h0)
//   (1 + g1): h = (p0 + i p3, p1 + i p2), full = (h0, h1, -i h1, -i h0)
//   (1 - g2): h = (p0 + p3,   p1 - p2),   full = (h0, h1, -h1,  h0)
//   (1 + g2): h = (p0 - p3,   p1 + p2),   full = (h0, h1,  h1, -h0)
//   (1 - g3): h = (p0 - i p2, p1 + i p3), full = (h0, h1,  i h0, -i h1)
//   (1 + g3): h = (p0 + i p2, p1 - i p3), full = (h0, h1, -i h0,  i h1)
//   (1 - g4): h = (p0 - p2,   p1 - p3),   full = (h0, h1, -h0, -h1)
//   (1 + g4): h = (p0 + p2,   p1 + p3),   full = (h0, h1,  h0,  h1)
// --------------------------------------------------------------------------
template <int MU, int SIGN, typename R>
__device__ __forceinline__ void spin_proj(const cx<R> p[4][3], cx<R> h[2][3]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if (MU == 0) {
            if (SIGN < 0) { h[0][c] = p[0][c] + times_mi(p[3][c]); h[1][c] = p[1][c] + times_mi(p[2][c]); }
            else          { h[0][c] = p[0][c] + times_i(p[3][c]);  h[1][c] = p[1][c] + times_i(p[2][c]); }
        } else if (MU == 1) {
            if (SIGN < 0) { h[0][c] = p[0][c] + p[3][c]; h[1][c] = p[1][c] - p[2][c]; }
            else          { h[0][c] = p[0][c] - p[3][c]; h[1][c] = p[1][c] + p[2][c]; }
        } else if (MU == 2) {
            if (SIGN < 0) { h[0][c] = p[0][c] + times_mi(p[2][c]); h[1][c] = p[1][c] + times_i(p[3][c]); }
            else          { h[0][c] = p[0][c] + times_i(p[2][c]);  h[1][c] = p[1][c] + times_mi(p[3][c]); }
        } else {
            if (SIGN < 0) { h[0][c] = p[0][c] - p[2][c]; h[1][c] = p[1][c] - p[3][c]; }
            else          { h[0][c] = p[0][c] + p[2][c]; h[1][c] = p[1][c] + p[3][c]; }
        }
    }
}

template <int MU, int SIGN, typename R>
__device__ __forceinline__ void spin_recon_acc(cx<R> acc[4][3], const cx<R> h[2][3], R w) {
    // acc += w * (the four-spinor rebuilt from the projected half spinor h);
    // w carries the storage scale and boundary sign, every term is one FMA
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const cx<R> a = h[0][c], b = h[1][c];
        acc[0][c] = axpy(w, a, acc[0][c]);
        acc[1][c] = axpy(w, b, acc[1][c]);
        if (MU == 0) {
            if (SIGN < 0) { acc[2][c] = axpy(w, times_i(b), acc[2][c]);  acc[3][c] = axpy(w, times_i(a), acc[3][c]); }
            else          { acc[2][c] = axpy(w, times_mi(b), acc[2][c]); acc[3][c] = axpy(w, times_mi(a), acc[3][c]); }
        } else if (MU == 1) {
            if (SIGN < 0) { acc[2][c] = axpy(w, -b, acc[2][c]); acc[3][c] = axpy(w, a, acc[3][c]); }
            else          { acc[2][c] = axpy(w, b, acc[2][c]);  acc[3][c] = axpy(w, -a, acc[3][c]); }
        } else if (MU == 2) {
            if (SIGN < 0) { acc[2][c] = axpy(w, times_i(a), acc[2][c]);  acc[3][c] = axpy(w, times_mi(b), acc[3][c]); }
            else          { acc[2][c] = axpy(w, times_mi(a), acc[2][c]); acc[3][c] = axpy(w, times_i(b), acc[3][c]); }
        } else {
            if (SIGN < 0) { acc[2][c] = axpy(w, -a, acc[2][c]); acc[3][c] = axpy(w, -b, acc[3][c]); }
            else          { acc[2][c] = axpy(w, a, acc[2][c]);  acc[3][c] = axpy(w, b, acc[3][c]); }
        }
    }
}

// --------------------------------------------------------------------------
// storage precisions
// --------------------------------------------------------------------------
enum Prec { P64 = 0, P32 = 1, P16 = 2 };

template <int P> struct Real { typedef float T; };
template <> struct Real<P64> { typedef double T; };

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef short s2 __attribute__((ext_vector_type(2)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef double d2 __attribute__((ext_vector_type(2)));

// spinor field view: base pointer of one parity field + norm array (FP16)
struct SpinorPtr {
    void* v;
    float* norm;
};

// One site's spinor exactly as stored (no conversion): a kernel can issue the
// loads of several neighbours before it decodes any of them.
template <int P> struct RawSp;
template <> struct RawSp<P64> { d2 v[12]; };
template <> struct RawSp<P32> { f4 v[6]; };
template <> struct RawSp<P16> { h8 v[3]; float n; };

template <int P> __device__ __forceinline__ void fetch_sp(const SpinorPtr& f, int s, int Vh, RawSp<P>& r) {
    if constexpr (P == P64) {
#pragma unroll
        for (int k = 0; k < 12; k++) r.v[k] = ((const d2*)f.v)[(size_t)k * Vh + s];
    } else if constexpr (P == P32) {
#pragma unroll
        for (int k = 0; k < 6; k++) r.v[k] = ((const f4*)f.v)[(size_t)k * Vh + s];
    } else {
#pragma unroll
        for (int k = 0; k < 3; k++) r.v[k] = ((const h8*)f.v)[(size_t)k * Vh + s];
        r.n = f.norm[s];
    }
}

template <int P, typename R> struct SpinorIO;

template <typename R> struct SpinorIO<P64, R> {
    static __device__ __forceinline__ void decode(const RawSp<P64>& r, cx<R> p[4][3]) {
#pragma unroll
        for (int k = 0; k < 12; k++) p[k / 3][k % 3] = {R(r.v[k].x), R(r.v[k].y)};
    }
    static __device__ __forceinline__ void load(const SpinorPtr& f, int s, int Vh, cx<R> p[4][3]) {
        const d2* b = (const d2*)f.v;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            d2 v = b[(size_t)k * Vh + s];
            p[k / 3][k % 3] = {R(v.x), R(v.y)};
        }
    }
    static __device__ __forceinline__ void store(const SpinorPtr& f, int s, int Vh, const cx<R> p[4][3]) {
        d2* b = (d2*)f.v;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            d2 v = {double(p[k / 3][k % 3].re), double(p[k / 3][k % 3].im)};
            b[(size_t)k * Vh + s] = v;
        }
    }
};

template <typename R> struct SpinorIO<P32, R> {
    static __device__ __forceinline__ void decode(const RawSp<P32>& r, cx<R> p[4][3]) {
#pragma unroll
        for (int k = 0; k < 6; k++) {
            p[(2 * k) / 3][(2 * k) % 3] = {R(r.v[k].x), R(r.v[k].y)};
            p[(2 * k + 1) / 3][(2 * k + 1) % 3] = {R(r.v[k].z), R(r.v[k].w)};
        }
    }
    static __device__ __forceinline__ void load(const SpinorPtr& f, int s, int Vh, cx<R> p[4][3]) {
        const f4* b = (const f4*)f.v;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            f4 v = b[(size_t)k * Vh + s];
            p[(2 * k) / 3][(2 * k) % 3] = {R(v.x), R(v.y)};
            p[(2 * k + 1) / 3][(2 * k + 1) % 3] = {R(v.z), R(v.w)};
        }
    }
    static __device__ __forceinline__ void store(const SpinorPtr& f, int s, int Vh, const cx<R> p[4][3]) {
        f4* b = (f4*)f.v;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const cx<R>& a = p[(2 * k) / 3][(2 * k) % 3];
            const cx<R>& c = p[(2 * k + 1) / 3][(2 * k + 1) % 3];
            f4 v = {float(a.re), float(a.im), float(c.re), float(c.im)};
            b[(size_t)k * Vh + s] = v;
        }
    }
};

template <typename R> struct SpinorIO<P16, R> {
    static __device__ __forceinline__ void decode(const RawSp<P16>& r, cx<R> p[4][3]) {
#pragma unroll
        for (int k = 0; k < 3; k++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                int e = 4 * k + j;
                p[e / 3][e % 3] = {R(float(r.v[k][2 * j]) * r.n), R(float(r.v[k][2 * j + 1]) * r.n)};
            }
    }
    static __device__ __forceinline__ void load(const SpinorPtr& f, int s, int Vh, cx<R> p[4][3]) {
        const h8* b = (const h8*)f.v;
        float nrm = f.norm[s];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            h8 v = b[(size_t)k * Vh + s];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                int e = 4 * k + j;
                p[e / 3][e % 3] = {R(float(v[2 * j]) * nrm), R(float(v[2 * j + 1]) * nrm)};
            }
        }
    }
    static __device__ __forceinline__ void store(const SpinorPtr& f, int s, int Vh, const cx<R> p[4][3]) {
        h8* b = (h8*)f.v;
        float m = 0.f;
#pragma unroll
        for (int e = 0; e < 12; e++) {
            m = fmaxf(m, fabsf(float(p[e / 3][e % 3].re)));
            m = fmaxf(m, fabsf(float(p[e / 3][e % 3].im)));
        }
        float inv = m > 0.f ? 1.0f / m : 0.f;
        f.norm[s] = m;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            h8 v;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                int e = 4 * k + j;
                v[2 * j] = (_Float16)(float(p[e / 3][e % 3].re) * inv);
                v[2 * j + 1] = (_Float16)(float(p[e / 3][e % 3].im) * inv);
            }
            b[(size_t)k * Vh + s] = v;
        }
    }
};

// link field loads: base points at the whole gauge field; (mu, p, s) selects a link
template <int P, int RECON, typename R> struct LinkIO;

// one link exactly as stored, and its fetch
template <int P, int RECON> struct RawLink;
template <> struct RawLink<P64, 18> { d2 v[9]; };
template <> struct RawLink<P32, 18> { f2 v[9]; };
template <> struct RawLink<P32, 12> { f4 v[3]; };
template <> struct RawLink<P16, 12> { h4 v[3]; };
// 16-bit / 18: per (mu, p) a block of 36 Vh bytes holding two short8 arrays
// (entries 0-3 and 4-7 of the row-major matrix) and one short2 array (entry
// 8); every real r of the link is kept as the 16-bit fixed-point value
// q = round(32767 r) (an entry of a unitary matrix has |r| <= 1), an absolute
// error of 1.5e-5 against FP16's relative 4.9e-4 near 1: a link error is a
// fixed change of the operator the inner solver inverts, and costs CG
// iterations where rounding of the vectors does not
template <> struct RawLink<P16, 18> { s8 v[2]; s2 w; };
__device__ __forceinline__ const s8* link16x18_block(const void* base, int mu, int p, int Vh) {
    return (const s8*)((const char*)base + (size_t)((mu * 2 + p) * 36) * Vh);
}
// the factor that turns a decoded sloppy link into the link: the 16-bit /18
// format decodes to 32767 times the entries (the hop applies the factor once,
// with the spinor's weight), the other formats to the entries themselves
template <int P, int RECON> __host__ __device__ constexpr float link_unit() {
    return (P == P16 && RECON == 18) ? 1.0f / 32767.0f : 1.0f;
}

// nt: non-temporal loads, for link fields larger than the L2 caches together
// (each link is read once per launch; streaming them keeps the L2 for the
// neighbour spinors, which are read eight times)
// (a compile-time choice: a run-time branch between the two loads is merged
// by the compiler, which then drops the non-temporal hint)
template <int P, int RECON, bool NT>
__device__ __forceinline__ void fetch_link(const void* base, int mu, int p, int s, int Vh, RawLink<P, RECON>& r) {
    constexpr int N = RECON == 18 ? 9 : 3;
    typedef decltype(r.v[0]) T0;
    typedef typename std::remove_reference<T0>::type T;
    if constexpr (P == P16 && RECON == 18) {
        const s8* b = link16x18_block(base, mu, p, Vh);
        const s2* w = (const s2*)(b + 2 * (size_t)Vh);
        if constexpr (NT) {
            r.v[0] = __builtin_nontemporal_load(b + s);
            r.v[1] = __builtin_nontemporal_load(b + Vh + s);
            r.w = __builtin_nontemporal_load(w + s);
        } else {
            r.v[0] = b[s];
            r.v[1] = b[Vh + s];
            r.w = w[s];
        }
        return;
    }
    const T* b = (const T*)base + (size_t)((mu * 2 + p) * N) * Vh + s;
    if constexpr (NT) {
#pragma unroll
        for (int k = 0; k < N; k++) r.v[k] = __builtin_nontemporal_load(b + (size_t)k * Vh);
    } else {
#pragma unroll
        for (int k = 0; k < N; k++) r.v[k] = b[(size_t)k * Vh];
    }
}

template <typename R> struct LinkIO<P64, 18, R> {
    static __device__ __forceinline__ M3<R> decode(const RawLink<P64, 18>& r) {
        M3<R> u;
#pragma unroll
        for (int k = 0; k < 9; k++) u.e[k / 3][k % 3] = {R(r.v[k].x), R(r.v[k].y)};
        return u;
    }
    static __device__ __forceinline__ M3<R> load(const void* base, int mu, int p, int s, int Vh) {
        const d2* b = (const d2*)base + (size_t)((mu * 2 + p) * 9) * Vh + s;
        M3<R> u;
#pragma unroll
        for (int k = 0; k < 9; k++) {
            d2 v = b[(size_t)k * Vh];
            u.e[k / 3][k % 3] = {R(v.x), R(v.y)};
        }
        return u;
    }
};

template <typename R> struct LinkIO<P32, 18, R> {
    static __device__ __forceinline__ M3<R> decode(const RawLink<P32, 18>& r) {
        M3<R> u;
#pragma unroll
        for (int k = 0; k < 9; k++) u.e[k / 3][k % 3] = {R(r.v[k].x), R(r.v[k].y)};
        return u;
    }
    static __device__ __forceinline__ M3<R> load(const void* base, int mu, int p, int s, int Vh) {
        const f2* b = (const f2*)base + (size_t)((mu * 2 + p) * 9) * Vh + s;
        M3<R> u;
#pragma unroll
        for (int k = 0; k < 9; k++) {
            f2 v = b[(size_t)k * Vh];
            u.e[k / 3][k % 3] = {R(v.x), R(v.y)};
        }
        return u;
    }
};

// third row of an SU(3) matrix from the first two: row2 = conj(row0 x row1)
template <typename R> __device__ __forceinline__ void recon_row2(M3<R>& u) {
    u.e[2][0] = conj_cross(u.e[0][1], u.e[1][2], u.e[0][2], u.e[1][1]);
    u.e[2][1] = conj_cross(u.e[0][2], u.e[1][0], u.e[0][0], u.e[1][2]);
    u.e[2][2] = conj_cross(u.e[0][0], u.e[1][1], u.e[0][1], u.e[1][0]);
}

template <typename R> struct LinkIO<P32, 12, R> {
    static __device__ __forceinline__ M3<R> decode(const RawLink<P32, 12>& r) {
        M3<R> u;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            int e0 = 2 * k, e1 = 2 * k + 1;
            u.e[e0 / 3][e0 % 3] = {R(r.v[k].x), R(r.v[k].y)};
            u.e[e1 / 3][e1 % 3] = {R(r.v[k].z), R(r.v[k].w)};
        }
        recon_row2(u);
        return u;
    }
    static __device__ __forceinline__ M3<R> load(const void* base, int mu, int p, int s, int Vh) {
        const f4* b = (const f4*)base + (size_t)((mu * 2 + p) * 3) * Vh + s;
        M3<R> u;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            f4 v = b[(size_t)k * Vh];
            int e0 = 2 * k, e1 = 2 * k + 1;
            u.e[e0 / 3][e0 % 3] = {R(v.x), R(v.y)};
            u.e[e1 / 3][e1 % 3] = {R(v.z), R(v.w)};
        }
        recon_row2(u);
        return u;
    }
};

template <typename R> struct LinkIO<P16, 12, R> {
    static __device__ __forceinline__ M3<R> decode(const RawLink<P16, 12>& r) {
        M3<R> u;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            int e0 = 2 * k, e1 = 2 * k + 1;
            u.e[e0 / 3][e0 % 3] = {R(float(r.v[k].x)), R(float(r.v[k].y))};
            u.e[e1 / 3][e1 % 3] = {R(float(r.v[k].z)), R(float(r.v[k].w))};
        }
        recon_row2(u);
        return u;
    }
    static __device__ __forceinline__ M3<R> load(const void* base, int mu, int p, int s, int Vh) {
        const h4* b = (const h4*)base + (size_t)((mu * 2 + p) * 3) * Vh + s;
        M3<R> u;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            h4 v = b[(size_t)k * Vh];
            int e0 = 2 * k, e1 = 2 * k + 1;
            u.e[e0 / 3][e0 % 3] = {R(float(v.x)), R(float(v.y))};
            u.e[e1 / 3][e1 % 3] = {R(float(v.z)), R(float(v.w))};
        }
        recon_row2(u);
        return u;
    }
};

template <typename R> struct LinkIO<P16, 18, R> {
    // 32767 times the link (see link_unit)
    static __device__ __forceinline__ M3<R> decode(const RawLink<P16, 18>& r) {
        M3<R> u;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            u.e[k / 3][k % 3] = {R(float(r.v[0][2 * k])), R(float(r.v[0][2 * k + 1]))};
            u.e[(k + 4) / 3][(k + 4) % 3] = {R(float(r.v[1][2 * k])), R(float(r.v[1][2 * k + 1]))};
        }
        u.e[2][2] = {R(float(r.w.x)), R(float(r.w.y))};
        return u;
    }
    static __device__ __forceinline__ M3<R> load(const void* base, int mu, int p, int s, int Vh) {
        RawLink<P16, 18> r;
        fetch_link<P16, 18, false>(base, mu, p, s, Vh, r);
        M3<R> u = decode(r);
        m3_scale(u, R(link_unit<P16, 18>()));
        return u;
    }
};

// a real in [-1, 1] as 16-bit fixed point, rounded to nearest (ties to even)
__device__ __forceinline__ short fixed16(double x) {
    return (short)rint(fmin(fmax(x, -1.0), 1.0) * 32767.0);
}

// A link written to a sloppy copy in storage (prec, recon): row-major
// entries e[0..8] in FP64; r = mu * 2 + p selects the (direction, parity) part.
__device__ __forceinline__ void store_sloppy_link(void* out, int prec, int recon, int r, int s, int Vh,
                                                  const cx<double> e[9]) {
    if (prec == P32 && recon == 18) {
        f2* o = (f2*)out + (size_t)(r * 9) * Vh + s;
#pragma unroll
        for (int k = 0; k < 9; k++) o[(size_t)k * Vh] = f2{(float)e[k].re, (float)e[k].im};
    } else if (prec == P32) {
        f4* o = (f4*)out + (size_t)(r * 3) * Vh + s;
#pragma unroll
        for (int k = 0; k < 3; k++)
            o[(size_t)k * Vh] = f4{(float)e[2 * k].re, (float)e[2 * k].im, (float)e[2 * k + 1].re, (float)e[2 * k + 1].im};
    } else if (recon == 18) {
        s8* o = (s8*)((char*)out + (size_t)(r * 36) * Vh);
#pragma unroll
        for (int j = 0; j < 2; j++) {
            s8 v;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                v[2 * k] = fixed16(e[4 * j + k].re);
                v[2 * k + 1] = fixed16(e[4 * j + k].im);
            }
            o[(size_t)j * Vh + s] = v;
        }
        ((s2*)(o + 2 * (size_t)Vh))[s] = s2{fixed16(e[8].re), fixed16(e[8].im)};
    } else {
        h4* o = (h4*)out + (size_t)(r * 3) * Vh + s;
#pragma unroll
        for (int k = 0; k < 3; k++)
            o[(size_t)k * Vh] = h4{(_Float16)e[2 * k].re, (_Float16)e[2 * k].im, (_Float16)e[2 * k + 1].re,
                                   (_Float16)e[2 * k + 1].im};
    }
}

// bytes of one link in a sloppy copy
__host__ __device__ __forceinline__ size_t sloppy_link_bytes(int prec, int recon) {
    return prec == P32 ? (recon == 18 ? 72 : 48) : (recon == 18 ? 36 : 24);
}

// FP64 master gauge field access (double2 chunks)
__device__ __forceinline__ M3<double> gauge_load(const d2* U, int mu, int p, int s, int Vh) {
    return LinkIO<P64, 18, double>::load(U, mu, p, s, Vh);
}

__device__ __forceinline__ void gauge_store(d2* U, int mu, int p, int s, int Vh, const M3<double>& u) {
    d2* b = U + (size_t)((mu * 2 + p) * 9) * Vh + s;
#pragma unroll
    for (int k = 0; k < 9; k++) b[(size_t)k * Vh] = d2{u.e[k / 3][k % 3].re, u.e[k / 3][k % 3].im};
}

__device__ __forceinline__ void mom_load(const double* P, int mu, int p, int s, int Vh, double x[8]) {
    const double* b = P + (size_t)((mu * 2 + p) * 8) * Vh + s;
#pragma unroll
    for (int a = 0; a < 8; a++) x[a] = b[(size_t)a * Vh];
}

__device__ __forceinline__ void mom_store(double* P, int mu, int p, int s, int Vh, const double x[8]) {
    double* b = P + (size_t)((mu * 2 + p) * 8) * Vh + s;
#pragma unroll
    for (int a = 0; a < 8; a++) b[(size_t)a * Vh] = x[a];
}

// --------------------------------------------------------------------------
// deterministic block reductions (fixed shuffle tree, fixed wave order)
// --------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// sum over the block of NV values per thread; result valid in every thread.
// lds must hold NV * (blockDim.x / 64) doubles.
template <int NV>
__device__ __forceinline__ void block_sum(double v[NV], double* lds) {
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; k++) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; k++) lds[k * nw + wid] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; k++) {
        double s = 0;
        for (int w = 0; w < nw; w++) s += lds[k * nw + w];
        v[k] = s;
    }
}

// sum of n partial values (written by an earlier kernel), computed the same
// way in every block that asks: thread t takes t, t + bs, ... then block_sum.
__device__ __forceinline__ double sum_partials(const double* part, int n, double* lds) {
    double v[1] = {0.0};
    for (int k = threadIdx.x; k < n; k += blockDim.x) v[0] += part[k];
    block_sum<1>(v, lds);
    return v[0];
}

}  // namespace fgi
