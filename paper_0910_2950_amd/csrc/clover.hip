// Clover (Sheikholeslami-Wohlert) term of the Wilson operator, FP64.
//
// The paper's conclusions state that its integrators apply to the usual
// improved actions; the clover term is the standard O(a) improvement of the
// fermion matrix.  In the hopping normalisation of M = 1 - kappa D:
//     M = A - kappa D,  A(x) = 1 + i kappa csw sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}(x),
//     sigma_{mu nu} = (i/2)[g_mu, g_nu],  Fhat = (Q - Q^+) / 8,
// Q_{mu nu}(x) the sum of the four plaquette leaves at x.  In the chiral
// (DeGrand-Rossi) basis A(x) is two Hermitian 6x6 blocks, one per pair of
// spin components {0,1} and {2,3}.  Even-odd: det M = det A_oo det Mhat with
//     Mhat = A_ee - kappa^2 D_eo A_oo^-1 D_oe,   Mhat^+ = g5 Mhat g5,
// so the two-flavour action is phi^+ (Mhat^+ Mhat)^-1 phi - 2 sum_{x odd} log det A(x).
//
// Storage: blk[(b * 36 + r * 6 + c) * V + p * Vh + s], block b, row r, column
// c (index spin' * 3 + colour within the block), site s of parity p; even
// sites hold A, odd sites A^-1 (or A, for the read-out entry point).
#include <algorithm>
#include <cmath>
#include <complex>

#include "fgi_coord.h"
#include "fgi_internal.h"

namespace fgi {
namespace {

constexpr int CBS = 256;

// sigma_{mu nu} restricted to its two diagonal 2x2 spin blocks, planes in
// the order (0,1), (0,2), (0,3), (1,2), (1,3), (2,3)
struct SigmaBlk {
    double re[6][2][2][2];
    double im[6][2][2][2];
};

SigmaBlk make_sigma() {
    // DeGrand-Rossi g_1..g_4 (x, y, z, t), the basis of the hopping term
    typedef std::complex<double> C;
    const C i(0.0, 1.0);
    C G[4][4][4] = {};
    G[0][0][3] = i;   G[0][1][2] = i;   G[0][2][1] = -i;  G[0][3][0] = -i;
    G[1][0][3] = -1;  G[1][1][2] = 1;   G[1][2][1] = 1;   G[1][3][0] = -1;
    G[2][0][2] = i;   G[2][1][3] = -i;  G[2][2][0] = -i;  G[2][3][1] = i;
    G[3][0][2] = 1;   G[3][1][3] = 1;   G[3][2][0] = 1;   G[3][3][1] = 1;
    SigmaBlk sb{};
    int q = 0;
    for (int mu = 0; mu < 4; mu++)
        for (int nu = mu + 1; nu < 4; nu++, q++) {
            C s[4][4];
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) {
                    C v = 0;
                    for (int k = 0; k < 4; k++) v += G[mu][a][k] * G[nu][k][b] - G[nu][a][k] * G[mu][k][b];
                    s[a][b] = 0.5 * i * v;
                }
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) {
                    if ((a < 2) != (b < 2)) {
                        if (std::abs(s[a][b]) != 0.0) throw Error(-1, "sigma is not block diagonal");
                        continue;
                    }
                    const int bl = a / 2;
                    sb.re[q][bl][a % 2][b % 2] = s[a][b].real();
                    sb.im[q][bl][a % 2][b % 2] = s[a][b].imag();
                }
        }
    return sb;
}

// the blocks in device memory, read with run-time plane indices:
// sig[k] = Re, sig[48 + k] = Im of block entry k = ((q * 2 + b) * 2 + s) * 2 + t
const double* sigma_blocks(Ctx& c) {
    static const SigmaBlk sb = make_sigma();
    const bool fresh = c.cl_sig.bytes == 0;
    double* d = (double*)c.cl_sig.get(sizeof(SigmaBlk));
    if (fresh) FGI_HIP(hipMemcpyAsync(d, &sb, sizeof(SigmaBlk), hipMemcpyHostToDevice, c.stream));
    return d;
}

__device__ __forceinline__ cx<double> sig_at(const double* __restrict__ sig, int q, int b, int s, int t) {
    const int k = ((q * 2 + b) * 2 + s) * 2 + t;
    return {sig[k], sig[48 + k]};
}

__device__ __forceinline__ int plane_index(int mu, int nu) {
    // (0,1)=0 (0,2)=1 (0,3)=2 (1,2)=3 (1,3)=4 (2,3)=5 for mu < nu
    return mu == 0 ? nu - 1 : (mu == 1 ? nu + 1 : 5);
}

__device__ __forceinline__ int site_of(const Geom& g, const Coord& y) { return coord_parity(y) * g.Vh + cb_index(g, y); }

// Fhat_{mu nu}(x) for the six planes, one thread per site (both parities)
__global__ void __launch_bounds__(CBS) k_clover_fhat(Geom g, const d2* __restrict__ U, d2* __restrict__ fh) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.V) return;
    const int p = t / g.Vh, s = t % g.Vh;
    const Coord x = cb_coords(g, p, s);
#pragma unroll 1
    for (int mu = 0; mu < 4; mu++)
#pragma unroll 1
        for (int nu = mu + 1; nu < 4; nu++) {
            Coord xm = x, xn = x, xbm = x, xbn = x;
            coord_step(g, xm, mu, 1);
            coord_step(g, xn, nu, 1);
            coord_step(g, xbm, mu, 0);
            coord_step(g, xbn, nu, 0);
            Coord xbmn = xbm, xbmbn = xbm, xmbn = xm;
            coord_step(g, xbmn, nu, 1);
            coord_step(g, xbmbn, nu, 0);
            coord_step(g, xmbn, nu, 0);
            const M3<double> umx = link_at(g, U, mu, x), unx = link_at(g, U, nu, x);
            // leaf from x: +mu +nu -mu -nu
            M3<double> Q = m3_mul_nd(m3_mul_nd(m3_mul(umx, link_at(g, U, nu, xm)), link_at(g, U, mu, xn)), unx);
            // +nu -mu -nu +mu
            m3_acc(Q, m3_mul(m3_mul_nd(m3_mul_nd(unx, link_at(g, U, mu, xbmn)), link_at(g, U, nu, xbm)),
                             link_at(g, U, mu, xbm)));
            // -mu -nu +mu +nu
            m3_acc(Q, m3_mul_dn(link_at(g, U, mu, xbm),
                                m3_mul(m3_mul_dn(link_at(g, U, nu, xbmbn), link_at(g, U, mu, xbmbn)),
                                       link_at(g, U, nu, xbn))));
            // -nu +mu +nu -mu
            m3_acc(Q, m3_mul_nd(m3_mul(m3_mul_dn(link_at(g, U, nu, xbn), link_at(g, U, mu, xbn)),
                                       link_at(g, U, nu, xmbn)),
                                umx));
            const int q = plane_index(mu, nu);
#pragma unroll
            for (int a = 0; a < 3; a++)
#pragma unroll
                for (int b = 0; b < 3; b++)
                    fh[(size_t)(q * 9 + a * 3 + b) * g.V + t] =
                        d2{0.125 * (Q.e[a][b].re - Q.e[b][a].re), 0.125 * (Q.e[a][b].im + Q.e[b][a].im)};
        }
}

// One 6x6 block of A(x) per thread: b = thread / V, site = thread % V.
// A = 1 + i kc sum_q sigma_q^b (x) Fhat_q.  Inverse and log |det| by
// Gauss-Jordan elimination with partial pivoting: A is Hermitian, positive
// definite for kappa csw < 1/6 on any field but possibly indefinite above,
// so the pivot row of column k is the row >= k of largest modulus; the
// interchanges are undone on the columns of the inverse in reverse order.
// The Nf = 2 weight is det(A)^2, so log |det| = sum log |pivot| enters the
// action.  A zero pivot (a singular block) leaves NaN in the block's log det
// and inverse, which the solver and the energy sum report as non-finite.
// Writes A, or A^-1 at odd sites when invert_odd; ld[b V + site] = log |det|
// of the block at odd sites, 0 at even ones.
__global__ void __launch_bounds__(CBS) k_clover_blocks(Geom g, const double* __restrict__ sig, double kc, const d2* __restrict__ fh,
                                                       d2* __restrict__ blk, double* __restrict__ ld, int invert_odd) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= 2 * g.V) return;
    const int b = id / g.V, t = id % g.V;
    const bool odd = t >= g.Vh;
    cx<double> a[6][6];
#pragma unroll
    for (int r = 0; r < 6; r++)
#pragma unroll
        for (int c = 0; c < 6; c++) a[r][c] = {r == c ? 1.0 : 0.0, 0.0};
#pragma unroll 1
    for (int q = 0; q < 6; q++) {
        cx<double> f[3][3];
#pragma unroll
        for (int e = 0; e < 9; e++) {
            const d2 v = fh[(size_t)(q * 9 + e) * g.V + t];
            f[e / 3][e % 3] = {v.x, v.y};
        }
#pragma unroll
        for (int s = 0; s < 2; s++)
#pragma unroll
            for (int u = 0; u < 2; u++) {
                // i kc sigma_su
                const cx<double> sg = sig_at(sig, q, b, s, u);
                const cx<double> w = {-kc * sg.im, kc * sg.re};
#pragma unroll
                for (int i = 0; i < 3; i++)
#pragma unroll
                    for (int j = 0; j < 3; j++) a[s * 3 + i][u * 3 + j] = a[s * 3 + i][u * 3 + j] + w * f[i][j];
            }
    }
    double logdet = 0.0;
    if (odd) {
        cx<double> m[6][6];
#pragma unroll
        for (int r = 0; r < 6; r++)
#pragma unroll
            for (int c = 0; c < 6; c++) m[r][c] = a[r][c];
        // in-place Gauss-Jordan inversion with partial pivoting; row
        // interchanges are predicated selects over the unrolled rows, so the
        // block stays in registers
        int perm[6];
#pragma unroll
        for (int k = 0; k < 6; k++) {
            int p = k;
            double best = m[k][k].re * m[k][k].re + m[k][k].im * m[k][k].im;
#pragma unroll
            for (int i = k + 1; i < 6; i++) {
                const double v = m[i][k].re * m[i][k].re + m[i][k].im * m[i][k].im;
                if (v > best) {
                    best = v;
                    p = i;
                }
            }
            perm[k] = p;
#pragma unroll
            for (int i = k + 1; i < 6; i++) {
                const bool sw = i == p;
#pragma unroll
                for (int j = 0; j < 6; j++) {
                    const cx<double> rk = m[k][j], ri = m[i][j];
                    m[k][j] = sw ? ri : rk;
                    m[i][j] = sw ? rk : ri;
                }
            }
            const cx<double> piv = m[k][k];
            const double den = piv.re * piv.re + piv.im * piv.im;
            logdet += den > 0.0 ? 0.5 * log(den) : __builtin_nan("");
            const cx<double> inv = {piv.re / den, -piv.im / den};
            m[k][k] = {1.0, 0.0};
#pragma unroll
            for (int j = 0; j < 6; j++) m[k][j] = m[k][j] * inv;
#pragma unroll
            for (int i = 0; i < 6; i++) {
                if (i == k) continue;
                const cx<double> fct = m[i][k];
                m[i][k] = {0.0, 0.0};
#pragma unroll
                for (int j = 0; j < 6; j++) m[i][j] = m[i][j] - fct * m[k][j];
            }
        }
        // undo the interchanges on the columns, last first
#pragma unroll
        for (int k = 5; k >= 0; k--)
#pragma unroll
            for (int j = k + 1; j < 6; j++) {
                const bool sw = perm[k] == j;
#pragma unroll
                for (int i = 0; i < 6; i++) {
                    const cx<double> ck = m[i][k], cj = m[i][j];
                    m[i][k] = sw ? cj : ck;
                    m[i][j] = sw ? ck : cj;
                }
            }
        if (invert_odd) {
#pragma unroll
            for (int r = 0; r < 6; r++)
#pragma unroll
                for (int c = 0; c < 6; c++) a[r][c] = m[r][c];
        }
    }
#pragma unroll
    for (int r = 0; r < 6; r++)
#pragma unroll
        for (int c = 0; c < 6; c++) blk[(size_t)(b * 36 + r * 6 + c) * g.V + t] = d2{a[r][c].re, a[r][c].im};
    ld[(size_t)b * g.V + t] = logdet;
}

// out = g5^go (A (g5^gi in) - k2 u) at the Vh sites of one parity (u may be
// null); in-place (out == in) is allowed
__global__ void __launch_bounds__(CBS) k_clover_apply(int Vh, int V, int poff, const d2* __restrict__ blk,
                                                      const d2* in, const d2* __restrict__ u, double k2, int gi,
                                                      int go, d2* out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= Vh) return;
    const size_t site = (size_t)poff + s;
    cx<double> v[12];
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const d2 w = in[(size_t)k * Vh + s];
        v[k] = (gi && k >= 6) ? cx<double>{-w.x, -w.y} : cx<double>{w.x, w.y};
    }
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
        for (int r = 0; r < 6; r++) {
            cx<double> acc = {0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 6; c++) {
                const d2 e = blk[(size_t)(b * 36 + r * 6 + c) * V + site];
                acc = acc + cx<double>{e.x, e.y} * v[b * 6 + c];
            }
            const int k = b * 6 + r;
            if (u) {
                const d2 w = u[(size_t)k * Vh + s];
                acc = acc - k2 * cx<double>{w.x, w.y};
            }
            if (go && k >= 6) acc = -acc;
            out[(size_t)k * Vh + s] = d2{acc.re, acc.im};
        }
}

// Colour matrices Kt_q(x) = (K - K^+) / 8, K = i (cw Z + cd Z') per site and
// plane, with
//   Z_{ba}  = sum_{s,t} sigma_{st} X_{t b} conj(Y_{s a})        (pseudofermion part, weight cw by parity)
//   Z'_{ba} = sum_{s,t} sigma_{st} A^-1[(t,b),(s,a)]            (log det part, odd sites)
// so that the derivative of the clover terms along e_a is
// sum_x sum_q Re Tr[e_a Q_q(x) Kt_q(x)].
__global__ void __launch_bounds__(CBS) k_clover_kt(Geom g, const double* __restrict__ sig, double cw_even, double cw_odd, double cd,
                                                   const d2* __restrict__ Xe, const d2* __restrict__ Xo,
                                                   const d2* __restrict__ Ye, const d2* __restrict__ Yo,
                                                   const d2* __restrict__ blk, d2* __restrict__ kt) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.V) return;
    const int p = t / g.Vh, s = t % g.Vh;
    const double cw = p ? cw_odd : cw_even;
    const d2* X = p ? Xo : Xe;
    const d2* Y = p ? Yo : Ye;
    const bool pf = X && cw != 0.0;
    const bool det = p == 1 && cd != 0.0;
#pragma unroll 1
    for (int q = 0; q < 6; q++) {
        cx<double> Z[3][3];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) Z[i][j] = {0.0, 0.0};
#pragma unroll 1
        for (int bst = 0; bst < 8; bst++) {
            const int b = bst >> 2, ss = (bst >> 1) & 1, tt = bst & 1;
            const cx<double> sg = sig_at(sig, q, b, ss, tt);
            if (sg.re == 0.0 && sg.im == 0.0) continue;
#pragma unroll
            for (int bb = 0; bb < 3; bb++) {
                cx<double> xv = {0.0, 0.0};
                if (pf) {
                    const d2 a = X[(size_t)((2 * b + tt) * 3 + bb) * g.Vh + s];
                    xv = {cw * a.x, cw * a.y};
                }
#pragma unroll
                for (int aa = 0; aa < 3; aa++) {
                    cx<double> v = {0.0, 0.0};
                    if (pf) {
                        const d2 c = Y[(size_t)((2 * b + ss) * 3 + aa) * g.Vh + s];
                        v = xv * cx<double>{c.x, -c.y};
                    }
                    if (det) {
                        const d2 e = blk[(size_t)(b * 36 + (tt * 3 + bb) * 6 + ss * 3 + aa) * g.V + t];
                        v = v + cd * cx<double>{e.x, e.y};
                    }
                    Z[bb][aa] = Z[bb][aa] + sg * v;
                }
            }
        }
        // K = i Z, Kt = (K - K^+)/8 = i (Z + Z^+)/8
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const cx<double> h = Z[i][j] + conj(Z[j][i]);
                kt[(size_t)(q * 9 + i * 3 + j) * g.V + t] = d2{-0.125 * h.im, 0.125 * h.re};
            }
    }
}

__device__ __forceinline__ M3<double> kt_at(const Geom& g, const d2* __restrict__ kt, int q, double sgn,
                                            const Coord& y) {
    const int t = site_of(g, y);
    M3<double> m;
#pragma unroll
    for (int e = 0; e < 9; e++) {
        const d2 v = kt[(size_t)(q * 9 + e) * g.V + t];
        m.e[e / 3][e % 3] = {sgn * v.x, sgn * v.y};
    }
    return m;
}

// Force of sum_x sum_{mu<nu} Re Tr[Q_{mu nu}(x) Kt_{mu nu}(x)], gathered per
// link U_mu(x): for every nu != mu (with Kt_{nu mu} = -Kt_{mu nu}) the two
// plaquettes through the link, each entered as a leaf at its four corners.
// With B = U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ (the +nu staple) and
// C = U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) (the -nu path to x+mu),
//   S_up = B K(x) + K(x+mu) B + U_nu(x+mu) [K(x+mu+nu) U_mu(x+nu)^+ + U_mu(x+nu)^+ K(x+nu)] U_nu(x)^+,
//   S_dn = K(x) C + C K(x+mu) + U_nu(x-nu)^+ [K(x-nu) U_mu(x-nu) + U_mu(x-nu) K(x-nu+mu)] U_nu(x-nu+mu),
// e_a of the sum is Re Tr[T^a U (S_up + S_dn^+)], so F_a += coef [TA(U (S_up + S_dn^+))]_a / 2.
__global__ void __launch_bounds__(CBS) k_clover_force(Geom g, const d2* __restrict__ U, const d2* __restrict__ kt,
                                                      double coef, double* __restrict__ F) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * g.V) return;
    const int s = t % g.Vh, r = t / g.Vh, p = r & 1, mu = r >> 1;
    const Coord x = cb_coords(g, p, s);
    Coord xm = x;
    coord_step(g, xm, mu, 1);
    M3<double> S = m3_zero<double>();
#pragma unroll 1
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        const int q = mu < nu ? plane_index(mu, nu) : plane_index(nu, mu);
        const double sg = mu < nu ? 1.0 : -1.0;
        Coord xn = x, xbn = x, xmn = xm, xmbn = xm;
        coord_step(g, xn, nu, 1);
        coord_step(g, xbn, nu, 0);
        coord_step(g, xmn, nu, 1);
        coord_step(g, xmbn, nu, 0);
        const M3<double> Kx = kt_at(g, kt, q, sg, x), Kxm = kt_at(g, kt, q, sg, xm);
        {
            const M3<double> unxm = link_at(g, U, nu, xm), umxn = link_at(g, U, mu, xn), unx = link_at(g, U, nu, x);
            const M3<double> B = m3_mul_nd(m3_mul_nd(unxm, umxn), unx);
            m3_acc(S, m3_mul(B, Kx));
            m3_acc(S, m3_mul(Kxm, B));
            M3<double> in = m3_mul_nd(kt_at(g, kt, q, sg, xmn), umxn);
            m3_acc(in, m3_mul_dn(umxn, kt_at(g, kt, q, sg, xn)));
            m3_acc(S, m3_mul_nd(m3_mul(unxm, in), unx));
        }
        {
            const M3<double> unxbn = link_at(g, U, nu, xbn), umxbn = link_at(g, U, mu, xbn);
            const M3<double> unxmbn = link_at(g, U, nu, xmbn);
            const M3<double> C = m3_mul(m3_mul_dn(unxbn, umxbn), unxmbn);
            M3<double> D = m3_mul(Kx, C);
            m3_acc(D, m3_mul(C, Kxm));
            M3<double> in = m3_mul(kt_at(g, kt, q, sg, xbn), umxbn);
            m3_acc(in, m3_mul(umxbn, kt_at(g, kt, q, sg, xmbn)));
            m3_acc(D, m3_mul(m3_mul_dn(unxbn, in), unxmbn));
            m3_acc(S, m3_dag(D));
        }
    }
    const M3<double> W = m3_mul(gauge_load(U, mu, p, s, g.Vh), S);
    double xa[8];
    ta_components(W, xa);
    double* o = F + (size_t)(r * 8) * g.Vh + s;
#pragma unroll
    for (int a = 0; a < 8; a++) o[(size_t)a * g.Vh] += 0.5 * coef * xa[a];
}

// A(x) in the public layout: [V lexicographic][12][12] complex, zero between
// the chirality blocks
__global__ void __launch_bounds__(CBS) k_clover_unpack(Geom g, const d2* __restrict__ blk, d2* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.V) return;
    const int p = t / g.Vh, s = t % g.Vh;
    const Coord x = cb_coords(g, p, s);
    const size_t lex = (size_t)x.c[0] + (size_t)g.L[0] * (x.c[1] + (size_t)g.L[1] * (x.c[2] + (size_t)g.L[2] * x.c[3]));
    d2* o = out + lex * 144;
    for (int r = 0; r < 12; r++)
        for (int c = 0; c < 12; c++) {
            const int b = r / 6;
            o[r * 12 + c] = (c / 6 == b) ? blk[(size_t)(b * 36 + (r % 6) * 6 + c % 6) * g.V + t] : d2{0.0, 0.0};
        }
}

// partial[k] = sum of the block's odd-site log dets (both chirality blocks)
__global__ void __launch_bounds__(CBS) k_logdet_partials(Geom g, const double* __restrict__ ld,
                                                         double* __restrict__ partial) {
    __shared__ double sh[CBS];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (s < g.Vh) v = ld[(size_t)g.Vh + s] + ld[(size_t)g.V + g.Vh + s];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = CBS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

int nb_of(long n) { return (int)((n + CBS - 1) / CBS); }

size_t spinor_bytes(const Geom& g) { return sizeof(d2) * 12 * (size_t)g.Vh; }

double host_scalar(Ctx& c, const double* dev, int slot) {
    FGI_HIP(hipMemcpyAsync(c.host_scal + slot, dev, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    FGI_HIP(hipStreamSynchronize(c.stream));
    return c.host_scal[slot];
}

// Re <a, b> over the 12 Vh complex components of two even spinors
double dot_re(Ctx& c, const Geom& g, const d2* a, const d2* b, int slot) {
    double* part = partial_buf(c, g);
    double* scal = (double*)c.scal.get(sizeof(double) * 64);
    const int nb = dot_partials(c, 24L * g.Vh, (const double*)a, (const double*)b, part);
    final_sum(c, part, nb, scal + slot);
    return host_scalar(c, scal + slot, slot);
}

// ---- CG scalars on the device: st[0] = |r|^2, st[1] = alpha, st[2] = beta.
// Reductions sum per-block partials in a fixed order in one block.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int n) {
    __shared__ double sh[CBS];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += CBS) v += part[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = CBS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    return sh[0];
}

// mode 0: st[0] = sum (|r|^2 of a restart); 1: alpha = st[0] / sum (<p, A p>);
// 2: beta = sum / st[0], st[0] = sum (|r|^2 of the new residual)
__global__ void __launch_bounds__(CBS) k_cl_scalar(const double* __restrict__ part, int n, int mode,
                                                   double* __restrict__ st) {
    const double v = sum_partials(part, n);
    if (threadIdx.x != 0) return;
    if (mode == 0) {
        st[0] = v;
    } else if (mode == 1) {
        st[1] = st[0] / v;
    } else {
        st[2] = v / st[0];
        st[0] = v;
    }
}

// x += alpha p, r -= alpha A p; partial[b] = sum over the block of |r|^2
__global__ void __launch_bounds__(CBS) k_cl_xr(int Vh, const double* __restrict__ st, const d2* __restrict__ p,
                                               const d2* __restrict__ ap, d2* __restrict__ x, d2* __restrict__ r,
                                               double* __restrict__ part) {
    __shared__ double sh[CBS];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (s < Vh) {
        const double a = st[1];
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const size_t i = (size_t)k * Vh + s;
            const d2 pv = p[i], qv = ap[i];
            d2 xv = x[i], rv = r[i];
            xv.x += a * pv.x;
            xv.y += a * pv.y;
            rv.x -= a * qv.x;
            rv.y -= a * qv.y;
            x[i] = xv;
            r[i] = rv;
            acc += rv.x * rv.x + rv.y * rv.y;
        }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = CBS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// p = r + beta p
__global__ void __launch_bounds__(CBS) k_cl_p(int Vh, const double* __restrict__ st, const d2* __restrict__ r,
                                              d2* __restrict__ p) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= Vh) return;
    const double b = st[2];
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const size_t i = (size_t)k * Vh + s;
        const d2 rv = r[i], pv = p[i];
        p[i] = d2{rv.x + b * pv.x, rv.y + b * pv.y};
    }
}

// ---- FP32 inner solver of the mixed-precision clover CG.  FP32 spinors are
// [6][Vh] float4 (component k in the x,y or z,w half of float4 k / 2), the
// blocks [72][V] float2 in the FP64 blocks' order.
__global__ void __launch_bounds__(CBS) k_blk_to_f32(size_t n, const d2* __restrict__ a, f2* __restrict__ b) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = f2{(float)a[t].x, (float)a[t].y};
}

__device__ __forceinline__ cx<float> ld32(const float* __restrict__ v, int Vh, int s, int k) {
    const size_t o = 4 * ((size_t)(k >> 1) * Vh + s) + 2 * (k & 1);
    return {v[o], v[o + 1]};
}
__device__ __forceinline__ void st32(float* __restrict__ v, int Vh, int s, int k, cx<float> z) {
    const size_t o = 4 * ((size_t)(k >> 1) * Vh + s) + 2 * (k & 1);
    v[o] = z.re;
    v[o + 1] = z.im;
}

// out = g5^go (A (g5^gi in) - k2 u), FP32 storage and arithmetic
__global__ void __launch_bounds__(CBS) k_clover_apply32(int Vh, int V, int poff, const f2* __restrict__ blk,
                                                        const float* in, const float* __restrict__ u, float k2,
                                                        int gi, int go, float* out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= Vh) return;
    const size_t site = (size_t)poff + s;
    cx<float> v[12];
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const cx<float> w = ld32(in, Vh, s, k);
        v[k] = (gi && k >= 6) ? cx<float>{-w.re, -w.im} : w;
    }
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
        for (int r = 0; r < 6; r++) {
            cx<float> acc = {0.0f, 0.0f};
#pragma unroll
            for (int c = 0; c < 6; c++) {
                const f2 e = blk[(size_t)(b * 36 + r * 6 + c) * V + site];
                acc = acc + cx<float>{e.x, e.y} * v[b * 6 + c];
            }
            const int k = b * 6 + r;
            if (u) acc = acc - k2 * ld32(u, Vh, s, k);
            if (go && k >= 6) acc = -acc;
            st32(out, Vh, s, k, acc);
        }
}

// partial[b] = sum over the block of Re <a, b> (FP32 vectors, FP64 sums)
__global__ void __launch_bounds__(CBS) k_dot32(int Vh, const float* __restrict__ a, const float* __restrict__ b,
                                               double* __restrict__ part) {
    __shared__ double sh[CBS];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (s < Vh)
#pragma unroll
        for (int k = 0; k < 24; k++) {
            const size_t o = (size_t)(k >> 2) * Vh * 4 + 4 * (size_t)s + (k & 3);
            acc += (double)a[o] * (double)b[o];
        }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = CBS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// x += alpha p, r -= alpha A p (FP32); partial[b] = block sum of |r|^2
__global__ void __launch_bounds__(CBS) k_cl_xr32(int Vh, const double* __restrict__ st, const float* __restrict__ p,
                                                 const float* __restrict__ ap, float* __restrict__ x,
                                                 float* __restrict__ r, double* __restrict__ part) {
    __shared__ double sh[CBS];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (s < Vh) {
        const float a = (float)st[1];
#pragma unroll
        for (int k = 0; k < 24; k++) {
            const size_t o = (size_t)(k >> 2) * Vh * 4 + 4 * (size_t)s + (k & 3);
            x[o] += a * p[o];
            const float rv = r[o] - a * ap[o];
            r[o] = rv;
            acc += (double)rv * (double)rv;
        }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = CBS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// p = r + beta p (FP32)
__global__ void __launch_bounds__(CBS) k_cl_p32(int Vh, const double* __restrict__ st, const float* __restrict__ r,
                                                float* __restrict__ p) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= Vh) return;
    const float b = (float)st[2];
#pragma unroll
    for (int k = 0; k < 24; k++) {
        const size_t o = (size_t)(k >> 2) * Vh * 4 + 4 * (size_t)s + (k & 3);
        p[o] = r[o] + b * p[o];
    }
}

}  // namespace

void clover_build(Ctx& c, const Geom& g, double kappa, double csw, const d2* U, d2* blk, int invert_odd,
                  double* det_action) {
    d2* fh = (d2*)c.cl_fh.get(sizeof(d2) * 54 * (size_t)g.V);
    double* ld = (double*)c.cl_ld.get(sizeof(double) * 2 * (size_t)g.V);
    hipLaunchKernelGGL(k_clover_fhat, dim3(nb_of(g.V)), dim3(CBS), 0, c.stream, g, U, fh);
    FGI_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_clover_blocks, dim3(nb_of(2L * g.V)), dim3(CBS), 0, c.stream, g, sigma_blocks(c),
                       kappa * csw, (const d2*)fh, blk, ld, invert_odd);
    FGI_LAUNCH_CHECK();
    if (det_action) {
        double* part = partial_buf(c, g);
        double* scal = (double*)c.scal.get(sizeof(double) * 64);
        const int nb = nb_of(g.Vh);
        hipLaunchKernelGGL(k_logdet_partials, dim3(nb), dim3(CBS), 0, c.stream, g, (const double*)ld, part);
        FGI_LAUNCH_CHECK();
        final_sum(c, part, nb, scal + 48);
        *det_action = -2.0 * host_scalar(c, scal + 48, 48);
    }
}

void clover_unpack(Ctx& c, const Geom& g, const d2* blk, void* out) {
    hipLaunchKernelGGL(k_clover_unpack, dim3(nb_of(g.V)), dim3(CBS), 0, c.stream, g, blk, (d2*)out);
    FGI_LAUNCH_CHECK();
}

void clover_apply(Ctx& c, const Geom& g, const d2* blk, int parity, const d2* in, const d2* u, double k2, int g5in,
                  int g5out, d2* out) {
    hipLaunchKernelGGL(k_clover_apply, dim3(nb_of(g.Vh)), dim3(CBS), 0, c.stream, g.Vh, g.V, parity * g.Vh, blk, in,
                       u, k2, g5in, g5out, out);
    FGI_LAUNCH_CHECK();
}

// out_e = Mhat in_e = A_ee in_e - kappa^2 D_eo A_oo^-1 D_oe in_e, or with
// dagger g5 Mhat g5 in_e (the g5 on the input folded into the first hop and
// into the A_ee product, the one on the output into that product's store)
void clover_mhat(Ctx& c, const FermionOp& op, const d2* blk, const d2* in_e, d2* out_e, int dagger) {
    const Geom& g = *op.g;
    d2* to = (d2*)c.cl_to.get(spinor_bytes(g));
    if (dagger) hop_oe_g5(c, op, in_e, to);
    else dslash(c, op, 1, P64, SpinorPtr{(void*)in_e, nullptr}, P64, SpinorPtr{to, nullptr});
    clover_apply(c, g, blk, 1, to, nullptr, 0.0, 0, 0, to);
    d2* ue = (d2*)c.cl_ue.get(spinor_bytes(g));
    dslash(c, op, 0, P64, SpinorPtr{to, nullptr}, P64, SpinorPtr{ue, nullptr});
    clover_apply(c, g, blk, 0, in_e, ue, op.kappa * op.kappa, dagger, dagger, out_e);
}

// CG on Mhat^+ Mhat with the clover Mhat, FP64.  The recurrence scalars stay
// on the device (k_cl_scalar); the host reads |r|^2 once per batch of
// CL_BATCH iterations.  Stopping rule as in the fused solver: once the
// recursive residual has passed tol |phi|, the true residual is formed and
// decides; if it has not passed, CG restarts from it.  A batch may run a few
// iterations past the point where the recursive residual first passed.
constexpr int CL_BATCH = 8;

CGResult clover_cg(Ctx& c, const FermionOp& op, const d2* blk, const d2* phi, d2* x, double tol, int maxiter,
                   bool guess) {
    const Geom& g = *op.g;
    const size_t nb = spinor_bytes(g);
    d2* r = (d2*)c.cl_r.get(nb);
    d2* p = (d2*)c.cl_p.get(nb);
    d2* ap = (d2*)c.cl_ap.get(nb);
    d2* t = (d2*)c.cl_t.get(nb);
    double* part = partial_buf(c, g);
    const long ndot = 24L * g.Vh;
    double* part2 = part + (ndot + 255) / 256 + 64;   // after the dot partials
    double* scal = (double*)c.scal.get(sizeof(double) * 64);
    double* st = scal + 56;                           // rr, alpha, beta
    const int nbv = nb_of(g.Vh);
    auto normal = [&](const d2* in, d2* out) {
        clover_mhat(c, op, blk, in, t, 0);
        clover_mhat(c, op, blk, t, out, 1);
    };
    auto true_residual = [&]() {
        normal(x, ap);
        spinor_lincomb(c, g, 1.0, phi, -1.0, ap, 0, r);
    };
    auto set_rr = [&]() {   // st[0] = |r|^2, returned to the host
        const int n = dot_partials(c, ndot, (const double*)r, (const double*)r, part);
        hipLaunchKernelGGL(k_cl_scalar, dim3(1), dim3(CBS), 0, c.stream, (const double*)part, n, 0, st);
        FGI_LAUNCH_CHECK();
        return host_scalar(c, st, 56);
    };
    CGResult res{};
    const double bb = dot_re(c, g, phi, phi, 49);
    const double target = tol * tol * bb;
    if (guess) {
        true_residual();
    } else {
        spinor_lincomb(c, g, 0.0, phi, 0.0, phi, 0, x);
        FGI_HIP(hipMemcpyAsync(r, phi, nb, hipMemcpyDeviceToDevice, c.stream));
    }
    FGI_HIP(hipMemcpyAsync(p, r, nb, hipMemcpyDeviceToDevice, c.stream));
    double rr = set_rr();
    int it = 0;
    bool conv = bb == 0.0 || rr <= target;
    while (!conv && it < maxiter) {
        const int nbatch = std::min(CL_BATCH, maxiter - it);
        for (int k = 0; k < nbatch; k++) {
            normal(p, ap);
            const int n1 = dot_partials(c, ndot, (const double*)p, (const double*)ap, part);
            hipLaunchKernelGGL(k_cl_scalar, dim3(1), dim3(CBS), 0, c.stream, (const double*)part, n1, 1, st);
            hipLaunchKernelGGL(k_cl_xr, dim3(nbv), dim3(CBS), 0, c.stream, g.Vh, (const double*)st, (const d2*)p,
                               (const d2*)ap, x, r, part2);
            hipLaunchKernelGGL(k_cl_scalar, dim3(1), dim3(CBS), 0, c.stream, (const double*)part2, nbv, 2, st);
            hipLaunchKernelGGL(k_cl_p, dim3(nbv), dim3(CBS), 0, c.stream, g.Vh, (const double*)st, (const d2*)r, p);
            FGI_LAUNCH_CHECK();
        }
        it += nbatch;
        rr = host_scalar(c, st, 56);
        if (!(rr > target)) {   // passed (or not a number: the true residual decides)
            true_residual();
            rr = set_rr();
            if (rr <= target) {
                conv = true;
                break;
            }
            FGI_HIP(hipMemcpyAsync(p, r, nb, hipMemcpyDeviceToDevice, c.stream));
            res.reliable_updates++;
        }
    }
    res.iters = it;
    res.converged = conv ? 1 : 0;
    res.rel_resid = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
    return res;
}

// Mixed precision: defect correction around an FP32 CG.  Each outer step forms
// the FP64 true residual r = phi - A x, solves A e = r in FP32 (FP32 links of
// op32, FP32 blocks, device scalars, |r32|^2 read every CL_BATCH iterations)
// until its residual has dropped by CL_INNER or below what the outer target
// needs, and adds e to x in FP64.  The FP64 true residual decides convergence,
// so the solution meets tol exactly as the FP64 solver's does.
constexpr double CL_INNER = 1e-5;

CGResult clover_cg_mp(Ctx& c, const FermionOp& op, const FermionOp& op32, const d2* blk, const d2* phi, d2* x,
                      double tol, int maxiter, bool guess) {
    const Geom& g = *op.g;
    const size_t nb = spinor_bytes(g), nb32 = nb / 2;
    d2* r = (d2*)c.cl_r.get(nb);
    d2* ap = (d2*)c.cl_ap.get(nb);
    d2* t = (d2*)c.cl_t.get(nb);
    f2* blk32 = (f2*)c.cl_blk32.get(sizeof(f2) * 72 * (size_t)g.V);
    float* s32 = (float*)c.cl_s32.get(nb32 * 7);
    float *r32 = s32, *p32 = s32 + nb32 / 4, *q32 = s32 + 2 * (nb32 / 4), *e32 = s32 + 3 * (nb32 / 4);
    float *t32 = s32 + 4 * (nb32 / 4), *to32 = s32 + 5 * (nb32 / 4), *ue32 = s32 + 6 * (nb32 / 4);
    double* part = partial_buf(c, g);
    double* part2 = part + nb_of(g.Vh) + 64;
    double* scal = (double*)c.scal.get(sizeof(double) * 64);
    double* st = scal + 56;
    const int nbv = nb_of(g.Vh);
    {
        const size_t n = 72 * (size_t)g.V;
        hipLaunchKernelGGL(k_blk_to_f32, dim3((unsigned)((n + CBS - 1) / CBS)), dim3(CBS), 0, c.stream, n, blk, blk32);
        FGI_LAUNCH_CHECK();
    }
    const float k2 = (float)(op.kappa * op.kappa);
    auto mhat32 = [&](float* in, float* out, int dagger) {
        if (dagger) hop_oe_g5_p32(c, op32, in, to32);
        else dslash(c, op32, 1, P32, SpinorPtr{in, nullptr}, P32, SpinorPtr{to32, nullptr});
        hipLaunchKernelGGL(k_clover_apply32, dim3(nbv), dim3(CBS), 0, c.stream, g.Vh, g.V, g.Vh,
                           (const f2*)blk32, (const float*)to32, (const float*)nullptr, 0.0f, 0, 0, to32);
        dslash(c, op32, 0, P32, SpinorPtr{to32, nullptr}, P32, SpinorPtr{ue32, nullptr});
        hipLaunchKernelGGL(k_clover_apply32, dim3(nbv), dim3(CBS), 0, c.stream, g.Vh, g.V, 0, (const f2*)blk32,
                           (const float*)in, (const float*)ue32, k2, dagger, dagger, out);
        FGI_LAUNCH_CHECK();
    };
    auto normal64 = [&](const d2* in, d2* out) {
        clover_mhat(c, op, blk, in, t, 0);
        clover_mhat(c, op, blk, t, out, 1);
    };
    auto dot32 = [&](const float* a, const float* b, int mode) {
        hipLaunchKernelGGL(k_dot32, dim3(nbv), dim3(CBS), 0, c.stream, g.Vh, a, b, part);
        hipLaunchKernelGGL(k_cl_scalar, dim3(1), dim3(CBS), 0, c.stream, (const double*)part, nbv, mode, st);
        FGI_LAUNCH_CHECK();
    };
    CGResult res{};
    const double bb = dot_re(c, g, phi, phi, 49);
    const double target = tol * tol * bb;
    if (!guess) spinor_lincomb(c, g, 0.0, phi, 0.0, phi, 0, x);
    int it = 0;
    bool conv = bb == 0.0;
    double rr = bb;
    while (!conv) {
        normal64(x, ap);
        spinor_lincomb(c, g, 1.0, phi, -1.0, ap, 0, r);
        rr = dot_re(c, g, r, r, 50);
        if (rr <= target) {
            conv = true;
            break;
        }
        if (it >= maxiter) break;
        if (it > 0) res.reliable_updates++;
        // inner FP32 solve of A e = r from e = 0
        convert_spinor(c, g, P64, SpinorPtr{r, nullptr}, P32, SpinorPtr{r32, nullptr});
        FGI_HIP(hipMemcpyAsync(p32, r32, nb32, hipMemcpyDeviceToDevice, c.stream));
        FGI_HIP(hipMemsetAsync(e32, 0, nb32, c.stream));
        dot32(r32, r32, 0);
        const double rr0 = host_scalar(c, st, 56);
        const double inner = std::max(CL_INNER * CL_INNER * rr0, 0.25 * target);
        double rri = rr0;
        const int before = it;
        bool inner_finite = std::isfinite(rr0);
        while (inner_finite && rri > inner && it < maxiter) {
            const int nbatch = std::min(CL_BATCH, maxiter - it);
            for (int k = 0; k < nbatch; k++) {
                mhat32(p32, t32, 0);
                mhat32(t32, q32, 1);
                dot32(p32, q32, 1);
                hipLaunchKernelGGL(k_cl_xr32, dim3(nbv), dim3(CBS), 0, c.stream, g.Vh, (const double*)st,
                                   (const float*)p32, (const float*)q32, e32, r32, part2);
                hipLaunchKernelGGL(k_cl_scalar, dim3(1), dim3(CBS), 0, c.stream, (const double*)part2, nbv, 2, st);
                hipLaunchKernelGGL(k_cl_p32, dim3(nbv), dim3(CBS), 0, c.stream, g.Vh, (const double*)st,
                                   (const float*)r32, p32);
                FGI_LAUNCH_CHECK();
            }
            it += nbatch;
            rri = host_scalar(c, st, 56);
            inner_finite = std::isfinite(rri);
        }
        if (!inner_finite) {
            // the FP32 residual is not finite (the recursion broke down, or the
            // residual does not fit FP32): its correction is discarded and the
            // FP64 solver continues from the current x
            const CGResult r64 = clover_cg(c, op, blk, phi, x, tol, std::max(maxiter - it, 0), true);
            res.iters = it + r64.iters;
            res.converged = r64.converged;
            res.rel_resid = r64.rel_resid;
            res.reliable_updates += r64.reliable_updates + 1;
            return res;
        }
        if (it == before) break;   // no FP32 progress possible: report the FP64 residual
        // x += e
        convert_spinor(c, g, P32, SpinorPtr{e32, nullptr}, P64, SpinorPtr{ap, nullptr});
        spinor_lincomb(c, g, 1.0, x, 1.0, ap, 0, x);
    }
    res.iters = it;
    res.converged = conv ? 1 : 0;
    res.rel_resid = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
    return res;
}

// F += coef * (pf_scale F_pf + det_scale F_det) with F_pf the force of
// phi^+ (Mhat^+ Mhat)^-1 phi given its solution X_e and F_det that of
// -2 sum_{x odd} log det A(x); blk must hold A_ee and A_oo^-1 of the links of op.
// With Ye_given, F_pf is the bilinear 2 Re[Y^+ (e_a Mhat) X] of that Y_e (the
// chi-dependent part of the Hasenbusch ratio term takes it at scale -1).
// With Y_e = Mhat X_e, X_o = A_oo^-1 D_oe X_e, Y_o = A_oo^-1 g5 D_oe g5 Y_e the
// hopping part is the Wilson bilinear of (X, Y) at kappa^2; the clover parts
// go through Kt (k_clover_kt) and the leaf derivatives (k_clover_force):
//   e_a S_F clover = -2 sum_x w_x Re[Y(x)^+ e_a A(x) X(x)], w = 1 even, kappa^2 odd,
//   e_a S_det      = -2 sum_{x odd} Tr[A(x)^-1 e_a A(x)],
// e_a A = i kappa csw sum sigma (x) e_a Fhat.
void clover_force(Ctx& c, const FermionOp& op, double csw, const d2* blk, const d2* Xe, double* F, double coef,
                  double pf_scale, double det_scale, const d2* Ye_given) {
    const Geom& g = *op.g;
    const double k = op.kappa, kc = k * csw;
    const size_t nb = spinor_bytes(g);
    d2* kt = (d2*)c.cl_fh.get(sizeof(d2) * 54 * (size_t)g.V);
    d2 *ye = nullptr, *xo = nullptr, *yo = nullptr;
    const bool pf = Xe && pf_scale != 0.0;
    if (pf) {
        ye = (d2*)c.cl_ye.get(nb);
        xo = (d2*)c.cl_xo.get(nb);
        yo = (d2*)c.cl_yo.get(nb);
        d2* te = (d2*)c.cl_t.get(nb);
        if (Ye_given) ye = (d2*)Ye_given;
        else clover_mhat(c, op, blk, Xe, ye, 0);
        dslash(c, op, 1, P64, SpinorPtr{(void*)Xe, nullptr}, P64, SpinorPtr{xo, nullptr});
        clover_apply(c, g, blk, 1, xo, nullptr, 0.0, 0, 0, xo);
        spinor_lincomb(c, g, 0.0, ye, 1.0, ye, 1, te);   // te = g5 Y_e
        dslash(c, op, 1, P64, SpinorPtr{te, nullptr}, P64, SpinorPtr{yo, nullptr});
        clover_apply(c, g, blk, 1, yo, nullptr, 0.0, 1, 0, yo);   // A^-1 g5 (D_oe g5 Y_e)
        fermion_force_xyo(c, op, Xe, xo, ye, yo, F, coef * pf_scale * k * k);
    }
    hipLaunchKernelGGL(k_clover_kt, dim3(nb_of(g.V)), dim3(CBS), 0, c.stream, g, sigma_blocks(c),
                       pf ? -2.0 * kc * pf_scale : 0.0, pf ? -2.0 * k * k * kc * pf_scale : 0.0,
                       -2.0 * kc * det_scale, (const d2*)Xe, (const d2*)xo, (const d2*)ye, (const d2*)yo, blk, kt);
    FGI_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_clover_force, dim3(nb_of(4L * g.V)), dim3(CBS), 0, c.stream, g, (const d2*)op.links,
                       (const d2*)kt, coef, F);
    FGI_LAUNCH_CHECK();
}

}  // namespace fgi
