// Fermion-side kernels: the even/odd Wilson hopping term (Dslash) with fused
// Schur-complement and conjugate-gradient epilogues, the reliable-update CG
// driver, the pseudofermion heatbath and the pseudofermion force.
//
// Wilson operator M = 1 - kappa D, D psi(x) = sum_mu [(1 - g_mu) U_mu(x) psi(x+mu)
// + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)], antiperiodic in t; even/odd Schur
// operator Mhat = 1 - kappa^2 D_eo D_oe on even sites, Mhat^+ = g5 Mhat g5, so
//   Mhat v   : t = D_oe v,      out = v - kappa^2 D_eo t
//   Mhat^+ v : t = D_oe g5 v,   out = v - kappa^2 g5 D_eo t.
// Every Dslash-shaped kernel computes acc = D_{p_out, 1-p_out} [g5] in and the
// epilogue  out = center - kappa^2 [g5] acc  (or out = [g5] acc for a bare hop).
#include <algorithm>
#include <climits>
#include <cmath>

#include "fgi_internal.h"

namespace fgi {

// Threads per block of the Dslash-shaped kernels: at most DBS (launch bounds and
// LDS sizes); the block size in use (64, 128 or 256) is part of the tuned
// schedule, as is the XCD-aware block order.  Helper kernels use DBS.
static const int DBS = 256;
static inline int nblk(long n, int bs) { return (int)((n + bs - 1) / bs); }

// --------------------------------------------------------------- hop sum ---
template <typename R> __device__ __forceinline__ void flip_lower(cx<R> v[4][3]) {
#pragma unroll
    for (int k = 0; k < 3; k++) { v[2][k] = -v[2][k]; v[3][k] = -v[3][k]; }
}

// Round a spinor to FP16 storage with the per-site scale exactly as
// SpinorIO<P16>::store followed by ::load does, in registers.
template <typename R> __device__ __forceinline__ void quantize16(cx<R> v[4][3]) {
    float m = 0.f;
#pragma unroll
    for (int e = 0; e < 12; e++) {
        m = fmaxf(m, fabsf(float(v[e / 3][e % 3].re)));
        m = fmaxf(m, fabsf(float(v[e / 3][e % 3].im)));
    }
    float inv = m > 0.f ? 1.0f / m : 0.f;
#pragma unroll
    for (int e = 0; e < 12; e++) {
        cx<R>& a = v[e / 3][e % 3];
        a.re = R(float((_Float16)(float(a.re) * inv)) * m);
        a.im = R(float((_Float16)(float(a.im) * inv)) * m);
    }
}

// p_new = r + beta p_old (explicit FMAs so every kernel rounds identically)
template <typename R>
__device__ __forceinline__ void p_update(const cx<R> r[4][3], cx<R> p[4][3], R beta) {
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) {
            p[i][k].re = fma(beta, p[i][k].re, r[i][k].re);
            p[i][k].im = fma(beta, p[i][k].im, r[i][k].im);
        }
}

// Neighbour spinor loaders used by the hop sum: fetch() issues the raw loads
// of one site, get() converts them to the working precision (the FP16
// conversion and its per-site scale fuse into one mixed-precision FMA) and
// returns the factor the hop applies with its accumulating FMAs (1 here).
template <int PIN, int G5IN, typename R> struct LoadPlain {
    SpinorPtr in;
    typedef RawSp<PIN> Raw;
    __device__ __forceinline__ void fetch(int s, int Vh, Raw& raw) const { fetch_sp<PIN>(in, s, Vh, raw); }
    __device__ __forceinline__ R get(const Raw& raw, cx<R> psi[4][3]) const {
        SpinorIO<PIN, R>::decode(raw, psi);
        if (G5IN) flip_lower(psi);
        return R(1);
    }
};

// The eight hops of D, k = 2 mu + d: d = 0 the forward hop (1 - g_mu) U_mu(x)
// psi(x + mu), d = 1 the backward hop (1 + g_mu) U_mu(x - mu)^+ psi(x - mu).
// Each hop projects to a half spinor, multiplies by the link and accumulates
// the rebuilt spinor times w = (storage scale) x (link unit) x (antiperiodic
// sign in t).
template <int K, int PL, int RECON, bool NT, typename R, typename L>
__device__ __forceinline__ void hop(const Geom& g, int p, int s, const Coord& c, const void* links, const L& load,
                                    cx<R> acc[4][3]) {
    constexpr int MU = K >> 1;
    constexpr bool FWD = (K & 1) == 0;
    const int sn = cb_neighbour(g, c, MU, FWD ? +1 : -1);
    cx<R> psi[4][3], h[2][3], uh[2][3];
    typename L::Raw rs;
    load.fetch(sn, g.Vh, rs);
    R w = load.get(rs, psi) * R(link_unit<PL, RECON>());
    spin_proj<MU, FWD ? -1 : +1>(psi, h);
    // the link is loaded after the projection: loads issued any earlier only
    // raise the register count (and lower occupancy on large lattices)
    RawLink<PL, RECON> rl;
    fetch_link<PL, RECON, NT>(links, MU, FWD ? p : 1 - p, FWD ? s : sn, g.Vh, rl);
    const M3<R> u = LinkIO<PL, RECON, R>::decode(rl);
    if constexpr (FWD) {
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int a = 0; a < 3; a++)
                uh[j][a] = cdot3(u.e[a][0], h[j][0], u.e[a][1], h[j][1], u.e[a][2], h[j][2]);
        if (MU == 3 && c.c[3] == g.L[3] - 1) w = -w;
    } else {
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int a = 0; a < 3; a++)
                uh[j][a] = cdot3c(u.e[0][a], h[j][0], u.e[1][a], h[j][1], u.e[2][a], h[j][2]);
        if (MU == 3 && c.c[3] == 0) w = -w;
    }
    spin_recon_acc<MU, FWD ? -1 : +1>(acc, uh, w);
}

template <int PL, int RECON, bool NT, typename R, typename L>
__device__ __forceinline__ void hop_sum(const Geom& g, int p, int s, const void* links, const L& load,
                                        cx<R> acc[4][3]) {
    Coord c = cb_coords(g, p, s);
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) acc[i][k] = {R(0), R(0)};
    hop<0, PL, RECON, NT>(g, p, s, c, links, load, acc);
    hop<1, PL, RECON, NT>(g, p, s, c, links, load, acc);
    hop<2, PL, RECON, NT>(g, p, s, c, links, load, acc);
    hop<3, PL, RECON, NT>(g, p, s, c, links, load, acc);
    hop<4, PL, RECON, NT>(g, p, s, c, links, load, acc);
    hop<5, PL, RECON, NT>(g, p, s, c, links, load, acc);
    hop<6, PL, RECON, NT>(g, p, s, c, links, load, acc);
    hop<7, PL, RECON, NT>(g, p, s, c, links, load, acc);
}

// ------------------------------------------------------------ reductions ---
// No atomics and no grid-scope fences: a reducing kernel writes one partial per
// block (indexed by the block's logical number inside its chain), and the
// kernel after it on the stream sums them in a fixed order (sum_partials), so
// every value is independent of block scheduling and identical wherever it is
// computed.  A last-block-done scheme would need an agent-scope release per
// block, i.e. a write-back of the XCD's L2, which costs several microseconds
// per launch on this part.

// ---------------------------------------------------------- the kernel ---
enum Mode {
    M_HOP = 0,    // out = [g5] acc
    M_SCHUR = 1,  // out = center - kappa^2 [g5] acc          [|out|^2 partials]
    M_CGQ = 2,    // CG: q = p - kappa^2 acc (center p), |q|^2 partials (pAp)
    M_CGX = 3,    // CG: Ap = q - kappa^2 g5 acc; x += alpha p; r -= alpha Ap; |r|^2 partials
    M_RESID = 4,  // r = aux - (center - kappa^2 g5 acc), |r|^2 partials
    M_CGS = 5     // CG, Chronopoulos-Gear form: w = q - kappa^2 g5 acc; p = rt + beta p;
                  // s = w + beta s; x += alpha p; r -= alpha s; the hops' copy rt of r;
                  // |r|^2, Re<rt, s>, Re<p, s> partials
};
// With a CG state and partials, an M_HOP launch carries one extra block per
// chain (logical index nb) that sums the M_CGQ partials into st->pAp, or with
// cgs set the three M_CGS partials into the state (cgs_state_update).

struct DArgs {
    Geom g;
    int p_out;
    double kappa2;
    const void* links;
    SpinorPtr in, center, out, aux, x, r;
    double* partial;   // per-block partials written (reducing modes) or read (M_HOP in CG)
    CGState* st;
    int iter;   // absolute index, or the offset from st->base inside a CG batch
    int g5out;
    int gate;   // with st: 0 skip once st->stop_at <= iteration, 1 skip unless st->act
    int xcd;    // XCD-aware block order
    int cgs;    // M_HOP reduction block of the Chronopoulos-Gear form
    SpinorPtr dir, adir;   // M_CGS: p and s = A p, in the precision of x and r
};

// Chronopoulos-Gear form (Chronopoulos and Gear, J. Comput. Appl. Math. 25
// (1989) 153): the operator is applied to the residual, w = A rt with rt the
// residual as the hops read it, and the direction and its image follow by
// recurrence, p_k = rt_k + beta_k p_{k-1}, s_k = w_k + beta_k s_{k-1}, so one
// kernel updates p, s, x and r and the direction update needs no launch of its
// own.  <p_k, A p_k> is not taken from the usual recurrence (it assumes
// rt = r and exact conjugacy, which FP16 storage and reliable updates break)
// but expanded exactly: |Mhat rt_k|^2 + 2 beta Re<rt_k, s_{k-1}> + beta^2
// Re<p_{k-1}, s_{k-1}>, the last two summed by the update kernel before.
// First kernel of iteration k (the reduction block of its hop): the previous
// update's partials |r_k|^2, Re<rt_k, s_{k-1}>, Re<p_{k-1}, s_{k-1}> give
// rr_k, beta_k = rr_k / rr_{k-1} and the correction; the stop test on rr_k.
__device__ __forceinline__ void cgs_state_update(CGState* st, const StateView& S, int iter, const double* part,
                                                 int nb, double* lds) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
        v[0] += part[k];
        v[1] += part[nb + k];
        v[2] += part[2 * nb + k];
    }
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) {
        // a select, not S.rr[(iter - 1) & 1]: a run-time index into the state
        // copy makes the compiler place it in LDS, one copy per thread
        const double beta = v[0] / ((iter & 1) ? S.rr[0] : S.rr[1]);
        st->rr[iter & 1] = v[0];
        st->beta = beta;
        st->corr = 2.0 * beta * v[1] + beta * beta * v[2];
        if (v[0] <= S.rr_stop) st->stop_at = iter;
    }
}

// NT: the links are streamed with non-temporal loads (see links_streamed)
template <int MODE, int PIN, int PC, int POUT, int PX, int PL, int RECON, int G5IN, bool NT>
__device__ __forceinline__ void dslash_body(const DArgs& A, int b, int nb, double* lds) {
    typedef typename Real<PIN == P64 ? P64 : P32>::T R;
    const Geom& g = A.g;
    // Solver state, read up front in one batch of loads (reading each field
    // where it is used puts a memory round trip per branch in front of the
    // data loads).  Nothing read here is written by the same launch.
    StateView S{INT_MAX, 0, 0, 1, {0.0, 0.0}, 0.0, 0.0, 0.0};
    if (A.st) S = load_state(A.st);
    const int iter = S.base + A.iter;
    if (A.st) {  // uniform over the chain's blocks: converged / masked chains no-op
        if (A.gate ? !S.act : S.stop_at <= iter) return;
        if constexpr (MODE == M_HOP) {
            if (b >= nb) {  // the reduction block: pAp of this iteration, or the CG-form state
                if (A.cgs) {
                    cgs_state_update(A.st, S, iter, A.partial, nb, lds);
                } else if (A.partial) {
                    const double pAp = sum_partials(A.partial, nb, lds);
                    if (threadIdx.x == 0) A.st->pAp = pAp;
                }
                return;
            }
        }
    }
    int s = b * blockDim.x + threadIdx.x;
    double nrm = 0.0, rs = 0.0, ps = 0.0;
    if (s < g.Vh) {
        cx<R> acc[4][3];
        LoadPlain<PIN, G5IN, R> ld{A.in};
        hop_sum<PL, RECON, NT, R>(g, A.p_out, s, A.links, ld, acc);
        if (A.g5out) flip_lower(acc);
        if (MODE == M_HOP) {
            SpinorIO<POUT, R>::store(A.out, s, g.Vh, acc);
        } else {
            cx<R> cen[4][3];
            SpinorIO<PC, R>::load(A.center, s, g.Vh, cen);
            const R k2 = R(A.kappa2);
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int k = 0; k < 3; k++) acc[i][k] = cen[i][k] - k2 * acc[i][k];
            if (MODE == M_SCHUR || MODE == M_CGQ) {
                SpinorIO<POUT, R>::store(A.out, s, g.Vh, acc);
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int k = 0; k < 3; k++)
                        nrm += double(acc[i][k].re) * double(acc[i][k].re) + double(acc[i][k].im) * double(acc[i][k].im);
            } else if (MODE == M_RESID) {
                cx<R> ph[4][3];
                SpinorIO<PC, R>::load(A.aux, s, g.Vh, ph);
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        acc[i][k] = ph[i][k] - acc[i][k];
                        nrm += double(acc[i][k].re) * double(acc[i][k].re) + double(acc[i][k].im) * double(acc[i][k].im);
                    }
                SpinorIO<POUT, R>::store(A.out, s, g.Vh, acc);
            } else if (MODE == M_CGX) {
                typedef typename Real<PX>::T RX;
                const RX al = RX(((iter & 1) ? S.rr[1] : S.rr[0]) / S.pAp);
                cx<RX> pv[4][3], xv[4][3], rv[4][3];
                SpinorIO<PC, RX>::load(A.aux, s, g.Vh, pv);  // p has the precision of q
                SpinorIO<PX, RX>::load(A.x, s, g.Vh, xv);
                SpinorIO<PX, RX>::load(A.r, s, g.Vh, rv);
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        cx<RX> ap = {RX(acc[i][k].re), RX(acc[i][k].im)};
                        xv[i][k] = xv[i][k] + al * pv[i][k];
                        rv[i][k] = rv[i][k] - al * ap;
                        nrm += double(rv[i][k].re) * double(rv[i][k].re) + double(rv[i][k].im) * double(rv[i][k].im);
                    }
                SpinorIO<PX, RX>::store(A.x, s, g.Vh, xv);
                SpinorIO<PX, RX>::store(A.r, s, g.Vh, rv);
            } else if (MODE == M_CGS) {
                typedef typename Real<PX>::T RX;
                const RX be = RX(S.beta);
                const RX al = RX(((iter & 1) ? S.rr[1] : S.rr[0]) / (S.pAp + S.corr));
                cx<RX> tv[4][3], pv[4][3], sv[4][3], xv[4][3], rv[4][3];
                SpinorIO<PC, RX>::load(A.aux, s, g.Vh, tv);  // rt_k, as the hops read it
                SpinorIO<PX, RX>::load(A.dir, s, g.Vh, pv);
                SpinorIO<PX, RX>::load(A.adir, s, g.Vh, sv);
                SpinorIO<PX, RX>::load(A.x, s, g.Vh, xv);
                SpinorIO<PX, RX>::load(A.r, s, g.Vh, rv);
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        const cx<RX> w = {RX(acc[i][k].re), RX(acc[i][k].im)};
                        pv[i][k].re = fma(be, pv[i][k].re, tv[i][k].re);
                        pv[i][k].im = fma(be, pv[i][k].im, tv[i][k].im);
                        sv[i][k].re = fma(be, sv[i][k].re, w.re);
                        sv[i][k].im = fma(be, sv[i][k].im, w.im);
                        xv[i][k] = xv[i][k] + al * pv[i][k];
                        rv[i][k] = rv[i][k] - al * sv[i][k];
                        nrm += double(rv[i][k].re) * double(rv[i][k].re) + double(rv[i][k].im) * double(rv[i][k].im);
                        ps += double(pv[i][k].re) * double(sv[i][k].re) + double(pv[i][k].im) * double(sv[i][k].im);
                    }
                SpinorIO<PX, RX>::store(A.dir, s, g.Vh, pv);
                SpinorIO<PX, RX>::store(A.adir, s, g.Vh, sv);
                SpinorIO<PX, RX>::store(A.x, s, g.Vh, xv);
                SpinorIO<PX, RX>::store(A.r, s, g.Vh, rv);
                if constexpr (PC != PX) {  // the hops' copy of r, and Re<rt, s> with the stored values
                    static_assert(PC == P16, "a separate copy of r is kept for FP16 hops only");
                    SpinorIO<PC, RX>::store(A.aux, s, g.Vh, rv);
                    quantize16(rv);
                }
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int k = 0; k < 3; k++)
                        rs += double(rv[i][k].re) * double(sv[i][k].re) + double(rv[i][k].im) * double(sv[i][k].im);
            }
        }
    }
    if (MODE == M_HOP || !A.partial) return;
    if constexpr (MODE == M_CGS) {
        double v[3] = {nrm, rs, ps};
        block_sum<3>(v, lds);
        if (threadIdx.x == 0) {
            A.partial[b] = v[0];
            A.partial[nb + b] = v[1];
            A.partial[2 * nb + b] = v[2];
        }
        return;
    }
    double v[1] = {nrm};
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) A.partial[b] = v[0];
}

template <int MODE, int PIN, int PC, int POUT, int PX, int PL, int RECON, int G5IN, bool NT>
__global__ void __launch_bounds__(DBS) k_dslash(DArgs A) {
    __shared__ double lds[3 * DBS / 64];
    // site blocks in XCD-aware order (the same order in every kernel of the
    // solver, so a site stays on one XCD); a reduction block comes last
    const int nb = (A.g.Vh + blockDim.x - 1) / blockDim.x;
    const int b = (int)blockIdx.x < nb ? (A.xcd ? xcd_block(blockIdx.x, nb) : (int)blockIdx.x) : blockIdx.x;
    dslash_body<MODE, PIN, PC, POUT, PX, PL, RECON, G5IN, NT>(A, b, nb, lds);
}

// one chain's part of a concatenated spinor field / link field
template <int P> __device__ __forceinline__ SpinorPtr spin_off(SpinorPtr p, const ChainDesc& d) {
    if (!p.v) return p;
    SpinorPtr q = p;
    if (P == P64) q.v = (d2*)p.v + 12 * (size_t)d.site0;
    else if (P == P32) q.v = (f4*)p.v + 6 * (size_t)d.site0;
    else {
        q.v = (h8*)p.v + 3 * (size_t)d.site0;
        q.norm = p.norm + d.site0;
    }
    return q;
}

template <int PL, int RECON> __device__ __forceinline__ size_t link_byte_off(const ChainDesc& d) {
    if (PL == P64) return 9 * (size_t)d.link0 * sizeof(d2);
    return (size_t)d.link0 * sloppy_link_bytes(PL, RECON);
}

// batched launch: every chain of the batch with its own geometry, kappa,
// solver state (base.st[c]) and partials slice; nsb site blocks in all, and
// blocks past them (an M_HOP with partials) are the chains' reduction blocks
template <int MODE, int PIN, int PC, int POUT, int PX, int PL, int RECON, int G5IN>
__global__ void __launch_bounds__(DBS) k_dslash_b(DArgs base, const ChainDesc* __restrict__ cd, int nc, int nsb) {
    __shared__ double lds[3 * DBS / 64];
    const int gb = (int)blockIdx.x < nsb ? (base.xcd ? xcd_block(blockIdx.x, nsb) : (int)blockIdx.x) : blockIdx.x;
    const int c = gb < nsb ? find_chain(cd, nc, gb, GRID_DS) : gb - nsb;
    const ChainDesc& d = cd[c];
    DArgs A = base;
    A.g = d.g;
    A.kappa2 = d.kappa * d.kappa;
    A.links = (const char*)base.links + link_byte_off<PL, RECON>(d);
    A.in = spin_off<PIN>(base.in, d);
    A.center = spin_off<PC>(base.center, d);
    A.aux = spin_off<PC>(base.aux, d);
    A.out = spin_off<POUT>(base.out, d);
    A.x = spin_off<PX>(base.x, d);
    A.r = spin_off<PX>(base.r, d);
    A.partial = base.partial ? base.partial + d.blk0[GRID_DS] : nullptr;
    A.st = base.st ? base.st + c : nullptr;
    const int b = gb < nsb ? gb - d.blk0[GRID_DS] : d.nblk[GRID_DS];
    dslash_body<MODE, PIN, PC, POUT, PX, PL, RECON, G5IN, false>(A, b, d.nblk[GRID_DS], lds);
}

// First kernel of a CG iteration: p = r + beta p, stored in p's precision.
// Later iterations of a run take |r_iter|^2 from the previous M_CGX's
// partials, summed in every block in the same order (so all blocks agree
// bitwise), and beta = rr / rr_prev; block 0 records rr and beta, or the
// stop once rr <= rr_stop, for the kernels after it.  The first iteration of
// a run (start or reliable update) takes rr and beta from the host.
template <int PP, int PX>
__device__ __forceinline__ void cg_p_body(int Vh, SpinorPtr p, SpinorPtr r, CGState* st, const double* partial,
                                          int j, int b, int nb, double* lds) {
    typedef typename Real<PP == P64 ? P64 : P32>::T R;
    // the state and the site's r and p are loaded before anything waits on
    // them, so their latencies overlap with each other and with the partials
    const StateView S = load_state(st);
    const int s = b * blockDim.x + threadIdx.x;
    const int sl = s < Vh ? s : Vh - 1;
    RawSp<PX> rr_raw;
    RawSp<PP> pp_raw;
    fetch_sp<PX>(r, sl, Vh, rr_raw);
    fetch_sp<PP>(p, sl, Vh, pp_raw);
    const int iter = S.base + j;
    if (S.stop_at <= iter) return;
    double beta = S.beta;
    if (iter != S.base0) {
        const double rr = sum_partials(partial, nb, lds);
        const bool stop = rr <= S.rr_stop;
        beta = rr / ((iter & 1) ? S.rr[0] : S.rr[1]);  // |r|^2 of iteration iter - 1
        if (b == 0 && threadIdx.x == 0) {
            st->rr[iter & 1] = rr;
            if (stop) st->stop_at = iter;
            else st->beta = beta;
        }
        if (stop) return;
    }
    if (s >= Vh) return;
    cx<R> rv[4][3], pv[4][3];
    SpinorIO<PX, R>::decode(rr_raw, rv);
    SpinorIO<PP, R>::decode(pp_raw, pv);
    p_update(rv, pv, R(beta));
    SpinorIO<PP, R>::store(p, s, Vh, pv);
}

template <int PP, int PX>
// np: the number of |r|^2 partials (blocks of the M_CGX launch, the same grid)
__global__ void __launch_bounds__(DBS) k_cg_p(int Vh, SpinorPtr p, SpinorPtr r, CGState* st, const double* partial,
                                              int np, int xcd, int j) {
    __shared__ double lds[DBS / 64];
    cg_p_body<PP, PX>(Vh, p, r, st, partial, j, xcd ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x, np, lds);
}

template <int PP, int PX>
__global__ void __launch_bounds__(DBS) k_cg_p_b(const ChainDesc* __restrict__ cd, int nc, SpinorPtr p, SpinorPtr r,
                                                CGState* st, const double* partial, int xcd, int j) {
    __shared__ double lds[DBS / 64];
    const int gb = xcd ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int c = find_chain(cd, nc, gb, GRID_DS);
    const ChainDesc& d = cd[c];
    cg_p_body<PP, PX>(d.g.Vh, spin_off<PP>(p, d), spin_off<PX>(r, d), st + c, partial + d.blk0[GRID_DS], j,
                      gb - d.blk0[GRID_DS], d.nblk[GRID_DS], lds);
}

// Last node of a CG batch: fold the |r|^2 partials of the batch's last
// iteration into the state (so the host sees a finished run at once) and
// move the batch base.  The next batch's first direction update sums the
// same partials again, in the same order, and agrees bitwise.
__device__ __forceinline__ void advance_body(CGState* st, const double* partial, int nb, int n, double* lds) {
    const int it = st->base + n;  // first iteration of the next batch
    if (st->stop_at == INT_MAX) {
        const double rr = sum_partials(partial, nb, lds);
        if (threadIdx.x == 0) {
            st->rr[it & 1] = rr;
            if (rr <= st->rr_stop) st->stop_at = it;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) st->base = it;
}

__global__ void __launch_bounds__(DBS) k_advance(CGState* st, const double* partial, int nb, int n) {
    __shared__ double lds[DBS / 64];
    advance_body(st, partial, nb, n, lds);
}

// one block per chain
__global__ void __launch_bounds__(DBS) k_advance_b(const ChainDesc* __restrict__ cd, CGState* st,
                                                   const double* partial, int n) {
    __shared__ double lds[DBS / 64];
    const ChainDesc& d = cd[blockIdx.x];
    advance_body(st + blockIdx.x, partial + d.blk0[GRID_DS], d.nblk[GRID_DS], n, lds);
}

// conversion between storage precisions (through FP64 registers)
template <int PA, int PB>
__global__ void k_convert(int Vh, SpinorPtr a, SpinorPtr b) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= Vh) return;
    cx<double> v[4][3];
    SpinorIO<PA, double>::load(a, s, Vh, v);
    SpinorIO<PB, double>::store(b, s, Vh, v);
}

// y(FP64) += x(PX)
template <int PX>
__global__ void k_add_to64(int Vh, SpinorPtr x, SpinorPtr y) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= Vh) return;
    cx<double> a[4][3], b[4][3];
    SpinorIO<PX, double>::load(x, s, Vh, a);
    SpinorIO<P64, double>::load(y, s, Vh, b);
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) b[i][k] = b[i][k] + a[i][k];
    SpinorIO<P64, double>::store(y, s, Vh, b);
}

// The three partials an M_CGS launch leaves (|r|^2, Re<rt, s>, Re<p, s>) for
// the vectors as they stand: the start of a Chronopoulos-Gear run and each
// reliable update, so the next iteration's first kernel finds them as after
// any other iteration.  Blocks of the solver's block size, indexed linearly.
template <int PP, int PX>
__global__ void __launch_bounds__(DBS) k_cgs_partials(int Vh, SpinorPtr r, SpinorPtr rt, SpinorPtr p, SpinorPtr sv,
                                                      double* partial) {
    __shared__ double lds[3 * DBS / 64];
    typedef typename Real<PX>::T RX;
    const int nb = gridDim.x, b = blockIdx.x;
    const int s = b * blockDim.x + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    if (s < Vh) {
        cx<RX> rv[4][3], tv[4][3], pv[4][3], w[4][3];
        SpinorIO<PX, RX>::load(r, s, Vh, rv);
        SpinorIO<PP, RX>::load(rt, s, Vh, tv);
        SpinorIO<PX, RX>::load(p, s, Vh, pv);
        SpinorIO<PX, RX>::load(sv, s, Vh, w);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
                v[0] += double(rv[i][k].re) * double(rv[i][k].re) + double(rv[i][k].im) * double(rv[i][k].im);
                v[1] += double(tv[i][k].re) * double(w[i][k].re) + double(tv[i][k].im) * double(w[i][k].im);
                v[2] += double(pv[i][k].re) * double(w[i][k].re) + double(pv[i][k].im) * double(w[i][k].im);
            }
    }
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) {
        partial[b] = v[0];
        partial[nb + b] = v[1];
        partial[2 * nb + b] = v[2];
    }
}

__global__ void k_set_state(CGState* st, CGState v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *st = v;
}

__global__ void k_zero(size_t n, double* p) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0;
}

__global__ void k_norm2_partials(int Vh, const d2* __restrict__ v, double* partial) {
    __shared__ double lds[DBS / 64];
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    double a[1] = {0.0};
    if (s < Vh) {
#pragma unroll
        for (int k = 0; k < 12; k++) {
            d2 e = v[(size_t)k * Vh + s];
            a[0] += e.x * e.x + e.y * e.y;
        }
    }
    block_sum<1>(a, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = a[0];
}

// Re phi^+ X - |eta|^2 per even site, block partials
__global__ void k_pf_density(int Vh, const d2* __restrict__ phi, const d2* __restrict__ X, const d2* __restrict__ eta,
                             double* partial) {
    __shared__ double lds[DBS / 64];
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    double a[1] = {0.0};
    if (s < Vh) {
#pragma unroll
        for (int k = 0; k < 12; k++) {
            d2 f = phi[(size_t)k * Vh + s], x = X[(size_t)k * Vh + s];
            a[0] += f.x * x.x + f.y * x.y;
            if (eta) {
                d2 e = eta[(size_t)k * Vh + s];
                a[0] -= e.x * e.x + e.y * e.y;
            }
        }
    }
    block_sum<1>(a, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = a[0];
}

// ----------------------------------------------------- fermion force ------
// For S = phi^+ (Mhat^+ Mhat)^-1 phi and full-lattice X = (X_e, D_oe X_e),
// Y = (Mhat X_e, g5 D_oe g5 Mhat X_e):  F_mu(x) = kappa^2 bc TA(U_mu(x) C) with
//   C = sum_k h-_k(X(x+mu)) h-_k(Y(x))^+ + h+_k(Y(x+mu)) h+_k(X(x))^+,
// h-/h+ the two independent spin components of (1 -/+ g_mu) (colour vectors),
// bc = -1 on the time boundary link.
// C(A, B) of the link (mu, x) for full-lattice vectors A, B (parity p site s,
// its forward neighbour sn of the other parity)
// A full-lattice field as its two parity halves seen from one site: `here`
// the half of the site's parity, `there` the other (its neighbours').  Chosen
// by selects once per thread: an array of the two indexed by the run-time
// parity would make the compiler keep a copy per thread in LDS.
struct PairAt {
    SpinorPtr here, there;
};
__device__ __forceinline__ PairAt pair_at(SpinorPtr even, SpinorPtr odd, int p) {
    return PairAt{p ? odd : even, p ? even : odd};
}

template <int MU>
__device__ __forceinline__ M3<double> outer_c(const Geom& g, int s, int sn, const PairAt& A, const PairAt& B) {
    cx<double> a[4][3], h1[2][3], h2[2][3], h3[2][3], h4[2][3];
    SpinorIO<P64, double>::load(A.there, sn, g.Vh, a);
    spin_proj<MU, -1>(a, h1);
    SpinorIO<P64, double>::load(B.here, s, g.Vh, a);
    spin_proj<MU, -1>(a, h2);
    SpinorIO<P64, double>::load(B.there, sn, g.Vh, a);
    spin_proj<MU, +1>(a, h3);
    SpinorIO<P64, double>::load(A.here, s, g.Vh, a);
    spin_proj<MU, +1>(a, h4);
    M3<double> C;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            C.e[i][j] = mulc(h1[0][i], h2[0][j]) + mulc(h1[1][i], h2[1][j]) + mulc(h3[0][i], h4[0][j]) +
                        mulc(h3[1][i], h4[1][j]);
    return C;
}

template <int MU>
__device__ __forceinline__ void ff_add(const Geom& g, int p, int s, const Coord& c, const M3<double>& W, double coef,
                                       double* F) {
    double x[8];
    ta_components(W, x);
    double f = coef * ((MU == 3 && c.c[3] == g.L[3] - 1) ? -1.0 : 1.0);
    double* o = F + (size_t)((MU * 2 + p) * 8) * g.Vh + s;
#pragma unroll
    for (int k = 0; k < 8; k++) o[(size_t)k * g.Vh] += f * x[k];
}

template <int MU>
__device__ __forceinline__ void ff_link(const Geom& g, int p, int s, const Coord& c, const d2* U,
                                        const PairAt& X, const PairAt& Y, double coef, double* F) {
    int sn = cb_neighbour(g, c, MU, +1);
    M3<double> C = outer_c<MU>(g, s, sn, X, Y);
    ff_add<MU>(g, p, s, c, m3_mul(gauge_load(U, MU, p, s, g.Vh), C), coef, F);
}

__global__ void __launch_bounds__(256) k_fermion_force(Geom g, const d2* __restrict__ U, SpinorPtr Xe, SpinorPtr Xo,
                                                      SpinorPtr Ye, SpinorPtr Yo, double coef, double* __restrict__ F,
                                                      int xcd) {
    int t = slab_thread(g.Vh, 2, xcd);
    if (t >= g.V) return;
    int p = t / g.Vh, s = t % g.Vh;
    Coord c = cb_coords(g, p, s);
    const PairAt X = pair_at(Xe, Xo, p), Y = pair_at(Ye, Yo, p);
    ff_link<0>(g, p, s, c, U, X, Y, coef, F);
    ff_link<1>(g, p, s, c, U, X, Y, coef, F);
    ff_link<2>(g, p, s, c, U, X, Y, coef, F);
    ff_link<3>(g, p, s, c, U, X, Y, coef, F);
}

// Derivative along V of the force kappa^2 bc TA(U C(X, Y)) (Section 4's
// Leibniz rule on the force): the vectors move to dX, dY and the link U to
// V U, so per link
//   J += coef bc TA( U [C(dX, Y) + C(X, dY)] + V U C(X, Y) ).
template <int MU>
__device__ __forceinline__ void ff_tangent_link(const Geom& g, int p, int s, const Coord& c, const d2* U,
                                                const double* Vd, const PairAt& X, const PairAt& Y,
                                                const PairAt& dX, const PairAt& dY, double coef,
                                                double* J) {
    int sn = cb_neighbour(g, c, MU, +1);
    M3<double> C1 = outer_c<MU>(g, s, sn, dX, Y);
    M3<double> C2 = outer_c<MU>(g, s, sn, X, dY);
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) C1.e[i][j] = C1.e[i][j] + C2.e[i][j];
    M3<double> u = gauge_load(U, MU, p, s, g.Vh);
    double v[8];
    mom_load(Vd, MU, p, s, g.Vh, v);
    M3<double> W0 = m3_mul(alg_matrix(v), m3_mul(u, outer_c<MU>(g, s, sn, X, Y)));
    M3<double> W = m3_mul(u, C1);
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) W.e[i][j] = W.e[i][j] + W0.e[i][j];
    ff_add<MU>(g, p, s, c, W, coef, J);
}

__global__ void __launch_bounds__(256) k_fermion_force_tangent(Geom g, const d2* __restrict__ U,
                                                              const double* __restrict__ Vd, SpinorPtr Xe,
                                                              SpinorPtr Xo, SpinorPtr Ye, SpinorPtr Yo, SpinorPtr dXe,
                                                              SpinorPtr dXo, SpinorPtr dYe, SpinorPtr dYo, double coef,
                                                              double* __restrict__ J, int xcd) {
    int t = slab_thread(g.Vh, 2, xcd);
    if (t >= g.V) return;
    int p = t / g.Vh, s = t % g.Vh;
    Coord c = cb_coords(g, p, s);
    const PairAt X = pair_at(Xe, Xo, p), Y = pair_at(Ye, Yo, p), dX = pair_at(dXe, dXo, p), dY = pair_at(dYe, dYo, p);
    ff_tangent_link<0>(g, p, s, c, U, Vd, X, Y, dX, dY, coef, J);
    ff_tangent_link<1>(g, p, s, c, U, Vd, X, Y, dX, dY, coef, J);
    ff_tangent_link<2>(g, p, s, c, U, Vd, X, Y, dX, dY, coef, J);
    ff_tangent_link<3>(g, p, s, c, U, Vd, X, Y, dX, dY, coef, J);
}

// out = a x + b [g5] y on FP64 even/odd vectors (out may alias x or y)
__global__ void k_sp_lincomb(int Vh, double a, const d2* x, double b, const d2* y, int g5y, d2* out) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= Vh) return;
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const double by = (g5y && k >= 6) ? -b : b;
        d2 u = x[(size_t)k * Vh + s], v = y[(size_t)k * Vh + s];
        out[(size_t)k * Vh + s] = d2{a * u.x + by * v.x, a * u.y + by * v.y};
    }
}

// ------------------------------------------------- batched small kernels ---
// chain of the calling block in a Vh-sized batched grid and its local site
#define FGI_CHAIN_SITE(cd, nc)                                             \
    const int c_ = find_chain(cd, nc, blockIdx.x, GRID_VH);                \
    const ChainDesc& d = cd[c_];                                           \
    const int s = (blockIdx.x - d.blk0[GRID_VH]) * blockDim.x + threadIdx.x

template <int PA, int PB>
__global__ void k_convert_b(const ChainDesc* __restrict__ cd, int nc, const CGState* st, SpinorPtr a, SpinorPtr b) {
    FGI_CHAIN_SITE(cd, nc);
    if (s >= d.g.Vh || (st && !st[c_].act)) return;
    cx<double> v[4][3];
    SpinorIO<PA, double>::load(spin_off<PA>(a, d), s, d.g.Vh, v);
    SpinorIO<PB, double>::store(spin_off<PB>(b, d), s, d.g.Vh, v);
}

template <int PX>
__global__ void k_add_to64_b(const ChainDesc* __restrict__ cd, int nc, const CGState* st, SpinorPtr x, SpinorPtr y) {
    FGI_CHAIN_SITE(cd, nc);
    if (s >= d.g.Vh || !st[c_].act) return;
    cx<double> a[4][3], b[4][3];
    SpinorIO<PX, double>::load(spin_off<PX>(x, d), s, d.g.Vh, a);
    SpinorPtr yy = spin_off<P64>(y, d);
    SpinorIO<P64, double>::load(yy, s, d.g.Vh, b);
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) b[i][k] = b[i][k] + a[i][k];
    SpinorIO<P64, double>::store(yy, s, d.g.Vh, b);
}

// zero a chain's FP32 / FP64 spinor (only chains with act set when st is given)
template <int P>
__global__ void k_zero_spinor_b(const ChainDesc* __restrict__ cd, int nc, const CGState* st, SpinorPtr v) {
    FGI_CHAIN_SITE(cd, nc);
    if (s >= d.g.Vh || (st && !st[c_].act)) return;
    cx<double> z[4][3];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) z[i][k] = {0.0, 0.0};
    SpinorIO<P, double>::store(spin_off<P>(v, d), s, d.g.Vh, z);
}

__global__ void k_norm2_partials_b(const ChainDesc* __restrict__ cd, int nc, const d2* __restrict__ v,
                                   double* __restrict__ partial) {
    __shared__ double lds[DBS / 64];
    FGI_CHAIN_SITE(cd, nc);
    const d2* w = v + 12 * (size_t)d.site0;
    double a[1] = {0.0};
    if (s < d.g.Vh) {
#pragma unroll
        for (int k = 0; k < 12; k++) {
            d2 e = w[(size_t)k * d.g.Vh + s];
            a[0] += e.x * e.x + e.y * e.y;
        }
    }
    block_sum<1>(a, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = a[0];
}

__global__ void k_pf_density_b(const ChainDesc* __restrict__ cd, int nc, const d2* __restrict__ phi,
                               const d2* __restrict__ X, const d2* __restrict__ eta, double* __restrict__ partial) {
    __shared__ double lds[DBS / 64];
    FGI_CHAIN_SITE(cd, nc);
    const size_t o = 12 * (size_t)d.site0;
    const int Vh = d.g.Vh;
    double a[1] = {0.0};
    if (s < Vh) {
#pragma unroll
        for (int k = 0; k < 12; k++) {
            d2 f = phi[o + (size_t)k * Vh + s], x = X[o + (size_t)k * Vh + s];
            a[0] += f.x * x.x + f.y * x.y;
            if (eta) {
                d2 e = eta[o + (size_t)k * Vh + s];
                a[0] -= e.x * e.x + e.y * e.y;
            }
        }
    }
    block_sum<1>(a, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = a[0];
}

// batched fermion force: coef times kappa_c^2 for chain c (Y_e = Mhat X_e form)
__global__ void __launch_bounds__(256) k_fermion_force_b(const ChainDesc* __restrict__ cd, int nc,
                                                        const d2* __restrict__ U, SpinorPtr Xe, SpinorPtr Xo,
                                                        SpinorPtr Ye, SpinorPtr Yo, double coef,
                                                        double* __restrict__ F) {
    const int c_ = find_chain(cd, nc, blockIdx.x, GRID_V);
    const ChainDesc& d = cd[c_];
    const Geom& g = d.g;
    const int t = (blockIdx.x - d.blk0[GRID_V]) * blockDim.x + threadIdx.x;
    if (t >= g.V) return;
    int p = t / g.Vh, s = t % g.Vh;
    Coord c = cb_coords(g, p, s);
    const PairAt X = pair_at(spin_off<P64>(Xe, d), spin_off<P64>(Xo, d), p);
    const PairAt Y = pair_at(spin_off<P64>(Ye, d), spin_off<P64>(Yo, d), p);
    const d2* u = U + 9 * d.link0;
    double* f = F + 8 * d.link0;
    const double cf = coef * d.kappa * d.kappa;
    ff_link<0>(g, p, s, c, u, X, Y, cf, f);
    ff_link<1>(g, p, s, c, u, X, Y, cf, f);
    ff_link<2>(g, p, s, c, u, X, Y, cf, f);
    ff_link<3>(g, p, s, c, u, X, Y, cf, f);
}

// ------------------------------------------------------- host launchers ---
static SpinorPtr sp(const void* v, float* norm = nullptr) { return SpinorPtr{(void*)v, norm}; }

// Links are streamed (non-temporal loads) when the whole link field of the
// operator is larger than the L2 caches together (8 XCDs x 4 MB): then they
// cannot stay cached between launches anyway, and streaming them keeps the
// neighbour spinors in L2.  Smaller fields are reused from L2 across the CG's
// kernels, so they are loaded normally.  Batched launches always load them
// normally (batches are many small lattices).
static const double kL2Bytes = 32.0 * (1 << 20);
static int links_streamed(const FermionOp& op, long nlinks) {
    const double per = op.prec == P64 ? 144 : (double)sloppy_link_bytes(op.prec, op.recon);
    return per * (double)nlinks > kL2Bytes ? 1 : 0;
}

template <int MODE, int PIN, int PC, int POUT, int PX, int PL, int RECON, int G5IN>
static void launch_dslash_nt(Ctx& c, bool nt, int nb, DArgs& a) {
    if (nt) hipLaunchKernelGGL((k_dslash<MODE, PIN, PC, POUT, PX, PL, RECON, G5IN, true>), dim3(nb), dim3(c.ds_bs), 0, c.stream, a);
    else hipLaunchKernelGGL((k_dslash<MODE, PIN, PC, POUT, PX, PL, RECON, G5IN, false>), dim3(nb), dim3(c.ds_bs), 0, c.stream, a);
}

template <int MODE, int PIN, int PC, int POUT, int PX, int G5IN>
static void launch_dslash(Ctx& c, const FermionOp& op, DArgs& a) {
    const bool nt = links_streamed(op, 4L * a.g.V);
    a.xcd = c.ds_xcd;
    // an M_HOP inside CG (state and partials) carries the pAp reduction block
    int nb = nblk(a.g.Vh, c.ds_bs) + ((MODE == M_HOP && a.st && a.partial) ? 1 : 0);
    if constexpr (PIN == P64) {
        if (op.prec != P64) throw Error(-1, "FP64 spinors need FP64 links");
        launch_dslash_nt<MODE, PIN, PC, POUT, PX, P64, 18, G5IN>(c, nt, nb, a);
    } else {
        if (op.prec == P32 && op.recon == 18) launch_dslash_nt<MODE, PIN, PC, POUT, PX, P32, 18, G5IN>(c, nt, nb, a);
        else if (op.prec == P32) launch_dslash_nt<MODE, PIN, PC, POUT, PX, P32, 12, G5IN>(c, nt, nb, a);
        else if (op.prec == P16 && op.recon == 18) launch_dslash_nt<MODE, PIN, PC, POUT, PX, P16, 18, G5IN>(c, nt, nb, a);
        else if (op.prec == P16) launch_dslash_nt<MODE, PIN, PC, POUT, PX, P16, 12, G5IN>(c, nt, nb, a);
        else throw Error(-1, "sloppy spinors need sloppy links");
    }
    FGI_LAUNCH_CHECK();
}

static DArgs base_args(const FermionOp& op, int p_out) {
    DArgs a{};
    a.g = *op.g;
    a.p_out = p_out;
    a.kappa2 = op.kappa * op.kappa;
    a.links = op.links;
    return a;
}

static CGState* dev_state(Ctx& c) { return (CGState*)c.state.get(sizeof(CGState)); }

void dslash(Ctx& c, const FermionOp& op, int out_parity, int prec_in, SpinorPtr in, int prec_out, SpinorPtr out) {
    DArgs a = base_args(op, out_parity);
    a.in = in;
    a.out = out;
    if (prec_in == P64 && prec_out == P64) launch_dslash<M_HOP, P64, P64, P64, P64, 0>(c, op, a);
    else if (prec_in == P32 && prec_out == P32) launch_dslash<M_HOP, P32, P32, P32, P32, 0>(c, op, a);
    else if (prec_in == P16 && prec_out == P16) launch_dslash<M_HOP, P16, P16, P16, P32, 0>(c, op, a);
    else throw Error(-1, "dslash: unsupported precision pair");
}

void mhat(Ctx& c, const FermionOp& op, int prec, SpinorPtr in_e, SpinorPtr tmp_o, SpinorPtr out_e, int dagger) {
    if (prec != P64) throw Error(-1, "mhat: FP64 only");
    DArgs a = base_args(op, 1);
    a.in = in_e;
    a.out = tmp_o;
    if (dagger) launch_dslash<M_HOP, P64, P64, P64, P64, 1>(c, op, a);
    else launch_dslash<M_HOP, P64, P64, P64, P64, 0>(c, op, a);
    DArgs b = base_args(op, 0);
    b.in = tmp_o;
    b.center = in_e;
    b.out = out_e;
    b.g5out = dagger;
    launch_dslash<M_SCHUR, P64, P64, P64, P64, 0>(c, op, b);
}

void pf_heatbath(Ctx& c, const FermionOp& op64, const d2* eta, d2* phi) {
    d2* t = (d2*)c.tmp_o.get(sizeof(d2) * 12 * (size_t)op64.g->Vh);
    mhat(c, op64, P64, sp(eta), sp(t), sp(phi), 1);
}

void spinor_copy(Ctx& c, const Geom& g, const d2* src, d2* dst) {
    FGI_HIP(hipMemcpyAsync(dst, src, sizeof(d2) * 12 * (size_t)g.Vh, hipMemcpyDeviceToDevice, c.stream));
}

int pf_density_partials(Ctx& c, const Geom& g, const d2* phi, const d2* X, const d2* eta, double* partial) {
    int nb = nblk(g.Vh, DBS);
    hipLaunchKernelGGL(k_pf_density, dim3(nb), dim3(DBS), 0, c.stream, g.Vh, phi, X, eta, partial);
    FGI_LAUNCH_CHECK();
    return nb;
}

// F += coef * TA(U C(X, Y)) with X = (X_e, D_oe X_e), Y = (Y_e, g5 D_oe g5 Y_e):
// the derivative -d/dt of 2 Re[Y^+ D X] / 2 per link (coef carries the kappas)
void fermion_force_xy(Ctx& c, const FermionOp& op64, const d2* Xe, const d2* Ye, double* F, double coef) {
    const Geom& g = *op64.g;
    size_t n = sizeof(d2) * 12 * (size_t)g.Vh;
    d2* Xo = (d2*)c.Xo.get(n);
    d2* Yo = (d2*)c.Yo.get(n);
    dslash(c, op64, 1, P64, sp(Xe), P64, sp(Xo));          // X_o = D_oe X_e
    {                                                       // Y_o = g5 D_oe g5 Y_e
        DArgs a = base_args(op64, 1);
        a.in = sp(Ye);
        a.out = sp(Yo);
        a.g5out = 1;
        launch_dslash<M_HOP, P64, P64, P64, P64, 1>(c, op64, a);
    }
    hipLaunchKernelGGL(k_fermion_force, dim3(slab_blocks(g.Vh, 2, 256, c.ds_xcd)), dim3(256), 0, c.stream, g,
                       (const d2*)op64.links, sp(Xe), sp(Xo), sp(Ye), sp(Yo), coef, F, c.ds_xcd);
    FGI_LAUNCH_CHECK();
}

// pseudofermion force of phi^+ (Mhat^+ Mhat)^-1 phi at op64.kappa: Y_e = Mhat X_e
void fermion_force(Ctx& c, const FermionOp& op64, const d2* Xe, double* F, double coef) {
    const Geom& g = *op64.g;
    size_t n = sizeof(d2) * 12 * (size_t)g.Vh;
    d2* Ye = (d2*)c.Ye.get(n);
    d2* t = (d2*)c.tmp_o.get(n);
    mhat(c, op64, P64, sp(Xe), sp(t), sp(Ye), 0);
    fermion_force_xy(c, op64, Xe, Ye, F, coef * op64.kappa * op64.kappa);
}

// ------------------------------------------------ force gradient (Section 4) ---
// J_V[F_F] = d/dt F_F(exp(tV) U) for S = phi^+ A^-1 phi, A = Mhat^+ Mhat.
// With dD the hopping term on the tangent links V U (opW):
//   dMhat = -kappa^2 (dD_eo D_oe + D_eo dD_oe),
//   Z = d_V X_e = -A^-1 (dMhat^+ Y_e + Mhat^+ dMhat X_e),   Y_e = Mhat X_e,
//   dX = (Z, dD_oe X_e + D_oe Z),
//   dY = (dMhat X_e + Mhat Z, g5 dD_oe g5 Y_e + g5 D_oe g5 dY_e),
//   J += coef kappa^2 bc TA(U [C(dX, Y) + C(X, dY)] + V U C(X, Y)).
namespace {
void lincomb(Ctx& c, const Geom& g, double a, const d2* x, double b, const d2* y, int g5y, d2* out) {
    hipLaunchKernelGGL(k_sp_lincomb, dim3(nblk(g.Vh, DBS)), dim3(DBS), 0, c.stream, g.Vh, a, x, b, y, g5y, out);
    FGI_LAUNCH_CHECK();
}
// out_o = [g5] D_oe g5 in_e  (the odd half of the Y vectors)
void hop_g5(Ctx& c, const FermionOp& op, const d2* in, d2* out, int g5out) {
    DArgs a = base_args(op, 1);
    a.in = sp(in);
    a.out = sp(out);
    a.g5out = g5out;
    launch_dslash<M_HOP, P64, P64, P64, P64, 1>(c, op, a);
}
}  // namespace

void fermion_tangent_rhs(Ctx& c, const FermionOp& op64, const FermionOp& opW, const d2* Xe, d2* rhs) {
    const Geom& g = *op64.g;
    const size_t n = sizeof(d2) * 12 * (size_t)g.Vh;
    const double k2 = op64.kappa * op64.kappa;
    d2 *Ye = (d2*)c.Ye.get(n), *Yo = (d2*)c.Yo.get(n), *Xo = (d2*)c.Xo.get(n);
    d2 *to = (d2*)c.tmp_o.get(n), *te = (d2*)c.tmp_e.get(n);
    d2 *dmx = (d2*)c.tg_dmx.get(n), *dxo = (d2*)c.tg_dxo.get(n), *dye = (d2*)c.tg_dye.get(n);
    d2* dyo = (d2*)c.tg_dyo.get(n);
    mhat(c, op64, P64, sp(Xe), sp(to), sp(Ye), 0);            // Y_e = Mhat X_e
    dslash(c, op64, 1, P64, sp(Xe), P64, sp(Xo));             // X_o = D_oe X_e
    hop_g5(c, op64, Ye, Yo, 1);                                // Y_o = g5 D_oe g5 Y_e
    // dMhat X_e = -kappa^2 (dD_eo X_o + D_eo dD_oe X_e)
    dslash(c, opW, 1, P64, sp(Xe), P64, sp(dxo));             // dD_oe X_e (first part of dX_o)
    dslash(c, op64, 0, P64, sp(dxo), P64, sp(te));
    dslash(c, opW, 0, P64, sp(Xo), P64, sp(dmx));
    lincomb(c, g, -k2, te, -k2, dmx, 0, dmx);
    // dMhat^+ Y_e = -kappa^2 g5 (dD_eo D_oe g5 Y_e + D_eo dD_oe g5 Y_e), with D_oe g5 Y_e = g5 Y_o
    hop_g5(c, opW, Ye, dyo, 0);                                // dD_oe g5 Y_e (g5 of it: first part of dY_o)
    dslash(c, op64, 0, P64, sp(dyo), P64, sp(dye));            // D_eo dD_oe g5 Y_e
    {
        DArgs a = base_args(opW, 0);                           // dD_eo g5 Y_o
        a.in = sp(Yo);
        a.out = sp(te);
        launch_dslash<M_HOP, P64, P64, P64, P64, 1>(c, opW, a);
    }
    lincomb(c, g, 1.0, te, 1.0, dye, 0, te);
    mhat(c, op64, P64, sp(dmx), sp(to), sp(rhs), 1);          // Mhat^+ dMhat X_e
    lincomb(c, g, -1.0, rhs, k2, te, 1, rhs);                  // -(Mhat^+ dMhat X_e + dMhat^+ Y_e)
}

void fermion_force_tangent(Ctx& c, const FermionOp& op64, const FermionOp& opW, const double* Vd, const d2* Xe,
                           const d2* Z, double* J, double coef) {
    const Geom& g = *op64.g;
    const size_t n = sizeof(d2) * 12 * (size_t)g.Vh;
    d2 *Ye = (d2*)c.Ye.get(n), *Yo = (d2*)c.Yo.get(n), *Xo = (d2*)c.Xo.get(n);
    d2* to = (d2*)c.tmp_o.get(n);
    d2 *dmx = (d2*)c.tg_dmx.get(n), *dxo = (d2*)c.tg_dxo.get(n), *dye = (d2*)c.tg_dye.get(n);
    d2* dyo = (d2*)c.tg_dyo.get(n);
    dslash(c, op64, 1, P64, sp(Z), P64, sp(to));               // dX_o = dD_oe X_e + D_oe Z
    lincomb(c, g, 1.0, dxo, 1.0, to, 0, dxo);
    mhat(c, op64, P64, sp(Z), sp(to), sp(dye), 0);             // dY_e = dMhat X_e + Mhat Z
    lincomb(c, g, 1.0, dye, 1.0, dmx, 0, dye);
    hop_g5(c, op64, dye, to, 1);                               // dY_o = g5 D_oe g5 dY_e + g5 dD_oe g5 Y_e
    lincomb(c, g, 1.0, to, 1.0, dyo, 1, dyo);
    hipLaunchKernelGGL(k_fermion_force_tangent, dim3(slab_blocks(g.Vh, 2, 256, c.ds_xcd)), dim3(256), 0, c.stream, g,
                       (const d2*)op64.links, Vd, sp(Xe), sp(Xo), sp(Ye), sp(Yo), sp(Z), sp(dxo), sp(dye), sp(dyo),
                       coef * op64.kappa * op64.kappa, J, c.ds_xcd);
    FGI_LAUNCH_CHECK();
}

static void zero_spinor(Ctx& c, const Geom& g, void* v, int prec);

// d_V chi for chi = Mhat^+ phi at op64.kappa: out_e = dMhat^+ in_e =
// -kappa^2 g5 (dD_eo D_oe + D_eo dD_oe) g5 in_e, dD the hopping term on the
// tangent links of opW (uses tmp_o, tmp_e and the hs_t1 scratch)
void dmhat_dag_apply(Ctx& c, const FermionOp& op64, const FermionOp& opW, const d2* in_e, d2* out_e) {
    const Geom& g = *op64.g;
    const size_t n = sizeof(d2) * 12 * (size_t)g.Vh;
    const double k2 = op64.kappa * op64.kappa;
    d2 *to = (d2*)c.tmp_o.get(n), *te = (d2*)c.tmp_e.get(n), *t1 = (d2*)c.hs_t1.get(n);
    hop_g5(c, op64, in_e, to, 0);                              // D_oe g5 in
    {
        DArgs a = base_args(opW, 0);                           // dD_eo D_oe g5 in
        a.in = sp(to);
        a.out = sp(te);
        launch_dslash<M_HOP, P64, P64, P64, P64, 0>(c, opW, a);
    }
    hop_g5(c, opW, in_e, t1, 0);                               // dD_oe g5 in
    dslash(c, op64, 0, P64, sp(t1), P64, sp(out_e));           // D_eo dD_oe g5 in
    lincomb(c, g, 0.0, out_e, -k2, te, 0, te);                 // -k2 dD_eo D_oe g5 in
    lincomb(c, g, -k2, out_e, 1.0, te, 0, out_e);              // -k2 (... + D_eo dD_oe g5 in)
    lincomb(c, g, 0.0, out_e, 1.0, out_e, 1, out_e);           // g5
}

// J += coef bc TA(U [C(dX, Y) + C(X, dY)] + V U C(X, Y)) for the bilinear force
// of fermion_force_xy with X = (X_e, D_oe X_e), Y = (Y_e, g5 D_oe g5 Y_e), when
// X_e moves by dX_e and Y_e is fixed: dX = (dX_e, dD_oe X_e + D_oe dX_e),
// dY = (0, g5 dD_oe g5 Y_e)
void fermion_force_xy_tangent(Ctx& c, const FermionOp& op64, const FermionOp& opW, const double* Vd, const d2* Xe,
                              const d2* Ye, const d2* dXe, double* J, double coef) {
    const Geom& g = *op64.g;
    const size_t n = sizeof(d2) * 12 * (size_t)g.Vh;
    d2 *xo = (d2*)c.hs_xo.get(n), *yo = (d2*)c.hs_yo.get(n), *dxo = (d2*)c.hs_dxo.get(n);
    d2 *dyo = (d2*)c.hs_dyo.get(n), *zero = (d2*)c.hs_zero.get(n), *t1 = (d2*)c.hs_t1.get(n);
    zero_spinor(c, g, zero, P64);
    dslash(c, op64, 1, P64, sp(Xe), P64, sp(xo));               // X_o = D_oe X_e
    hop_g5(c, op64, Ye, yo, 1);                                 // Y_o = g5 D_oe g5 Y_e
    dslash(c, opW, 1, P64, sp(Xe), P64, sp(dxo));               // dD_oe X_e
    dslash(c, op64, 1, P64, sp(dXe), P64, sp(t1));              // + D_oe dX_e
    lincomb(c, g, 1.0, dxo, 1.0, t1, 0, dxo);
    hop_g5(c, opW, Ye, dyo, 1);                                 // dY_o = g5 dD_oe g5 Y_e
    hipLaunchKernelGGL(k_fermion_force_tangent, dim3(slab_blocks(g.Vh, 2, 256, c.ds_xcd)), dim3(256), 0, c.stream, g,
                       (const d2*)op64.links, Vd, sp(Xe), sp(xo), sp(Ye), sp(yo), sp(dXe), sp(dxo), sp(zero), sp(dyo),
                       coef, J, c.ds_xcd);
    FGI_LAUNCH_CHECK();
}

void spinor_lincomb(Ctx& c, const Geom& g, double a, const d2* x, double b, const d2* y, int g5y, d2* out) {
    lincomb(c, g, a, x, b, y, g5y, out);
}

// F += coef * TA(U C(X, Y)) for given odd halves X_o, Y_o (operators whose odd
// reconstruction is not D_oe alone)
void fermion_force_xyo(Ctx& c, const FermionOp& op64, const d2* Xe, const d2* Xo, const d2* Ye, const d2* Yo,
                       double* F, double coef) {
    const Geom& g = *op64.g;
    hipLaunchKernelGGL(k_fermion_force, dim3(slab_blocks(g.Vh, 2, 256, c.ds_xcd)), dim3(256), 0, c.stream, g,
                       (const d2*)op64.links, sp(Xe), sp(Xo), sp(Ye), sp(Yo), coef, F, c.ds_xcd);
    FGI_LAUNCH_CHECK();
}

// out_o = D_oe g5 in_e (FP64): the first hop of Mhat^+ = g5 Mhat g5
void hop_oe_g5(Ctx& c, const FermionOp& op64, const d2* in_e, d2* out_o) { hop_g5(c, op64, in_e, out_o, 0); }

// the same with FP32 spinors on FP32 links
void hop_oe_g5_p32(Ctx& c, const FermionOp& op32, void* in_e, void* out_o) {
    DArgs a = base_args(op32, 1);
    a.in = sp(in_e);
    a.out = sp(out_o);
    launch_dslash<M_HOP, P32, P32, P32, P32, 1>(c, op32, a);
}

// ---------------------------------------------------------------- CG ------
static double norm2_sync(Ctx& c, const Geom& g, const d2* v) {
    double* part = partial_buf(c, g);
    double* scal = (double*)c.scal.get(sizeof(double) * 64);
    int nb = nblk(g.Vh, DBS);
    hipLaunchKernelGGL(k_norm2_partials, dim3(nb), dim3(DBS), 0, c.stream, g.Vh, v, part);
    FGI_LAUNCH_CHECK();
    final_sum(c, part, nb, scal);
    FGI_HIP(hipMemcpyAsync(c.host_scal, scal, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    FGI_HIP(hipStreamSynchronize(c.stream));
    return c.host_scal[0];
}

// r64 = phi - Mhat^+ Mhat X (FP64), returns |r64|^2
static double true_residual(Ctx& c, const FermionOp& op64, const d2* phi, const d2* X, d2* r64) {
    const Geom& g = *op64.g;
    size_t n = sizeof(d2) * 12 * (size_t)g.Vh;
    d2* t = (d2*)c.tmp_o.get(n);
    d2* q = (d2*)c.cg_q.get(n);
    double* scal = (double*)c.scal.get(sizeof(double) * 64);
    mhat(c, op64, P64, sp(X), sp(t), sp(q), 0);  // q = Mhat X
    DArgs a = base_args(op64, 1);                // t = D_oe g5 q
    a.in = sp(q);
    a.out = sp(t);
    launch_dslash<M_HOP, P64, P64, P64, P64, 1>(c, op64, a);
    DArgs b = base_args(op64, 0);                // r = phi - (q - k^2 g5 D_eo t)
    b.in = sp(t);
    b.center = sp(q);
    b.aux = sp(phi);
    b.out = sp(r64);
    b.g5out = 1;
    b.partial = partial_buf(c, g);
    launch_dslash<M_RESID, P64, P64, P64, P64, 0>(c, op64, b);
    final_sum(c, b.partial, nblk(g.Vh, c.ds_bs), scal + 1);
    FGI_HIP(hipMemcpyAsync(c.host_scal + 1, scal + 1, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    FGI_HIP(hipStreamSynchronize(c.stream));
    return c.host_scal[1];
}

struct CGVecs {
    SpinorPtr x, r, p, q, t;  // x, r in PX; p, q, t in PP
    SpinorPtr pf, sf, rt;     // Chronopoulos-Gear form: p, s = A p in PX; rt, the hops' r, in PP (r itself if PP = PX)
};

// One CG iteration on A = Mhat^+ Mhat: a direction update and four
// Dslash-shaped kernels; the iteration index is st->base + j so a captured
// batch can be replayed.
//   rr = sum of the previous |r|^2 partials, beta, stop test; p = r + beta p
//   t = D_oe p
//   q = p - k^2 D_eo t; |q|^2 partials
//   t = D_oe g5 q; pAp = sum of the |q|^2 partials  [one extra block]
//   Ap = q - k^2 g5 D_eo t; x += alpha p; r -= alpha Ap; |r|^2 partials
// Each reduction's partials are consumed by the next kernel that reads them,
// before the next reduction writes, so one buffer serves both.
template <int PP, int PX>
static void cg_iteration(Ctx& c, const FermionOp& ops, const CGVecs& v, int j) {
    CGState* st = dev_state(c);
    double* part = partial_buf(c, *ops.g);
    const int Vh = ops.g->Vh;
    hipLaunchKernelGGL((k_cg_p<PP, PX>), dim3(nblk(Vh, c.ds_bs)), dim3(c.ds_bs), 0, c.stream, Vh, v.p, v.r, st,
                       (const double*)part, nblk(Vh, c.ds_bs), c.ds_xcd, j);
    FGI_LAUNCH_CHECK();
    {
        DArgs a = base_args(ops, 1);
        a.in = v.p;
        a.out = v.t;
        a.st = st;
        a.iter = j;
        launch_dslash<M_HOP, PP, PP, PP, PX, 0>(c, ops, a);
    }
    {
        DArgs a = base_args(ops, 0);
        a.in = v.t;
        a.center = v.p;
        a.out = v.q;
        a.partial = part;
        a.st = st;
        a.iter = j;
        launch_dslash<M_CGQ, PP, PP, PP, PX, 0>(c, ops, a);
    }
    {
        DArgs a = base_args(ops, 1);
        a.in = v.q;
        a.out = v.t;
        a.partial = part;
        a.st = st;
        a.iter = j;
        launch_dslash<M_HOP, PP, PP, PP, PX, 1>(c, ops, a);
    }
    {
        DArgs a = base_args(ops, 0);
        a.in = v.t;
        a.center = v.q;
        a.aux = v.p;
        a.x = v.x;
        a.r = v.r;
        a.g5out = 1;
        a.partial = part;
        a.st = st;
        a.iter = j;
        launch_dslash<M_CGX, PP, PP, PP, PX, 0>(c, ops, a);
    }
}

// One iteration in the Chronopoulos-Gear form: four Dslash-shaped kernels.
//   t = D_oe rt; rr, beta and the <p, A p> correction from the partials  [one extra block]
//   q = rt - k^2 D_eo t; |q|^2 partials
//   t = D_oe g5 q; |q|^2 summed into pAp  [one extra block]
//   w = q - k^2 g5 D_eo t; p = rt + beta p; s = w + beta s; x += alpha p; r -= alpha s;
//   rt; |r|^2, Re<rt, s>, Re<p, s> partials
template <int PP, int PX>
static void cg_iteration_cgs(Ctx& c, const FermionOp& ops, const CGVecs& v, int j) {
    CGState* st = dev_state(c);
    double* part = partial_buf(c, *ops.g);
    {
        DArgs a = base_args(ops, 1);
        a.in = v.rt;
        a.out = v.t;
        a.partial = part;
        a.cgs = 1;
        a.st = st;
        a.iter = j;
        launch_dslash<M_HOP, PP, PP, PP, PX, 0>(c, ops, a);
    }
    {
        DArgs a = base_args(ops, 0);
        a.in = v.t;
        a.center = v.rt;
        a.out = v.q;
        a.partial = part;
        a.st = st;
        a.iter = j;
        launch_dslash<M_CGQ, PP, PP, PP, PX, 0>(c, ops, a);
    }
    {
        DArgs a = base_args(ops, 1);
        a.in = v.q;
        a.out = v.t;
        a.partial = part;
        a.st = st;
        a.iter = j;
        launch_dslash<M_HOP, PP, PP, PP, PX, 1>(c, ops, a);
    }
    {
        DArgs a = base_args(ops, 0);
        a.in = v.t;
        a.center = v.q;
        a.aux = v.rt;
        a.x = v.x;
        a.r = v.r;
        a.dir = v.pf;
        a.adir = v.sf;
        a.g5out = 1;
        a.partial = part;
        a.st = st;
        a.iter = j;
        launch_dslash<M_CGS, PP, PP, PP, PX, 0>(c, ops, a);
    }
}

// the M_CGS partials of the vectors as they stand (start of a run, reliable update)
template <int PP, int PX>
static void cgs_partials(Ctx& c, const Geom& g, const CGVecs& v) {
    hipLaunchKernelGGL((k_cgs_partials<PP, PX>), dim3(nblk(g.Vh, c.ds_bs)), dim3(c.ds_bs), 0, c.stream, g.Vh, v.r,
                       v.rt, v.pf, v.sf, partial_buf(c, g));
    FGI_LAUNCH_CHECK();
}

// B iterations then the batch's closing reduction and base += B, on c.stream
template <int PP, int PX>
static void cg_batch_eager(Ctx& c, const FermionOp& ops, const CGVecs& v, int B) {
    for (int j = 0; j < B; j++) {
        if (c.cg_form) cg_iteration_cgs<PP, PX>(c, ops, v, j);
        else cg_iteration<PP, PX>(c, ops, v, j);
    }
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(DBS), 0, c.stream, dev_state(c), (const double*)partial_buf(c, *ops.g),
                       nblk(ops.g->Vh, c.ds_bs), B);
    FGI_LAUNCH_CHECK();
}

// N bare hops t = D_oe g5 q on the solve's live operator and vectors (the
// sample that times the Dslash kernel; t is scratch, q is only read)
template <int PP, int PX>
static void hop_sample_eager(Ctx& c, const FermionOp& ops, const CGVecs& v, int N) {
    for (int j = 0; j < N; j++) {
        DArgs a = base_args(ops, 1);
        a.in = v.q;
        a.out = v.t;
        launch_dslash<M_HOP, PP, PP, PP, PX, 1>(c, ops, a);
    }
}

// Capture `body` on the private capture stream into an instantiated graph,
// cached under `key`.
template <typename Body>
static GraphEntry& cached_graph(Ctx& c, const std::string& key, Body body) {
    for (auto& e : c.graphs)
        if (e.key == key) return e;
    if (!c.cap_stream) FGI_HIP(hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking));
    if (c.graphs.size() >= 24) {
        hipGraphExecDestroy(c.graphs.front().exec);
        c.graphs.erase(c.graphs.begin());
    }
    GraphEntry e;
    e.key = key;
    hipStream_t saved = c.stream;
    c.stream = c.cap_stream;
    hipGraph_t graph = nullptr;
    try {
        FGI_HIP(hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeRelaxed));
        body();
        FGI_HIP(hipStreamEndCapture(c.cap_stream, &graph));
        FGI_HIP(hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0));
        FGI_HIP(hipGraphDestroy(graph));
    } catch (...) {
        c.stream = saved;
        hipStreamEndCapture(c.cap_stream, &graph);
        if (graph) hipGraphDestroy(graph);
        throw;
    }
    c.stream = saved;
    c.graphs.push_back(e);
    c.graph_captures++;
    return c.graphs.back();
}

template <int PP, int PX>
static std::string graph_key(const char* what, Ctx& c, const FermionOp& ops, const CGVecs& v, int n) {
    char key[512];
    snprintf(key, sizeof key, "%s/%d/%d/%p/%.17g/%d/%d/%d/%d/%d/%d/%d/%p/%p/%p/%p/%p/%p/%p/%p/%d/%d/%d/%d/%p/%p/%p/%p",
             what, PP, PX, ops.links, ops.kappa, ops.prec, ops.recon, ops.g->L[0], ops.g->L[1], ops.g->L[2],
             ops.g->L[3], ops.g->Vh, v.x.v, v.r.v, v.p.v, v.q.v, v.t.v, (void*)v.p.norm, (void*)dev_state(c),
             (void*)partial_buf(c, *ops.g), n, c.ds_bs, c.ds_xcd, c.cg_form, v.pf.v, v.sf.v, v.rt.v,
             (void*)v.rt.norm);
    return key;
}

template <int PA, int PB>
static void convert(Ctx& c, const Geom& g, SpinorPtr a, SpinorPtr b) {
    hipLaunchKernelGGL((k_convert<PA, PB>), dim3(nblk(g.Vh, DBS)), dim3(DBS), 0, c.stream, g.Vh, a, b);
    FGI_LAUNCH_CHECK();
}

void convert_spinor(Ctx& c, const Geom& g, int pa, SpinorPtr a, int pb, SpinorPtr b) {
    if (pa == P64 && pb == P32) convert<P64, P32>(c, g, a, b);
    else if (pa == P64 && pb == P16) convert<P64, P16>(c, g, a, b);
    else if (pa == P32 && pb == P64) convert<P32, P64>(c, g, a, b);
    else if (pa == P16 && pb == P64) convert<P16, P64>(c, g, a, b);
    else if (pa == P64 && pb == P64) convert<P64, P64>(c, g, a, b);
    else throw Error(-1, "convert_spinor: unsupported pair");
}

static void zero_spinor(Ctx& c, const Geom& g, void* v, int prec) {
    size_t n = prec == P64 ? 24 * (size_t)g.Vh : (prec == P32 ? 12 * (size_t)g.Vh : 0);
    if (prec == P16) throw Error(-1, "zero_spinor: FP16");
    hipLaunchKernelGGL(k_zero, dim3(nblk((long)n, 256)), dim3(256), 0, c.stream, n, (double*)v);
    FGI_LAUNCH_CHECK();
}

// s = A p at a reliable update of the Chronopoulos-Gear form, from p as the
// hops read it: with FP16 hops p is first rounded to FP16 storage (in q) and
// kept that way, so s stays the image of the p that x is moved along.
template <int PP, int PX>
static void cgs_refresh_s(Ctx& c, const FermionOp& ops, const CGVecs& v) {
    const Geom& g = *ops.g;
    SpinorPtr pin = v.pf;
    if constexpr (PP != PX) {
        convert<PX, PP>(c, g, v.pf, v.q);
        convert<PP, PX>(c, g, v.q, v.pf);
        pin = v.q;
    }
    {
        DArgs a = base_args(ops, 1);
        a.in = pin;
        a.out = v.t;
        launch_dslash<M_HOP, PP, PP, PP, PX, 0>(c, ops, a);
    }
    {
        DArgs a = base_args(ops, 0);
        a.in = v.t;
        a.center = pin;
        a.out = v.q;   // M pin, in place when pin is q (each site reads only its own centre)
        launch_dslash<M_SCHUR, PP, PP, PP, PX, 0>(c, ops, a);
    }
    {
        DArgs a = base_args(ops, 1);
        a.in = v.q;
        a.out = v.t;
        launch_dslash<M_HOP, PP, PP, PP, PX, 1>(c, ops, a);
    }
    {
        DArgs a = base_args(ops, 0);
        a.in = v.t;
        a.center = v.q;
        a.out = v.sf;
        a.g5out = 1;
        launch_dslash<M_SCHUR, PP, PP, PX, PX, 0>(c, ops, a);
    }
}

// guess: X holds the starting point on entry (else CG starts from zero); the
// run then begins like a reliable update, from the true residual phi - A X,
// and stops on |phi - A X| <= tol |phi| as always.
template <int PP, int PX>
static CGResult cg_run(Ctx& c, const FermionOp& op64, const FermionOp& ops, const d2* phi, d2* X, double tol,
                       int maxiter, bool guess) {
    const Geom& g = *op64.g;
    const size_t n64 = sizeof(d2) * 12 * (size_t)g.Vh;
    CGResult res{0, 0, 0.0, 0};
    double bb = norm2_sync(c, g, phi);
    if (!guess || bb == 0.0) zero_spinor(c, g, X, P64);
    if (bb == 0.0) {
        res.converged = 1;
        return res;
    }
    const double target = tol * tol * bb;
    d2* r64 = (d2*)c.cg_r.get(n64);
    double rr0 = bb;  // |r|^2 of the starting point
    if (guess) {
        rr0 = true_residual(c, op64, phi, X, r64);
        if (!std::isfinite(rr0)) throw Error(-4, "CG: non-finite residual of the starting point");
        if (rr0 <= target) {
            res.converged = 1;
            res.rel_resid = std::sqrt(rr0 / bb);
            return res;
        }
    }
    const d2* r_start = guess ? r64 : phi;
    CGVecs v{};   // every field null until set: the graph key reads them all
    float* norms = (float*)c.s_norms.get(sizeof(float) * 4 * (size_t)g.Vh);
    if (PX == P64) {
        if (!guess) spinor_copy(c, g, phi, r64);
        v.x = sp(X);
        v.r = sp(r64);
        v.p = sp(c.cg_p.get(n64));
        v.q = sp(c.cg_q.get(n64));
        v.t = sp(c.s_t.get(n64));
        spinor_copy(c, g, r_start, (d2*)v.p.v);
    } else {
        size_t nx = sizeof(float) * 24 * (size_t)g.Vh;
        size_t np = PP == P32 ? nx : sizeof(_Float16) * 24 * (size_t)g.Vh;
        v.x = sp(c.s_x.get(nx));
        v.r = sp(c.s_r.get(nx));
        v.p = sp(c.s_p.get(np), norms);
        v.q = sp(c.s_q.get(np), norms + g.Vh);
        v.t = sp(c.s_t.get(np), norms + 2 * (size_t)g.Vh);
        zero_spinor(c, g, v.x.v, P32);
        convert<P64, PX>(c, g, sp(r_start), v.r);
        convert<P64, PP>(c, g, sp(r_start), v.p);
    }
    partial_buf(c, g);  // allocate before any capture
    const bool cgs = c.cg_form != 0;
    if (cgs) {  // Chronopoulos-Gear form: p = s = 0, rt = r, and the partials its first iteration sums
        const size_t nx = PX == P64 ? n64 : sizeof(float) * 24 * (size_t)g.Vh;
        v.pf = sp(c.s_pf.get(nx));
        v.sf = sp(c.s_sf.get(nx));
        zero_spinor(c, g, v.pf.v, PX);
        zero_spinor(c, g, v.sf.v, PX);
        if constexpr (PP == PX) {
            v.rt = v.r;
        } else {
            v.rt = sp(c.s_rt.get(sizeof(_Float16) * 24 * (size_t)g.Vh), norms + 3 * (size_t)g.Vh);
            convert<PX, PP>(c, g, v.r, v.rt);
        }
        cgs_partials<PP, PX>(c, g, v);
    }
    CGState* st = dev_state(c);
    CGState h{};
    h.rr[0] = rr0;
    h.rr[1] = rr0;   // the CG form's first beta divides by it (p = s = 0 there, so its value does not matter)
    h.rr_stop = (PX == P64) ? target : std::max(c.ru_delta * c.ru_delta * rr0, target);
    h.beta = 0.0;
    h.stop_at = INT_MAX;
    h.base = 0;
    h.base0 = 0;
    hipLaunchKernelGGL(k_set_state, dim3(1), dim3(64), 0, c.stream, st, h);
    FGI_LAUNCH_CHECK();
    const bool prof = c.profile && (c.profile_prec < 0 || c.profile_prec == PP);
    const int B = c.cg_batch;
    GraphEntry* ge = nullptr;
    if (c.use_graphs)
        ge = &cached_graph(c, graph_key<PP, PX>("cg", c, ops, v, B), [&] { cg_batch_eager<PP, PX>(c, ops, v, B); });
    int k = 0;  // iteration index of the next batch
    for (;;) {
        if (ge) FGI_HIP(hipGraphLaunch(ge->exec, c.stream));
        else cg_batch_eager<PP, PX>(c, ops, v, B);
        FGI_HIP(hipMemcpyAsync(c.host_state, st, sizeof(CGState), hipMemcpyDeviceToHost, c.stream));
        FGI_HIP(hipStreamSynchronize(c.stream));
        const CGState hs = *c.host_state;
        const int kend = hs.stop_at <= k + B ? hs.stop_at : k + B;
        bool inner_done = hs.stop_at <= kend;
        if (inner_done || kend >= maxiter) {
            if (PX != P64) {
                hipLaunchKernelGGL((k_add_to64<PX>), dim3(nblk(g.Vh, DBS)), dim3(DBS), 0, c.stream, g.Vh, v.x, sp(X));
                FGI_LAUNCH_CHECK();
            }
            double rr = true_residual(c, op64, phi, X, r64);
            res.iters = kend;
            res.rel_resid = std::sqrt(rr / bb);
            if (!std::isfinite(rr)) throw Error(-4, "CG: non-finite residual");
            if (rr <= target) {
                res.converged = 1;
                break;
            }
            if (kend >= maxiter) break;
            // reliable update: continue from the true residual, keep the direction
            res.reliable_updates++;
            if (PX != P64) {
                convert<P64, PX>(c, g, sp(r64), v.r);
                zero_spinor(c, g, v.x.v, P32);
            }
            if (cgs) {  // the hops' copy of the new r, s = A p afresh, and the partials
                if constexpr (PP != PX) convert<PX, PP>(c, g, v.r, v.rt);
                cgs_refresh_s<PP, PX>(c, ops, v);
                cgs_partials<PP, PX>(c, g, v);
            }
            CGState u = hs;
            u.beta = rr / hs.rr[(kend - 1) & 1];
            u.rr[kend & 1] = rr;
            u.stop_at = INT_MAX;
            u.base = kend;
            u.base0 = kend;
            u.rr_stop = (PX == P64) ? target : std::max(c.ru_delta * c.ru_delta * rr, target);
            hipLaunchKernelGGL(k_set_state, dim3(1), dim3(64), 0, c.stream, st, u);
            FGI_LAUNCH_CHECK();
            k = kend;
        } else {
            k = kend;
        }
    }
    if (prof) {
        // live sample of the bare hop: N back-to-back launches between two events
        const int N = 16;
        if (c.ev_pool.empty()) {
            for (int i = 0; i < 2; i++) {
                hipEvent_t e;
                FGI_HIP(hipEventCreate(&e));
                c.ev_pool.push_back(e);
            }
        }
        GraphEntry* hg = nullptr;
        if (c.use_graphs)
            hg = &cached_graph(c, graph_key<PP, PX>("hop", c, ops, v, N), [&] { hop_sample_eager<PP, PX>(c, ops, v, N); });
        FGI_HIP(hipEventRecord(c.ev_pool[0], c.stream));
        if (hg) FGI_HIP(hipGraphLaunch(hg->exec, c.stream));
        else hop_sample_eager<PP, PX>(c, ops, v, N);
        FGI_HIP(hipEventRecord(c.ev_pool[1], c.stream));
        FGI_HIP(hipEventSynchronize(c.ev_pool[1]));
        float ms = 0.f;
        FGI_HIP(hipEventElapsedTime(&ms, c.ev_pool[0], c.ev_pool[1]));
        c.dslash_ms += ms;
        c.dslash_launches += N;
        c.dslash_sites += (long)N * g.Vh;
    }
    return res;
}

// ====================================================== batched chains ======
template <int MODE, int PIN, int PC, int POUT, int PX, int G5IN>
static void launch_dslash_b(Ctx& c, const Batch& B, const FermionOp& op, DArgs& a) {
    const int nsb = B.nblk[GRID_DS];
    a.xcd = c.ds_xcd;
    // an M_HOP inside CG (states and partials) carries one pAp reduction block per chain
    const int nb = nsb + ((MODE == M_HOP && a.st && a.partial) ? B.nc : 0);
    if constexpr (PIN == P64) {
        hipLaunchKernelGGL((k_dslash_b<MODE, PIN, PC, POUT, PX, P64, 18, G5IN>), dim3(nb), dim3(c.ds_bs), 0, c.stream, a,
                           B.cd, B.nc, nsb);
    } else {
        if (op.prec == P32 && op.recon == 18)
            hipLaunchKernelGGL((k_dslash_b<MODE, PIN, PC, POUT, PX, P32, 18, G5IN>), dim3(nb), dim3(c.ds_bs), 0, c.stream,
                               a, B.cd, B.nc, nsb);
        else if (op.prec == P32)
            hipLaunchKernelGGL((k_dslash_b<MODE, PIN, PC, POUT, PX, P32, 12, G5IN>), dim3(nb), dim3(c.ds_bs), 0, c.stream,
                               a, B.cd, B.nc, nsb);
        else if (op.recon == 18)
            hipLaunchKernelGGL((k_dslash_b<MODE, PIN, PC, POUT, PX, P16, 18, G5IN>), dim3(nb), dim3(c.ds_bs), 0, c.stream,
                               a, B.cd, B.nc, nsb);
        else
            hipLaunchKernelGGL((k_dslash_b<MODE, PIN, PC, POUT, PX, P16, 12, G5IN>), dim3(nb), dim3(c.ds_bs), 0, c.stream,
                               a, B.cd, B.nc, nsb);
    }
    FGI_LAUNCH_CHECK();
}

static DArgs base_args_b(const FermionOp& op, int p_out) {
    DArgs a{};
    a.p_out = p_out;
    a.links = op.links;
    return a;
}

#define FGI_B_LAUNCH(kernel, grid) \
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(DBS), 0, c.stream

// out = Mhat in (dagger: Mhat^+) for every chain (gated by st[c].act when st given)
static void mhat_b(Ctx& c, const Batch& B, const FermionOp& op64, const d2* in, d2* tmp, d2* out, int dagger,
                   CGState* st) {
    DArgs a = base_args_b(op64, 1);
    a.in = sp(in);
    a.out = sp(tmp);
    a.st = st;
    a.gate = 1;
    if (dagger) launch_dslash_b<M_HOP, P64, P64, P64, P64, 1>(c, B, op64, a);
    else launch_dslash_b<M_HOP, P64, P64, P64, P64, 0>(c, B, op64, a);
    DArgs b = base_args_b(op64, 0);
    b.in = sp(tmp);
    b.center = sp(in);
    b.out = sp(out);
    b.g5out = dagger;
    b.st = st;
    b.gate = 1;
    launch_dslash_b<M_SCHUR, P64, P64, P64, P64, 0>(c, B, op64, b);
}

void pf_heatbath_b(Ctx& c, const Batch& B, const FermionOp& op64, const d2* eta, d2* phi) {
    d2* t = (d2*)c.tmp_o.get(sizeof(d2) * 12 * (size_t)B.sites);
    mhat_b(c, B, op64, eta, t, phi, 1, nullptr);
}

void fermion_force_b(Ctx& c, const Batch& B, const FermionOp& op64, const d2* Xe, double* F, double coef) {
    size_t n = sizeof(d2) * 12 * (size_t)B.sites;
    d2* Xo = (d2*)c.Xo.get(n);
    d2* Ye = (d2*)c.Ye.get(n);
    d2* Yo = (d2*)c.Yo.get(n);
    d2* t = (d2*)c.tmp_o.get(n);
    {
        DArgs a = base_args_b(op64, 1);
        a.in = sp(Xe);
        a.out = sp(Xo);
        launch_dslash_b<M_HOP, P64, P64, P64, P64, 0>(c, B, op64, a);
    }
    mhat_b(c, B, op64, Xe, t, Ye, 0, nullptr);
    {
        DArgs a = base_args_b(op64, 1);
        a.in = sp(Ye);
        a.out = sp(Yo);
        a.g5out = 1;
        launch_dslash_b<M_HOP, P64, P64, P64, P64, 1>(c, B, op64, a);
    }
    hipLaunchKernelGGL(k_fermion_force_b, dim3(B.nblk[GRID_V]), dim3(256), 0, c.stream, B.cd, B.nc,
                       (const d2*)op64.links, sp(Xe), sp(Xo), sp(Ye), sp(Yo), coef, F);
    FGI_LAUNCH_CHECK();
}

void pf_density_b(Ctx& c, const Batch& B, const d2* phi, const d2* X, const d2* eta, double* partial, double* out) {
    hipLaunchKernelGGL(k_pf_density_b, dim3(B.nblk[GRID_VH]), dim3(DBS), 0, c.stream, B.cd, B.nc, phi, X, eta, partial);
    FGI_LAUNCH_CHECK();
    final_sums_b(c, B, partial, GRID_VH, out);
}

// r = phi - Mhat^+ Mhat X and |r|^2 -> res[c] for the chains with act set
// (res[c] of the other chains is meaningless)
static void true_residual_b(Ctx& c, const Batch& B, const FermionOp& op64, const d2* phi, const d2* X, d2* r64,
                            CGState* st, double* res) {
    size_t n = sizeof(d2) * 12 * (size_t)B.sites;
    d2* t = (d2*)c.tmp_o.get(n);
    d2* q = (d2*)c.cg_q.get(n);
    mhat_b(c, B, op64, X, t, q, 0, st);
    DArgs a = base_args_b(op64, 1);
    a.in = sp(q);
    a.out = sp(t);
    a.st = st;
    a.gate = 1;
    launch_dslash_b<M_HOP, P64, P64, P64, P64, 1>(c, B, op64, a);
    DArgs b = base_args_b(op64, 0);
    b.in = sp(t);
    b.center = sp(q);
    b.aux = sp(phi);
    b.out = sp(r64);
    b.g5out = 1;
    b.partial = partial_buf(c, B);
    b.st = st;
    b.gate = 1;
    launch_dslash_b<M_RESID, P64, P64, P64, P64, 0>(c, B, op64, b);
    final_sums_b(c, B, b.partial, GRID_DS, res);
}

template <int PP, int PX>
static void cg_iteration_b(Ctx& c, const Batch& B, const FermionOp& ops, const CGVecs& v, int j, CGState* st) {
    double* part = partial_buf(c, B);
    hipLaunchKernelGGL((k_cg_p_b<PP, PX>), dim3(B.nblk[GRID_DS]), dim3(c.ds_bs), 0, c.stream, B.cd, B.nc, v.p, v.r, st,
                       (const double*)part, c.ds_xcd, j);
    FGI_LAUNCH_CHECK();
    {
        DArgs a = base_args_b(ops, 1);
        a.in = v.p;
        a.out = v.t;
        a.st = st;
        a.iter = j;
        launch_dslash_b<M_HOP, PP, PP, PP, PX, 0>(c, B, ops, a);
    }
    {
        DArgs a = base_args_b(ops, 0);
        a.in = v.t;
        a.center = v.p;
        a.out = v.q;
        a.partial = part;
        a.st = st;
        a.iter = j;
        launch_dslash_b<M_CGQ, PP, PP, PP, PX, 0>(c, B, ops, a);
    }
    {
        DArgs a = base_args_b(ops, 1);
        a.in = v.q;
        a.out = v.t;
        a.partial = part;
        a.st = st;
        a.iter = j;
        launch_dslash_b<M_HOP, PP, PP, PP, PX, 1>(c, B, ops, a);
    }
    {
        DArgs a = base_args_b(ops, 0);
        a.in = v.t;
        a.center = v.q;
        a.aux = v.p;
        a.x = v.x;
        a.r = v.r;
        a.g5out = 1;
        a.partial = part;
        a.st = st;
        a.iter = j;
        launch_dslash_b<M_CGX, PP, PP, PP, PX, 0>(c, B, ops, a);
    }
}

template <int PP, int PX>
static void cg_batch_b(Ctx& c, const Batch& B, const FermionOp& ops, const CGVecs& v, int nit, CGState* st) {
    for (int j = 0; j < nit; j++) cg_iteration_b<PP, PX>(c, B, ops, v, j, st);
    hipLaunchKernelGGL(k_advance_b, dim3(B.nc), dim3(DBS), 0, c.stream, B.cd, st, (const double*)partial_buf(c, B), nit);
    FGI_LAUNCH_CHECK();
}

// The pinned staging buffer is rewritten only after the stream has drained, so
// an earlier upload still queued behind kernels cannot pick up a later state
// (two uploads in a row at a reliable update differ in the act flags).
static void upload_states(Ctx& c, CGState* dev, const std::vector<CGState>& h) {
    FGI_HIP(hipStreamSynchronize(c.stream));
    std::copy(h.begin(), h.end(), c.host_bstates);
    FGI_HIP(hipMemcpyAsync(dev, c.host_bstates, sizeof(CGState) * h.size(), hipMemcpyHostToDevice, c.stream));
}

static void download_states(Ctx& c, const CGState* dev, std::vector<CGState>& h) {
    FGI_HIP(hipMemcpyAsync(c.host_bstates, dev, sizeof(CGState) * h.size(), hipMemcpyDeviceToHost, c.stream));
    FGI_HIP(hipStreamSynchronize(c.stream));
    std::copy(c.host_bstates, c.host_bstates + h.size(), h.begin());
}

static void download_doubles(Ctx& c, const double* dev, int n) {
    FGI_HIP(hipMemcpyAsync(c.host_bscal, dev, sizeof(double) * n, hipMemcpyDeviceToHost, c.stream));
    FGI_HIP(hipStreamSynchronize(c.stream));
}

// All chains of the batch solved together: every kernel covers every chain,
// each chain with its own CG state; chains stop on their own and take their
// reliable updates in masked steps.
template <int PP, int PX>
static std::vector<CGResult> cg_run_b(Ctx& c, const Batch& B, const FermionOp& op64, const FermionOp& ops,
                                      const d2* phi, d2* X, double tol, int maxiter, bool guess) {
    const int nc = B.nc;
    const size_t n64 = sizeof(d2) * 12 * (size_t)B.sites;
    std::vector<CGResult> res(nc, CGResult{0, 0, 0.0, 0});
    double* part = partial_buf(c, B);
    double* dres = (double*)c.bscal.get(sizeof(double) * nc);
    CGState* st = (CGState*)c.bstate.get(sizeof(CGState) * nc);
    hipLaunchKernelGGL(k_norm2_partials_b, dim3(B.nblk[GRID_VH]), dim3(DBS), 0, c.stream, B.cd, nc, phi, part);
    FGI_LAUNCH_CHECK();
    final_sums_b(c, B, part, GRID_VH, dres);
    download_doubles(c, dres, nc);
    std::vector<double> bb(c.host_bscal, c.host_bscal + nc), target(nc), rr0(bb);
    if (!guess) zero_doubles(c, (double*)X, 24 * (size_t)B.sites);
    d2* r64 = (d2*)c.cg_r.get(n64);
    std::vector<CGState> hs(nc);
    std::vector<int> done(nc, 0);
    for (int i = 0; i < nc; i++) {
        target[i] = tol * tol * bb[i];
        hs[i] = CGState{};
        hs[i].act = bb[i] != 0.0;
    }
    if (guess) {  // every chain with a nonzero right-hand side starts from its true residual
        upload_states(c, st, hs);
        true_residual_b(c, B, op64, phi, X, r64, st, dres);
        download_doubles(c, dres, nc);
        bool any_zero = false;
        for (int i = 0; i < nc; i++) {
            hs[i].act = bb[i] == 0.0;
            any_zero = any_zero || bb[i] == 0.0;
            if (bb[i] == 0.0) continue;
            rr0[i] = c.host_bscal[i];
            if (!std::isfinite(rr0[i])) throw Error(-4, "batched CG: non-finite residual of the starting point");
        }
        if (any_zero) {  // phi = 0: the solution is 0, whatever the start
            upload_states(c, st, hs);
            FGI_B_LAUNCH((k_zero_spinor_b<P64>), B.nblk[GRID_VH]), B.cd, nc, st, sp(X));
            FGI_LAUNCH_CHECK();
        }
    }
    CGVecs v{};
    float* norms = (float*)c.s_norms.get(sizeof(float) * 3 * (size_t)B.sites);
    const d2* r_start = guess ? r64 : phi;
    if (PX == P64) {
        if (!guess) FGI_HIP(hipMemcpyAsync(r64, phi, n64, hipMemcpyDeviceToDevice, c.stream));
        v.x = sp(X);
        v.r = sp(r64);
        v.p = sp(c.cg_p.get(n64));
        v.q = sp(c.cg_q.get(n64));
        v.t = sp(c.s_t.get(n64));
        FGI_HIP(hipMemcpyAsync(v.p.v, r_start, n64, hipMemcpyDeviceToDevice, c.stream));
    } else {
        size_t nx = sizeof(float) * 24 * (size_t)B.sites;
        size_t np = PP == P32 ? nx : sizeof(_Float16) * 24 * (size_t)B.sites;
        v.x = sp(c.s_x.get(nx));
        v.r = sp(c.s_r.get(nx));
        v.p = sp(c.s_p.get(np), norms);
        v.q = sp(c.s_q.get(np), norms + B.sites);
        v.t = sp(c.s_t.get(np), norms + 2 * (size_t)B.sites);
        zero_doubles(c, (double*)v.x.v, 12 * (size_t)B.sites);
        FGI_B_LAUNCH((k_convert_b<P64, PX>), B.nblk[GRID_VH]), B.cd, nc, nullptr, sp(r_start), v.r);
        FGI_B_LAUNCH((k_convert_b<P64, PP>), B.nblk[GRID_VH]), B.cd, nc, nullptr, sp(r_start), v.p);
        FGI_LAUNCH_CHECK();
    }
    for (int i = 0; i < nc; i++) {
        CGState& h = hs[i];
        h = CGState{};
        h.rr[0] = rr0[i];
        h.rr_stop = (PX == P64) ? target[i] : std::max(c.ru_delta * c.ru_delta * rr0[i], target[i]);
        const bool zero = bb[i] == 0.0, there = guess && !zero && rr0[i] <= target[i];
        h.stop_at = (zero || there) ? 0 : INT_MAX;
        if (zero || there) {
            done[i] = 1;
            res[i].converged = 1;
            res[i].rel_resid = zero ? 0.0 : std::sqrt(rr0[i] / bb[i]);
        }
    }
    upload_states(c, st, hs);
    const int Bi = c.cg_batch;
    GraphEntry* ge = nullptr;
    if (c.use_graphs) {
        // the grid sizes are baked into the graph (the chain table is read at run time)
        char key[320];
        snprintf(key, sizeof key, "bcg/%d/%d/%p/%d/%d/%d/%d/%ld/%p/%p/%p/%p/%p/%p/%p/%p/%p/%d/%d/%d", PP, PX,
                 ops.links, ops.prec, ops.recon, nc, B.nblk[GRID_DS], B.sites, (void*)B.cd, v.x.v, v.r.v, v.p.v,
                 v.q.v, v.t.v, (void*)v.p.norm, (void*)st, (void*)part, Bi, c.ds_bs, c.ds_xcd);
        ge = &cached_graph(c, key, [&] { cg_batch_b<PP, PX>(c, B, ops, v, Bi, st); });
    }
    int left = 0;
    for (int i = 0; i < nc; i++) left += !done[i];
    while (left > 0) {
        if (ge) FGI_HIP(hipGraphLaunch(ge->exec, c.stream));
        else cg_batch_b<PP, PX>(c, B, ops, v, Bi, st);
        download_states(c, st, hs);
        bool any = false;
        std::vector<int> kend(nc, 0);
        for (int i = 0; i < nc; i++) {
            hs[i].act = 0;
            if (done[i]) continue;
            bool inner = hs[i].stop_at <= hs[i].base;
            kend[i] = inner ? hs[i].stop_at : hs[i].base;
            if (inner || kend[i] >= maxiter) {
                hs[i].act = 1;
                any = true;
            }
        }
        if (!any) continue;
        upload_states(c, st, hs);
        if (PX != P64) {
            FGI_B_LAUNCH((k_add_to64_b<PX>), B.nblk[GRID_VH]), B.cd, nc, st, v.x, sp(X));
            FGI_LAUNCH_CHECK();
        }
        true_residual_b(c, B, op64, phi, X, r64, st, dres);
        download_doubles(c, dres, nc);
        bool restart = false;
        for (int i = 0; i < nc; i++) {
            if (!hs[i].act) continue;
            double rr = c.host_bscal[i];
            if (!std::isfinite(rr)) throw Error(-4, "batched CG: non-finite residual");
            res[i].iters = kend[i];
            res[i].rel_resid = bb[i] > 0 ? std::sqrt(rr / bb[i]) : 0.0;
            if (rr <= target[i] || kend[i] >= maxiter) {
                res[i].converged = rr <= target[i];
                done[i] = 1;
                left--;
                hs[i].act = 0;
                hs[i].stop_at = hs[i].base;  // no-op from now on
                continue;
            }
            res[i].reliable_updates++;
            restart = true;
            hs[i].beta = rr / hs[i].rr[(kend[i] - 1) & 1];
            hs[i].rr[kend[i] & 1] = rr;
            hs[i].stop_at = INT_MAX;
            hs[i].base = kend[i];
            hs[i].base0 = kend[i];
            hs[i].rr_stop = (PX == P64) ? target[i] : std::max(c.ru_delta * c.ru_delta * rr, target[i]);
        }
        upload_states(c, st, hs);  // act still set for the restarting chains
        if (restart && PX != P64) {
            FGI_B_LAUNCH((k_convert_b<P64, PX>), B.nblk[GRID_VH]), B.cd, nc, st, sp(r64), v.r);
            FGI_B_LAUNCH((k_zero_spinor_b<PX>), B.nblk[GRID_VH]), B.cd, nc, st, v.x);
            FGI_LAUNCH_CHECK();
        }
        for (int i = 0; i < nc; i++) hs[i].act = 0;
        upload_states(c, st, hs);
    }
    return res;
}

std::vector<CGResult> cg_solve_b(Ctx& c, const Batch& B, const FermionOp& op64, const FermionOp& ops, int sprec,
                                 const d2* phi, d2* X, double tol, int maxiter, bool guess) {
    if ((size_t)B.nc > c.host_b_cap) {
        if (c.host_bstates) hipHostFree(c.host_bstates);
        if (c.host_bscal) hipHostFree(c.host_bscal);
        FGI_HIP(hipHostMalloc((void**)&c.host_bstates, sizeof(CGState) * B.nc, hipHostMallocDefault));
        FGI_HIP(hipHostMalloc((void**)&c.host_bscal, sizeof(double) * B.nc, hipHostMallocDefault));
        c.host_b_cap = B.nc;
    }
    if (sprec == P64) return cg_run_b<P64, P64>(c, B, op64, op64, phi, X, tol, maxiter, guess);
    if (sprec == P32) return cg_run_b<P32, P32>(c, B, op64, ops, phi, X, tol, maxiter, guess);
    return cg_run_b<P16, P32>(c, B, op64, ops, phi, X, tol, maxiter, guess);
}

CGResult cg_solve(Ctx& c, const FermionOp& op64, const FermionOp& ops, int sprec, const d2* phi, d2* X, double tol,
                  int maxiter, bool guess) {
    if (sprec == P64) return cg_run<P64, P64>(c, op64, op64, phi, X, tol, maxiter, guess);
    if (sprec == P32) return cg_run<P32, P32>(c, op64, ops, phi, X, tol, maxiter, guess);
    return cg_run<P16, P32>(c, op64, ops, phi, X, tol, maxiter, guess);
}

// ============================================ t-decomposed hopping term ======
// One GPU's share of a lattice split over GPUs in t: its local sub-lattice is
// an ordinary (L0, L1, L2, Lt) checkerboard, and the hops across its two
// t-faces go through halo buffers instead of the local field.  Face sites form
// one contiguous range of F = Vh / Lt checkerboard indices per t slice (t is
// the slowest coordinate), and the site (x, y, z) of the t = 0 face and of the
// t = Lt - 1 face share the face index f = s - t F, also across neighbouring
// ranks (Lt even keeps the local and global parities equal).
//
// The pack kernel forms, for an input field of parity p_in, what each
// neighbour rank needs from this one:
//   to_lo[f] = sign_lo (1 - g4) psi(x, t = 0)                (projected half spinor)
//   to_hi[f] = sign_hi U_t(x)^+ (1 + g4) psi(x, t = Lt - 1)   (already carried by its link)
// as 2 x 3 complex numbers in the working precision R.  The rank below reads
// our to_lo as its from_hi, the rank above our to_hi as its from_lo.  The
// signs carry the antiperiodic boundary: -1 on the lowest rank's to_lo and on
// the highest rank's to_hi, +1 elsewhere.  The halo hop then applies exactly
// the arithmetic of the local kernel's t hops (the link product of the forward
// hop, the spin reconstruction of both), so a decomposed hop is bitwise the
// hop of the whole lattice.
struct HaloArgs {
    Geom g;
    int p;       // output parity (hop) or input parity (pack)
    int s0, s1;  // hop: output sites s0 <= s < s1, or with faces the two face slices
    int faces;
    const void* links;
    SpinorPtr in, out;
    const void* lo;  // hop: from_lo (backward t hops at t = 0);  pack: to_lo
    const void* hi;  // hop: from_hi (forward t hops at t = Lt-1); pack: to_hi
    double sign_lo, sign_hi;
};

template <typename R> struct HaloT;
template <> struct HaloT<double> { typedef d2 T; };
template <> struct HaloT<float> { typedef f2 T; };

// component k = 3 j + a of face entry f: SoA over the F face sites
template <typename R>
__device__ __forceinline__ void halo_store(void* buf, int F, int f, const cx<R> v[2][3], R sign) {
    typedef typename HaloT<R>::T T;
    T* b = (T*)buf;
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
        for (int a = 0; a < 3; a++) b[(size_t)(3 * j + a) * F + f] = T{sign * v[j][a].re, sign * v[j][a].im};
}

template <typename R>
__device__ __forceinline__ void halo_load(const void* buf, int F, int f, cx<R> v[2][3]) {
    typedef typename HaloT<R>::T T;
    const T* b = (const T*)buf;
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const T x = b[(size_t)(3 * j + a) * F + f];
            v[j][a] = {x.x, x.y};
        }
}

template <int PIN, int PL, int RECON>
__global__ void __launch_bounds__(DBS) k_halo_pack(HaloArgs A) {
    typedef typename Real<PIN == P64 ? P64 : P32>::T R;
    const Geom& g = A.g;
    const int F = g.Vh / g.L[3];
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    LoadPlain<PIN, 0, R> ld{A.in};
    cx<R> psi[4][3], h[2][3];
    {   // t = 0: the forward hop of the rank below lands here
        typename LoadPlain<PIN, 0, R>::Raw rs;
        ld.fetch(f, g.Vh, rs);
        const R w = ld.get(rs, psi);
        spin_proj<3, -1>(psi, h);
        halo_store<R>(const_cast<void*>(A.lo), F, f, h, w * R(A.sign_lo));
    }
    {   // t = Lt - 1: the backward hop of the rank above, link product included
        const int s = (g.L[3] - 1) * F + f;
        typename LoadPlain<PIN, 0, R>::Raw rs;
        ld.fetch(s, g.Vh, rs);
        const R w = ld.get(rs, psi);
        spin_proj<3, +1>(psi, h);
        RawLink<PL, RECON> rl;
        fetch_link<PL, RECON, false>(A.links, 3, A.p, s, g.Vh, rl);
        const M3<R> u = LinkIO<PL, RECON, R>::decode(rl);
        cx<R> uh[2][3];
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int a = 0; a < 3; a++)
                uh[j][a] = cdot3c(u.e[0][a], h[j][0], u.e[1][a], h[j][1], u.e[2][a], h[j][2]);
        halo_store<R>(const_cast<void*>(A.hi), F, f, uh, w * R(A.sign_hi) * R(link_unit<PL, RECON>()));
    }
}

template <int PIN, int POUT, int PL, int RECON>
__global__ void __launch_bounds__(DBS) k_dslash_halo(HaloArgs A) {
    typedef typename Real<PIN == P64 ? P64 : P32>::T R;
    const Geom& g = A.g;
    const int F = g.Vh / g.L[3];
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    // faces: threads 0..F-1 take the t = 0 slice, F..2F-1 the t = Lt-1 slice
    const int s = A.faces ? (i < F ? i : g.Vh - 2 * F + i) : A.s0 + i;
    if (A.faces ? i >= 2 * F : s >= A.s1) return;
    const int p = A.p;
    LoadPlain<PIN, 0, R> ld{A.in};
    const Coord c = cb_coords(g, p, s);
    cx<R> acc[4][3];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) acc[i][k] = {R(0), R(0)};
    hop<0, PL, RECON, false>(g, p, s, c, A.links, ld, acc);
    hop<1, PL, RECON, false>(g, p, s, c, A.links, ld, acc);
    hop<2, PL, RECON, false>(g, p, s, c, A.links, ld, acc);
    hop<3, PL, RECON, false>(g, p, s, c, A.links, ld, acc);
    hop<4, PL, RECON, false>(g, p, s, c, A.links, ld, acc);
    hop<5, PL, RECON, false>(g, p, s, c, A.links, ld, acc);
    if (c.c[3] == g.L[3] - 1) {  // forward t hop: the projected spinor of the rank above
        cx<R> h[2][3];
        halo_load<R>(A.hi, F, s - (g.L[3] - 1) * F, h);
        RawLink<PL, RECON> rl;
        fetch_link<PL, RECON, false>(A.links, 3, p, s, g.Vh, rl);
        const M3<R> u = LinkIO<PL, RECON, R>::decode(rl);
        cx<R> uh[2][3];
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int a = 0; a < 3; a++)
                uh[j][a] = cdot3(u.e[a][0], h[j][0], u.e[a][1], h[j][1], u.e[a][2], h[j][2]);
        spin_recon_acc<3, -1>(acc, uh, R(link_unit<PL, RECON>()));
    } else {
        hop<6, PL, RECON, false>(g, p, s, c, A.links, ld, acc);
    }
    if (c.c[3] == 0) {  // backward t hop: the link product of the rank below
        cx<R> uh[2][3];
        halo_load<R>(A.lo, F, s, uh);
        spin_recon_acc<3, +1>(acc, uh, R(1));
    } else {
        hop<7, PL, RECON, false>(g, p, s, c, A.links, ld, acc);
    }
    SpinorIO<POUT, R>::store(A.out, s, g.Vh, acc);
}

size_t halo_bytes(const Geom& g, int prec) {
    return (size_t)6 * (g.Vh / g.L[3]) * (prec == P64 ? sizeof(d2) : sizeof(f2));
}

template <int PIN, int POUT>
static void halo_launch(Ctx& c, const FermionOp& op, HaloArgs& a, bool pack) {
    const int n = pack ? a.g.Vh / a.g.L[3] : (a.faces ? 2 * (a.g.Vh / a.g.L[3]) : a.s1 - a.s0);
    if (n <= 0) return;
    const int nb = nblk(n, DBS);
#define FGI_HALO_K(PL_, RC_)                                                                                   \
    do {                                                                                                         \
        if (pack) hipLaunchKernelGGL((k_halo_pack<PIN, PL_, RC_>), dim3(nb), dim3(DBS), 0, c.stream, a);         \
        else hipLaunchKernelGGL((k_dslash_halo<PIN, POUT, PL_, RC_>), dim3(nb), dim3(DBS), 0, c.stream, a);      \
    } while (0)
    if constexpr (PIN == P64) {
        FGI_HALO_K(P64, 18);
    } else {
        if (op.prec == P32 && op.recon == 18) FGI_HALO_K(P32, 18);
        else if (op.prec == P32) FGI_HALO_K(P32, 12);
        else if (op.prec == P16 && op.recon == 18) FGI_HALO_K(P16, 18);
        else if (op.prec == P16) FGI_HALO_K(P16, 12);
        else throw Error(-1, "sloppy spinors need sloppy links");
    }
#undef FGI_HALO_K
    FGI_LAUNCH_CHECK();
}

static HaloArgs halo_args(const FermionOp& op) {
    HaloArgs a{};
    a.g = *op.g;
    a.links = op.links;
    return a;
}

void halo_pack(Ctx& c, const FermionOp& op, int prec, int in_parity, SpinorPtr in, double sign_lo, double sign_hi,
               void* to_lo, void* to_hi) {
    HaloArgs a = halo_args(op);
    a.p = in_parity;
    a.in = in;
    a.lo = to_lo;
    a.hi = to_hi;
    a.sign_lo = sign_lo;
    a.sign_hi = sign_hi;
    if (prec == P64) halo_launch<P64, P64>(c, op, a, true);
    else if (prec == P32) halo_launch<P32, P32>(c, op, a, true);
    else halo_launch<P16, P16>(c, op, a, true);
}

// part: 0 every site, 1 the interior (1 <= t <= Lt - 2), 2 the two face slices (one launch)
void dslash_halo(Ctx& c, const FermionOp& op, int prec, int out_parity, SpinorPtr in, SpinorPtr out,
                 const void* from_lo, const void* from_hi, int part) {
    HaloArgs a = halo_args(op);
    a.p = out_parity;
    a.in = in;
    a.out = out;
    a.lo = from_lo;
    a.hi = from_hi;
    const int F = a.g.Vh / a.g.L[3];
    auto run = [&](int s0, int s1, int faces) {
        a.s0 = s0;
        a.s1 = s1;
        a.faces = faces;
        if (prec == P64) halo_launch<P64, P64>(c, op, a, false);
        else if (prec == P32) halo_launch<P32, P32>(c, op, a, false);
        else halo_launch<P16, P16>(c, op, a, false);
    };
    if (part == 0) run(0, a.g.Vh, 0);
    else if (part == 1) run(F, a.g.Vh - F, 0);
    else if (a.g.L[3] == 2) run(0, a.g.Vh, 0);  // both slices are faces
    else run(0, 0, 1);
}

}  // namespace fgi
