// Host-side internals of the force-gradient HMC library: the context that owns
// scratch memory, the kernel launchers of each translation unit, and error
// plumbing.  Nothing here crosses the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "fgi_device.h"

namespace fgi {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define FGI_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            throw ::fgi::Error(-2, std::string(#call) + ": " + hipGetErrorString(e_));      \
    } while (0)

#define FGI_LAUNCH_CHECK() FGI_HIP(hipGetLastError())

Geom make_geom(const int dims[4]);

// grow-only device buffer owned by the context
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    void* get(size_t n);
    void release();
};

// Device-resident iteration state of one CG solve.  Written by the solver
// kernels and by the host between batches; copied to pinned host memory when
// the host polls.  Reductions never use atomics: a kernel writes one partial
// per block and the kernel after it sums them in a fixed order.
struct alignas(64) CGState {
    int stop_at;       // first iteration index that must not run (INT_MAX while running)
    int base;          // iteration index of the first iteration of the current batch
    int base0;         // first iteration of the current run (start or reliable update):
                       // its rr and beta come from the host, later ones from partials
    int act;           // batched solves: 1 when this chain takes part in a masked step
    double rr[2];      // |r|^2 of the iteration vectors, slot k & 1 holds iteration k's
    double pAp;        // <p, A p> of the current iteration
    double rr_stop;    // inner stopping target
    double beta;       // p_k = r_k + beta p_{k-1} of the current iteration
    double corr;       // Chronopoulos-Gear form: <p_k, A p_k> = pAp + corr
};
static_assert(sizeof(CGState) == 64, "CGState is read as 16-byte vectors");

// All fields of a state in four 16-byte loads issued together (kernels read
// the state once, up front, instead of one memory round trip per use).
struct StateView {
    int stop_at, base, base0, act;
    double rr[2], pAp, rr_stop, beta, corr;
};
__device__ __forceinline__ StateView load_state(const CGState* st) {
    typedef int i4 __attribute__((ext_vector_type(4)));
    typedef double dd2 __attribute__((ext_vector_type(2)));
    const i4 a = *(const i4*)st;
    const dd2 r = *(const dd2*)&st->rr[0];
    const dd2 q = *(const dd2*)&st->pAp;
    const dd2 t = *(const dd2*)&st->beta;
    return StateView{a.x, a.y, a.z, a.w, {r.x, r.y}, q.x, q.y, t.x, t.y};
}

// one instantiated CG batch graph, keyed by everything its kernels capture
struct GraphEntry {
    std::string key;
    hipGraphExec_t exec = nullptr;
};

// field pointers of one gauge configuration in every storage the solver needs
struct GaugeSet {
    d2* u64;          // FP64 master
    void* sloppy;     // FP32/18, FP32/12 or FP16/12 copy (nullptr in FP64 mode)
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // persistent trajectory / call scratch
    DevBuf gauge, gauge_disp, sloppy, sloppy_disp, mom, force, force2, scratch_mom;
    DevBuf eta, phi, X, Xo, Ye, Yo, tmp_e, tmp_o, cg_r, cg_p, cg_q;
    DevBuf s_x, s_r, s_p, s_q, s_t, s_norms;
    DevBuf s_pf, s_sf, s_rt;   // Chronopoulos-Gear form: p and s = A p (FP32 or FP64), the hops' copy of r
    DevBuf h0, hf0, partial, scal, state;
    DevBuf phi2, eta2, user_tmp, chi, X2;
    // force gradient of the pseudofermion force: tangent links and vectors
    DevBuf gauge_tan, tg_dmx, tg_rhs, tg_z, tg_dxo, tg_dye, tg_dyo, force3;
    DevBuf chain_U;   // the accepted links of an on-device Markov chain
    // stout smearing: the smeared levels, the fermion force on the top level and
    // its back-propagation scratch, the sloppy copy of the smeared links
    DevBuf stout_lev, stout_F, stout_ga, stout_gb, stout_part, stout_M, stout_sloppy;
    // exact force gradient of the Hasenbusch ratio term
    DevBuf hs_dchi, hs_xo, hs_yo, hs_dxo, hs_dyo, hs_zero, hs_t1;
    // clover term: blocks (A_ee, A_oo^-1), field strengths / force matrices,
    // log dets, and the vectors of its operator, solver and force
    DevBuf cl_sig, cl_blk, cl_blk2, cl_blk32, cl_s32, cl_fh, cl_ld, cl_to, cl_te, cl_ue, cl_r, cl_p, cl_ap, cl_t, cl_ye, cl_xo, cl_yo;
    DevBuf cdesc, bstate, bscal, bh0, bh1, bres;  // batched chains
    DevBuf br_jp, br_jf, br_jj;   // force gradients of the dt^4 brackets
    DevBuf halo_a, halo_b;        // face buffers of the t-decomposed hop (timing)
    CGState* host_bstates = nullptr;          // pinned [host_b_cap]
    double* host_bscal = nullptr;             // pinned [host_b_cap]
    size_t host_b_cap = 0;
    double* host_scal = nullptr;   // pinned, 64 doubles
    CGState* host_state = nullptr; // pinned
    // Live profile of the bare Dslash hop inside CG: when on, after every solve
    // 16 back-to-back launches of t = D_oe g5 q (the solve's operator and
    // vectors, one captured graph) are bracketed by HIP events on the solve's
    // stream and their time accumulated.
    bool profile = false;
    int profile_prec = -1;     // only solves whose inner precision is this (-1: all)
    std::vector<hipEvent_t> ev_pool;
    double dslash_ms = 0.0;
    long dslash_launches = 0;
    long dslash_sites = 0;     // output sites summed over profiled launches
    // inner CG: batches of per-phase kernels replayed as HIP graphs (default)
    // or launched eagerly
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;
    std::vector<GraphEntry> graphs;
    long graph_captures = 0;   // graphs captured and instantiated so far (a steady state adds none)
    // solver tuning
    int cg_batch = 8;          // iterations launched between host polls
    // schedule of the Dslash-shaped kernels (set by hand or by fgi_autotune_cg):
    // threads (= even sites) per block, and XCD-aware block order on/off
    int ds_bs = 256;
    int ds_xcd = 1;
    double ru_delta = 0.1;     // reliable-update trigger |r| drop
    // single-lattice CG iteration: 0 the classic form (five launches), 1 the
    // Chronopoulos-Gear form with exact <p, A p> (four launches; fermion.hip)
    int cg_form = 0;
    // FG displacement form: the solves of the displaced force start from the
    // undisplaced solutions (a deterministic function of the stage's links, so
    // the stage stays reversible); 0 starts them from zero
    int fg_start = 1;
    // device address of the fixed scratch array of the allocation-free entry
    // point on this context's device (looked up once per device at fgi_create)
    d2* noalloc_scratch = nullptr;
};

// A batch of independent chains: their descriptors on the device and the
// total block counts of the Vh-, V- and 4V-sized grids over all of them.
struct Batch {
    const ChainDesc* cd = nullptr;   // device array [nc]
    int nc = 0;
    int nblk[4] = {0, 0, 0, 0};
    long sites = 0, vol = 0, links = 0;  // totals: sum Vh, sum V, sum 4V
};

// Block-partial buffer of the reductions, with room for every grid launched
// over `vol` sites in `nchains` chains: the largest reduction grid (64 doubles
// per even site, blocks of 256) has vol / 8 blocks plus one rounding block per
// chain.  Every caller asks with the same arguments for a given lattice or
// batch, so the buffer never moves while a call is using it.
inline double* partial_buf(Ctx& c, long vol, long nchains = 1) {
    long n = vol / 4 + 8 * nchains + 64;
    if (n < 65536) n = 65536;
    return (double*)c.partial.get(sizeof(double) * (size_t)n);
}
inline double* partial_buf(Ctx& c, const Geom& g) { return partial_buf(c, g.V, 1); }
inline double* partial_buf(Ctx& c, const Batch& B) { return partial_buf(c, B.vol, B.nc); }

// blocks of `bs` threads for slab_thread over nt arrays of Vh sites
inline int slab_blocks(long Vh, int nt, int bs, int xcd) {
    return xcd ? nt * (int)((Vh + bs - 1) / bs) : (int)((nt * Vh + bs - 1) / bs);
}

// ---------------- gauge.hip ----------------
void pack_gauge(Ctx&, const Geom&, const void* user, d2* internal);
void unpack_gauge(Ctx&, const Geom&, const d2* internal, void* user);
void pack_mom(Ctx&, const Geom&, const double* user, double* internal);
void unpack_mom(Ctx&, const Geom&, const double* internal, double* user);
void pack_even_spinor(Ctx&, const Geom&, const void* user, d2* internal);
void unpack_even_spinor(Ctx&, const Geom&, const d2* internal, void* user);
void make_sloppy(Ctx&, const Geom&, const d2* u64, void* sloppy, int prec, int recon);
// per-site h = beta * sum_{mu<nu}(1 - ReTr U_P/3) [when U != null] + kinetic of P [when P != null]
// h = gauge action density (plaquettes at beta (1 - 8 c1), rectangles at
// beta c1; none when U is null) + kinetic density (when P is given)
void ham_density(Ctx&, const Geom&, double beta, const d2* U, const double* P, double* h, double c1 = 0.0);
// partial[b] = sum over block b of (h1 - h0) [or h1 when h0 == null]; returns nblocks
int diff_partials(Ctx&, int n, const double* h1, const double* h0, double* partial);
void final_sum(Ctx&, const double* partial, int n, double* out);
// F_G into F: mode 0: F = c * F_G; 1: F += c * F_G
// F (+)= c F_G(U) for the gauge action with rectangle coefficient c1
void gauge_force(Ctx&, const Geom&, double beta, const d2* U, double* F, double c, int accumulate,
                 double c1 = 0.0);
// mode 0: J = c * d/dt F_G(exp(t V) U); mode 1: J = c * (-J_V[F_G] + [V, F_G]/2),
// the Hessian of S_G in the chart exp(omega) U at omega = 0 applied to V (+ J when accumulate)
void gauge_force_tangent(Ctx&, const Geom&, double beta, const d2* U, const double* Vd, double* J,
                         double c, int accumulate, int mode = 0, double c1 = 0.0);
// dst = exp(h X) src on every link; sloppy copy of dst written when sloppy != null
void link_update(Ctx&, const Geom&, double h, const double* X, const d2* src, d2* dst, void* sloppy,
                 int prec, int recon);
// W = V U on every link (FP64 internal layout): the links of the derivative of D along V
void tangent_links(Ctx&, const Geom&, const double* Vd, const d2* U, d2* W);
// n stout levels of U into levels (n consecutive gauge fields); returns the top level
const d2* stout_smear(Ctx&, const Geom&, double rho, int n, const d2* U, d2* levels);
// F (+)= coef * (force on the thin links U) given the force Fs on the top smeared
// level; levels as written by stout_smear for the same U
void stout_backprop(Ctx&, const Geom&, double rho, int n, const d2* U, const d2* levels, const double* Fs,
                    double* F, double coef, int accumulate);
// y += a x over the 4 * 2 * 8 * Vh momentum components
void mom_axpy(Ctx&, const Geom&, double a, const double* x, double* y);
void reunitarize(Ctx&, const Geom&, d2* U);
// partial[b] = sum over block b of x[k] y[k], k < n; returns nblocks
int dot_partials(Ctx&, long n, const double* x, const double* y, double* partial);
// p[0..n) = 0 (a kernel, not a memset, so it can sit in a captured graph)
void zero_doubles(Ctx&, double* p, size_t n);
// exp of one su(3) element (test hook of the device exponential)
void exp_su3_batch(Ctx&, int n, const double* p, double h, void* out);

// batched versions (every chain with its own geometry, beta, kappa)
void pack_b(Ctx&, const Batch&, void* internal, int field /*0 U, 1 P, 2 eta*/, int to_internal);
void make_sloppy_b(Ctx&, const Batch&, const d2* U, void* sloppy, int prec, int recon);
void ham_density_b(Ctx&, const Batch&, const d2* U, const double* P, double* h, double c1 = 0.0);
void diff_sums_b(Ctx&, const Batch&, const double* h1, const double* h0, double* partial, double* out);
void final_sums_b(Ctx&, const Batch&, const double* partial, int kind, double* out);
void gauge_force_b(Ctx&, const Batch&, const d2* U, double* F, double coef, int accumulate, double c1 = 0.0);
// stout smearing and its force back-propagation for every chain of a batch
const d2* stout_smear_b(Ctx&, const Batch&, double rho, int n, const d2* U, d2* levels);
void stout_backprop_b(Ctx&, const Batch&, double rho, int n, const d2* U, const d2* levels, const double* Fs,
                      double* F, double coef, int accumulate);
void link_update_b(Ctx&, const Batch&, double h, const double* X, const d2* src, d2* dst, void* sloppy, int prec,
                   int recon);

// ---------------- chain.hip ----------------
// Heatbath draws of trajectory traj of the chain with this seed (rng.h streams):
// P internal momenta, eta internal even noise of stream 1 (eta1) or 2 (eta2)
void refresh_momenta(Ctx&, const Geom&, uint64_t seed, uint32_t traj, double* P);
void refresh_noise(Ctx&, const Geom&, uint64_t seed, uint32_t traj, int stream, d2* eta);
// the Metropolis uniform of trajectory traj (host)
double metropolis_uniform(uint64_t seed, uint32_t traj);
void philox_host(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

// ---------------- fermion.hip ----------------
struct FermionOp {
    const Geom* g;
    double kappa;
    const void* links;   // gauge storage for this operator
    int prec, recon;     // link storage precision / reconstruction
};
// out_{1-p} = D_{(1-p) p} in_p  (hopping term between parities)
void dslash(Ctx&, const FermionOp&, int out_parity, int prec_in, SpinorPtr in, int prec_out,
            SpinorPtr out);
// out_e = [g5] (in_e - kappa^2 D_eo t_o)  where t_o = D_oe in_e is computed too
void mhat(Ctx&, const FermionOp&, int prec, SpinorPtr in_e, SpinorPtr tmp_o, SpinorPtr out_e,
          int dagger);
struct CGResult {
    int iters;
    int converged;
    double rel_resid;
    int reliable_updates;
};
// X = (Mhat^+ Mhat)^-1 phi from a zero start, or (guess) from the X given on
// entry; FP64 op64 for the true residual, sloppy op for the inner iterations
// (same op for FP64 mode)
CGResult cg_solve(Ctx&, const FermionOp& op64, const FermionOp& ops, int sprec, const d2* phi, d2* X,
                  double tol, int maxiter, bool guess = false);
// phi = Mhat^+ eta
void pf_heatbath(Ctx&, const FermionOp& op64, const d2* eta, d2* phi);
// F += c * F_F(X_e) (pseudofermion force given the solution X_e)
void fermion_force(Ctx&, const FermionOp& op64, const d2* Xe, double* F, double c);
// F += coef * TA(U C(X, Y)), X = (X_e, D_oe X_e), Y = (Y_e, g5 D_oe g5 Y_e)
void fermion_force_xy(Ctx&, const FermionOp& op64, const d2* Xe, const d2* Ye, double* F, double coef);
// Force gradient of the pseudofermion force along V (Section 4), in two halves
// around the one extra solve.  opW is the operator on the tangent links V U.
//   rhs = -(d_V A) X_e,  A = Mhat^+ Mhat     (also keeps Y_e, X_o, ... for the second half)
void fermion_tangent_rhs(Ctx&, const FermionOp& op64, const FermionOp& opW, const d2* Xe, d2* rhs);
// out_e = dMhat^+ in_e along the tangent links of opW (d_V of Mhat^+ phi)
void dmhat_dag_apply(Ctx&, const FermionOp& op64, const FermionOp& opW, const d2* in_e, d2* out_e);
// J += coef * d_V of the bilinear force of fermion_force_xy(X_e, Y_e) when X_e moves by dX_e, Y_e fixed
void fermion_force_xy_tangent(Ctx&, const FermionOp& op64, const FermionOp& opW, const double* Vd, const d2* Xe,
                              const d2* Ye, const d2* dXe, double* J, double coef);
// out = a x + b [g5] y on FP64 even vectors
void spinor_lincomb(Ctx&, const Geom&, double a, const d2* x, double b, const d2* y, int g5y, d2* out);
// F += coef * TA(U C(X, Y)) for given even and odd halves of X and Y
void fermion_force_xyo(Ctx&, const FermionOp& op64, const d2* Xe, const d2* Xo, const d2* Ye, const d2* Yo,
                       double* F, double coef);
// out_o = D_oe g5 in_e (FP64)
void hop_oe_g5(Ctx&, const FermionOp& op64, const d2* in_e, d2* out_o);
void hop_oe_g5_p32(Ctx&, const FermionOp& op32, void* in_e, void* out_o);
//   J += coef * J_V[F_F] given Z = A^-1 rhs (after fermion_tangent_rhs on the same X_e)
void fermion_force_tangent(Ctx&, const FermionOp& op64, const FermionOp& opW, const double* Vd, const d2* Xe,
                           const d2* Z, double* J, double coef);
// partials of Re phi^+ X - |eta|^2 (eta may be null) per even site; returns nblocks
int pf_density_partials(Ctx&, const Geom&, const d2* phi, const d2* X, const d2* eta, double* partial);
// for the Hasenbusch pair: out = Mhat(kappa2)^+ in etc. use mhat with another op
void spinor_copy(Ctx&, const Geom&, const d2* src, d2* dst);
// b = a with storage conversion (P64/P32/P16 -> P64/P32/P16)
void convert_spinor(Ctx&, const Geom&, int prec_a, SpinorPtr a, int prec_b, SpinorPtr b);
// t-decomposed hopping term (one GPU's share of a lattice split in t)
size_t halo_bytes(const Geom&, int prec);
void halo_pack(Ctx&, const FermionOp&, int prec, int in_parity, SpinorPtr in, double sign_lo, double sign_hi,
               void* to_lo, void* to_hi);
void dslash_halo(Ctx&, const FermionOp&, int prec, int out_parity, SpinorPtr in, SpinorPtr out, const void* from_lo,
                 const void* from_hi, int part);

// batched fermion operations (all chains of B; FP64 fields concatenated chain by chain)
void pf_heatbath_b(Ctx&, const Batch&, const FermionOp& op64, const d2* eta, d2* phi);
void fermion_force_b(Ctx&, const Batch&, const FermionOp& op64, const d2* Xe, double* F, double coef);
void pf_density_b(Ctx&, const Batch&, const d2* phi, const d2* X, const d2* eta, double* partial, double* out);
std::vector<CGResult> cg_solve_b(Ctx&, const Batch&, const FermionOp& op64, const FermionOp& ops, int sprec,
                                 const d2* phi, d2* X, double tol, int maxiter, bool guess = false);


// ---------------- clover.hip ----------------
// A_ee and A_oo^-1 (A everywhere when invert_odd == 0) of the clover term at
// kappa, csw on the FP64 links U into blk (72 d2 per site); with det_action,
// -2 sum_{x odd} log det A(x) (synchronises)
void clover_build(Ctx&, const Geom&, double kappa, double csw, const d2* U, d2* blk, int invert_odd,
                  double* det_action);
// A(x) as [V][12][12] complex in lexicographic site order (blk built with invert_odd == 0)
void clover_unpack(Ctx&, const Geom&, const d2* blk, void* out);
// out_e = [g5] Mhat [g5] in_e with the clover Mhat (dagger)
void clover_mhat(Ctx&, const FermionOp& op64, const d2* blk, const d2* in_e, d2* out_e, int dagger);
CGResult clover_cg(Ctx&, const FermionOp& op64, const d2* blk, const d2* phi, d2* x, double tol, int maxiter,
                   bool guess);
// the same solve with an FP32 inner CG on the FP32 links of ops (defect
// correction: the FP64 true residual decides convergence)
CGResult clover_cg_mp(Ctx&, const FermionOp& op64, const FermionOp& op32, const d2* blk, const d2* phi, d2* x,
                      double tol, int maxiter, bool guess);
// F += coef (pf_scale F_pf(X_e) + det_scale F_det); Xe may be null when pf_scale == 0
void clover_force(Ctx&, const FermionOp& op64, double csw, const d2* blk, const d2* Xe, double* F, double coef,
                  double pf_scale, double det_scale, const d2* Ye_given = nullptr);

}  // namespace fgi
