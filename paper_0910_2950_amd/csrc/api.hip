// C-ABI entry points, context and the integrator driver (host side).
#include <hip/hip_runtime.h>

#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fgi.h"
#include "fgi_internal.h"
#include "rng.h"

struct fgi_ctx {
    fgi::Ctx c;
};

namespace fgi {

static thread_local std::string g_last_error;
void set_last_error(const std::string& m) { g_last_error = m; }

void* DevBuf::get(size_t n) {
    if (n > bytes) {
        if (p) {
            hipFree(p);
            p = nullptr;
            bytes = 0;
        }
        FGI_HIP(hipMalloc(&p, n));
        bytes = n;
    }
    return p;
}

void DevBuf::release() {
    if (p) hipFree(p);
    p = nullptr;
    bytes = 0;
}

Geom make_geom(const int dims[4]) {
    Geom g;
    long V = 1;
    for (int m = 0; m < 4; m++) {
        if (dims[m] < 2 || (dims[m] & 1)) throw Error(FGI_EINVAL, "every lattice extent must be even and >= 2");
        g.L[m] = dims[m];
        V *= dims[m];
    }
    if (V > (1L << 30)) throw Error(FGI_EINVAL, "lattice volume too large");
    g.Lxh = dims[0] / 2;
    g.V = (int)V;
    g.Vh = (int)(V / 2);
    return g;
}

}  // namespace fgi

using namespace fgi;

// Scratch of the allocation-free entry point (fgi_mhat_packed_noalloc): the
// odd intermediate D_oe in of one Schur application, FGI_NOALLOC_MAX_VH odd
// FP64 spinors in the internal layout.  Every GPU the library runs on holds
// its own copy until the process ends.  In host code this name is only a
// stand-in: kernels and copies take the per-device address from
// hipGetSymbolAddress (noalloc_scratch_address), never the name itself.
static __device__ __align__(256) d2 scratch[12 * (size_t)FGI_NOALLOC_MAX_VH];

namespace {

std::mutex g_scratch_mu;
std::vector<d2*> g_scratch_addr;   // per device index; null until looked up

// The device address of `scratch` on `device`, which must be current: looked
// up once per device, then served from the table.
d2* noalloc_scratch_address(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_addr.size() <= device) g_scratch_addr.resize(device + 1, nullptr);
    if (!g_scratch_addr[device]) {
        void* ptr = nullptr;
        FGI_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw Error(FGI_EHIP, "hipGetSymbolAddress returned a null address for the scratch array");
        g_scratch_addr[device] = (d2*)ptr;
    }
    return g_scratch_addr[device];
}

template <typename F>
int guarded(F&& f) {
    try {
        f();
        return FGI_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return FGI_EHIP;
    } catch (...) {
        set_last_error("unknown failure");
        return FGI_EHIP;
    }
}

void need(const void* p, const char* what, size_t align) {
    if (!p) throw Error(FGI_EINVAL, std::string("null pointer: ") + what);
    if (((uintptr_t)p) % align) throw Error(FGI_EINVAL, std::string("misaligned pointer: ") + what);
}

Ctx& ctx_of(fgi_ctx* c) {
    if (!c) throw Error(FGI_EINVAL, "null context");
    FGI_HIP(hipSetDevice(c->c.device));
    return c->c;
}

struct StreamScope {
    Ctx& c;
    StreamScope(Ctx& cc, void* s) : c(cc) { c.stream = (hipStream_t)s; }
    ~StreamScope() { c.stream = nullptr; }
};

size_t gauge_bytes(const Geom& g) { return sizeof(d2) * 9 * 4 * (size_t)g.V; }
size_t mom_bytes(const Geom& g) { return sizeof(double) * 8 * 4 * (size_t)g.V; }
size_t spinor_bytes(const Geom& g) { return sizeof(d2) * 12 * (size_t)g.Vh; }
size_t sloppy_bytes(const Geom& g) { return sizeof(float) * 18 * 4 * (size_t)g.V; }

double sync_scalar(Ctx& c, const double* dev, int slot) {
    FGI_HIP(hipMemcpyAsync(c.host_scal + slot, dev, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    FGI_HIP(hipStreamSynchronize(c.stream));
    return c.host_scal[slot];
}

void check_action(const fgi_action* a) {
    if (!a) throw Error(FGI_EINVAL, "null action");
    if (a->prec < FGI_FP64 || a->prec > FGI_MP16) throw Error(FGI_EINVAL, "bad precision");
    if (a->link_recon != 18 && a->link_recon != 12) throw Error(FGI_EINVAL, "link_recon must be 18 or 12");
    if (a->kappa != 0 && (a->cg_tol <= 0 || a->cg_maxiter <= 0)) throw Error(FGI_EINVAL, "bad CG settings");
    if (a->kappa_hasen != 0 && (a->kappa == 0 || a->kappa_hasen >= a->kappa))
        throw Error(FGI_EINVAL, "Hasenbusch kappa' must satisfy 0 < kappa' < kappa");
    if (!std::isfinite(a->c1)) throw Error(FGI_EINVAL, "the rectangle coefficient c1 must be finite");
    if (!(a->cg_tol_md >= 0.0 && a->cg_tol_md < 1.0)) throw Error(FGI_EINVAL, "cg_tol_md must be in [0, 1)");
    if (a->stout_n < 0 || a->stout_n > 8) throw Error(FGI_EINVAL, "stout_n must be in [0, 8]");
    if (!(a->stout_rho >= 0.0 && a->stout_rho <= 0.5)) throw Error(FGI_EINVAL, "stout_rho must be in [0, 0.5]");
    if (!(a->csw >= 0.0 && a->csw <= 10.0)) throw Error(FGI_EINVAL, "csw must be in [0, 10]");
    if (a->csw != 0.0 && a->kappa != 0.0) {
        if (a->prec == FGI_MP16) throw Error(FGI_EINVAL, "the clover operator takes FGI_FP64 or FGI_MP32");
    }
}

int sloppy_prec(const fgi_action* a) { return a->prec == FGI_FP64 ? P64 : (a->prec == FGI_MP32 ? P32 : P16); }
int sloppy_recon(const fgi_action* a) { return a->link_recon; }

void accumulate_stats(fgi_stats* st, const CGResult& r) {
    if (!st) return;
    st->solves++;
    st->cg_iters += r.iters;
    if (r.iters > st->cg_iters_max) st->cg_iters_max = r.iters;
    st->reliable_updates += r.reliable_updates;
    if (r.rel_resid > st->max_rel_resid) st->max_rel_resid = r.rel_resid;
}

// --------------------------------------------------------------------------
// The state of one trajectory (or one single call) in internal layouts.
// --------------------------------------------------------------------------
struct Fields {
    Ctx& c;
    Geom g;
    fgi_action act;
    d2* U = nullptr;      // FP64 master links
    void* Us = nullptr;   // sloppy links (MP modes)
    d2* Ud = nullptr;     // displaced links of an FG stage
    void* Uds = nullptr;
    double* P = nullptr;
    double* F = nullptr;  // force scratch
    d2* phi[2] = {nullptr, nullptr};  // S_F (or S_1) and the Hasenbusch ratio term S_2
    d2* X = nullptr;      // solution of the S_F / S_1 solve
    d2* X2 = nullptr;     // solution of the S_2 solve
    d2* chi = nullptr;    // Mhat2^+ phi2
    int sp, rc;
    bool nonconv = false;
    fgi_stats* st = nullptr;

    Fields(Ctx& cc, const Geom& gg, const fgi_action& a) : c(cc), g(gg), act(a) {
        sp = sloppy_prec(&act);
        rc = sloppy_recon(&act);
    }

    FermionOp op64(const d2* u, double kappa) const { return FermionOp{&g, kappa, u, P64, 18}; }
    FermionOp ops(const d2* u, const void* us, double kappa) const {
        if (sp == P64) return op64(u, kappa);
        return FermionOp{&g, kappa, us, sp, rc};
    }

    // md: a solve inside a force evaluation (tolerance cg_tol_md when set);
    // the heatbath and action solves keep cg_tol
    // the clover term of the links u is built into c.cl_blk by every clover
    // solve, so the force that follows a solve finds A_ee, A_oo^-1 of its links
    bool clover() const { return act.csw != 0.0 && act.kappa != 0.0; }
    // slot 0 is the solves' buffer; slot 1 holds a second kappa's blocks
    // (the Hasenbusch kappa2 operator, or the log det at kappa) meanwhile
    d2* clover_at(const d2* u, double kappa, double* det = nullptr, int slot = 0) {
        d2* blk = (d2*)(slot ? c.cl_blk2 : c.cl_blk).get(sizeof(d2) * 72 * (size_t)g.V);
        clover_build(c, g, kappa, act.csw, u, blk, 1, det);
        return blk;
    }

    CGResult solve(const d2* u, const void* us, double kappa, const d2* rhs, d2* x, bool guess = false,
                   bool md = false) {
        const double tol = (md && act.cg_tol_md > 0.0) ? act.cg_tol_md : act.cg_tol;
        CGResult r;
        if (clover() && sp == P32)
            r = clover_cg_mp(c, op64(u, kappa), ops(u, us, kappa), clover_at(u, kappa), rhs, x, tol, act.cg_maxiter,
                             guess);
        else if (clover())
            r = clover_cg(c, op64(u, kappa), clover_at(u, kappa), rhs, x, tol, act.cg_maxiter, guess);
        else
            r = cg_solve(c, op64(u, kappa), ops(u, us, kappa), sp, rhs, x, tol, act.cg_maxiter, guess);
        accumulate_stats(st, r);
        if (!r.converged) nonconv = true;
        return r;
    }

    // The links the fermion operator sees at thin links u: u itself, or its
    // stout smearing (levels kept in c.stout_lev for the force's
    // back-propagation) with a sloppy copy when the solves need one
    struct FLinks {
        const d2* u;
        const void* us;
    };
    FLinks flinks(const d2* u, const void* us) {
        if (act.stout_n <= 0) return {u, us};
        d2* lev = (d2*)c.stout_lev.get(gauge_bytes(g) * act.stout_n);
        const d2* top = stout_smear(c, g, act.stout_rho, act.stout_n, u, lev);
        void* s = nullptr;
        if (sp != P64) {
            s = c.stout_sloppy.get(sloppy_bytes(g));
            make_sloppy(c, g, top, s, sp, rc);
        }
        return {top, s};
    }

    // out (+)= coef * F_terms(u); guess: the solves start from the solutions
    // held in X, X2 (those of the previous force evaluation).  With stout
    // smearing the pseudofermion forces are taken on the smeared links and
    // carried back to u.
    void force(const d2* u, const void* us, int terms, double* out, double coef, bool accumulate,
               bool guess = false) {
        bool have = accumulate;
        if (st) st->force_evals++;
        if (terms & FGI_TERM_GAUGE) {
            gauge_force(c, g, act.beta, u, out, coef, have ? 1 : 0, act.c1);
            have = true;
        }
        bool ferm = act.kappa != 0.0 && (terms & (FGI_TERM_FERMION | FGI_TERM_HASEN));
        if (!ferm) {
            if (!have) zero_mom(out);
            return;
        }
        if (!have) zero_mom(out);
        const bool smear = act.stout_n > 0;
        const FLinks fl = flinks(u, us);
        double* fo = out;
        double fc = coef;
        if (smear) {
            fo = (double*)c.stout_F.get(mom_bytes(g));
            zero_mom(fo);
            fc = 1.0;
        }
        const double k1 = act.kappa_hasen != 0.0 ? act.kappa_hasen : act.kappa;
        if (terms & FGI_TERM_FERMION) {
            solve(fl.u, fl.us, k1, phi[0], X, guess, true);
            if (clover()) {   // S_F (S_1 at kappa2) and the -2 log det A_oo term at kappa
                const bool split = act.kappa_hasen != 0.0;
                clover_force(c, op64(fl.u, k1), act.csw, (const d2*)c.cl_blk.get(sizeof(d2) * 72 * (size_t)g.V), X,
                             fo, fc, 1.0, split ? 0.0 : 1.0);
                if (split)
                    clover_force(c, op64(fl.u, act.kappa), act.csw, clover_at(fl.u, act.kappa, nullptr, 1), nullptr,
                                 fo, fc, 0.0, 1.0);
            } else
                fermion_force(c, op64(fl.u, k1), X, fo, fc);
        }
        if ((terms & FGI_TERM_HASEN) && act.kappa_hasen != 0.0) {
            // S_2 = chi^+ (Mhat^+ Mhat)^-1 chi, chi = Mhat2^+ phi2: the ordinary force
            // of X2 at kappa plus -kappa2^2 TA(U C(X2, phi2)) from the U dependence of chi
            hasen_solve(fl.u, fl.us, guess, true);
            if (clover()) {
                // hasen_solve left A(kappa) in slot 0 and A(kappa2) in slot 1
                clover_force(c, op64(fl.u, act.kappa), act.csw, (const d2*)c.cl_blk.get(sizeof(d2) * 72 * (size_t)g.V),
                             X2, fo, fc, 1.0, 0.0);
                clover_force(c, op64(fl.u, act.kappa_hasen), act.csw,
                             (const d2*)c.cl_blk2.get(sizeof(d2) * 72 * (size_t)g.V), X2, fo, fc, -1.0, 0.0, phi[1]);
            } else {
                fermion_force(c, op64(fl.u, act.kappa), X2, fo, fc);
                fermion_force_xy(c, op64(fl.u, act.kappa_hasen), X2, phi[1], fo,
                                 -fc * act.kappa_hasen * act.kappa_hasen);
            }
        }
        if (smear)
            stout_backprop(c, g, act.stout_rho, act.stout_n, u, (const d2*)c.stout_lev.get(gauge_bytes(g) * act.stout_n),
                           fo, out, coef, 1);
    }

    // J = J_V[F_terms](u) = d/dt F_terms(exp(t V) u) at t = 0: the gauge part
    // analytic, the pseudofermion part by the Section 4 Leibniz rule with one
    // more solve (for d_V X).  X must hold the S_F solve at u.
    // With Hasenbusch terms, X and X2 must hold the S_1 and S_2 solves at u
    // (those of the force evaluation just before).  The S_2 part: chi =
    // Mhat2^+ phi2 moves with u, so d_V X2 = A^-1 (d_V chi - (d_V A) X2) (one
    // solve), and its chi-dependent force term -kappa2^2 TA(U C(X2, phi2))
    // differentiates through X2 and the links.
    void force_tangent(const d2* u, const void* us, int terms, const double* Vd, double* J) {
        const bool ferm = act.kappa != 0.0 && (terms & (FGI_TERM_FERMION | FGI_TERM_HASEN));
        const bool hasen = act.kappa_hasen != 0.0;
        if (ferm && act.stout_n > 0)
            throw Error(FGI_EINVAL, "the exact force gradient is not available with stout smearing");
        if (ferm && clover()) throw Error(FGI_EINVAL, "the exact force gradient is not available with the clover term");
        if (terms & FGI_TERM_GAUGE) gauge_force_tangent(c, g, act.beta, u, Vd, J, 1.0, 0, 0, act.c1);
        else zero_mom(J);
        if (!ferm) return;
        d2* W = (d2*)c.gauge_tan.get(gauge_bytes(g));
        tangent_links(c, g, Vd, u, W);
        d2* rhs = (d2*)c.tg_rhs.get(spinor_bytes(g));
        d2* Z = (d2*)c.tg_z.get(spinor_bytes(g));
        if (terms & FGI_TERM_FERMION) {
            const double k1 = hasen ? act.kappa_hasen : act.kappa;
            const FermionOp o64 = op64(u, k1), oW = op64(W, k1);
            fermion_tangent_rhs(c, o64, oW, X, rhs);
            solve(u, us, k1, rhs, Z, false, true);
            fermion_force_tangent(c, o64, oW, Vd, X, Z, J, 1.0);
        }
        if ((terms & FGI_TERM_HASEN) && hasen) {
            const FermionOp o64 = op64(u, act.kappa), oW = op64(W, act.kappa);
            const FermionOp o2 = op64(u, act.kappa_hasen), oW2 = op64(W, act.kappa_hasen);
            d2* dchi = (d2*)c.hs_dchi.get(spinor_bytes(g));
            dmhat_dag_apply(c, o2, oW2, phi[1], dchi);
            fermion_tangent_rhs(c, o64, oW, X2, rhs);
            spinor_lincomb(c, g, 1.0, rhs, 1.0, dchi, 0, rhs);
            solve(u, us, act.kappa, rhs, Z, false, true);
            fermion_force_tangent(c, o64, oW, Vd, X2, Z, J, 1.0);
            fermion_force_xy_tangent(c, o2, oW2, Vd, X2, phi[1], Z, J, -act.kappa_hasen * act.kappa_hasen);
        }
    }

    // chi = Mhat2^+ phi2 at u; X2 = (Mhat^+ Mhat)^-1 chi
    void hasen_solve(const d2* u, const void* us, bool guess = false, bool md = false) {
        d2* t = (d2*)c.tmp_o.get(spinor_bytes(g));
        if (clover())
            clover_mhat(c, op64(u, act.kappa_hasen), clover_at(u, act.kappa_hasen, nullptr, 1), phi[1], chi, 1);
        else
            mhat(c, op64(u, act.kappa_hasen), P64, SpinorPtr{phi[1], nullptr}, SpinorPtr{t, nullptr},
                 SpinorPtr{chi, nullptr}, 1);
        solve(u, us, act.kappa, chi, X2, guess, md);
    }

    // phi2 = Mhat2 (Mhat2^+ Mhat2)^-1 Mhat^+ eta2 at the fermion links of u
    // (one solve at kappa2)
    void hasen_heatbath(const d2* thin, const void* thin_s, const d2* eta2) {
        const FLinks fl = flinks(thin, thin_s);
        const d2* u = fl.u;
        const void* us = fl.us;
        d2* t = (d2*)c.tmp_o.get(spinor_bytes(g));
        if (clover()) {
            clover_mhat(c, op64(u, act.kappa), clover_at(u, act.kappa, nullptr, 1), eta2, chi, 1);
            solve(u, us, act.kappa_hasen, chi, X2);   // leaves A(kappa2) in slot 0
            clover_mhat(c, op64(u, act.kappa_hasen), (const d2*)c.cl_blk.get(sizeof(d2) * 72 * (size_t)g.V), X2,
                        phi[1], 0);
            return;
        }
        mhat(c, op64(u, act.kappa), P64, SpinorPtr{(void*)eta2, nullptr}, SpinorPtr{t, nullptr},
             SpinorPtr{chi, nullptr}, 1);
        solve(u, us, act.kappa_hasen, chi, X2);
        mhat(c, op64(u, act.kappa_hasen), P64, SpinorPtr{X2, nullptr}, SpinorPtr{t, nullptr},
             SpinorPtr{phi[1], nullptr}, 0);
    }

    // sum over the pseudofermion terms of Re phi^+ X - |eta|^2 (eta may be null):
    // the fermion part of H at the fermion links of u minus its heatbath value
    double pf_energy(const d2* thin, const void* thin_s, const d2* eta1, const d2* eta2, double* part,
                     double* scal) {
        const FLinks fl = flinks(thin, thin_s);
        const d2* u = fl.u;
        const void* us = fl.us;
        const double k1 = act.kappa_hasen != 0.0 ? act.kappa_hasen : act.kappa;
        solve(u, us, k1, phi[0], X);
        int nb = pf_density_partials(c, g, phi[0], X, eta1, part);
        final_sum(c, part, nb, scal + 4);
        double e = sync_scalar(c, scal + 4, 4);
        if (clover()) {   // -2 sum_{x odd} log det A(x) at kappa is part of H
            double det = 0.0;
            clover_at(u, act.kappa, &det, 1);
            e += det;
        }
        if (act.kappa_hasen != 0.0) {
            hasen_solve(u, us);
            nb = pf_density_partials(c, g, chi, X2, eta2, part);
            final_sum(c, part, nb, scal + 5);
            e += sync_scalar(c, scal + 5, 5);
        }
        return e;
    }

    void zero_mom(double* out) { zero_doubles(c, out, mom_bytes(g) / sizeof(double)); }
};

}  // namespace

// ==========================================================================
extern "C" {

const char* fgi_last_error(void) { return fgi::g_last_error.c_str(); }

int fgi_create(fgi_ctx** out, int device) {
    return guarded([&] {
        if (!out) throw Error(FGI_EINVAL, "null output");
        int n = 0;
        FGI_HIP(hipGetDeviceCount(&n));
        if (device < 0 || device >= n) throw Error(FGI_EINVAL, "bad device index");
        FGI_HIP(hipSetDevice(device));
        d2* scr = noalloc_scratch_address(device);
        fgi_ctx* c = new fgi_ctx();
        c->c.device = device;
        c->c.noalloc_scratch = scr;
        FGI_HIP(hipHostMalloc((void**)&c->c.host_scal, 64 * sizeof(double), hipHostMallocDefault));
        FGI_HIP(hipHostMalloc((void**)&c->c.host_state, sizeof(CGState), hipHostMallocDefault));
        void* st = c->c.state.get(sizeof(CGState));
        FGI_HIP(hipMemset(st, 0, sizeof(CGState)));
        FGI_HIP(hipDeviceSynchronize());
        *out = c;
    });
}

int fgi_destroy(fgi_ctx* ctx) {
    return guarded([&] {
        if (!ctx) throw Error(FGI_EINVAL, "null context");
        Ctx& c = ctx->c;
        FGI_HIP(hipSetDevice(c.device));
        FGI_HIP(hipDeviceSynchronize());
        DevBuf* bufs[] = {&c.gauge, &c.gauge_disp, &c.sloppy, &c.sloppy_disp, &c.mom, &c.force, &c.force2,
                          &c.scratch_mom, &c.eta, &c.phi, &c.X, &c.Xo, &c.Ye, &c.Yo, &c.tmp_e, &c.tmp_o,
                          &c.cg_r, &c.cg_p, &c.cg_q, &c.s_x, &c.s_r, &c.s_p, &c.s_q, &c.s_t, &c.s_norms,
                          &c.s_pf, &c.s_sf, &c.s_rt,
                          &c.h0, &c.hf0, &c.partial, &c.scal, &c.state, &c.phi2, &c.eta2, &c.user_tmp,
                          &c.chi, &c.X2, &c.cdesc, &c.bstate, &c.bscal, &c.bh0, &c.bh1, &c.bres,
                          &c.gauge_tan, &c.tg_dmx, &c.tg_rhs, &c.tg_z, &c.tg_dxo, &c.tg_dye, &c.tg_dyo,
                          &c.force3, &c.chain_U, &c.stout_lev, &c.stout_F, &c.stout_ga, &c.stout_gb,
                          &c.stout_part, &c.stout_M, &c.stout_sloppy, &c.hs_dchi, &c.hs_xo, &c.hs_yo,
                          &c.hs_dxo, &c.hs_dyo, &c.hs_zero, &c.hs_t1, &c.cl_sig, &c.cl_blk, &c.cl_blk2,
                          &c.cl_blk32, &c.cl_s32, &c.cl_fh,
                          &c.cl_ld, &c.cl_to, &c.cl_te, &c.cl_ue, &c.cl_r, &c.cl_p, &c.cl_ap, &c.cl_t,
                          &c.cl_ye, &c.cl_xo, &c.cl_yo, &c.br_jp, &c.br_jf, &c.br_jj, &c.halo_a, &c.halo_b};
        for (DevBuf* b : bufs) b->release();
        for (hipEvent_t e : c.ev_pool) hipEventDestroy(e);
        for (GraphEntry& e : c.graphs) hipGraphExecDestroy(e.exec);
        if (c.cap_stream) hipStreamDestroy(c.cap_stream);
        if (c.host_scal) hipHostFree(c.host_scal);
        if (c.host_state) hipHostFree(c.host_state);
        if (c.host_bstates) hipHostFree(c.host_bstates);
        if (c.host_bscal) hipHostFree(c.host_bscal);
        delete ctx;
    });
}

int fgi_set_option(fgi_ctx* ctx, const char* name, double value) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!name) throw Error(FGI_EINVAL, "null option name");
        std::string n(name);
        if (n == "cg_batch") {
            if (value < 1 || value > 1024) throw Error(FGI_EINVAL, "cg_batch out of range");
            c.cg_batch = (int)value;
        } else if (n == "ru_delta") {
            if (!(value > 0 && value < 1)) throw Error(FGI_EINVAL, "ru_delta must be in (0,1)");
            c.ru_delta = value;
        } else if (n == "dslash_block") {
            if (!(value == 64 || value == 128 || value == 256))
                throw Error(FGI_EINVAL, "dslash_block must be 64, 128 or 256");
            c.ds_bs = (int)value;
        } else if (n == "xcd_order") {
            c.ds_xcd = value != 0;
        } else if (n == "fg_start") {
            c.fg_start = value != 0;
        } else if (n == "cg_form") {
            if (!(value == 0 || value == 1)) throw Error(FGI_EINVAL, "cg_form must be 0 or 1");
            c.cg_form = (int)value;
        } else if (n == "graphs") {
            c.use_graphs = value != 0;
        } else if (n == "profile") {
            c.profile = value != 0;
        } else if (n == "profile_prec") {
            if (value < -1 || value > 2) throw Error(FGI_EINVAL, "profile_prec must be -1, 0, 1 or 2");
            c.profile_prec = (int)value;
        } else if (n == "profile_reset") {
            c.dslash_ms = 0;
            c.dslash_launches = 0;
            c.dslash_sites = 0;
        } else {
            throw Error(FGI_EINVAL, "unknown option " + n);
        }
    });
}

int fgi_get_profile(fgi_ctx* ctx, double* ms, long* launches, long* sites) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (ms) *ms = c.dslash_ms;
        if (launches) *launches = c.dslash_launches;
        if (sites) *sites = c.dslash_sites;
    });
}

int fgi_gauge_action(fgi_ctx* ctx, const fgi_geom* gg, double beta, const void* U, double* S, void* stream) {
    return fgi_improved_gauge_action(ctx, gg, beta, 0.0, U, S, stream);
}

int fgi_improved_gauge_action(fgi_ctx* ctx, const fgi_geom* gg, double beta, double c1, const void* U, double* S,
                              void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg || !S) throw Error(FGI_EINVAL, "null argument");
        if (!std::isfinite(c1)) throw Error(FGI_EINVAL, "the rectangle coefficient c1 must be finite");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        StreamScope ss(c, stream);
        d2* u = (d2*)c.gauge.get(gauge_bytes(g));
        pack_gauge(c, g, U, u);
        double* h = (double*)c.h0.get(sizeof(double) * g.V);
        ham_density(c, g, beta, u, nullptr, h, c1);
        double* part = partial_buf(c, g);
        double* scal = (double*)c.scal.get(sizeof(double) * 64);
        int nb = diff_partials(c, g.V, h, nullptr, part);
        final_sum(c, part, nb, scal);
        *S = sync_scalar(c, scal, 0);
    });
}

int fgi_kinetic(fgi_ctx* ctx, const fgi_geom* gg, const void* P, double* T, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg || !T) throw Error(FGI_EINVAL, "null argument");
        Geom g = make_geom(gg->dims);
        need(P, "P", 8);
        StreamScope ss(c, stream);
        double* pm = (double*)c.mom.get(mom_bytes(g));
        pack_mom(c, g, (const double*)P, pm);
        double* h = (double*)c.h0.get(sizeof(double) * g.V);
        ham_density(c, g, 0.0, nullptr, pm, h);
        double* part = partial_buf(c, g);
        double* scal = (double*)c.scal.get(sizeof(double) * 64);
        int nb = diff_partials(c, g.V, h, nullptr, part);
        final_sum(c, part, nb, scal);
        *T = sync_scalar(c, scal, 0);
    });
}

int fgi_gauge_force(fgi_ctx* ctx, const fgi_geom* gg, double beta, const void* U, void* F, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(F, "F", 8);
        StreamScope ss(c, stream);
        d2* u = (d2*)c.gauge.get(gauge_bytes(g));
        double* f = (double*)c.force.get(mom_bytes(g));
        pack_gauge(c, g, U, u);
        gauge_force(c, g, beta, u, f, 1.0, 0);
        unpack_mom(c, g, f, (double*)F);
    });
}

int fgi_stout_smear(fgi_ctx* ctx, const fgi_geom* gg, double rho, int n, const void* U, void* Us, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        if (n < 0 || n > 8 || !(rho >= 0.0 && rho <= 0.5)) throw Error(FGI_EINVAL, "need 0 <= n <= 8, 0 <= rho <= 0.5");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(Us, "Us", 16);
        StreamScope ss(c, stream);
        d2* u = (d2*)c.gauge.get(gauge_bytes(g));
        pack_gauge(c, g, U, u);
        if (n == 0) {
            unpack_gauge(c, g, u, Us);
            return;
        }
        d2* lev = (d2*)c.stout_lev.get(gauge_bytes(g) * n);
        unpack_gauge(c, g, stout_smear(c, g, rho, n, u, lev), Us);
    });
}

int fgi_stout_force(fgi_ctx* ctx, const fgi_geom* gg, double rho, int n, const void* U, const void* Fs, void* F,
                    void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        if (n < 0 || n > 8 || !(rho >= 0.0 && rho <= 0.5)) throw Error(FGI_EINVAL, "need 0 <= n <= 8, 0 <= rho <= 0.5");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(Fs, "Fs", 8);
        need(F, "F", 8);
        StreamScope ss(c, stream);
        d2* u = (d2*)c.gauge.get(gauge_bytes(g));
        double* fs = (double*)c.force2.get(mom_bytes(g));
        double* f = (double*)c.force.get(mom_bytes(g));
        pack_gauge(c, g, U, u);
        pack_mom(c, g, (const double*)Fs, fs);
        if (n == 0) {
            unpack_mom(c, g, fs, (double*)F);
            return;
        }
        d2* lev = (d2*)c.stout_lev.get(gauge_bytes(g) * n);
        stout_smear(c, g, rho, n, u, lev);
        stout_backprop(c, g, rho, n, u, lev, fs, f, 1.0, 0);
        unpack_mom(c, g, f, (double*)F);
    });
}

int fgi_force_gradient(fgi_ctx* ctx, const fgi_geom* gg, double beta, const void* U, const void* Vd, void* J,
                       void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(Vd, "V", 8);
        need(J, "J", 8);
        StreamScope ss(c, stream);
        d2* u = (d2*)c.gauge.get(gauge_bytes(g));
        double* v = (double*)c.force2.get(mom_bytes(g));
        double* j = (double*)c.force.get(mom_bytes(g));
        pack_gauge(c, g, U, u);
        pack_mom(c, g, (const double*)Vd, v);
        gauge_force_tangent(c, g, beta, u, v, j, 1.0, 0);
        unpack_mom(c, g, j, (double*)J);
    });
}

int fgi_gauge_hvp(fgi_ctx* ctx, const fgi_geom* gg, double beta, const void* U, const void* Vd, void* HV,
                  void* stream) {
    return fgi_improved_gauge_hvp(ctx, gg, beta, 0.0, U, Vd, HV, stream);
}

int fgi_improved_gauge_hvp(fgi_ctx* ctx, const fgi_geom* gg, double beta, double c1, const void* U, const void* Vd,
                           void* HV, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        if (!std::isfinite(c1)) throw Error(FGI_EINVAL, "the rectangle coefficient c1 must be finite");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(Vd, "V", 8);
        need(HV, "HV", 8);
        StreamScope ss(c, stream);
        d2* u = (d2*)c.gauge.get(gauge_bytes(g));
        double* v = (double*)c.force2.get(mom_bytes(g));
        double* j = (double*)c.force.get(mom_bytes(g));
        pack_gauge(c, g, U, u);
        pack_mom(c, g, (const double*)Vd, v);
        gauge_force_tangent(c, g, beta, u, v, j, 1.0, 0, 1, c1);
        unpack_mom(c, g, j, (double*)HV);
    });
}

int fgi_link_update(fgi_ctx* ctx, const fgi_geom* gg, double h, const void* P, void* U, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(P, "P", 8);
        StreamScope ss(c, stream);
        d2* u = (d2*)c.gauge.get(gauge_bytes(g));
        double* pm = (double*)c.mom.get(mom_bytes(g));
        pack_gauge(c, g, U, u);
        pack_mom(c, g, (const double*)P, pm);
        link_update(c, g, h, pm, u, u, nullptr, P64, 18);
        unpack_gauge(c, g, u, U);
    });
}

int fgi_reunitarize(fgi_ctx* ctx, const fgi_geom* gg, void* U, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        StreamScope ss(c, stream);
        d2* u = (d2*)c.gauge.get(gauge_bytes(g));
        pack_gauge(c, g, U, u);
        reunitarize(c, g, u);
        unpack_gauge(c, g, u, U);
    });
}

int fgi_exp_su3(fgi_ctx* ctx, int n, const void* p, double h, void* out, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (n < 0) throw Error(FGI_EINVAL, "negative count");
        if (n == 0) return;
        need(p, "p", 8);
        need(out, "out", 16);
        StreamScope ss(c, stream);
        exp_su3_batch(c, n, (const double*)p, h, out);
    });
}

int fgi_dslash(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* in, void* out,
               int out_parity, int prec, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        check_action(act);
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(in, "in", 16);
        need(out, "out", 16);
        if (out_parity != 0 && out_parity != 1) throw Error(FGI_EINVAL, "parity must be 0 or 1");
        if (prec < FGI_FP64 || prec > FGI_MP16) throw Error(FGI_EINVAL, "bad precision");
        StreamScope ss(c, stream);
        fgi_action a = *act;
        a.prec = prec;
        Fields f(c, g, a);
        d2* u = (d2*)c.gauge.get(gauge_bytes(g));
        pack_gauge(c, g, U, u);
        d2* vin = (d2*)c.tmp_e.get(spinor_bytes(g));
        d2* vout = (d2*)c.X.get(spinor_bytes(g));
        pack_even_spinor(c, g, in, vin);  // same layout for either parity
        FermionOp op = f.op64(u, a.kappa);
        if (f.sp == P64) {
            dslash(c, op, out_parity, P64, SpinorPtr{vin, nullptr}, P64, SpinorPtr{vout, nullptr});
        } else {
            void* us = c.sloppy.get(sloppy_bytes(g));
            make_sloppy(c, g, u, us, f.sp, f.rc);
            FermionOp os = f.ops(u, us, a.kappa);
            size_t nb = sizeof(float) * 24 * (size_t)g.Vh;
            float* norms = (float*)c.s_norms.get(sizeof(float) * 3 * (size_t)g.Vh);
            SpinorPtr si{c.s_p.get(nb), norms}, so{c.s_q.get(nb), norms + g.Vh};
            convert_spinor(c, g, P64, SpinorPtr{vin, nullptr}, f.sp, si);
            dslash(c, os, out_parity, f.sp, si, f.sp, so);
            convert_spinor(c, g, f.sp, so, P64, SpinorPtr{vout, nullptr});
        }
        unpack_even_spinor(c, g, vout, out);
    });
}

// ------------------------------------------ t-decomposed hopping term ---
namespace {
Geom halo_geom(const fgi_geom* gg) {
    if (!gg) throw Error(FGI_EINVAL, "null geometry");
    Geom g = make_geom(gg->dims);
    if (g.L[3] < 2) throw Error(FGI_EINVAL, "the local t extent must be at least 2");
    return g;
}

// the sloppy (or FP64) operator and the input converted to it, for one halo call
struct HaloOp {
    FermionOp op;
    SpinorPtr in;
    int prec;
};

HaloOp halo_setup(Ctx& c, const Geom& g, const fgi_action* act, const void* U, const void* in, int prec) {
    fgi_action a = *act;
    a.prec = prec;
    const int sp = sloppy_prec(&a), rc = sloppy_recon(&a);
    d2* u = (d2*)c.gauge.get(gauge_bytes(g));
    pack_gauge(c, g, U, u);
    d2* vin = (d2*)c.tmp_e.get(spinor_bytes(g));
    pack_even_spinor(c, g, in, vin);  // same layout for either parity
    if (sp == P64) return HaloOp{FermionOp{nullptr, a.kappa, u, P64, 18}, SpinorPtr{vin, nullptr}, P64};
    void* us = c.sloppy.get(sloppy_bytes(g));
    make_sloppy(c, g, u, us, sp, rc);
    const size_t nb = sizeof(float) * 24 * (size_t)g.Vh;
    float* norms = (float*)c.s_norms.get(sizeof(float) * 3 * (size_t)g.Vh);
    SpinorPtr si{c.s_p.get(nb), norms};
    convert_spinor(c, g, P64, SpinorPtr{vin, nullptr}, sp, si);
    return HaloOp{FermionOp{nullptr, a.kappa, us, sp, rc}, si, sp};
}

void halo_checks(const fgi_action* act, const void* U, const void* in, int prec) {
    check_action(act);
    need(U, "U", 16);
    need(in, "in", 16);
    if (prec < FGI_FP64 || prec > FGI_MP16) throw Error(FGI_EINVAL, "bad precision");
}
}  // namespace

int fgi_halo_bytes(const fgi_geom* gg, int prec, size_t* bytes) {
    return guarded([&] {
        Geom g = halo_geom(gg);
        if (prec < FGI_FP64 || prec > FGI_MP16) throw Error(FGI_EINVAL, "bad precision");
        if (!bytes) throw Error(FGI_EINVAL, "null bytes");
        *bytes = halo_bytes(g, prec == FGI_FP64 ? P64 : P32);
    });
}

int fgi_halo_pack(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* in,
                  int in_parity, double sign_lo, double sign_hi, void* to_lo, void* to_hi, int prec, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        Geom g = halo_geom(gg);
        halo_checks(act, U, in, prec);
        const size_t hal = prec == FGI_FP64 ? 16 : 8;  // one complex number of the working precision
        need(to_lo, "to_lo", hal);
        need(to_hi, "to_hi", hal);
        if (to_lo == to_hi) throw Error(FGI_EINVAL, "to_lo and to_hi must be different buffers");
        if (in_parity != 0 && in_parity != 1) throw Error(FGI_EINVAL, "parity must be 0 or 1");
        if (!((sign_lo == 1.0 || sign_lo == -1.0) && (sign_hi == 1.0 || sign_hi == -1.0)))
            throw Error(FGI_EINVAL, "face signs must be +1 or -1");
        StreamScope ss(c, stream);
        HaloOp h = halo_setup(c, g, act, U, in, prec);
        h.op.g = &g;
        halo_pack(c, h.op, h.prec, in_parity, h.in, sign_lo, sign_hi, to_lo, to_hi);
    });
}

int fgi_dslash_halo(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* in,
                    void* out, int out_parity, const void* from_lo, const void* from_hi, int split, int prec,
                    void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        Geom g = halo_geom(gg);
        halo_checks(act, U, in, prec);
        need(out, "out", 16);
        const size_t hal = prec == FGI_FP64 ? 16 : 8;
        need(from_lo, "from_lo", hal);
        need(from_hi, "from_hi", hal);
        if (out_parity != 0 && out_parity != 1) throw Error(FGI_EINVAL, "parity must be 0 or 1");
        if (split != 0 && split != 1) throw Error(FGI_EINVAL, "split must be 0 or 1");
        StreamScope ss(c, stream);
        HaloOp h = halo_setup(c, g, act, U, in, prec);
        h.op.g = &g;
        d2* vout = (d2*)c.X.get(spinor_bytes(g));
        if (h.prec == P64) {
            SpinorPtr so{vout, nullptr};
            if (split) {
                dslash_halo(c, h.op, P64, out_parity, h.in, so, from_lo, from_hi, 1);
                dslash_halo(c, h.op, P64, out_parity, h.in, so, from_lo, from_hi, 2);
            } else {
                dslash_halo(c, h.op, P64, out_parity, h.in, so, from_lo, from_hi, 0);
            }
        } else {
            const size_t nb = sizeof(float) * 24 * (size_t)g.Vh;
            float* norms = (float*)c.s_norms.get(sizeof(float) * 3 * (size_t)g.Vh);
            SpinorPtr so{c.s_q.get(nb), norms + g.Vh};
            if (split) {
                dslash_halo(c, h.op, h.prec, out_parity, h.in, so, from_lo, from_hi, 1);
                dslash_halo(c, h.op, h.prec, out_parity, h.in, so, from_lo, from_hi, 2);
            } else {
                dslash_halo(c, h.op, h.prec, out_parity, h.in, so, from_lo, from_hi, 0);
            }
            convert_spinor(c, g, h.prec, so, P64, SpinorPtr{vout, nullptr});
        }
        unpack_even_spinor(c, g, vout, out);
    });
}

int fgi_halo_time(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* in,
                  int reps, fgi_halo_timing* out, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        Geom g = halo_geom(gg);
        halo_checks(act, U, in, act ? act->prec : FGI_FP64);
        if (!out) throw Error(FGI_EINVAL, "null output");
        if (reps < 1 || reps > 100000) throw Error(FGI_EINVAL, "reps must be in [1, 100000]");
        StreamScope ss(c, stream);
        HaloOp h = halo_setup(c, g, act, U, in, act->prec);
        h.op.g = &g;
        const size_t hb = halo_bytes(g, h.prec == P64 ? P64 : P32);
        void* ha = c.halo_a.get(hb);
        void* hb_ = c.halo_b.get(hb);
        SpinorPtr so;
        if (h.prec == P64) {
            so = SpinorPtr{c.X.get(spinor_bytes(g)), nullptr};
        } else {
            const size_t nb = sizeof(float) * 24 * (size_t)g.Vh;
            float* norms = (float*)c.s_norms.get(sizeof(float) * 3 * (size_t)g.Vh);
            so = SpinorPtr{c.s_q.get(nb), norms + g.Vh};
        }
        // one rank holding the whole t ring: its faces are its own neighbours
        halo_pack(c, h.op, h.prec, 0, h.in, -1.0, -1.0, ha, hb_);
        hipEvent_t e0, e1;
        FGI_HIP(hipEventCreate(&e0));
        FGI_HIP(hipEventCreate(&e1));
        auto timed = [&](auto body) {
            body();  // untimed first launch
            FGI_HIP(hipEventRecord(e0, c.stream));
            for (int k = 0; k < reps; k++) body();
            FGI_HIP(hipEventRecord(e1, c.stream));
            FGI_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            FGI_HIP(hipEventElapsedTime(&ms, e0, e1));
            return 1e3 * ms / reps;
        };
        fgi_halo_timing t{};
        t.pack_us = timed([&] { halo_pack(c, h.op, h.prec, 0, h.in, -1.0, -1.0, ha, hb_); });
        t.interior_us = timed([&] { dslash_halo(c, h.op, h.prec, 1, h.in, so, hb_, ha, 1); });
        t.faces_us = timed([&] { dslash_halo(c, h.op, h.prec, 1, h.in, so, hb_, ha, 2); });
        t.all_us = timed([&] { dslash_halo(c, h.op, h.prec, 1, h.in, so, hb_, ha, 0); });
        t.local_us = timed([&] { dslash(c, h.op, 1, h.prec, h.in, h.prec, so); });
        t.face_sites = g.Vh / g.L[3];
        t.halo_bytes = (long)hb;
        FGI_HIP(hipEventDestroy(e0));
        FGI_HIP(hipEventDestroy(e1));
        *out = t;
    });
}

int fgi_mhat(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* in, void* out,
             int dagger, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        check_action(act);
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(in, "in", 16);
        need(out, "out", 16);
        StreamScope ss(c, stream);
        d2* u = (d2*)c.gauge.get(gauge_bytes(g));
        pack_gauge(c, g, U, u);
        d2* vin = (d2*)c.tmp_e.get(spinor_bytes(g));
        d2* vout = (d2*)c.X.get(spinor_bytes(g));
        d2* t = (d2*)c.Xo.get(spinor_bytes(g));
        pack_even_spinor(c, g, in, vin);
        FermionOp op{&g, act->kappa, u, P64, 18};
        if (act->csw != 0.0 && act->kappa != 0.0) {
            d2* blk = (d2*)c.cl_blk.get(sizeof(d2) * 72 * (size_t)g.V);
            clover_build(c, g, act->kappa, act->csw, u, blk, 1, nullptr);
            clover_mhat(c, op, blk, vin, vout, dagger ? 1 : 0);
        } else {
            mhat(c, op, P64, SpinorPtr{vin, nullptr}, SpinorPtr{t, nullptr}, SpinorPtr{vout, nullptr},
                 dagger ? 1 : 0);
        }
        unpack_even_spinor(c, g, vout, out);
    });
}

int fgi_mhat_packed_noalloc(fgi_ctx* ctx, const fgi_geom* gg, double kappa, const void* U, const void* in, void* out,
                            int dagger, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        Geom g = make_geom(gg->dims);
        if (g.Vh > FGI_NOALLOC_MAX_VH)
            throw Error(FGI_EINVAL, "fgi_mhat_packed_noalloc: V/2 = " + std::to_string(g.Vh) +
                                        " odd sites exceed the fixed scratch of FGI_NOALLOC_MAX_VH = " +
                                        std::to_string(FGI_NOALLOC_MAX_VH));
        if (!std::isfinite(kappa)) throw Error(FGI_EINVAL, "kappa must be finite");
        need(U, "U", 16);
        need(in, "in", 16);
        need(out, "out", 16);
        const uintptr_t nb = spinor_bytes(g), a0 = (uintptr_t)in, b0 = (uintptr_t)out;
        if (a0 < b0 + nb && b0 < a0 + nb) throw Error(FGI_EINVAL, "in and out must not overlap");
        if (!c.noalloc_scratch) throw Error(FGI_EHIP, "the scratch array has no device address");
        StreamScope ss(c, stream);
        FermionOp op{&g, kappa, U, P64, 18};
        mhat(c, op, P64, SpinorPtr{(void*)in, nullptr}, SpinorPtr{c.noalloc_scratch, nullptr}, SpinorPtr{out, nullptr},
             dagger ? 1 : 0);
    });
}

int fgi_pf_heatbath(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* eta,
                    void* phi, void* stream) {
    return fgi_mhat(ctx, gg, act, U, eta, phi, 1, stream);
}

int fgi_cg_solve(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* phi, void* X,
                 fgi_stats* st, void* stream) {
    int rc = guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        check_action(act);
        if (act->kappa == 0) throw Error(FGI_EINVAL, "kappa must be nonzero");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(phi, "phi", 16);
        need(X, "X", 16);
        auto t0 = std::chrono::steady_clock::now();
        const long cap0 = c.graph_captures;
        StreamScope ss(c, stream);
        Fields f(c, g, *act);
        f.st = st;
        f.U = (d2*)c.gauge.get(gauge_bytes(g));
        pack_gauge(c, g, U, f.U);
        if (f.sp != P64) {
            f.Us = c.sloppy.get(sloppy_bytes(g));
            make_sloppy(c, g, f.U, f.Us, f.sp, f.rc);
        }
        d2* ph = (d2*)c.phi.get(spinor_bytes(g));
        d2* x = (d2*)c.X.get(spinor_bytes(g));
        pack_even_spinor(c, g, phi, ph);
        f.solve(f.U, f.Us, act->kappa, ph, x);
        unpack_even_spinor(c, g, x, X);
        FGI_HIP(hipStreamSynchronize(c.stream));
        if (st) {
            st->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            st->graph_captures += c.graph_captures - cap0;
        }
        if (f.nonconv) throw Error(FGI_ENOCONV, "CG reached cg_maxiter");
    });
    return rc;
}

int fgi_pf_action(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* phi,
                  double* SF, fgi_stats* st, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg || !SF) throw Error(FGI_EINVAL, "null argument");
        check_action(act);
        if (act->kappa == 0) throw Error(FGI_EINVAL, "kappa must be nonzero");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(phi, "phi", 16);
        StreamScope ss(c, stream);
        Fields f(c, g, *act);
        f.st = st;
        f.U = (d2*)c.gauge.get(gauge_bytes(g));
        pack_gauge(c, g, U, f.U);
        if (f.sp != P64) {
            f.Us = c.sloppy.get(sloppy_bytes(g));
            make_sloppy(c, g, f.U, f.Us, f.sp, f.rc);
        }
        d2* ph = (d2*)c.phi.get(spinor_bytes(g));
        d2* x = (d2*)c.X.get(spinor_bytes(g));
        pack_even_spinor(c, g, phi, ph);
        f.solve(f.U, f.Us, act->kappa, ph, x);
        double* part = partial_buf(c, g);
        double* scal = (double*)c.scal.get(sizeof(double) * 64);
        int nb = pf_density_partials(c, g, ph, x, nullptr, part);
        final_sum(c, part, nb, scal);
        *SF = sync_scalar(c, scal, 0);
        if (f.nonconv) throw Error(FGI_ENOCONV, "CG reached cg_maxiter");
    });
}

int fgi_force(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* phi, void* F,
              fgi_stats* st, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        check_action(act);
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(F, "F", 8);
        bool ferm = act->kappa != 0 && phi;
        if (ferm) need(phi, "phi", 16);
        StreamScope ss(c, stream);
        fgi_action a = *act;
        if (!ferm) a.kappa = 0;
        Fields f(c, g, a);
        f.st = st;
        f.U = (d2*)c.gauge.get(gauge_bytes(g));
        pack_gauge(c, g, U, f.U);
        if (ferm && f.sp != P64) {
            f.Us = c.sloppy.get(sloppy_bytes(g));
            make_sloppy(c, g, f.U, f.Us, f.sp, f.rc);
        }
        if (ferm) {
            f.phi[0] = (d2*)c.phi.get(spinor_bytes(g));
            pack_even_spinor(c, g, phi, f.phi[0]);
            f.X = (d2*)c.X.get(spinor_bytes(g));
        }
        double* fm = (double*)c.force.get(mom_bytes(g));
        f.force(f.U, f.Us, FGI_TERM_GAUGE | FGI_TERM_FERMION, fm, 1.0, false);
        unpack_mom(c, g, fm, (double*)F);
        FGI_HIP(hipStreamSynchronize(c.stream));
        if (f.nonconv) throw Error(FGI_ENOCONV, "CG reached cg_maxiter");
    });
}

int fgi_total_force_gradient(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U,
                             const void* phi, const void* Vd, void* J, fgi_stats* st, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        check_action(act);
        if (act->kappa_hasen != 0)
            throw Error(FGI_EINVAL, "this call takes one pseudofermion: no Hasenbusch terms (trajectories with "
                                    "fg_exact take them)");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(J, "J", 8);
        if (Vd) need(Vd, "V", 8);
        const bool ferm = act->kappa != 0 && phi;
        if (ferm) need(phi, "phi", 16);
        StreamScope ss(c, stream);
        fgi_action a = *act;
        if (!ferm) a.kappa = 0;
        Fields f(c, g, a);
        f.st = st;
        f.U = (d2*)c.gauge.get(gauge_bytes(g));
        pack_gauge(c, g, U, f.U);
        if (ferm && f.sp != P64) {
            f.Us = c.sloppy.get(sloppy_bytes(g));
            make_sloppy(c, g, f.U, f.Us, f.sp, f.rc);
        }
        if (ferm) {
            f.phi[0] = (d2*)c.phi.get(spinor_bytes(g));
            pack_even_spinor(c, g, phi, f.phi[0]);
            f.X = (d2*)c.X.get(spinor_bytes(g));
        }
        const int terms = FGI_TERM_GAUGE | FGI_TERM_FERMION;
        double* fm = (double*)c.force.get(mom_bytes(g));
        double* v = fm;
        f.force(f.U, f.Us, terms, fm, 1.0, false);   // F(U), and X at U
        if (Vd) {
            v = (double*)c.force2.get(mom_bytes(g));
            pack_mom(c, g, (const double*)Vd, v);
        }
        double* jm = (double*)c.force3.get(mom_bytes(g));
        f.force_tangent(f.U, f.Us, terms, v, jm);
        unpack_mom(c, g, jm, (double*)J);
        FGI_HIP(hipStreamSynchronize(c.stream));
        if (f.nonconv) throw Error(FGI_ENOCONV, "CG reached cg_maxiter");
    });
}

int fgi_fermion_force(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* X,
                      void* F, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        check_action(act);
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(X, "X", 16);
        need(F, "F", 8);
        StreamScope ss(c, stream);
        d2* u = (d2*)c.gauge.get(gauge_bytes(g));
        pack_gauge(c, g, U, u);
        d2* x = (d2*)c.X.get(spinor_bytes(g));
        pack_even_spinor(c, g, X, x);
        double* fm = (double*)c.force.get(mom_bytes(g));
        zero_doubles(c, fm, mom_bytes(g) / sizeof(double));
        const FermionOp op{&g, act->kappa, u, P64, 18};
        if (act->csw != 0.0 && act->kappa != 0.0) {
            d2* blk = (d2*)c.cl_blk.get(sizeof(d2) * 72 * (size_t)g.V);
            clover_build(c, g, act->kappa, act->csw, u, blk, 1, nullptr);
            clover_force(c, op, act->csw, blk, x, fm, 1.0, 1.0, 0.0);
        } else {
            fermion_force(c, op, x, fm, 1.0);
        }
        unpack_mom(c, g, fm, (double*)F);
    });
}

int fgi_clover_field(fgi_ctx* ctx, const fgi_geom* gg, double kappa, double csw, const void* U, void* A,
                     double* S_det, void* F_det, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        if (!std::isfinite(kappa) || !(csw >= 0.0 && csw <= 10.0)) throw Error(FGI_EINVAL, "bad kappa or csw");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        if (A) need(A, "A", 16);
        if (F_det) need(F_det, "F_det", 8);
        StreamScope ss(c, stream);
        d2* u = (d2*)c.gauge.get(gauge_bytes(g));
        pack_gauge(c, g, U, u);
        d2* blk = (d2*)c.cl_blk.get(sizeof(d2) * 72 * (size_t)g.V);
        if (A) {
            clover_build(c, g, kappa, csw, u, blk, 0, nullptr);
            clover_unpack(c, g, blk, A);
        }
        if (S_det || F_det) clover_build(c, g, kappa, csw, u, blk, 1, S_det);
        if (F_det) {
            double* fm = (double*)c.force.get(mom_bytes(g));
            zero_doubles(c, fm, mom_bytes(g) / sizeof(double));
            clover_force(c, FermionOp{&g, kappa, u, P64, 18}, csw, blk, nullptr, fm, 1.0, 0.0, 1.0);
            unpack_mom(c, g, fm, (double*)F_det);
        }
        FGI_HIP(hipStreamSynchronize(c.stream));
    });
}

// prepare a Fields object with packed links (and sloppy copy) for the fermion entry points
namespace {
void setup_fermion_fields(Ctx& c, Fields& f, const Geom& g, const void* U) {
    f.U = (d2*)c.gauge.get(gauge_bytes(g));
    pack_gauge(c, g, U, f.U);
    if (f.sp != P64) {
        f.Us = c.sloppy.get(sloppy_bytes(g));
        make_sloppy(c, g, f.U, f.Us, f.sp, f.rc);
    }
    f.phi[0] = (d2*)c.phi.get(spinor_bytes(g));
    f.phi[1] = (d2*)c.phi2.get(spinor_bytes(g));
    f.X = (d2*)c.X.get(spinor_bytes(g));
    f.X2 = (d2*)c.X2.get(spinor_bytes(g));
    f.chi = (d2*)c.chi.get(spinor_bytes(g));
}
void check_hasen(const fgi_action* act) {
    check_action(act);
    if (act->kappa == 0 || act->kappa_hasen == 0) throw Error(FGI_EINVAL, "needs kappa and kappa_hasen");
}
}  // namespace

int fgi_hasen_heatbath(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* eta2,
                       void* phi2, fgi_stats* st, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        check_hasen(act);
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(eta2, "eta2", 16);
        need(phi2, "phi2", 16);
        StreamScope ss(c, stream);
        Fields f(c, g, *act);
        f.st = st;
        setup_fermion_fields(c, f, g, U);
        d2* e = (d2*)c.eta2.get(spinor_bytes(g));
        pack_even_spinor(c, g, eta2, e);
        f.hasen_heatbath(f.U, f.Us, e);
        unpack_even_spinor(c, g, f.phi[1], phi2);
        FGI_HIP(hipStreamSynchronize(c.stream));
        if (f.nonconv) throw Error(FGI_ENOCONV, "CG reached cg_maxiter");
    });
}

int fgi_hasen_action(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* phi2,
                     double* S2, fgi_stats* st, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg || !S2) throw Error(FGI_EINVAL, "null argument");
        check_hasen(act);
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(phi2, "phi2", 16);
        StreamScope ss(c, stream);
        Fields f(c, g, *act);
        f.st = st;
        setup_fermion_fields(c, f, g, U);
        pack_even_spinor(c, g, phi2, f.phi[1]);
        f.hasen_solve(f.U, f.Us);
        double* part = partial_buf(c, g);
        double* scal = (double*)c.scal.get(sizeof(double) * 64);
        int nb = pf_density_partials(c, g, f.chi, f.X2, nullptr, part);
        final_sum(c, part, nb, scal);
        *S2 = sync_scalar(c, scal, 0);
        if (f.nonconv) throw Error(FGI_ENOCONV, "CG reached cg_maxiter");
    });
}

int fgi_force_terms(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* phi1,
                    const void* phi2, int terms, void* F, fgi_stats* st, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        check_action(act);
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(F, "F", 8);
        if (terms & ~(FGI_TERM_GAUGE | FGI_TERM_FERMION | FGI_TERM_HASEN)) throw Error(FGI_EINVAL, "bad term mask");
        if (act->kappa != 0 && (terms & FGI_TERM_FERMION)) need(phi1, "phi1", 16);
        if (act->kappa_hasen != 0 && (terms & FGI_TERM_HASEN)) need(phi2, "phi2", 16);
        StreamScope ss(c, stream);
        Fields f(c, g, *act);
        f.st = st;
        setup_fermion_fields(c, f, g, U);
        if (phi1) pack_even_spinor(c, g, phi1, f.phi[0]);
        if (phi2) pack_even_spinor(c, g, phi2, f.phi[1]);
        double* fm = (double*)c.force.get(mom_bytes(g));
        f.force(f.U, f.Us, terms, fm, 1.0, false);
        unpack_mom(c, g, fm, (double*)F);
        FGI_HIP(hipStreamSynchronize(c.stream));
        if (f.nonconv) throw Error(FGI_ENOCONV, "CG reached cg_maxiter");
    });
}

int fgi_poisson_brackets(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* P,
                         const void* phi, double h, double* SST, double* TST, fgi_stats* st, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg || !SST || !TST) throw Error(FGI_EINVAL, "null argument");
        check_action(act);
        if (!(h > 0)) throw Error(FGI_EINVAL, "h must be positive");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(P, "P", 8);
        bool ferm = act->kappa != 0 && phi;
        StreamScope ss(c, stream);
        fgi_action a = *act;
        if (!ferm) a.kappa = 0;
        Fields f(c, g, a);
        f.st = st;
        f.U = (d2*)c.gauge.get(gauge_bytes(g));
        f.Ud = (d2*)c.gauge_disp.get(gauge_bytes(g));
        pack_gauge(c, g, U, f.U);
        double* pm = (double*)c.mom.get(mom_bytes(g));
        pack_mom(c, g, (const double*)P, pm);
        if (ferm) {
            f.phi[0] = (d2*)c.phi.get(spinor_bytes(g));
            pack_even_spinor(c, g, phi, f.phi[0]);
            f.X = (d2*)c.X.get(spinor_bytes(g));
            if (f.sp != P64) {
                f.Us = c.sloppy.get(sloppy_bytes(g));
                f.Uds = c.sloppy_disp.get(sloppy_bytes(g));
                make_sloppy(c, g, f.U, f.Us, f.sp, f.rc);
            }
        }
        double* fm = (double*)c.force.get(mom_bytes(g));
        double* part = partial_buf(c, g);
        double* scal = (double*)c.scal.get(sizeof(double) * 64);
        const int terms = FGI_TERM_GAUGE | FGI_TERM_FERMION;
        // SST = sum F^2
        f.force(f.U, f.Us, terms, fm, 1.0, false);
        int nb = dot_partials(c, 4L * 2 * 8 * g.Vh, fm, fm, part);
        final_sum(c, part, nb, scal);
        double sst = sync_scalar(c, scal, 0);
        // TST = d/dt <p, F(exp(tP) U)> by central difference
        double v[2];
        for (int k = 0; k < 2; k++) {
            double hh = k == 0 ? h : -h;
            link_update(c, g, hh, pm, f.U, f.Ud, f.Uds, f.sp, f.rc);
            f.force(f.Ud, f.Uds, terms, fm, 1.0, false);
            nb = dot_partials(c, 4L * 2 * 8 * g.Vh, pm, fm, part);
            final_sum(c, part, nb, scal + 1 + k);
            v[k] = sync_scalar(c, scal + 1 + k, 1 + k);
        }
        *SST = sst;
        *TST = (v[0] - v[1]) / (2.0 * h);
        if (f.nonconv) throw Error(FGI_ENOCONV, "CG reached cg_maxiter");
    });
}

int fgi_poisson_brackets4(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* P,
                          const void* phi, double h, double* out, fgi_stats* st, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg || !out) throw Error(FGI_EINVAL, "null argument");
        check_action(act);
        if (!(h > 0)) throw Error(FGI_EINVAL, "h must be positive");
        if (act->kappa_hasen != 0) throw Error(FGI_EINVAL, "the dt^4 brackets take one pseudofermion");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(P, "P", 8);
        const bool ferm = act->kappa != 0 && phi;
        if (ferm) need(phi, "phi", 16);
        StreamScope ss(c, stream);
        fgi_action a = *act;
        if (!ferm) a.kappa = 0;
        Fields f(c, g, a);
        f.st = st;
        f.U = (d2*)c.gauge.get(gauge_bytes(g));
        f.Ud = (d2*)c.gauge_disp.get(gauge_bytes(g));
        pack_gauge(c, g, U, f.U);
        double* pm = (double*)c.mom.get(mom_bytes(g));
        pack_mom(c, g, (const double*)P, pm);
        if (ferm) {
            f.phi[0] = (d2*)c.phi.get(spinor_bytes(g));
            pack_even_spinor(c, g, phi, f.phi[0]);
            f.X = (d2*)c.X.get(spinor_bytes(g));
            if (f.sp != P64) {
                f.Us = c.sloppy.get(sloppy_bytes(g));
                f.Uds = c.sloppy_disp.get(sloppy_bytes(g));
                make_sloppy(c, g, f.U, f.Us, f.sp, f.rc);
            }
        }
        const size_t mb = mom_bytes(g);
        double* fm = (double*)c.force.get(mb);    // F(U)
        double* fd = (double*)c.force2.get(mb);   // F at a moved U (its solve sets X there)
        double* jd = (double*)c.force3.get(mb);   // J_P at a moved U
        double* jp = (double*)c.br_jp.get(mb);
        double* jf = (double*)c.br_jf.get(mb);
        double* jj = (double*)c.br_jj.get(mb);
        double* part = partial_buf(c, g);
        double* scal = (double*)c.scal.get(sizeof(double) * 64);
        const long nm = 4L * 2 * 8 * g.Vh;
        auto dot = [&](const double* x, const double* y) {
            const int nb = dot_partials(c, nm, x, y, part);
            final_sum(c, part, nb, scal);
            return sync_scalar(c, scal, 0);
        };
        const int terms = FGI_TERM_GAUGE | FGI_TERM_FERMION;
        // at U: F, J_P, J_F and J_{J_P} (all with X at U)
        f.force(f.U, f.Us, terms, fm, 1.0, false);
        f.force_tangent(f.U, f.Us, terms, pm, jp);
        f.force_tangent(f.U, f.Us, terms, fm, jf);
        f.force_tangent(f.U, f.Us, terms, jp, jj);
        const double sst = dot(fm, fm), tst = dot(pm, jp), fjf = dot(fm, jf), jpjp = dot(jp, jp), pjj = dot(pm, jj);
        // J_P at exp(+-hP) U (<F, .> and <P, .>) and at exp(+-hF) U (<P, .>)
        double fjd[2], pjd[2], pjf[2];
        for (int k = 0; k < 2; k++) {
            const double hh = k == 0 ? h : -h;
            link_update(c, g, hh, pm, f.U, f.Ud, f.Uds, f.sp, f.rc);
            f.force(f.Ud, f.Uds, terms, fd, 1.0, false);
            f.force_tangent(f.Ud, f.Uds, terms, pm, jd);
            fjd[k] = dot(fm, jd);
            pjd[k] = dot(pm, jd);
        }
        for (int k = 0; k < 2; k++) {
            const double hh = k == 0 ? h : -h;
            link_update(c, g, hh, fm, f.U, f.Ud, f.Uds, f.sp, f.rc);
            f.force(f.Ud, f.Uds, terms, fd, 1.0, false);
            f.force_tangent(f.Ud, f.Uds, terms, pm, jd);
            pjf[k] = dot(pm, jd);
        }
        out[0] = sst;
        out[1] = tst;
        out[2] = 2.0 * fjf;
        out[3] = (pjf[0] - pjf[1]) / (2.0 * h) - jpjp - pjj;
        out[4] = 2.0 * jpjp + 2.0 * (fjd[0] - fjd[1]) / (2.0 * h);
        out[5] = (pjd[0] - 2.0 * tst + pjd[1]) / (h * h);
        if (f.nonconv) throw Error(FGI_ENOCONV, "CG reached cg_maxiter");
    });
}

int fgi_integrator_builtin(int which, double alpha, fgi_integrator* out) {
    return guarded([&] {
        if (!out) throw Error(FGI_EINVAL, "null output");
        std::memset(out, 0, sizeof(*out));
        out->nlevels = 1;
        fgi_level& L = out->lev[0];
        L.terms = FGI_TERM_GAUGE | FGI_TERM_FERMION | FGI_TERM_HASEN;
        L.nsub = 1;
        auto add = [&](int kind, double w, double xi) {
            fgi_stage& s = L.st[L.nstages++];
            s.kind = kind;
            s.w = w;
            s.xi = xi;
        };
        switch (which) {
        case FGI_PQP:
            add('P', 0.5, 0); add('Q', 1.0, 0); add('P', 0.5, 0);
            break;
        case FGI_QPQ:
            add('Q', 0.5, 0); add('P', 1.0, 0); add('Q', 0.5, 0);
            break;
        case FGI_PQPQP:
            if (!(alpha > 0 && alpha < 0.5)) throw Error(FGI_EINVAL, "alpha must be in (0, 1/2)");
            add('P', alpha, 0); add('Q', 0.5, 0); add('P', 1 - 2 * alpha, 0); add('Q', 0.5, 0); add('P', alpha, 0);
            break;
        case FGI_CAMPOSTRINI: {
            // Table 1 row 5: coefficients a cbrt4 + b cbrt2 + c over 12, 6, 12, 3
            const double c2 = std::cbrt(2.0), c4 = std::cbrt(4.0);
            const double q1 = (c4 + 2 * c2 + 4) / 12, p1 = (c4 + 2 * c2 + 4) / 6;
            const double q2 = (-c4 - 2 * c2 + 2) / 12, p2 = -(c4 + 2 * c2 + 1) / 3;
            add('Q', q1, 0); add('P', p1, 0); add('Q', q2, 0); add('P', p2, 0);
            add('Q', q2, 0); add('P', p1, 0); add('Q', q1, 0);
            break;
        }
        case FGI_FG:
            add('P', 1.0 / 6, 0); add('Q', 0.5, 0); add('G', 2.0 / 3, 1.0 / 72); add('Q', 0.5, 0); add('P', 1.0 / 6, 0);
            break;
        default:
            throw Error(FGI_EINVAL, "unknown integrator");
        }
    });
}

}  // extern "C"

// ==========================================================================
// trajectory driver
// ==========================================================================
namespace {

void check_integrator(const fgi_integrator* I) {
    if (!I) throw Error(FGI_EINVAL, "null integrator");
    if (I->nlevels < 1 || I->nlevels > FGI_MAX_LEVELS) throw Error(FGI_EINVAL, "bad number of levels");
    for (int l = 0; l < I->nlevels; l++) {
        const fgi_level& L = I->lev[l];
        if (L.nstages < 1 || L.nstages > FGI_MAX_STAGES) throw Error(FGI_EINVAL, "bad number of stages");
        if (l > 0 && L.nsub < 1) throw Error(FGI_EINVAL, "nsub must be >= 1");
        for (int k = 0; k < L.nstages; k++) {
            int kd = L.st[k].kind;
            if (kd != 'P' && kd != 'Q' && kd != 'G') throw Error(FGI_EINVAL, "stage kind must be P, Q or G");
            if (kd == 'G' && L.st[k].w == 0) throw Error(FGI_EINVAL, "G stage needs w != 0");
        }
    }
}

struct Driver {
    Fields& f;
    const fgi_integrator& I;
    Driver(Fields& ff, const fgi_integrator& ii) : f(ff), I(ii) {}

    // run level l for n steps of size h (P stages merged across steps)
    void run(int l, int n, double h) {
        const fgi_level& L = I.lev[l];
        double pending = 0.0;  // P weight waiting to be applied
        for (int step = 0; step < n; step++) {
            for (int k = 0; k < L.nstages; k++) {
                const fgi_stage& s = L.st[k];
                if (s.kind == 'P') {
                    pending += s.w;
                    continue;
                }
                flush(l, pending, h);
                pending = 0.0;
                if (s.kind == 'Q') {
                    if (l + 1 < I.nlevels) {
                        int ns = I.lev[l + 1].nsub;
                        run(l + 1, ns, s.w * h / ns);
                    } else {
                        link_update(f.c, f.g, s.w * h, f.P, f.U, f.U, f.Us, f.sp, f.rc);
                    }
                } else {
                    fg_stage(l, s.w, s.xi, h);
                }
            }
        }
        flush(l, pending, h);
    }

    void flush(int l, double w, double h) {
        if (w == 0.0) return;
        f.force(f.U, f.Us, I.lev[l].terms, f.P, w * h, true);
    }

    void fg_stage(int l, double w, double xi, double h) {
        int terms = I.lev[l].terms;
        if (f.act.fg_exact) {
            // p += w h F + 2 xi h^3 J_F[F]: F, then its derivative along itself
            // (one solve each for the pseudofermion force)
            double* J = (double*)f.c.force3.get(mom_bytes(f.g));
            f.force(f.U, f.Us, terms, f.F, 1.0, false);
            f.force_tangent(f.U, f.Us, terms, f.F, J);
            mom_axpy(f.c, f.g, w * h, f.F, f.P);
            mom_axpy(f.c, f.g, 2.0 * xi * h * h * h, J, f.P);
            return;
        }
        f.force(f.U, f.Us, terms, f.F, 1.0, false);
        link_update(f.c, f.g, 2.0 * xi / w * h * h, f.F, f.U, f.Ud, f.Uds, f.sp, f.rc);
        f.force(f.Ud, f.Uds, terms, f.P, w * h, true, f.c.fg_start != 0);
    }
};

}  // namespace

namespace {

void check_trajectory_args(const fgi_action* act, const fgi_integrator* integ, int nsteps, double tau) {
    check_action(act);
    check_integrator(integ);
    if (act->fg_exact && act->kappa != 0 && act->stout_n > 0)
        throw Error(FGI_EINVAL, "the exact force gradient is not available with stout smearing");
    if (act->fg_exact && act->kappa != 0 && act->csw != 0)
        throw Error(FGI_EINVAL, "the exact force gradient is not available with the clover term");
    if (nsteps < 1) throw Error(FGI_EINVAL, "nsteps must be >= 1");
    if (!std::isfinite(tau)) throw Error(FGI_EINVAL, "tau must be finite");
}

// Scratch of one trajectory in the internal layouts (links f.U are set by the caller)
void trajectory_buffers(Ctx& c, const Geom& g, Fields& f) {
    const bool ferm = f.act.kappa != 0.0, hasen = f.act.kappa_hasen != 0.0;
    f.Ud = (d2*)c.gauge_disp.get(gauge_bytes(g));
    f.P = (double*)c.mom.get(mom_bytes(g));
    f.F = (double*)c.force.get(mom_bytes(g));
    if (ferm && f.sp != P64) {
        f.Us = c.sloppy.get(sloppy_bytes(g));
        f.Uds = c.sloppy_disp.get(sloppy_bytes(g));
    }
    if (ferm) {
        f.phi[0] = (d2*)c.phi.get(spinor_bytes(g));
        f.X = (d2*)c.X.get(spinor_bytes(g));
        if (hasen) {
            f.phi[1] = (d2*)c.phi2.get(spinor_bytes(g));
            f.X2 = (d2*)c.X2.get(spinor_bytes(g));
            f.chi = (d2*)c.chi.get(spinor_bytes(g));
        }
    }
}

// One trajectory on packed fields: f.U and f.P hold the start, and for
// fermions either the noise (eta, eta_2: pseudofermions by heatbath) or, with
// phi_given, the pseudofermions themselves in f.phi.  f.U, f.P end as the
// final fields; returns dH (per-site differences of the gauge and kinetic
// densities plus the pseudofermion energies).
double trajectory_packed(Fields& f, const fgi_integrator& integ, double tau, int nsteps, const d2* eta,
                         const d2* eta_2, bool phi_given) {
    Ctx& c = f.c;
    const Geom& g = f.g;
    const bool ferm = f.act.kappa != 0.0, hasen = f.act.kappa_hasen != 0.0;
    if (ferm && f.sp != P64) make_sloppy(c, g, f.U, f.Us, f.sp, f.rc);
    double* h0 = (double*)c.h0.get(sizeof(double) * g.V);
    double* h1 = (double*)c.hf0.get(sizeof(double) * g.V);
    double* part = partial_buf(c, g);
    double* scal = (double*)c.scal.get(sizeof(double) * 64);
    double sf0 = 0.0;
    if (ferm) {
        const double k1 = hasen ? f.act.kappa_hasen : f.act.kappa;
        if (phi_given) {
            sf0 = f.pf_energy(f.U, f.Us, nullptr, nullptr, part, scal);
        } else if (f.clover()) {
            // phi = Mhat^+ eta (Mhat2 with the Hasenbusch split); the start's
            // -2 log det A_oo at kappa enters H
            const d2* fu = f.flinks(f.U, f.Us).u;
            f.clover_at(fu, f.act.kappa, &sf0, 1);
            const d2* blk = f.clover_at(fu, k1);
            clover_mhat(c, f.op64(fu, k1), blk, eta, f.phi[0], 1);
            if (hasen) f.hasen_heatbath(f.U, f.Us, eta_2);
        } else {
            pf_heatbath(c, f.op64(f.flinks(f.U, f.Us).u, k1), eta, f.phi[0]);
            if (hasen) f.hasen_heatbath(f.U, f.Us, eta_2);
        }
    }
    ham_density(c, g, f.act.beta, f.U, f.P, h0, f.act.c1);
    Driver d(f, integ);
    d.run(0, nsteps, tau / nsteps);
    ham_density(c, g, f.act.beta, f.U, f.P, h1, f.act.c1);
    int nb = diff_partials(c, g.V, h1, h0, part);
    final_sum(c, part, nb, scal);
    double dh = sync_scalar(c, scal, 0);
    if (ferm) dh += f.pf_energy(f.U, f.Us, phi_given ? nullptr : eta, phi_given ? nullptr : eta_2, part, scal) - sf0;
    return dh;
}

}  // namespace

extern "C" int fgi_trajectory(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const fgi_integrator* integ,
                              double tau, int nsteps, void* U, void* P, const void* eta1, const void* eta2,
                              int pf_is_phi, double* dH, fgi_stats* st, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg || !dH) throw Error(FGI_EINVAL, "null argument");
        check_trajectory_args(act, integ, nsteps, tau);
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(P, "P", 8);
        const bool ferm = act->kappa != 0.0;
        const bool hasen = act->kappa_hasen != 0.0;
        if (ferm) need(eta1, "eta1", 16);
        if (hasen) need(eta2, "eta2", 16);
        auto t0 = std::chrono::steady_clock::now();
        const long cap0 = c.graph_captures;
        StreamScope ss(c, stream);
        Fields f(c, g, *act);
        f.st = st;
        f.U = (d2*)c.gauge.get(gauge_bytes(g));
        trajectory_buffers(c, g, f);
        pack_gauge(c, g, U, f.U);
        pack_mom(c, g, (const double*)P, f.P);
        d2 *eta = nullptr, *eta_2 = nullptr;
        if (ferm && pf_is_phi) {
            pack_even_spinor(c, g, eta1, f.phi[0]);
            if (hasen) pack_even_spinor(c, g, eta2, f.phi[1]);
        } else if (ferm) {
            eta = (d2*)c.eta.get(spinor_bytes(g));
            pack_even_spinor(c, g, eta1, eta);
            if (hasen) {
                eta_2 = (d2*)c.eta2.get(spinor_bytes(g));
                pack_even_spinor(c, g, eta2, eta_2);
            }
        }
        const double dh = trajectory_packed(f, *integ, tau, nsteps, eta, eta_2, pf_is_phi != 0);
        unpack_gauge(c, g, f.U, U);
        unpack_mom(c, g, f.P, (double*)P);
        FGI_HIP(hipStreamSynchronize(c.stream));
        *dH = dh;
        if (st) {
            st->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            st->graph_captures += c.graph_captures - cap0;
        }
        if (!std::isfinite(dh)) throw Error(FGI_ENONFINITE, "dH is not finite");
        if (f.nonconv) throw Error(FGI_ENOCONV, "a CG solve reached cg_maxiter");
    });
}

extern "C" int fgi_field_bytes(const fgi_geom* gg, int kind, size_t* bytes) {
    return guarded([&] {
        if (!gg || !bytes) throw Error(FGI_EINVAL, "null argument");
        Geom g = make_geom(gg->dims);
        if (kind == FGI_FIELD_LINKS) *bytes = gauge_bytes(g);
        else if (kind == FGI_FIELD_MOMENTA) *bytes = mom_bytes(g);
        else if (kind == FGI_FIELD_EVEN) *bytes = spinor_bytes(g);
        else throw Error(FGI_EINVAL, "unknown field kind");
    });
}

namespace {
void field_convert(fgi_ctx* ctx, const fgi_geom* gg, int kind, const void* src, void* dst, void* stream, bool pack) {
    Ctx& c = ctx_of(ctx);
    if (!gg) throw Error(FGI_EINVAL, "null geometry");
    Geom g = make_geom(gg->dims);
    const size_t align = kind == FGI_FIELD_MOMENTA ? 8 : 16;
    if (kind < FGI_FIELD_LINKS || kind > FGI_FIELD_EVEN) throw Error(FGI_EINVAL, "unknown field kind");
    need(src, "source", align);
    need(dst, "destination", align);
    StreamScope ss(c, stream);
    if (kind == FGI_FIELD_LINKS) {
        if (pack) pack_gauge(c, g, src, (d2*)dst);
        else unpack_gauge(c, g, (const d2*)src, dst);
    } else if (kind == FGI_FIELD_MOMENTA) {
        if (pack) pack_mom(c, g, (const double*)src, (double*)dst);
        else unpack_mom(c, g, (const double*)src, (double*)dst);
    } else {
        if (pack) pack_even_spinor(c, g, src, (d2*)dst);
        else unpack_even_spinor(c, g, (const d2*)src, dst);
    }
}
}  // namespace

extern "C" int fgi_field_pack(fgi_ctx* ctx, const fgi_geom* gg, int kind, const void* user, void* internal,
                              void* stream) {
    return guarded([&] { field_convert(ctx, gg, kind, user, internal, stream, true); });
}

extern "C" int fgi_field_unpack(fgi_ctx* ctx, const fgi_geom* gg, int kind, const void* internal, void* user,
                                void* stream) {
    return guarded([&] { field_convert(ctx, gg, kind, internal, user, stream, false); });
}

extern "C" int fgi_trajectory_packed(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act,
                                     const fgi_integrator* integ, double tau, int nsteps, void* U, void* P,
                                     const void* eta1, const void* eta2, int pf_is_phi, double* dH, fgi_stats* st,
                                     void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg || !dH) throw Error(FGI_EINVAL, "null argument");
        check_trajectory_args(act, integ, nsteps, tau);
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(P, "P", 8);
        const bool ferm = act->kappa != 0.0, hasen = act->kappa_hasen != 0.0;
        if (ferm) need(eta1, "eta1", 16);
        if (hasen) need(eta2, "eta2", 16);
        auto t0 = std::chrono::steady_clock::now();
        const long cap0 = c.graph_captures;
        StreamScope ss(c, stream);
        Fields f(c, g, *act);
        f.st = st;
        f.U = (d2*)U;
        trajectory_buffers(c, g, f);
        f.P = (double*)P;
        if (ferm && pf_is_phi) {  // the pseudofermions are only read
            f.phi[0] = (d2*)eta1;
            if (hasen) f.phi[1] = (d2*)eta2;
        }
        const double dh = trajectory_packed(f, *integ, tau, nsteps, pf_is_phi ? nullptr : (const d2*)eta1,
                                            pf_is_phi ? nullptr : (const d2*)eta2, pf_is_phi != 0);
        FGI_HIP(hipStreamSynchronize(c.stream));
        *dH = dh;
        if (st) {
            st->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            st->graph_captures += c.graph_captures - cap0;
        }
        if (!std::isfinite(dh)) throw Error(FGI_ENONFINITE, "dH is not finite");
        if (f.nonconv) throw Error(FGI_ENOCONV, "a CG solve reached cg_maxiter");
    });
}

extern "C" int fgi_refresh(fgi_ctx* ctx, const fgi_geom* gg, uint64_t seed, uint64_t traj, void* P, void* eta1,
                           void* eta2, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        if (traj > 0xffffffffull) throw Error(FGI_EINVAL, "trajectory index beyond 2^32 - 1");
        Geom g = make_geom(gg->dims);
        StreamScope ss(c, stream);
        if (P) {
            need(P, "P", 8);
            double* pm = (double*)c.mom.get(mom_bytes(g));
            refresh_momenta(c, g, seed, (uint32_t)traj, pm);
            unpack_mom(c, g, pm, (double*)P);
        }
        void* etas[2] = {eta1, eta2};
        for (int k = 0; k < 2; k++) {
            if (!etas[k]) continue;
            need(etas[k], k ? "eta2" : "eta1", 16);
            d2* e = (d2*)c.eta.get(spinor_bytes(g));
            refresh_noise(c, g, seed, (uint32_t)traj, k ? RNG_ETA2 : RNG_ETA1, e);
            unpack_even_spinor(c, g, e, etas[k]);
        }
        FGI_HIP(hipStreamSynchronize(c.stream));
    });
}

extern "C" int fgi_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
    return guarded([&] {
        if (!ctr || !key || !out) throw Error(FGI_EINVAL, "null argument");
        philox_host(ctr, key, out);
    });
}

extern "C" int fgi_hmc_run(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const fgi_integrator* integ,
                           double tau, int nsteps, void* U, uint64_t seed, uint64_t traj0, int ntraj, int metropolis,
                           double* dH, int* accepted, double* plaq, fgi_stats* st, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        check_trajectory_args(act, integ, nsteps, tau);
        if (ntraj < 0) throw Error(FGI_EINVAL, "negative trajectory count");
        if (traj0 + (uint64_t)ntraj > 0x100000000ull) throw Error(FGI_EINVAL, "trajectory index beyond 2^32 - 1");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        if (ntraj == 0) return;
        const bool ferm = act->kappa != 0.0, hasen = act->kappa_hasen != 0.0;
        auto t0 = std::chrono::steady_clock::now();
        const long cap0 = c.graph_captures;
        StreamScope ss(c, stream);
        Fields f(c, g, *act);
        f.st = st;
        d2* Ucur = (d2*)c.chain_U.get(gauge_bytes(g));   // the chain's links
        f.U = (d2*)c.gauge.get(gauge_bytes(g));         // the trial trajectory's links
        trajectory_buffers(c, g, f);
        d2* eta = ferm ? (d2*)c.eta.get(spinor_bytes(g)) : nullptr;
        d2* eta_2 = hasen ? (d2*)c.eta2.get(spinor_bytes(g)) : nullptr;
        double* scal = (double*)c.scal.get(sizeof(double) * 64);
        double* part = partial_buf(c, g);
        pack_gauge(c, g, U, Ucur);
        bool nonconv = false;
        for (int k = 0; k < ntraj; k++) {
            const uint32_t t = (uint32_t)(traj0 + (uint64_t)k);
            FGI_HIP(hipMemcpyAsync(f.U, Ucur, gauge_bytes(g), hipMemcpyDeviceToDevice, c.stream));
            refresh_momenta(c, g, seed, t, f.P);
            if (ferm) refresh_noise(c, g, seed, t, RNG_ETA1, eta);
            if (hasen) refresh_noise(c, g, seed, t, RNG_ETA2, eta_2);
            f.nonconv = false;
            const double dh = trajectory_packed(f, *integ, tau, nsteps, eta, eta_2, false);
            if (!std::isfinite(dh)) throw Error(FGI_ENONFINITE, "dH is not finite");
            nonconv = nonconv || f.nonconv;
            const bool acc = !metropolis || metropolis_uniform(seed, t) < std::exp(-dh);
            if (acc) std::swap(Ucur, f.U);
            reunitarize(c, g, Ucur);
            if (dH) dH[k] = dh;
            if (accepted) accepted[k] = acc ? 1 : 0;
            if (plaq) {  // average plaquette ReTr U_P / 3 = 1 - S_G(beta = 1) / (6 V)
                ham_density(c, g, 1.0, Ucur, nullptr, (double*)c.h0.get(sizeof(double) * g.V));
                int nb = diff_partials(c, g.V, (const double*)c.h0.get(sizeof(double) * g.V), nullptr, part);
                final_sum(c, part, nb, scal + 8);
                plaq[k] = 1.0 - sync_scalar(c, scal + 8, 8) / (6.0 * g.V);
            }
        }
        unpack_gauge(c, g, Ucur, U);
        FGI_HIP(hipStreamSynchronize(c.stream));
        if (st) {
            st->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            st->graph_captures += c.graph_captures - cap0;
        }
        if (nonconv) throw Error(FGI_ENOCONV, "a CG solve reached cg_maxiter");
    });
}

// ==========================================================================
// batched independent chains
// ==========================================================================
namespace {

struct BFields {
    Ctx& c;
    Batch B;
    fgi_action act;
    int sp, rc;
    d2 *U = nullptr, *Ud = nullptr;
    void *Us = nullptr, *Uds = nullptr;
    double *P = nullptr, *F = nullptr;
    d2 *phi = nullptr, *X = nullptr;
    bool fermions = false, nonconv = false;
    fgi_stats* st = nullptr;

    BFields(Ctx& cc, const fgi_action& a) : c(cc), act(a) {
        sp = sloppy_prec(&act);
        rc = sloppy_recon(&act);
    }
    FermionOp op64(const d2* u) const { return FermionOp{nullptr, 0.0, u, P64, 18}; }
    FermionOp ops(const d2* u, const void* us) const {
        if (sp == P64) return op64(u);
        return FermionOp{nullptr, 0.0, us, sp, rc};
    }
    void solve(const d2* u, const void* us, const d2* rhs, d2* x, bool guess = false, bool md = false) {
        const double tol = (md && act.cg_tol_md > 0.0) ? act.cg_tol_md : act.cg_tol;
        std::vector<CGResult> r = cg_solve_b(c, B, op64(u), ops(u, us), sp, rhs, x, tol, act.cg_maxiter, guess);
        for (const CGResult& q : r) {
            accumulate_stats(st, q);
            if (!q.converged) nonconv = true;
        }
    }
    // the links the fermion operator sees (Fields::flinks for every chain)
    struct FLinks {
        const d2* u;
        const void* us;
    };
    FLinks flinks(const d2* u, const void* us) {
        if (act.stout_n <= 0) return {u, us};
        d2* lev = (d2*)c.stout_lev.get(sizeof(d2) * 9 * (size_t)B.links * act.stout_n);
        const d2* top = stout_smear_b(c, B, act.stout_rho, act.stout_n, u, lev);
        void* s = nullptr;
        if (sp != P64) {
            s = c.stout_sloppy.get(sizeof(float) * 18 * (size_t)B.links);
            make_sloppy_b(c, B, top, s, sp, rc);
        }
        return {top, s};
    }
    void force(const d2* u, const void* us, int terms, double* out, double coef, bool accumulate,
               bool guess = false) {
        bool have = accumulate;
        if (st) st->force_evals++;
        if (terms & FGI_TERM_GAUGE) {
            gauge_force_b(c, B, u, out, coef, have ? 1 : 0, act.c1);
            have = true;
        }
        if (!have) zero_doubles(c, out, 8 * (size_t)B.links);
        if (fermions && (terms & FGI_TERM_FERMION)) {
            const FLinks fl = flinks(u, us);
            if (act.stout_n > 0) {
                const size_t nm = 8 * (size_t)B.links;
                double* fo = (double*)c.stout_F.get(sizeof(double) * nm);
                zero_doubles(c, fo, nm);
                solve(fl.u, fl.us, phi, X, guess, true);
                fermion_force_b(c, B, op64(fl.u), X, fo, 1.0);
                stout_backprop_b(c, B, act.stout_rho, act.stout_n, u,
                                 (const d2*)c.stout_lev.get(sizeof(d2) * 9 * (size_t)B.links * act.stout_n), fo, out,
                                 coef, 1);
            } else {
                solve(u, us, phi, X, guess, true);
                fermion_force_b(c, B, op64(u), X, out, coef);
            }
        }
    }
};

struct BDriver {
    BFields& f;
    const fgi_integrator& I;
    void run(int l, int n, double h) {
        const fgi_level& L = I.lev[l];
        double pending = 0.0;
        for (int step = 0; step < n; step++) {
            for (int k = 0; k < L.nstages; k++) {
                const fgi_stage& s = L.st[k];
                if (s.kind == 'P') {
                    pending += s.w;
                    continue;
                }
                if (pending != 0.0) f.force(f.U, f.Us, L.terms, f.P, pending * h, true);
                pending = 0.0;
                if (s.kind == 'Q') {
                    if (l + 1 < I.nlevels) run(l + 1, I.lev[l + 1].nsub, s.w * h / I.lev[l + 1].nsub);
                    else link_update_b(f.c, f.B, s.w * h, f.P, f.U, f.U, f.Us, f.sp, f.rc);
                } else {
                    f.force(f.U, f.Us, L.terms, f.F, 1.0, false);
                    link_update_b(f.c, f.B, 2.0 * s.xi / s.w * h * h, f.F, f.U, f.Ud, f.Uds, f.sp, f.rc);
                    f.force(f.Ud, f.Uds, L.terms, f.P, s.w * h, true, f.c.fg_start != 0);
                }
            }
        }
        if (pending != 0.0) f.force(f.U, f.Us, L.terms, f.P, pending * h, true);
    }
};

}  // namespace

namespace {
// Chain table and block counts of a batch (host side).  The Dslash grid
// (GRID_DS) uses the context's current Dslash block size.
void describe_batch(Ctx& c, int nchains, const fgi_chain* chains, std::vector<ChainDesc>& cd, Batch& B) {
    const bool ferm = chains[0].kappa != 0.0;
    cd.assign(nchains, ChainDesc{});
    B = Batch{};
    B.nc = nchains;
    for (int i = 0; i < nchains; i++) {
        const fgi_chain& ch = chains[i];
        if ((ch.kappa != 0.0) != ferm) throw Error(FGI_EINVAL, "all chains need fermions or none");
        need(ch.U, "chain U", 16);
        need(ch.P, "chain P", 8);
        if (ferm) need(ch.eta, "chain eta", 16);
        ChainDesc& d = cd[i];
        d.g = make_geom(ch.dims);
        d.site0 = B.sites;
        d.vol0 = B.vol;
        d.link0 = B.links;
        d.beta = ch.beta;
        d.kappa = ch.kappa;
        const long n[4] = {d.g.Vh, d.g.V, 4L * d.g.V, d.g.Vh};
        const int bsz[4] = {256, 256, 256, c.ds_bs};
        for (int k = 0; k < 4; k++) {
            d.blk0[k] = B.nblk[k];
            d.nblk[k] = (int)((n[k] + bsz[k] - 1) / bsz[k]);
            B.nblk[k] += d.nblk[k];
        }
        d.user_U = ch.U;
        d.user_P = ch.P;
        d.user_eta = ch.eta;
        B.sites += d.g.Vh;
        B.vol += d.g.V;
        B.links += 4L * d.g.V;
    }
}

void upload_batch(Ctx& c, const std::vector<ChainDesc>& cd, Batch& B) {
    ChainDesc* dcd = (ChainDesc*)c.cdesc.get(sizeof(ChainDesc) * cd.size());
    FGI_HIP(hipMemcpyAsync(dcd, cd.data(), sizeof(ChainDesc) * cd.size(), hipMemcpyHostToDevice, c.stream));
    B.cd = dcd;
}
}  // namespace

extern "C" int fgi_trajectory_batched(fgi_ctx* ctx, int nchains, const fgi_chain* chains, const fgi_action* act,
                                      const fgi_integrator* integ, double tau, int nsteps, double* dH, fgi_stats* st,
                                      void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (nchains < 1 || !chains || !dH) throw Error(FGI_EINVAL, "need chains and a dH array");
        check_action(act);
        check_integrator(integ);
        if (nsteps < 1 || !std::isfinite(tau)) throw Error(FGI_EINVAL, "bad tau / nsteps");
        if (act->kappa_hasen != 0.0) throw Error(FGI_EINVAL, "batched chains take one pseudofermion");
        if (act->csw != 0.0) throw Error(FGI_EINVAL, "batched chains have no clover term");
        if (act->fg_exact) throw Error(FGI_EINVAL, "batched chains use the displacement force-gradient form");
        const bool ferm = chains[0].kappa != 0.0;
        std::vector<ChainDesc> cd;
        Batch B;
        describe_batch(c, nchains, chains, cd, B);
        auto t0 = std::chrono::steady_clock::now();
        const long cap0 = c.graph_captures;
        StreamScope ss(c, stream);
        upload_batch(c, cd, B);
        BFields f(c, *act);
        f.B = B;
        f.st = st;
        f.fermions = ferm;
        const size_t gb = sizeof(d2) * 9 * (size_t)B.links, mb = sizeof(double) * 8 * (size_t)B.links;
        const size_t sb = sizeof(d2) * 12 * (size_t)B.sites, slb = sizeof(float) * 18 * (size_t)B.links;
        f.U = (d2*)c.gauge.get(gb);
        f.Ud = (d2*)c.gauge_disp.get(gb);
        f.P = (double*)c.mom.get(mb);
        f.F = (double*)c.force.get(mb);
        pack_b(c, B, f.U, 0, 1);
        pack_b(c, B, f.P, 1, 1);
        d2* eta = nullptr;
        if (ferm) {
            f.phi = (d2*)c.phi.get(sb);
            f.X = (d2*)c.X.get(sb);
            eta = (d2*)c.eta.get(sb);
            pack_b(c, B, eta, 2, 1);
            if (f.sp != P64) {
                f.Us = c.sloppy.get(slb);
                f.Uds = c.sloppy_disp.get(slb);
                make_sloppy_b(c, B, f.U, f.Us, f.sp, f.rc);
            }
            pf_heatbath_b(c, B, f.op64(f.flinks(f.U, f.Us).u), eta, f.phi);
        }
        double* h0 = (double*)c.bh0.get(sizeof(double) * B.vol);
        double* h1 = (double*)c.bh1.get(sizeof(double) * B.vol);
        double* part = partial_buf(c, B);
        double* res = (double*)c.bres.get(sizeof(double) * 2 * nchains);  // not shared with the solver's scalars
        ham_density_b(c, B, f.U, f.P, h0, f.act.c1);

        BDriver d{f, *integ};
        d.run(0, nsteps, tau / nsteps);

        ham_density_b(c, B, f.U, f.P, h1, f.act.c1);
        diff_sums_b(c, B, h1, h0, part, res);
        if (ferm) {
            const BFields::FLinks fl = f.flinks(f.U, f.Us);
            f.solve(fl.u, fl.us, f.phi, f.X);
            pf_density_b(c, B, f.phi, f.X, eta, part, res + nchains);
        }
        std::vector<double> out(2 * nchains, 0.0);
        FGI_HIP(hipMemcpyAsync(out.data(), res, sizeof(double) * (ferm ? 2 : 1) * nchains, hipMemcpyDeviceToHost,
                               c.stream));
        pack_b(c, B, f.U, 0, 0);
        pack_b(c, B, f.P, 1, 0);
        FGI_HIP(hipStreamSynchronize(c.stream));
        bool finite = true;
        for (int i = 0; i < nchains; i++) {
            dH[i] = out[i] + (ferm ? out[nchains + i] : 0.0);
            finite = finite && std::isfinite(dH[i]);
        }
        if (st) {
            st->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            st->graph_captures += c.graph_captures - cap0;
        }
        if (!finite) throw Error(FGI_ENONFINITE, "dH is not finite");
        if (f.nonconv) throw Error(FGI_ENOCONV, "a CG solve reached cg_maxiter");
    });
}

// ------------------------------------------------------------ autotuner ---
// Schedules of the CG kernels picked by measurement on the caller's own
// system: the Dslash block size (64, 128 or 256 even sites per block) and
// block order (XCD-aware or linear) by timing a 64-iteration solve with each,
// then the iterations per host poll (cg_batch 4 ... 64) by timing full solves
// at the caller's tolerance.  Every candidate runs once untimed first (it
// captures its HIP graphs).  The winners stay set in the context.
namespace {
const int kTuneBlocks[3] = {64, 128, 256};
const int kTuneBatches[5] = {4, 8, 16, 32, 64};

template <typename Solve>
double time_solve(Ctx& c, Solve solve) {
    solve();  // untimed: graph capture, first touch
    FGI_HIP(hipStreamSynchronize(c.stream));
    auto t0 = std::chrono::steady_clock::now();
    int iters = solve();
    FGI_HIP(hipStreamSynchronize(c.stream));
    double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return iters > 0 ? s / iters : s;
}

// phase 1 with `solve64` (returns iterations), phase 2 with `solve_full`
template <typename S64, typename SFull, typename Rebuild>
void tune(Ctx& c, S64 solve64, SFull solve_full, Rebuild rebuild, fgi_tuning* out, bool forms) {
    fgi_tuning t{};
    const int saved_batch = c.cg_batch;
    double best = 1e300;
    int bb = 256, bx = 1;
    c.cg_batch = 16;
    for (int k = 0; k < 3; k++)
        for (int x = 0; x < 2; x++) {
            c.ds_bs = kTuneBlocks[k];
            c.ds_xcd = x;
            rebuild();
            const double us = 1e6 * time_solve(c, solve64);
            t.sched_us_per_iter[2 * k + x] = us;
            if (us < best) {
                best = us;
                bb = kTuneBlocks[k];
                bx = x;
            }
        }
    c.ds_bs = bb;
    c.ds_xcd = bx;
    rebuild();
    // the CG form (single-lattice solves only), on full solves: the
    // Chronopoulos-Gear form saves a launch per iteration but may take a few
    // more iterations
    int bf = c.cg_form;
    if (forms) {
        best = 1e300;
        for (int f = 0; f < 2; f++) {
            c.cg_form = f;
            const double ms = 1e3 * time_solve(c, [&] { solve_full(); return 1; });
            t.form_ms_per_solve[f] = ms;
            if (ms < best) {
                best = ms;
                bf = f;
            }
        }
    }
    c.cg_form = bf;   // unchanged unless timed
    best = 1e300;
    int bn = saved_batch;
    for (int k = 0; k < 5; k++) {
        c.cg_batch = kTuneBatches[k];
        const double ms = 1e3 * time_solve(c, [&] { solve_full(); return 1; });
        t.batch_ms_per_solve[k] = ms;
        if (ms < best) {
            best = ms;
            bn = kTuneBatches[k];
        }
    }
    c.cg_batch = bn;
    t.dslash_block = bb;
    t.xcd_order = bx;
    t.cg_batch = bn;
    t.cg_form = bf;
    if (out) *out = t;
}
}  // namespace

int fgi_autotune_cg(fgi_ctx* ctx, const fgi_geom* gg, const fgi_action* act, const void* U, const void* phi,
                    fgi_tuning* out, void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (!gg) throw Error(FGI_EINVAL, "null geometry");
        check_action(act);
        if (act->kappa == 0) throw Error(FGI_EINVAL, "kappa must be nonzero");
        Geom g = make_geom(gg->dims);
        need(U, "U", 16);
        need(phi, "phi", 16);
        StreamScope ss(c, stream);
        fgi_action a64 = *act;
        a64.cg_maxiter = 64;
        Fields f(c, g, *act), f64(c, g, a64);
        f.U = (d2*)c.gauge.get(gauge_bytes(g));
        pack_gauge(c, g, U, f.U);
        if (f.sp != P64) {
            f.Us = c.sloppy.get(sloppy_bytes(g));
            make_sloppy(c, g, f.U, f.Us, f.sp, f.rc);
        }
        f64.U = f.U;
        f64.Us = f.Us;
        d2* ph = (d2*)c.phi.get(spinor_bytes(g));
        d2* x = (d2*)c.X.get(spinor_bytes(g));
        pack_even_spinor(c, g, phi, ph);
        tune(
            c, [&] { return f64.solve(f.U, f.Us, act->kappa, ph, x).iters; },
            [&] { f.solve(f.U, f.Us, act->kappa, ph, x); }, [] {}, out, true);
    });
}

int fgi_autotune_batched(fgi_ctx* ctx, int nchains, const fgi_chain* chains, const fgi_action* act, fgi_tuning* out,
                         void* stream) {
    return guarded([&] {
        Ctx& c = ctx_of(ctx);
        if (nchains < 1 || !chains) throw Error(FGI_EINVAL, "need chains");
        check_action(act);
        if (chains[0].kappa == 0.0) throw Error(FGI_EINVAL, "the CG schedule is tuned on chains with fermions");
        std::vector<ChainDesc> cd;
        Batch B;
        describe_batch(c, nchains, chains, cd, B);
        StreamScope ss(c, stream);
        upload_batch(c, cd, B);
        fgi_action a64 = *act;
        a64.cg_maxiter = 64;
        BFields f(c, *act), f64(c, a64);
        f.B = B;
        f.fermions = true;
        const size_t gb = sizeof(d2) * 9 * (size_t)B.links, sb = sizeof(d2) * 12 * (size_t)B.sites;
        const size_t slb = sizeof(float) * 18 * (size_t)B.links;
        f.U = (d2*)c.gauge.get(gb);
        pack_b(c, B, f.U, 0, 1);
        f.phi = (d2*)c.phi.get(sb);
        f.X = (d2*)c.X.get(sb);
        d2* eta = (d2*)c.eta.get(sb);
        pack_b(c, B, eta, 2, 1);
        if (f.sp != P64) {
            f.Us = c.sloppy.get(slb);
            make_sloppy_b(c, B, f.U, f.Us, f.sp, f.rc);
        }
        pf_heatbath_b(c, B, f.op64(f.U), eta, f.phi);
        f64.U = f.U;
        f64.Us = f.Us;
        f64.phi = f.phi;
        f64.X = f.X;
        f64.fermions = true;
        auto rebuild = [&] {  // the Dslash grid follows the block size
            describe_batch(c, nchains, chains, cd, B);
            upload_batch(c, cd, B);
            f.B = B;
            f64.B = B;
        };
        tune(
            c,
            [&] {
                f64.solve(f.U, f.Us, f.phi, f.X);
                return 64;
            },
            [&] { f.solve(f.U, f.Us, f.phi, f.X); }, rebuild, out, false);
    });
}
