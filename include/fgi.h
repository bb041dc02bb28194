/*
 * fgi.h -- C ABI of the MI355X force-gradient HMC library (libfgi.so).
 *
 * The library implements the molecular-dynamics hot path of Kennedy, Clark
 * and Silva, "Force Gradient Integrators" (LAT2009, arXiv:0910.2950):
 * Hamiltonian H(U, p) = S(U) + T(p) (Section 2), integrators built as
 * products of the exactly integrable flows of S, T and of the force-gradient
 * bracket {S,{S,T}} (Section 3, Table 1), the gauge force gradient and the
 * pseudofermion force of Section 4, and the change dH over one trajectory
 * (Section 5, Figure 1).  All of it runs on one GPU in hand-written HIP.
 *
 * Conventions fixed by this library (the paper leaves them open):
 *   - site index i = x + Lx*(y + Ly*(z + Lz*t)); every extent even and >= 2;
 *     parity of a site = (x+y+z+t) mod 2; time direction antiperiodic for the
 *     fermions, everything else periodic.
 *   - su(3) basis T^a = i lambda^a / 2 (Gell-Mann lambda); a momentum or force
 *     is stored as its 8 real components, P = sum_a p_a T^a, T(p) = 1/2 sum p_a^2.
 *   - link update (the T-hat flow of Section 2): U <- exp(h P) U;
 *     momentum update (S-hat flow): p <- p + h F with F_a = -d/dt S(exp(t T^a) U)
 *     at t = 0 on each link.
 *   - gauge action S_G = beta sum_{x, mu<nu} (1 - Re Tr U_{mu nu}(x) / 3).
 *   - Wilson operator M = 1 - kappa D,
 *       D psi(x) = sum_mu [(1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)],
 *     DeGrand-Rossi gamma matrices; even-odd Schur operator on even sites
 *     Mhat = 1 - kappa^2 D_eo D_oe; pseudofermion action (Section 4 with the
 *     kernel Mhat^+ Mhat)  S_F = phi^+ (Mhat^+ Mhat)^-1 phi,  phi = Mhat^+ eta.
 *
 * User layouts (all DEVICE pointers, caller-owned, C-contiguous):
 *   links      complex128 [4][V][3][3]     U_mu(x), row-major colour matrix
 *   momenta    float64    [4][V][8]        components p_a (also forces)
 *   even field complex128 [V/2][4][3]      entry k = k-th even site in
 *                                          lexicographic order (spin, colour)
 *   odd field  complex128 [V/2][4][3]      same for odd sites
 * Links and momenta must be 16- resp. 8-byte aligned.
 *
 * Streams: every call takes a hipStream_t (as void*, NULL = legacy default
 * stream); all device work is ordered on it.  Calls that return host
 * scalars (actions, dH, statistics) synchronise that stream before returning.
 * A context is not thread-safe: one host thread per context at a time.
 *
 * Errors: every call returns FGI_OK (0) or a negative code; the text of the
 * last failure of the calling thread is in fgi_last_error().  Arguments are
 * checked on the host before any launch (FGI_EINVAL leaves outputs untouched).
 * No C++ exception crosses this boundary.
 */
#ifndef FGI_H
#define FGI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FGI_OK 0
#define FGI_EINVAL (-1)     /* bad geometry, null/misaligned pointer, bad option */
#define FGI_EHIP (-2)       /* HIP runtime failure (text in fgi_last_error) */
#define FGI_ENOCONV (-3)    /* a CG solve reached cg_maxiter; outputs are written */
#define FGI_ENONFINITE (-4) /* NaN/Inf in a residual or in dH */

#define FGI_FP64 0 /* everything FP64 */
#define FGI_MP32 1 /* CG inner iterations FP32 (links and vectors), FP64 reliable updates */
#define FGI_MP16 2 /* CG inner iterations with 16-bit links (12 reals in FP16, or
                      18 reals in 16-bit fixed point, round(32767 r)) and FP16
                      vectors (per-site scale), FP32 accumulation, FP64
                      reliable updates */

typedef struct fgi_ctx fgi_ctx;

typedef struct {
    int dims[4]; /* Lx, Ly, Lz, Lt */
} fgi_geom;

typedef struct {
    double beta;        /* Wilson gauge coupling */
    double kappa;       /* Wilson hopping parameter; 0 = pure gauge (no fermions) */
    double kappa_hasen; /* Hasenbusch mass-preconditioning kappa' (< kappa); 0 = off */
    double cg_tol;      /* CG stop: |phi - A x| <= cg_tol |phi| (true residual) */
    int cg_maxiter;     /* CG iteration cap */
    int prec;           /* FGI_FP64 | FGI_MP32 | FGI_MP16 (CG inner precision) */
    int link_recon;     /* 18 or 12: reals stored per sloppy link (FP32, or 16-bit: FP16 for 12, fixed point for 18); 12 keeps rows 0, 1 and rebuilds row 2.
                           Both compressions assume unitary links: 12 rebuilds row 2 from
                           unitarity, and the 16-bit fixed point of 18 holds reals in
                           [-1, 1] (larger ones are clamped; the FP64 reliable updates
                           still decide convergence) */
    int fg_exact;       /* G stages: 0 = displacement form, 1 = exact force gradient
                           (Section 4; every action term, the Hasenbusch ratio
                           term included; not with stout smearing, not for
                           batched chains) */
    double c1;          /* rectangle coefficient of the gauge action (finite):
                           S_G = beta sum_x [c0 sum_{mu<nu} (1 - ReTr P_{mu nu}(x)/3)
                                 + c1 sum_{mu!=nu} (1 - ReTr R_{mu nu}(x)/3)],
                           c0 = 1 - 8 c1, R the 2x1 rectangle two links along mu;
                           0 = Wilson, -1/12 tree-level Symanzik, -0.331 Iwasaki.
                           Forces, force gradients, brackets, trajectories and
                           chains (batched ones too) all take it. */
    double stout_rho;   /* stout smearing of the links the fermion operator sees
                           (Morningstar-Peardon): 0 <= rho <= 0.5 ... */
    int stout_n;        /* ... applied stout_n times (0 = thin links, at most 8).
                           It applies where the library builds the fermion
                           operator itself: fgi_force, fgi_poisson_brackets,
                           fgi_trajectory(_packed), fgi_hmc_run,
                           fgi_trajectory_batched; the fermion force
                           on the smeared links is carried back to the thin links
                           (fgi_stout_force); batched chains too.  Not with
                           fg_exact (FGI_EINVAL).  The operator-level entry points
                           (dslash, mhat, cg_solve, pf_*, fermion_force, hasen_*)
                           act on the links they are given. */
    int pad;
    double cg_tol_md;   /* tolerance of the solves inside force evaluations
                           (forces, force gradients, brackets, the MD of
                           trajectories and chains); 0 = cg_tol.  The heatbath
                           and action solves that enter dH keep cg_tol, so a
                           looser MD tolerance leaves the accept/reject step
                           exact.  In [0, 1), else FGI_EINVAL. */
    double csw;         /* clover (Sheikholeslami-Wohlert) coefficient of the
                           fermion matrix, M = A - kappa D with
                           A(x) = 1 + i kappa csw sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}(x),
                           sigma_{mu nu} = (i/2)[g_mu, g_nu], Fhat = (Q - Q^+)/8 of
                           the four-leaf clover Q; even-odd Mhat = A_ee -
                           kappa^2 D_eo A_oo^-1 D_oe and the action gains
                           -2 sum_{x odd} log det A(x).  0 = Wilson; in [0, 10],
                           else FGI_EINVAL.  With kappa != 0 it takes prec =
                           FGI_FP64, or FGI_MP32 (an FP32 inner CG on the FP32
                           links with FP64 defect correction; the FP64 true
                           residual decides, so cg_tol holds as in FP64), not
                           FGI_MP16 (FGI_EINVAL); with the Hasenbusch split
                           S_1 and S_2 use the clover operators at kappa' and
                           kappa and the log det is taken at kappa, on the
                           S_1 scale; not with fg_exact or for batched chains
                           (FGI_EINVAL).
                           fgi_mhat, fgi_pf_heatbath, fgi_cg_solve,
                           fgi_pf_action (S_F only), fgi_fermion_force (the S_F
                           force only), fgi_force (with the log det force),
                           fgi_force_terms, trajectories and fgi_hmc_run take
                           it; fgi_dslash stays the hopping term. */
} fgi_action;

/* One stage of an integrator step (Table 1), coefficients multiply the step h:
 *   kind 'P': p += w h F                       (flow of S)
 *   kind 'Q': U <- exp(w h P) U                (flow of T); on an outer level
 *             of a nested scheme it runs the next level for time w h instead
 *   kind 'G': the stage exp(w h S-hat - xi h^3 C-hat), C = {S,{S,T}}:
 *             exact form        p += w h F + 2 xi h^3 J_F[F],
 *                               J_F[F] = d/dt F(exp(t F) U) at t = 0
 *             displacement form U' = exp((2 xi / w) h^2 F(U)) U, p += w h F(U')
 * Neighbouring P stages of consecutive steps are merged into one. */
#define FGI_MAX_STAGES 16
#define FGI_MAX_LEVELS 4
typedef struct {
    int kind; /* 'P', 'Q' or 'G' */
    int pad;
    double w;
    double xi;
} fgi_stage;

#define FGI_TERM_GAUGE 1     /* S_G */
#define FGI_TERM_FERMION 2   /* S_F (or the heavy Hasenbusch term S_1) */
#define FGI_TERM_HASEN 4     /* Hasenbusch ratio term S_2 */

typedef struct {
    int nstages;
    int terms;    /* FGI_TERM_* mask: action terms whose force this level applies */
    int nsub;     /* steps of this level per Q stage of the level above (>= 1) */
    int pad;
    fgi_stage st[FGI_MAX_STAGES];
} fgi_level;

typedef struct {
    int nlevels;  /* level 0 is the outermost time scale */
    int pad;
    fgi_level lev[FGI_MAX_LEVELS];
} fgi_integrator;

typedef struct {
    long solves;           /* CG solves (the cost unit of Section 5) */
    long cg_iters;         /* CG iterations summed over solves */
    int cg_iters_max;      /* largest single solve */
    int reliable_updates;  /* FP64 residual replacements summed over solves */
    double max_rel_resid;  /* largest final true relative residual */
    long force_evals;      /* force evaluations (gauge + fermion counted once) */
    double seconds;        /* host wall time of the call */
    long graph_captures;   /* HIP graphs of CG batches captured during the call: the first call with a
                              given operator and vectors captures, repeated calls reuse them (0) */
} fgi_stats;

#define FGI_PQP 0          /* leapfrog, P first (Table 1 row 1) */
#define FGI_QPQ 1          /* leapfrog, Q first (row 2) */
#define FGI_PQPQP 2        /* Omelyan PQPQP with parameter alpha (Section 3) */
#define FGI_CAMPOSTRINI 3  /* 4th order, 7 stages, Q first (row 5) */
#define FGI_FG 4           /* force-gradient PQPQP (row 6) */

/* ---------------------------------------------------------------- context */
/* Create a context on HIP device `device` (owns scratch memory only). */
int fgi_create(fgi_ctx** out, int device);
/* Free all scratch of the context; the context pointer is invalid afterwards. */
int fgi_destroy(fgi_ctx* ctx);
/* Text of the calling thread's last failure ("" if none). */
const char* fgi_last_error(void);
/* Tuning/diagnostic options: "cg_batch" (CG iterations launched between host
 * polls; each batch is one replay of a captured HIP graph), "dslash_block"
 * (64, 128 or 256 even sites per block of the Dslash-shaped kernels),
 * "xcd_order" (1: XCD-aware block order, 0: linear; also the block order of
 * the force kernels), "fg_start" (1, the default: in the displacement form of
 * an FG stage the solves of the displaced force start from the solutions at
 * the undisplaced links, which are a function of the stage's links alone, so
 * the stage stays reversible; 0: from zero), "graphs" (0: launch the batch
 * kernels one by one instead), "ru_delta" (reliable-update residual drop),
 * "cg_form" (0, the default: the classic CG iteration, five launches; 1: the
 * Chronopoulos-Gear form, four launches, which applies the operator to the
 * residual and carries the direction's image by recurrence, with <p, A p>
 * expanded exactly; single-lattice Wilson solves only, the same tolerance and
 * true-residual stop; Chronopoulos and Gear, J. Comput. Appl. Math. 25 (1989)
 * 153), "profile" (1: after every CG solve, time 16 back-to-back launches of the
 * bare Dslash hop on the solve's operator with HIP events), "profile_prec"
 * (profile only solves whose inner precision is 0 FP64 / 1 FP32 / 2 FP16;
 * -1 all), "profile_reset".  An unknown name is FGI_EINVAL. */
int fgi_set_option(fgi_ctx* ctx, const char* name, double value);
/* Accumulated Dslash profile since the last reset: total ms of the timed bare
 * hop launches, their number, and output sites summed over them. */
int fgi_get_profile(fgi_ctx* ctx, double* ms, long* launches, long* sites);

/* Schedule of the CG kernels chosen by fgi_autotune_* (also settable with
 * fgi_set_option: "dslash_block", "xcd_order", "cg_batch", "cg_form"). */
typedef struct {
    int dslash_block;             /* even sites (threads) per block of the Dslash-shaped kernels: 64, 128, 256 */
    int xcd_order;                /* 1: blocks ordered so each XCD owns a contiguous slab of sites; 0: linear */
    int cg_batch;                 /* CG iterations launched between host polls */
    int cg_form;                  /* single-lattice CG: 0 classic (five launches per iteration), 1 the
                                     Chronopoulos-Gear form (four); batched solves use the classic form */
    double sched_us_per_iter[6];  /* measured: candidate (block 64, 128, 256) x (order 0, 1), index 2 k + order */
    double batch_ms_per_solve[5]; /* measured: full solve with cg_batch 4, 8, 16, 32, 64 */
    double form_ms_per_solve[2];  /* measured: full solve in each CG form (fgi_autotune_cg only; else 0) */
} fgi_tuning;
/* Autotuner: times every (block, order) schedule on a 64-iteration solve of
 * the caller's system (U, phi in the user layout, act's precision), then
 * every cg_batch on full solves at act->cg_tol, each candidate once untimed
 * first; leaves the fastest choices set in the context and reports all
 * timings in *out (may be NULL).  Results of later calls do not depend on
 * the schedule beyond rounding of the reductions (the same schedule always
 * gives the same bits).  Synchronises the stream. */
int fgi_autotune_cg(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* phi,
                    fgi_tuning* out, void* stream);

/* ------------------------------------------------ Hamiltonian (Section 2) */
/* *S = S_G(U) (FP64), Wilson plaquette action. */
int fgi_gauge_action(fgi_ctx* ctx, const fgi_geom* g, double beta, const void* U, double* S, void* stream);
/* *S = S_G(U) (FP64) of the improved gauge action with rectangle coefficient
 * c1 (as fgi_action.c1; the conclusions of the paper note that the
 * force-gradient construction holds for any common action).  FGI_EINVAL for a
 * non-finite c1. */
int fgi_improved_gauge_action(fgi_ctx* ctx, const fgi_geom* g, double beta, double c1, const void* U, double* S,
                              void* stream);
/* *T = 1/2 sum p_a^2 over all links (FP64). */
int fgi_kinetic(fgi_ctx* ctx, const fgi_geom* g, const void* P, double* T, void* stream);

/* ------------------------------------------- forces (Sections 2 and 4) */
/* F = gauge force -e_a S_G on every link (momentum layout). */
int fgi_gauge_force(fgi_ctx* ctx, const fgi_geom* g, double beta, const void* U, void* F, void* stream);
/* ------------------------------------------------------- stout smearing */
/* Us = n levels of stout smearing of U (Morningstar and Peardon, Phys. Rev. D
 * 69 (2004) 054501): per level U' = exp(TA(Omega)) U, Omega = C U^+,
 * C = rho * (sum of the six staples); the conclusions of the paper count
 * smearing among the settings the force-gradient construction covers.
 * Links layout in and out; 0 <= n <= 8, 0 <= rho <= 0.5, else FGI_EINVAL. */
int fgi_stout_smear(fgi_ctx* ctx, const fgi_geom* g, double rho, int n, const void* U, void* Us, void* stream);
/* F = the force on the thin links U of an action that depends on U only
 * through its smearing, given Fs, that action's force on the smeared links
 * (momentum layout; the adjoint of the smearing's tangent map, level by
 * level).  Same limits as fgi_stout_smear. */
int fgi_stout_force(fgi_ctx* ctx, const fgi_geom* g, double rho, int n, const void* U, const void* Fs, void* F,
                    void* stream);

/* J = d/dt F_G(exp(t V) U) at t = 0 for a field V of su(3) components
 * (momentum layout).  With V = F_G this is the gauge force gradient of
 * Section 4 that enters the Table 1 force-gradient stage. */
int fgi_force_gradient(fgi_ctx* ctx, const fgi_geom* g, double beta, const void* U, const void* V, void* J,
                       void* stream);
/* HV = H V with H the Hessian of S_G(exp(omega) U) in the chart omega (su(3)
 * components per link) at omega = 0, i.e. the symmetrised second derivative
 * (e_a e_b + e_b e_a) S_G / 2.  Per link HV = -J_V[F_G] + [V, F_G] / 2 with
 * J_V as in fgi_force_gradient; along V = F_G the commutator vanishes and HV is
 * minus the Section 4 force gradient.  (Backs the double backward of the
 * PyTorch autograd wrapper.) */
int fgi_gauge_hvp(fgi_ctx* ctx, const fgi_geom* g, double beta, const void* U, const void* V, void* HV,
                  void* stream);
/* The same Hessian-vector product for the improved gauge action with
 * rectangle coefficient c1 (as fgi_action.c1); FGI_EINVAL for a non-finite c1. */
int fgi_improved_gauge_hvp(fgi_ctx* ctx, const fgi_geom* g, double beta, double c1, const void* U, const void* V,
                           void* HV, void* stream);
/* F = F_G + F_F, the total force of S_G + S_F at U for pseudofermion phi
 * (even field; NULL or act->kappa == 0 for pure gauge).  One CG solve. */
int fgi_force(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* phi, void* F,
              fgi_stats* st, void* stream);
/* J = J_V[F] = d/dt F(exp(t V) U) at t = 0 for the total force F = F_G + F_F
 * of fgi_force (pure gauge when phi is NULL or act->kappa == 0), V a field of
 * su(3) components in the momentum layout; V == NULL takes V = F(U), which
 * gives the Section 4 force gradient G = J_F[F] itself.  The pseudofermion
 * part follows Section 4's Leibniz rule: with X = A^-1 phi, A = Mhat^+ Mhat,
 * one more CG solve gives d_V X = -A^-1 (d_V A) X, then
 *   J_F = kappa^2 bc TA(U [C(dX, Y) + C(X, dY)] + V U C(X, Y))
 * over the full-lattice force vectors.  Two solves (one for X, one for d_V X),
 * counted in *st (may be NULL), both in act->prec to act->cg_tol.  FGI_EINVAL
 * with act->kappa_hasen != 0 (this call takes one pseudofermion; trajectories
 * with fg_exact take the Hasenbusch terms' gradient); FGI_ENOCONV when a solve
 * hits cg_maxiter (J is still written).
 * Synchronises the stream. */
int fgi_total_force_gradient(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U,
                             const void* phi, const void* V, void* J, fgi_stats* st, void* stream);
/* F = F_F(X): the pseudofermion force of Section 4, e_a S = -X^+ e_a(A) X
 * for A = Mhat^+ Mhat, given the solution X = A^-1 phi (even field). */
int fgi_fermion_force(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* X,
                      void* F, void* stream);

/* Clover term at (kappa, csw) of the links U (the definition at
 * fgi_action.csw; the paper's conclusions leave the choice of fermion action
 * open and this is its standard O(a)-improved form).  Each output is optional
 * (NULL skips it):
 *   A      [V][12][12] complex: A(x) in lexicographic site order, index
 *          spin * 3 + colour (DeGrand-Rossi basis; zero between the spin
 *          pairs {0,1} and {2,3});
 *   S_det  host double: -2 sum_{x odd} log det A(x);
 *   F_det  [4][V][8] real: the force -e_a S_det on every link.
 * kappa csw < 1/6 keeps A(x) positive definite for any links; above it a
 * block may be indefinite, and since the Nf = 2 weight is det(A)^2 the term
 * is -2 sum log |det A(x)|, taken from the moduli of the pivots of a
 * partially pivoted elimination (a singular block gives NaN, reported as
 * FGI_ENONFINITE by the calls that sum or solve with it).  FGI_EINVAL for a
 * non-finite kappa or csw outside [0, 10].  Synchronises the stream. */
int fgi_clover_field(fgi_ctx* ctx, const fgi_geom* g, double kappa, double csw, const void* U, void* A,
                     double* S_det, void* F_det, void* stream);

/* ------------------------------------------- Wilson operator and solver */
/* out = D_{p,1-p} in: the hopping term from the other parity to parity
 * `out_parity` (in: field of parity 1-out_parity, out: parity out_parity),
 * evaluated in storage precision `prec` (FGI_FP64/MP32/MP16, links as in act). */
int fgi_dslash(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* in, void* out,
               int out_parity, int prec, void* stream);
/* out = Mhat in (dagger = 0) or Mhat^+ in (dagger = 1), even fields, FP64. */
int fgi_mhat(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* in, void* out,
             int dagger, void* stream);
/* X = (Mhat^+ Mhat)^-1 phi by CG from a zero start in act->prec with FP64
 * reliable updates, to act->cg_tol.  FGI_ENOCONV when act->cg_maxiter is hit
 * (X holds the last iterate). */
int fgi_cg_solve(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* phi, void* X,
                 fgi_stats* st, void* stream);
/* phi = Mhat^+ eta (pseudofermion heatbath for Gaussian eta, P ~ exp(-eta^+ eta)). */
int fgi_pf_heatbath(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* eta,
                    void* phi, void* stream);
/* *SF = Re phi^+ (Mhat^+ Mhat)^-1 phi (one CG solve). */
int fgi_pf_action(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* phi,
                  double* SF, fgi_stats* st, void* stream);

/* ------------------------- Hasenbusch mass preconditioning (two pseudofermions)
 * With act->kappa_hasen = kappa2 (< kappa) the pseudofermion action is split
 * S_F = S_1 + S_2, S_1 = phi1^+ (Mhat2^+ Mhat2)^-1 phi1 (Mhat2 at kappa2) and
 * S_2 = chi^+ (Mhat^+ Mhat)^-1 chi, chi = Mhat2^+ phi2, each with the Section 4
 * force; the integrator's term masks put them on separate time scales. */
/* phi2 = Mhat2 (Mhat2^+ Mhat2)^-1 Mhat^+ eta2, so that S_2 = eta2^+ eta2 (one solve). */
int fgi_hasen_heatbath(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* eta2,
                       void* phi2, fgi_stats* st, void* stream);
/* *S2 = Re chi^+ (Mhat^+ Mhat)^-1 chi with chi = Mhat2^+ phi2 (one solve). */
int fgi_hasen_action(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* phi2,
                     double* S2, fgi_stats* st, void* stream);
/* F = sum of the forces of the FGI_TERM_* terms selected by `terms` at U
 * (phi1: S_F or S_1 pseudofermion, phi2: S_2's; NULL when not selected). */
int fgi_force_terms(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* phi1,
                    const void* phi2, int terms, void* F, fgi_stats* st, void* stream);

/* ------------------------------------------ Poisson brackets (Section 3) */
/* *SST = {S,{S,T}} = sum |F|^2 and *TST = {T,{S,T}} = d/dt <p, F(exp(tP) U)>
 * at t = 0, the latter by a central difference of step h (two more force
 * evaluations).  phi may be NULL for pure gauge. */
int fgi_poisson_brackets(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* P,
                         const void* phi, double h, double* SST, double* TST, fgi_stats* st, void* stream);
/* The dt^4 Poisson brackets of Table 1 that enter the fourth-order shadow
 * Hamiltonians (the paper's nesting): out[6] = {SST, TST, STSST, STTST,
 * TTSST, TTTST} with STSST = {{S,T},{S,{S,T}}}, STTST = {{S,T},{T,{S,T}}},
 * TTSST = {T,{T,{S,{S,T}}}}, TTTST = {T,{T,{T,{S,T}}}} ({S,{S,{S,{S,T}}}}
 * and {T,{S,{S,{S,T}}}} vanish for T quadratic in p).  With the T-hat and
 * S-hat flows as derivations (L_T W = d/dt W(exp(tP) U, P), L_S W = d/ds
 * W(U, P + s F)), {T, W} = -L_T W, {S, W} = -L_S W and {{S,T}, W} =
 * [L_S, L_T] W, so with J_V the exact force gradient of the total force
 * along V and D_b its derivative along exp(t b) U:
 *   STSST = 2 <F, J_F>,  STTST = <P, D_F J_P> - |J_P|^2 - <P, J_{J_P}>,
 *   TTSST = 2 |J_P|^2 + 2 <F, D_P J_P>,  TTTST = d^2/dt^2 <P, J_P(exp(tP) U)>,
 * SST = |F|^2 and TST = <P, J_P>; the derivatives of J_P by central
 * differences with step h (eight force gradients and five forces in all,
 * two solves each with fermions).  The total force as in fgi_force (gauge
 * action with act->c1, Wilson pseudofermions when kappa != 0 and phi given);
 * not with Hasenbusch, stout or clover terms (FGI_EINVAL).  Synchronises. */
int fgi_poisson_brackets4(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* P,
                          const void* phi, double h, double* out, fgi_stats* st, void* stream);

/* ----------------------------------------------- integrators (Table 1) */
/* Fill a one-level integrator for a Table 1 scheme (alpha used by PQPQP). */
int fgi_integrator_builtin(int which, double alpha, fgi_integrator* out);

/* One molecular-dynamics trajectory of length tau in nsteps outer steps.
 * U, P (user layout) are updated in place.  Fermions (act->kappa != 0):
 * eta1 is the heatbath noise of the pseudofermion (phi = Mhat^+ eta1, S_F at
 * the start = eta1^+ eta1), or phi itself when pf_is_phi = 1 (S_F at the
 * start then costs one solve); eta2 is the noise of the Hasenbusch ratio
 * term (act->kappa_hasen != 0), else NULL.  *dH = H(end) - H(start), summed
 * as per-site differences.  Synchronises the stream. */
int fgi_trajectory(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const fgi_integrator* integ, double tau,
                   int nsteps, void* U, void* P, const void* eta1, const void* eta2, int pf_is_phi, double* dH,
                   fgi_stats* st, void* stream);

/* ------------------------------------------- internal layouts */
/* The internal (structure-of-arrays, checkerboard) layout of a field kind,
 * for callers that keep fields packed between calls: bytes to allocate
 * (device memory, 256-byte aligned from hipMalloc suffices); pack converts
 * the user layout into it, unpack back (bitwise round trip).  Asynchronous
 * on the stream.  FGI_EINVAL for an unknown kind or a null/misaligned pointer. */
#define FGI_FIELD_LINKS 0   /* complex128 [4][V][3][3] <-> double2 [4][2][9][V/2] */
#define FGI_FIELD_MOMENTA 1 /* float64 [4][V][8] <-> double [4][2][8][V/2] */
#define FGI_FIELD_EVEN 2    /* complex128 [V/2][4][3] <-> double2 [12][V/2] */
int fgi_field_bytes(const fgi_geom* g, int kind, size_t* bytes);
int fgi_field_pack(fgi_ctx* ctx, const fgi_geom* g, int kind, const void* user, void* internal, void* stream);
int fgi_field_unpack(fgi_ctx* ctx, const fgi_geom* g, int kind, const void* internal, void* user, void* stream);
/* fgi_trajectory on packed fields: U, P (updated in place) and eta1, eta2 (or
 * the pseudofermions with pf_is_phi) in the internal layouts; no packing or
 * unpacking inside.  Same results as fgi_trajectory, bitwise. */
int fgi_trajectory_packed(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const fgi_integrator* integ,
                          double tau, int nsteps, void* U, void* P, const void* eta1, const void* eta2, int pf_is_phi,
                          double* dH, fgi_stats* st, void* stream);

/* ------------------------- domain decomposition in t: one GPU's share */
/* The hopping term of Section 5's even-odd operator on a local sub-lattice of a
 * lattice split over GPUs in t (g = the local extents, L_t even and >= 2; its
 * sites in the user layouts of the local lattice).  The hops that cross the two
 * local t-faces take their operands from halo buffers filled by the
 * neighbouring ranks' fgi_halo_pack instead of from the local field, so the
 * caller moves only the faces between GPUs (peer stores or send/recv): two
 * buffers of fgi_halo_bytes each way per hop, 6 complex numbers per face site in
 * the working precision (FP64 for FGI_FP64, FP32 for FGI_MP32 and FGI_MP16), in a
 * layout only these calls read.  The antiperiodic t boundary travels in the
 * signs: sign_lo = -1 on the rank holding global t = 0, sign_hi = -1 on the rank
 * holding the last global t slice, +1 otherwise (one rank alone: both -1, which
 * gives the antiperiodic local lattice).  The decomposed hop is bitwise the
 * hop of the whole lattice (fgi_dslash in the same precision) on every rank's
 * sites.  All pointers are device memory; in, out in the even/odd user layout;
 * halo buffers 16-byte aligned for FGI_FP64, 8-byte otherwise, the two of a
 * pack distinct and neither overlapping in or out; prec as fgi_dslash
 * (act->link_recon applies to the sloppy links).
 * FGI_EINVAL for a null or misaligned pointer, a bad parity, precision or sign,
 * or L_t < 2.  Asynchronous on the stream. */
int fgi_halo_bytes(const fgi_geom* g, int prec, size_t* bytes);
/* to_lo (for the rank below): sign_lo (1 - g_4) psi at the local t = 0 sites;
 * to_hi (for the rank above): sign_hi U_t(x)^+ (1 + g_4) psi at t = L_t - 1;
 * psi = in, of parity in_parity. */
int fgi_halo_pack(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* in,
                  int in_parity, double sign_lo, double sign_hi, void* to_lo, void* to_hi, int prec, void* stream);
/* out_{out_parity} = D in_{1 - out_parity} with the forward t hops of the
 * t = L_t - 1 sites taken from from_hi (the rank above's to_lo) and the
 * backward t hops of the t = 0 sites from from_lo (the rank below's to_hi).
 * split = 1 computes the interior slices (1 <= t <= L_t - 2, which need no
 * halo and can run while the faces travel) and then the two face slices in
 * one launch; split = 0 one launch over every site.  Both give the same bits. */
int fgi_dslash_halo(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* in,
                    void* out, int out_parity, const void* from_lo, const void* from_hi, int split, int prec,
                    void* stream);
/* Kernel times of the decomposed hop at act->prec on a rank that is its own
 * neighbour (HIP events around reps launches each, after one untimed launch):
 * the face pack, the interior launch, the face launch, one launch over every
 * site, and the plain local hop (fgi_dslash's kernel) for comparison. */
typedef struct {
    double pack_us, interior_us, faces_us, all_us, local_us;
    long face_sites;  /* F = V/2 / L_t face sites per parity and face */
    long halo_bytes;  /* bytes of one halo buffer */
} fgi_halo_timing;
int fgi_halo_time(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const void* U, const void* in, int reps,
                  fgi_halo_timing* out, void* stream);

/* ------------------------------------------- allocation-free operator */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * Wilson Schur operator of fgi_mhat on packed fields, out = Mhat in
 * (dagger = 0) or Mhat^+ in (dagger = 1), Mhat = 1 - kappa^2 D_eo D_oe, with
 * U in the FGI_FIELD_LINKS layout and in, out in the FGI_FIELD_EVEN layout
 * (fgi_field_pack; all device memory, caller-owned, 16-byte aligned).
 * Its odd intermediate D_oe in lives in a fixed library-owned device array
 * of FGI_NOALLOC_MAX_VH odd sites (25.2 MB per GPU, held until the process
 * ends); the call allocates and frees nothing.  Asynchronous on the stream
 * (no synchronisation).  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (other streams, threads or contexts) race and must
 * be ordered by the caller.  Bitwise the result of fgi_mhat on the same
 * fields and kappa.  FGI_EINVAL, before any launch, when V/2 exceeds
 * FGI_NOALLOC_MAX_VH (16^3 x 64 is the largest 16^3 x T lattice), kappa is
 * not finite, a pointer is null or misaligned, or in and out overlap. */
#define FGI_NOALLOC_MAX_VH 131072
int fgi_mhat_packed_noalloc(fgi_ctx* ctx, const fgi_geom* g, double kappa, const void* U, const void* in, void* out,
                            int dagger, void* stream);

/* ------------------------------------------- Markov chain (HMC, Section 2) */
/* The heatbath draws of trajectory `traj` of the chain with this seed, from
 * the counter-based generator Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
 * SC11, 2011; key = the seed's low and high 32-bit words):
 *   P    (momentum layout, may be NULL): p_a ~ N(0, 1), component 2j + b of
 *        link l = mu V + i from counter (4 l + j, traj, 0, 0), b = 0, 1 the
 *        Box-Muller pair;
 *   eta1, eta2 (even layout, may be NULL): Re, Im ~ N(0, 1/2), spin-colour
 *        component e of even site k from counter (12 k + e, traj, 1 | 2, 0).
 * A counter's four words give two uniforms (m + 1/2) 2^-52 (m from words 0,1
 * and 2,3: 32 + 20 bits) and z0, z1 = sqrt(-2 ln u1) (cos, sin)(2 pi u2).
 * traj < 2^32.  Synchronises the stream. */
int fgi_refresh(fgi_ctx* ctx, const fgi_geom* g, uint64_t seed, uint64_t traj, void* P, void* eta1, void* eta2,
                void* stream);
/* Philox4x32-10 of one counter (host; the library's generator, for tests). */
int fgi_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out);
/* ntraj HMC trajectories of a Markov chain on U (user layout, updated in
 * place), entirely on the device: trajectory t = traj0 + k draws its momenta
 * and noise with fgi_refresh(seed, t), runs one fgi_trajectory from the
 * chain's links, and is accepted when metropolis == 0 or u < exp(-dH) with
 * u the uniform of counter (0, t, 3, 0); the links are reunitarised after
 * every trajectory.  dH[k], accepted[k] and the average plaquette
 * plaq[k] = ReTr U_P / 3 of the chain after trajectory k (each may be NULL)
 * are written for k < ntraj.  The chain's state is U and the next index, so
 * a run of n then m trajectories gives the same bits as one run of n + m.
 * traj0 + ntraj <= 2^32.  FGI_ENOCONV (after the last trajectory, U written)
 * when a solve hit cg_maxiter; FGI_ENONFINITE on a non-finite dH: the run
 * stops there and U is left as it was before the call (the outputs of the
 * finished trajectories are written).  Synchronises the stream. */
int fgi_hmc_run(fgi_ctx* ctx, const fgi_geom* g, const fgi_action* act, const fgi_integrator* integ, double tau,
                int nsteps, void* U, uint64_t seed, uint64_t traj0, int ntraj, int metropolis, double* dH,
                int* accepted, double* plaq, fgi_stats* st, void* stream);

/* ------------------------------------------------ batched chains
 * Many independent chains of different lattice sizes and couplings advanced
 * together: every MD sub-step is one set of kernel launches covering all
 * chains (each chain keeps its own geometry, beta, kappa and CG state, and
 * stops its solves on its own).  Chain buffers are caller-owned device
 * memory in the user layouts above.  The action supplies the precision and
 * CG settings (its beta and kappa are ignored); either every chain has
 * fermions (kappa != 0) or none; one pseudofermion per chain. */
typedef struct {
    int dims[4];
    int pad;
    double beta;
    double kappa;
    void* U;          /* links, updated in place */
    void* P;          /* momenta, updated in place */
    const void* eta;  /* pseudofermion heatbath noise (even sites) */
} fgi_chain;

/* One trajectory of every chain with the same integrator, tau and nsteps;
 * dH[i] = H_i(end) - H_i(start).  Synchronises the stream. */
int fgi_trajectory_batched(fgi_ctx* ctx, int nchains, const fgi_chain* chains, const fgi_action* act,
                           const fgi_integrator* integ, double tau, int nsteps, double* dH, fgi_stats* st,
                           void* stream);
/* The autotuner of fgi_autotune_cg on a batch of chains (every chain with
 * fermions; phi = Mhat^+ eta per chain): the block size sets the Dslash grid
 * of every chain, the order and cg_batch apply to the whole batch. */
int fgi_autotune_batched(fgi_ctx* ctx, int nchains, const fgi_chain* chains, const fgi_action* act,
                         fgi_tuning* out, void* stream);

/* --------------------------------------------------------- utilities */
/* U <- exp(h P) U on every link (exact su(3) exponential). */
int fgi_link_update(fgi_ctx* ctx, const fgi_geom* g, double h, const void* P, void* U, void* stream);
/* Project every link back onto SU(3) (Gram-Schmidt of rows 0, 1; row 2 = conj(row0 x row1)). */
int fgi_reunitarize(fgi_ctx* ctx, const fgi_geom* g, void* U, void* stream);
/* out[k] = exp(h sum_a p[k][a] T^a) for n elements (p: float64 [n][8],
 * out: complex128 [n][3][3], device pointers). */
int fgi_exp_su3(fgi_ctx* ctx, int n, const void* p, double h, void* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FGI_H */
