/*
 * fgi_oracle.c -- plain, slow, FP64 CPU oracle for the force-gradient HMC
 * hot path of Kennedy, Clark and Silva, "Force Gradient Integrators"
 * (arXiv:0910.2950).
 *
 * THIS IS TEST INFRASTRUCTURE.  It exists only so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the GPU library
 * against an independent implementation.  The GPU library never calls it,
 * links it or includes anything from it, and it includes nothing of the GPU
 * library.
 *
 * Everything is double precision, lexicographic, array-of-structures, full
 * lattice.  Even/odd structure appears only as a parity test on a site.
 * Reductions are sequential sums over per-site arrays in lexicographic order
 * (deterministic regardless of the OpenMP thread count).
 *
 * Conventions (the paper fixes none of these; each is a reading):
 *  - site index i = x + Lx*(y + Ly*(z + Lz*t)); parity(i) = (x+y+z+t) mod 2.
 *  - links U[mu][i][a][b] complex; momenta P[mu][i][8] real components p_a of
 *    the anti-Hermitian matrix P = sum_a p_a T^a with T^a = i*lambda^a/2
 *    (Gell-Mann lambda), so Tr(T^a T^b) = -delta_ab/2 and T(p) = 1/2 sum p_a^2.
 *  - component of an anti-Hermitian traceless X:  x_a = -2 Tr(T^a X).
 *  - e_a f(U) = d/dt f(exp(t T^a) U_l) at t=0 for one link l (the paper's
 *    left-invariant operators of Section 4, e_i(U) = -T_i U, up to the sign
 *    of the generator, which cancels in every quantity computed here).
 *  - force F_a = -e_a S (the S-hat flow of Section 2: p' = p + h F),
 *    link flow (T-hat): U' = exp(h P) U.
 *  - gauge action S_G = beta * sum_x [c0 sum_{mu<nu} (1 - Re Tr U_{mu nu}(x) / 3)
 *                                      + c1 sum_{mu!=nu} (1 - Re Tr R_{mu nu}(x) / 3)],
 *    c0 = 1 - 8 c1, R_{mu nu}(x) the 2x1 rectangle two links along mu and one
 *    along nu; c1 = 0 is the Wilson action, c1 = -1/12 the tree-level
 *    Symanzik action of Luscher and Weisz (1985), c1 = -0.331 Iwasaki's.
 *  - Wilson operator M = 1 - kappa D, with
 *      D psi(x) = sum_mu [(1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^+ psi(x-mu)],
 *    DeGrand-Rossi gamma matrices, antiperiodic in t, periodic in space.
 *  - even-odd Schur operator on even sites: Mhat = 1 - kappa^2 D_eo D_oe,
 *    Mhat^+ = g5 Mhat g5.  Pseudofermion action S_F = phi^+ (Mhat^+ Mhat)^-1 phi,
 *    phi = Mhat^+ eta, so S_F at the start equals eta^+ eta (Section 4: the
 *    generic pseudofermion action with kernel Mhat^+ Mhat).
 *  - even-site vectors are stored compactly: the k-th even site in
 *    lexicographic order is entry k.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* number of OpenMP threads the oracle's parallel loops use */
int oracle_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* lattice geometry                                                    */
/* ------------------------------------------------------------------ */

static long lat_volume(const int L[4]) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void lat_coords(const int L[4], long i, int c[4]) {
    c[0] = (int)(i % L[0]); i /= L[0];
    c[1] = (int)(i % L[1]); i /= L[1];
    c[2] = (int)(i % L[2]); i /= L[2];
    c[3] = (int)i;
}

static long lat_index(const int L[4], const int c[4]) {
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

static int lat_parity(const int L[4], long i) {
    int c[4];
    lat_coords(L, i, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* neighbour of site i one step in direction mu, forward (s=+1) or backward */
static long lat_step(const int L[4], long i, int mu, int s) {
    int c[4];
    lat_coords(L, i, c);
    c[mu] = (c[mu] + s + L[mu]) % L[mu];
    return lat_index(L, c);
}

/* fermion boundary sign of the hop from x to x+mu (s=+1) or x-mu (s=-1):
 * -1 when the hop wraps around the time direction. */
static double lat_bc(const int L[4], long i, int mu, int s) {
    int c[4];
    if (mu != 3) return 1.0;
    lat_coords(L, i, c);
    if (s > 0 && c[3] == L[3] - 1) return -1.0;
    if (s < 0 && c[3] == 0) return -1.0;
    return 1.0;
}

/* ------------------------------------------------------------------ */
/* 3x3 complex matrices                                                */
/* ------------------------------------------------------------------ */

typedef struct { cplx m[3][3]; } mat3;

static mat3 m_zero(void) { mat3 r; memset(&r, 0, sizeof r); return r; }
static mat3 m_unit(void) { mat3 r = m_zero(); r.m[0][0] = r.m[1][1] = r.m[2][2] = 1.0; return r; }

static mat3 m_mul(mat3 a, mat3 b) {
    mat3 r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx s = 0;
            for (int k = 0; k < 3; k++) s += a.m[i][k] * b.m[k][j];
            r.m[i][j] = s;
        }
    return r;
}

static mat3 m_dag(mat3 a) {
    mat3 r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r.m[i][j] = conj(a.m[j][i]);
    return r;
}

static mat3 m_add(mat3 a, mat3 b) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) a.m[i][j] += b.m[i][j];
    return a;
}

static mat3 m_scale(mat3 a, cplx s) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) a.m[i][j] *= s;
    return a;
}

static cplx m_trace(mat3 a) { return a.m[0][0] + a.m[1][1] + a.m[2][2]; }

static mat3 link_get(const cplx *U, long V, int mu, long i) {
    mat3 r;
    memcpy(&r, U + ((long)mu * V + i) * 9, sizeof r);
    return r;
}

static void link_put(cplx *U, long V, int mu, long i, mat3 a) {
    memcpy(U + ((long)mu * V + i) * 9, &a, sizeof a);
}

/* ------------------------------------------------------------------ */
/* su(3) basis: T^a = i lambda^a / 2                                   */
/* ------------------------------------------------------------------ */

static mat3 gen_T(int a) {
    mat3 l = m_zero();
    const double r3 = 1.0 / sqrt(3.0);
    switch (a) {
    case 0: l.m[0][1] = 1; l.m[1][0] = 1; break;
    case 1: l.m[0][1] = -I; l.m[1][0] = I; break;
    case 2: l.m[0][0] = 1; l.m[1][1] = -1; break;
    case 3: l.m[0][2] = 1; l.m[2][0] = 1; break;
    case 4: l.m[0][2] = -I; l.m[2][0] = I; break;
    case 5: l.m[1][2] = 1; l.m[2][1] = 1; break;
    case 6: l.m[1][2] = -I; l.m[2][1] = I; break;
    case 7: l.m[0][0] = r3; l.m[1][1] = r3; l.m[2][2] = -2 * r3; break;
    }
    return m_scale(l, 0.5 * I);
}

/* X = sum_a p_a T^a */
static mat3 alg_from_components(const double p[8]) {
    mat3 r = m_zero();
    for (int a = 0; a < 8; a++) r = m_add(r, m_scale(gen_T(a), p[a]));
    return r;
}

/* x_a = -2 Tr(T^a X), exact for traceless anti-Hermitian X */
static void alg_components(mat3 X, double x[8]) {
    for (int a = 0; a < 8; a++) x[a] = creal(-2.0 * m_trace(m_mul(gen_T(a), X)));
}

/* traceless anti-Hermitian part: (W - W^+)/2 - Tr(W - W^+)/6 */
static mat3 traceless_antiherm(mat3 W) {
    mat3 A = m_scale(m_add(W, m_scale(m_dag(W), -1.0)), 0.5);
    cplx t = m_trace(A) / 3.0;
    for (int i = 0; i < 3; i++) A.m[i][i] -= t;
    return A;
}

/* exp(X) by Taylor series with scaling and squaring.  X is scaled by 2^-s so
 * that its Frobenius norm is below 1/8, the series is summed to 24 terms
 * (remainder far below one ulp), and the result squared s times. */
static mat3 mat_exp(mat3 X) {
    double nrm = 0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) nrm += creal(X.m[i][j] * conj(X.m[i][j]));
    nrm = sqrt(nrm);
    int s = 0;
    while (nrm > 0.125) { nrm *= 0.5; s++; }
    mat3 Y = m_scale(X, ldexp(1.0, -s));
    mat3 term = m_unit(), sum = m_unit();
    for (int k = 1; k <= 24; k++) {
        term = m_scale(m_mul(term, Y), 1.0 / k);
        sum = m_add(sum, term);
    }
    for (int k = 0; k < s; k++) sum = m_mul(sum, sum);
    return sum;
}

/* ------------------------------------------------------------------ */
/* gauge action and force                                              */
/* ------------------------------------------------------------------ */

static mat3 plaquette(const int L[4], const cplx *U, long i, int mu, int nu) {
    long V = lat_volume(L);
    long ip = lat_step(L, i, mu, +1), in = lat_step(L, i, nu, +1);
    mat3 a = link_get(U, V, mu, i), b = link_get(U, V, nu, ip);
    mat3 c = link_get(U, V, mu, in), d = link_get(U, V, nu, i);
    return m_mul(m_mul(a, b), m_mul(m_dag(c), m_dag(d)));
}

/* Ordered product of the links along a lattice path starting at site i: step
 * +(d+1) goes forward along d (factor U_d(y), then y -> y + d), step -(d+1)
 * goes back (y -> y - d, then factor U_d(y)^+).  When Vm is given, *dP is the
 * derivative of the product under U_l -> exp(t V_l) U_l at t = 0 for every
 * link l at once (product rule with dU = V U and d(U^+) = -U^+ V). */
static mat3 path_product(const int L[4], const cplx *U, long i, const int *steps, int n,
                         const mat3 *Vm, mat3 *dP) {
    long V = lat_volume(L), y = i;
    mat3 P = m_unit(), D = m_zero();
    for (int k = 0; k < n; k++) {
        int d = abs(steps[k]) - 1;
        mat3 f, df = m_zero();
        if (steps[k] > 0) {
            f = link_get(U, V, d, y);
            if (Vm) df = m_mul(Vm[(long)d * V + y], f);
            y = lat_step(L, y, d, +1);
        } else {
            y = lat_step(L, y, d, -1);
            f = m_dag(link_get(U, V, d, y));
            if (Vm) df = m_scale(m_mul(f, Vm[(long)d * V + y]), -1.0);
        }
        if (Vm) D = m_add(m_mul(D, f), m_mul(P, df));
        P = m_mul(P, f);
    }
    if (dP) *dP = D;
    return P;
}

/* the 2x1 rectangle R_{mu nu}(x): two steps along mu, one along nu, back */
static mat3 rectangle(const int L[4], const cplx *U, long i, int mu, int nu) {
    int m = mu + 1, n = nu + 1;
    int steps[6] = {m, m, n, -m, -m, -n};
    return path_product(L, U, i, steps, 6, NULL, NULL);
}

/* per-site gauge action density
 * h_G(x) = beta [c0 sum_{mu<nu} (1 - ReTr U_mn / 3) + c1 sum_{mu!=nu} (1 - ReTr R_mn / 3)] */
static void gauge_density(const int L[4], double beta, double c1, const cplx *U, double *h) {
    long V = lat_volume(L);
    double c0 = 1.0 - 8.0 * c1;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        double sp = 0, sr = 0;
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++)
                sp += 1.0 - creal(m_trace(plaquette(L, U, i, mu, nu))) / 3.0;
        if (c1 != 0.0)
            for (int mu = 0; mu < 4; mu++)
                for (int nu = 0; nu < 4; nu++)
                    if (nu != mu) sr += 1.0 - creal(m_trace(rectangle(L, U, i, mu, nu))) / 3.0;
        h[i] = beta * (c0 * sp + c1 * sr);
    }
}

double oracle_gauge_action(const int L[4], double beta, double c1, const cplx *U) {
    long V = lat_volume(L);
    double *h = malloc(sizeof(double) * V), s = 0;
    gauge_density(L, beta, c1, U, h);
    for (long i = 0; i < V; i++) s += h[i];
    free(h);
    return s;
}

/* average plaquette ReTr U_P / 3 over all 6V plaquettes */
double oracle_plaquette(const int L[4], const cplx *U) {
    long V = lat_volume(L);
    return 1.0 - oracle_gauge_action(L, 1.0, 0.0, U) / (6.0 * V);
}

/* Sum of the 18 rectangle staples of link (mu, x): the 5-link paths from
 * x + mu back to x that close a 2x1 rectangle through U_mu(x).  For each
 * nu != mu: the rectangle two long along mu with U_mu(x) as its first or
 * second mu link, on the +nu or the -nu side (4 paths), and the rectangle two
 * long along nu on either side (2 paths).  Every rectangle of the action that
 * contains U_mu(x) appears once, so the part of S_G holding U_mu(x) is
 * -beta c1 / 3 ReTr(U_mu(x) A^R_mu(x)).  With Vm, *dA is the derivative of the
 * sum along V (path_product). */
static mat3 rect_staple_sum(const int L[4], const cplx *U, long i, int mu, const mat3 *Vm, mat3 *dA) {
    long xpm = lat_step(L, i, mu, +1);
    int m = mu + 1;
    mat3 A = m_zero(), D = m_zero();
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        int n = nu + 1;
        const int shapes[6][5] = {
            {m, n, -m, -m, -n},   /* along mu, +nu side, U_mu(x) first */
            {n, -m, -m, -n, m},   /* along mu, +nu side, U_mu(x) second */
            {m, -n, -m, -m, n},   /* along mu, -nu side, first */
            {-n, -m, -m, n, m},   /* along mu, -nu side, second */
            {n, n, -m, -n, -n},   /* along nu, +nu side */
            {-n, -n, -m, n, n},   /* along nu, -nu side */
        };
        for (int k = 0; k < 6; k++) {
            mat3 dP;
            A = m_add(A, path_product(L, U, xpm, shapes[k], 5, Vm, Vm ? &dP : NULL));
            if (Vm) D = m_add(D, dP);
        }
    }
    if (dA) *dA = D;
    return A;
}

/* sum of the 6 staples attached to link (mu, x):
 * A = sum_{nu != mu} [U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
 *                     + U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)]
 * so that the part of S_G containing U_mu(x) is -beta/3 ReTr(U_mu(x) A). */
static mat3 staple_sum(const int L[4], const cplx *U, long i, int mu) {
    long V = lat_volume(L);
    mat3 A = m_zero();
    long ipm = lat_step(L, i, mu, +1);
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        long ipn = lat_step(L, i, nu, +1), imn = lat_step(L, i, nu, -1);
        long ipm_mn = lat_step(L, ipm, nu, -1);
        mat3 up = m_mul(m_mul(link_get(U, V, nu, ipm), m_dag(link_get(U, V, mu, ipn))),
                        m_dag(link_get(U, V, nu, i)));
        mat3 dn = m_mul(m_mul(m_dag(link_get(U, V, nu, ipm_mn)), m_dag(link_get(U, V, mu, imn))),
                        link_get(U, V, nu, imn));
        A = m_add(A, m_add(up, dn));
    }
    return A;
}

/* F_a(mu,x) = -e_a S_G = -(beta/6) [TA(U_mu(x) (c0 A_mu(x) + c1 A^R_mu(x)))]_a
 * (e_a of -beta/3 ReTr(U A) is -beta/3 ReTr(T^a U A) = +beta/6 [TA(UA)]_a) */
void oracle_gauge_force(const int L[4], double beta, double c1, const cplx *U, double *F) {
    long V = lat_volume(L);
    double c0 = 1.0 - 8.0 * c1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int mu = 0; mu < 4; mu++)
        for (long i = 0; i < V; i++) {
            mat3 A = m_scale(staple_sum(L, U, i, mu), c0);
            if (c1 != 0.0) A = m_add(A, m_scale(rect_staple_sum(L, U, i, mu, NULL, NULL), c1));
            mat3 W = m_mul(link_get(U, V, mu, i), A);
            double x[8];
            alg_components(traceless_antiherm(W), x);
            for (int a = 0; a < 8; a++) F[((long)mu * V + i) * 8 + a] = -beta / 6.0 * x[a];
        }
}

/* Directional derivative of the gauge force along a field of algebra
 * elements V_l (components v[mu][i][8]):
 *   J_V[F_G](l) = d/dt F_G(exp(t V) U) at t = 0,
 * written out with the product rule on U_mu(x) A_mu(x), using
 * d U_l = V_l U_l and d U_l^+ = -U_l^+ V_l for every link l (the rectangle
 * staples through path_product). */
void oracle_gauge_force_tangent(const int L[4], double beta, double c1, const cplx *U, const double *v,
                                double *J) {
    double c0 = 1.0 - 8.0 * c1;
    long V = lat_volume(L);
    mat3 *Vm = malloc(sizeof(mat3) * 4 * V);
    for (long l = 0; l < 4 * V; l++) Vm[l] = alg_from_components(v + l * 8);
#pragma omp parallel for collapse(2) schedule(static)
    for (int mu = 0; mu < 4; mu++)
        for (long i = 0; i < V; i++) {
            mat3 u = link_get(U, V, mu, i);
            mat3 du = m_mul(Vm[(long)mu * V + i], u);
            mat3 A = m_zero(), dA = m_zero();
            long ipm = lat_step(L, i, mu, +1);
            for (int nu = 0; nu < 4; nu++) {
                if (nu == mu) continue;
                long ipn = lat_step(L, i, nu, +1), imn = lat_step(L, i, nu, -1);
                long ipm_mn = lat_step(L, ipm, nu, -1);
                /* upper staple a b^+ c^+ with a = U_nu(x+mu), b = U_mu(x+nu), c = U_nu(x) */
                mat3 a = link_get(U, V, nu, ipm), b = link_get(U, V, mu, ipn), c = link_get(U, V, nu, i);
                mat3 da = m_mul(Vm[(long)nu * V + ipm], a);
                mat3 dbd = m_scale(m_mul(m_dag(b), Vm[(long)mu * V + ipn]), -1.0); /* d(b^+) */
                mat3 dcd = m_scale(m_mul(m_dag(c), Vm[(long)nu * V + i]), -1.0);  /* d(c^+) */
                A = m_add(A, m_mul(m_mul(a, m_dag(b)), m_dag(c)));
                dA = m_add(dA, m_mul(m_mul(da, m_dag(b)), m_dag(c)));
                dA = m_add(dA, m_mul(m_mul(a, dbd), m_dag(c)));
                dA = m_add(dA, m_mul(m_mul(a, m_dag(b)), dcd));
                /* lower staple d^+ e^+ f with d = U_nu(x+mu-nu), e = U_mu(x-nu), f = U_nu(x-nu) */
                mat3 d = link_get(U, V, nu, ipm_mn), e = link_get(U, V, mu, imn), f = link_get(U, V, nu, imn);
                mat3 ddd = m_scale(m_mul(m_dag(d), Vm[(long)nu * V + ipm_mn]), -1.0);
                mat3 ded = m_scale(m_mul(m_dag(e), Vm[(long)mu * V + imn]), -1.0);
                mat3 df = m_mul(Vm[(long)nu * V + imn], f);
                A = m_add(A, m_mul(m_mul(m_dag(d), m_dag(e)), f));
                dA = m_add(dA, m_mul(m_mul(ddd, m_dag(e)), f));
                dA = m_add(dA, m_mul(m_mul(m_dag(d), ded), f));
                dA = m_add(dA, m_mul(m_mul(m_dag(d), m_dag(e)), df));
            }
            A = m_scale(A, c0);
            dA = m_scale(dA, c0);
            if (c1 != 0.0) {
                mat3 dR;
                A = m_add(A, m_scale(rect_staple_sum(L, U, i, mu, Vm, &dR), c1));
                dA = m_add(dA, m_scale(dR, c1));
            }
            mat3 dW = m_add(m_mul(du, A), m_mul(u, dA));
            double x[8];
            alg_components(traceless_antiherm(dW), x);
            for (int k = 0; k < 8; k++) J[((long)mu * V + i) * 8 + k] = -beta / 6.0 * x[k];
        }
    free(Vm);
}

/* ------------------------------------------------------------------ */
/* momenta and link updates                                            */
/* ------------------------------------------------------------------ */

static void kinetic_density(const int L[4], const double *P, double *h) {
    long V = lat_volume(L);
    for (long i = 0; i < V; i++) {
        double s = 0;
        for (int mu = 0; mu < 4; mu++)
            for (int a = 0; a < 8; a++) {
                double p = P[((long)mu * V + i) * 8 + a];
                s += p * p;
            }
        h[i] = 0.5 * s;
    }
}

double oracle_kinetic(const int L[4], const double *P) {
    long V = lat_volume(L);
    double *h = malloc(sizeof(double) * V), s = 0;
    kinetic_density(L, P, h);
    for (long i = 0; i < V; i++) s += h[i];
    free(h);
    return s;
}

/* exp(h X) with X = sum_a p_a T^a; out is 3x3 row-major complex */
void oracle_exp_su3(const double p[8], double h, cplx *out) {
    double q[8];
    for (int a = 0; a < 8; a++) q[a] = h * p[a];
    mat3 E = mat_exp(alg_from_components(q));
    memcpy(out, &E, sizeof E);
}

/* T-hat flow for time h: U_l <- exp(h P_l) U_l on every link */
void oracle_link_update(const int L[4], double h, const double *P, cplx *U) {
    long V = lat_volume(L);
#pragma omp parallel for schedule(static)
    for (long l = 0; l < 4 * V; l++) {
        double q[8];
        for (int a = 0; a < 8; a++) q[a] = h * P[l * 8 + a];
        mat3 E = mat_exp(alg_from_components(q));
        mat3 u;
        memcpy(&u, U + l * 9, sizeof u);
        u = m_mul(E, u);
        memcpy(U + l * 9, &u, sizeof u);
    }
}

/* Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1): the closest
 * special-unitary matrix in the usual lattice sense. */
void oracle_reunitarize(const int L[4], cplx *U) {
    long V = lat_volume(L);
#pragma omp parallel for schedule(static)
    for (long l = 0; l < 4 * V; l++) {
        cplx *u = U + l * 9;
        double n0 = 0;
        for (int j = 0; j < 3; j++) n0 += creal(u[j] * conj(u[j]));
        n0 = 1.0 / sqrt(n0);
        for (int j = 0; j < 3; j++) u[j] *= n0;
        cplx d = 0;
        for (int j = 0; j < 3; j++) d += conj(u[j]) * u[3 + j];
        for (int j = 0; j < 3; j++) u[3 + j] -= d * u[j];
        double n1 = 0;
        for (int j = 0; j < 3; j++) n1 += creal(u[3 + j] * conj(u[3 + j]));
        n1 = 1.0 / sqrt(n1);
        for (int j = 0; j < 3; j++) u[3 + j] *= n1;
        u[6] = conj(u[1] * u[5] - u[2] * u[4]);
        u[7] = conj(u[2] * u[3] - u[0] * u[5]);
        u[8] = conj(u[0] * u[4] - u[1] * u[3]);
    }
}

/* ------------------------------------------------------------------ */
/* Wilson-Dirac operator                                               */
/* ------------------------------------------------------------------ */

/* DeGrand-Rossi gamma matrices, g[0..3] = gamma_1..gamma_4 (x, y, z, t) */
static cplx GAM[4][4][4];
static int gam_ready = 0;

static void gamma_init(void) {
    if (gam_ready) return;
    memset(GAM, 0, sizeof GAM);
    GAM[0][0][3] = I;  GAM[0][1][2] = I;  GAM[0][2][1] = -I; GAM[0][3][0] = -I;
    GAM[1][0][3] = -1; GAM[1][1][2] = 1;  GAM[1][2][1] = 1;  GAM[1][3][0] = -1;
    GAM[2][0][2] = I;  GAM[2][1][3] = -I; GAM[2][2][0] = -I; GAM[2][3][1] = I;
    GAM[3][0][2] = 1;  GAM[3][1][3] = 1;  GAM[3][2][0] = 1;  GAM[3][3][1] = 1;
    gam_ready = 1;
}

/* for tests: copy gamma_{mu+1} (mu = 0..3) as a 4x4 row-major complex matrix */
void oracle_gamma(int mu, cplx *out) {
    gamma_init();
    memcpy(out, GAM[mu], sizeof GAM[mu]);
}

/* out(s) = (1 + sign*gamma_mu) in(s), for one 4x3 spinor */
static void spin_proj(int mu, double sign, const cplx *in, cplx *out) {
    for (int s = 0; s < 4; s++)
        for (int c = 0; c < 3; c++) {
            cplx v = in[s * 3 + c];
            for (int t = 0; t < 4; t++) v += sign * GAM[mu][s][t] * in[t * 3 + c];
            out[s * 3 + c] = v;
        }
}

/* out = u * in on the colour index of each spin component */
static void colour_mul(mat3 u, const cplx *in, cplx *out) {
    for (int s = 0; s < 4; s++)
        for (int a = 0; a < 3; a++) {
            cplx v = 0;
            for (int b = 0; b < 3; b++) v += u.m[a][b] * in[s * 3 + b];
            out[s * 3 + a] = v;
        }
}

/* full-lattice hopping term out = D in (in, out: [V][4][3]) */
void oracle_dhop(const int L[4], const cplx *U, const cplx *in, cplx *out) {
    long V = lat_volume(L);
    gamma_init();
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        cplx acc[12] = {0}, t1[12], t2[12];
        for (int mu = 0; mu < 4; mu++) {
            long f = lat_step(L, i, mu, +1), b = lat_step(L, i, mu, -1);
            double sf = lat_bc(L, i, mu, +1), sb = lat_bc(L, i, mu, -1);
            colour_mul(link_get(U, V, mu, i), in + f * 12, t1);
            spin_proj(mu, -1.0, t1, t2);
            for (int k = 0; k < 12; k++) acc[k] += sf * t2[k];
            colour_mul(m_dag(link_get(U, V, mu, b)), in + b * 12, t1);
            spin_proj(mu, +1.0, t1, t2);
            for (int k = 0; k < 12; k++) acc[k] += sb * t2[k];
        }
        memcpy(out + i * 12, acc, sizeof acc);
    }
}

/* out = (1 - kappa D) in, full lattice */
void oracle_wilson(const int L[4], double kappa, const cplx *U, const cplx *in, cplx *out) {
    long V = lat_volume(L);
    oracle_dhop(L, U, in, out);
    for (long k = 0; k < V * 12; k++) out[k] = in[k] - kappa * out[k];
}

/* compact even-site vector <-> full-lattice vector (odd sites zero) */
static void even_to_full(const int L[4], const cplx *e, cplx *full) {
    long V = lat_volume(L), k = 0;
    for (long i = 0; i < V; i++) {
        if (lat_parity(L, i) == 0) { memcpy(full + i * 12, e + k * 12, 12 * sizeof(cplx)); k++; }
        else memset(full + i * 12, 0, 12 * sizeof(cplx));
    }
}

static void full_to_even(const int L[4], const cplx *full, cplx *e) {
    long V = lat_volume(L), k = 0;
    for (long i = 0; i < V; i++)
        if (lat_parity(L, i) == 0) { memcpy(e + k * 12, full + i * 12, 12 * sizeof(cplx)); k++; }
}

static void zero_parity(const int L[4], cplx *full, int par) {
    long V = lat_volume(L);
    for (long i = 0; i < V; i++)
        if (lat_parity(L, i) == par) memset(full + i * 12, 0, 12 * sizeof(cplx));
}

static void apply_g5(long nsites, cplx *v) {
    for (long i = 0; i < nsites; i++)
        for (int k = 6; k < 12; k++) v[i * 12 + k] = -v[i * 12 + k];
}

/* Clover term of the fermion matrix (not in the paper, which only states that
 * the integrators apply to any action): per-site 12x12 Hermitian matrices
 * A(x) = 1 + i kappa csw sum_{mu<nu} sigma_{mu nu} (x) Fhat_{mu nu}(x), index
 * s*3 + colour, and their inverses; NULL everywhere means the Wilson
 * operator (A = 1). */
typedef struct {
    double csw;
    cplx *A, *Ainv;   /* [V][12][12] */
} clover_t;

static void site_mul12(const cplx *A, const cplx *in, cplx *out) {
    for (int r = 0; r < 12; r++) {
        cplx v = 0;
        for (int k = 0; k < 12; k++) v += A[r * 12 + k] * in[k];
        out[r] = v;
    }
}

/* Mhat psi_e = psi_e - kappa^2 D_eo D_oe psi_e on compact even vectors, or
 * with a clover term A_ee psi_e - kappa^2 D_eo A_oo^-1 D_oe psi_e (the Schur
 * complement of the odd block); dagger != 0 applies Mhat^+ = g5 Mhat g5
 * (A commutes with g5 and is Hermitian). */
static void mhat_cl(const int L[4], double kappa, const cplx *U, const clover_t *cl, const cplx *in, cplx *out,
                    int dagger) {
    long V = lat_volume(L), Vh = V / 2;
    cplx *f = malloc(sizeof(cplx) * 12 * V), *g = malloc(sizeof(cplx) * 12 * V);
    cplx *tmp = malloc(sizeof(cplx) * 12 * Vh);
    memcpy(tmp, in, sizeof(cplx) * 12 * Vh);
    if (dagger) apply_g5(Vh, tmp);
    even_to_full(L, tmp, f);
    oracle_dhop(L, U, f, g);   /* odd part of g = D_oe psi_e */
    zero_parity(L, g, 0);
    if (cl) {
        for (long i = 0; i < V; i++)
            if (lat_parity(L, i) == 1) {
                cplx t[12];
                site_mul12(cl->Ainv + i * 144, g + i * 12, t);
                memcpy(g + i * 12, t, sizeof t);
            }
    }
    oracle_dhop(L, U, g, f);   /* even part of f = D_eo (A_oo^-1) D_oe psi_e */
    full_to_even(L, f, out);
    if (cl) {
        long k = 0;
        for (long i = 0; i < V; i++)
            if (lat_parity(L, i) == 0) {
                cplx t[12];
                site_mul12(cl->A + i * 144, tmp + k * 12, t);
                for (int r = 0; r < 12; r++) out[k * 12 + r] = t[r] - kappa * kappa * out[k * 12 + r];
                k++;
            }
    } else {
        for (long k = 0; k < Vh * 12; k++) out[k] = tmp[k] - kappa * kappa * out[k];
    }
    if (dagger) apply_g5(Vh, out);
    free(f); free(g); free(tmp);
}

void oracle_mhat(const int L[4], double kappa, const cplx *U, const cplx *in, cplx *out, int dagger) {
    mhat_cl(L, kappa, U, NULL, in, out, dagger);
}

static double vdot_re(long n, const cplx *a, const cplx *b) {
    double s = 0;
    for (long k = 0; k < n; k++) s += creal(conj(a[k]) * b[k]);
    return s;
}

/* A = Mhat^+ Mhat */
static void normal_op(const int L[4], double kappa, const cplx *U, const clover_t *cl, const cplx *in, cplx *out,
                      cplx *tmp) {
    mhat_cl(L, kappa, U, cl, in, tmp, 0);
    mhat_cl(L, kappa, U, cl, tmp, out, 1);
}

/* Conjugate gradient on A = Mhat^+ Mhat from a zero start, or (start != 0)
 * from the x given on entry, whose true residual phi - A x is then the first
 * residual and direction.  Stops when the true residual |phi - A x| <=
 * tol |phi| (when the recursive residual first passes the target the true
 * residual is formed; if it has not passed, CG restarts from it).  Returns
 * the iteration count, or -1 on maxiter. */
static int cg_cl(const int L[4], double kappa, const cplx *U, const clover_t *cl, const cplx *phi, cplx *x,
                 double tol, int maxiter, double *rel_resid, int start) {
    long n = (lat_volume(L) / 2) * 12;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *Ap = malloc(sizeof(cplx) * n), *tmp = malloc(sizeof(cplx) * n);
    double bb = vdot_re(n, phi, phi), target = tol * tol * bb;
    if (!start || bb == 0.0) {
        memset(x, 0, sizeof(cplx) * n);
        memcpy(r, phi, sizeof(cplx) * n);
    } else {
        normal_op(L, kappa, U, cl, x, Ap, tmp);
        for (long k = 0; k < n; k++) r[k] = phi[k] - Ap[k];
    }
    memcpy(p, r, sizeof(cplx) * n);
    double rr = vdot_re(n, r, r);
    int it = 0, status = -1;
    if (bb == 0.0 || rr <= target) { status = 0; goto done; }
    while (it < maxiter) {
        normal_op(L, kappa, U, cl, p, Ap, tmp);
        double alpha = rr / vdot_re(n, p, Ap);
        for (long k = 0; k < n; k++) { x[k] += alpha * p[k]; r[k] -= alpha * Ap[k]; }
        double rr_new = vdot_re(n, r, r);
        it++;
        if (rr_new <= target) {
            normal_op(L, kappa, U, cl, x, Ap, tmp);
            for (long k = 0; k < n; k++) r[k] = phi[k] - Ap[k];
            rr_new = vdot_re(n, r, r);
            if (rr_new <= target) { status = it; break; }
            memcpy(p, r, sizeof(cplx) * n);
            rr = rr_new;
            continue;
        }
        double beta = rr_new / rr;
        for (long k = 0; k < n; k++) p[k] = r[k] + beta * p[k];
        rr = rr_new;
    }
done:
    if (rel_resid) {
        normal_op(L, kappa, U, cl, x, Ap, tmp);
        for (long k = 0; k < n; k++) r[k] = phi[k] - Ap[k];
        *rel_resid = bb > 0 ? sqrt(vdot_re(n, r, r) / bb) : 0.0;
    }
    free(r); free(p); free(Ap); free(tmp);
    return status;
}

int oracle_cg_from(const int L[4], double kappa, const cplx *U, const cplx *phi, cplx *x, double tol,
                   int maxiter, double *rel_resid, int start) {
    return cg_cl(L, kappa, U, NULL, phi, x, tol, maxiter, rel_resid, start);
}

int oracle_cg(const int L[4], double kappa, const cplx *U, const cplx *phi, cplx *x, double tol,
              int maxiter, double *rel_resid) {
    return oracle_cg_from(L, kappa, U, phi, x, tol, maxiter, rel_resid, 0);
}

/* heatbath: phi = Mhat^+ eta */
void oracle_pf_heatbath(const int L[4], double kappa, const cplx *U, const cplx *eta, cplx *phi) {
    oracle_mhat(L, kappa, U, eta, phi, 1);
}

/* per even site: Re phi(x)^+ X(x), compact even order */
static void pf_density(long Vh, const cplx *phi, const cplx *X, double *h) {
    for (long k = 0; k < Vh; k++) h[k] = vdot_re(12, phi + k * 12, X + k * 12);
}

/* S_F = Re phi^+ X with X = (Mhat^+ Mhat)^-1 phi (zero-start CG) */
double oracle_pf_action(const int L[4], double kappa, const cplx *U, const cplx *phi, double tol,
                        int maxiter, int *iters) {
    long Vh = lat_volume(L) / 2;
    cplx *X = malloc(sizeof(cplx) * 12 * Vh);
    double *h = malloc(sizeof(double) * Vh), s = 0;
    int it = oracle_cg(L, kappa, U, phi, X, tol, maxiter, NULL);
    if (iters) *iters = it;
    pf_density(Vh, phi, X, h);
    for (long k = 0; k < Vh; k++) s += h[k];
    free(X); free(h);
    return s;
}

/* Full-lattice vectors of the force: X = (X_e, D_oe X_e) and
 * Y = (Y_e, g5 D_oe g5 Y_e), so that Y_o = D_eo^+ Y_e. */
static void full_xy(const int L[4], const cplx *U, const cplx *Xe, const cplx *Ye, cplx *X, cplx *Y) {
    long V = lat_volume(L);
    cplx *t = malloc(sizeof(cplx) * 12 * V);
    even_to_full(L, Xe, X);
    oracle_dhop(L, U, X, t);
    for (long i = 0; i < V; i++)
        if (lat_parity(L, i) == 1) memcpy(X + i * 12, t + i * 12, 12 * sizeof(cplx));
    even_to_full(L, Ye, Y);
    apply_g5(V, Y);
    oracle_dhop(L, U, Y, t);
    apply_g5(V, t);
    even_to_full(L, Ye, Y);
    for (long i = 0; i < V; i++)
        if (lat_parity(L, i) == 1) memcpy(Y + i * 12, t + i * 12, 12 * sizeof(cplx));
    free(t);
}

/* Generic bilinear force of full-lattice vectors X, Y.  The derivative of
 * 2 Re[Y^+ D X] along link (mu, x) is
 *     2 Re Tr[T^a W] * bc,  W = sum_s [U X(x+mu)]_s [(1-g_mu) Y(x)]_s^+
 *                             + sum_s [U (1+g_mu) Y(x+mu)]_s [X(x)]_s^+,
 * with Re Tr[T^a W] = -[TA(W)]_a / 2; this adds coef * bc * [TA W]_a to F.
 * When Vm is given, W is replaced by Vm_l W: the same bilinear with the
 * link U_l replaced by its derivative V_l U_l inside e_a D (both the link
 * and its adjoint in the backward hop, where d(-U^+ T^a) = U^+ V T^a). */
static void bilinear_add(const int L[4], const cplx *U, const cplx *X, const cplx *Y, const mat3 *Vm,
                         double coef, double *F) {
    long V = lat_volume(L);
    gamma_init();
#pragma omp parallel for collapse(2) schedule(static)
    for (int mu = 0; mu < 4; mu++)
        for (long i = 0; i < V; i++) {
            long f = lat_step(L, i, mu, +1);
            double bc = lat_bc(L, i, mu, +1);
            mat3 u = link_get(U, V, mu, i);
            cplx a1[12], b1[12], a2[12], b2[12];
            colour_mul(u, X + f * 12, a1);
            spin_proj(mu, -1.0, Y + i * 12, b1);
            spin_proj(mu, +1.0, Y + f * 12, b2);
            colour_mul(u, b2, a2);
            const cplx *x0 = X + i * 12;
            mat3 W = m_zero();
            for (int s = 0; s < 4; s++)
                for (int p = 0; p < 3; p++)
                    for (int q = 0; q < 3; q++)
                        W.m[p][q] += a1[s * 3 + p] * conj(b1[s * 3 + q]) + a2[s * 3 + p] * conj(x0[s * 3 + q]);
            if (Vm) W = m_mul(Vm[(long)mu * V + i], W);
            double x[8];
            alg_components(traceless_antiherm(W), x);
            for (int a = 0; a < 8; a++) F[((long)mu * V + i) * 8 + a] += coef * bc * x[a];
        }
}

/* bilinear force of the even parts X_e, Y_e (odd parts from full_xy) */
static void force_xy_add(const int L[4], const cplx *U, const cplx *Xe, const cplx *Ye, double coef, double *F) {
    long V = lat_volume(L);
    cplx *X = malloc(sizeof(cplx) * 12 * V), *Y = malloc(sizeof(cplx) * 12 * V);
    full_xy(L, U, Xe, Ye, X, Y);
    bilinear_add(L, U, X, Y, NULL, coef, F);
    free(X); free(Y);
}

/* Pseudofermion force for S = phi^+ (Mhat^+ Mhat)^-1 phi given the solution
 * X_e.  From the Section 4 relation e_a(S) = -X^+ e_a(M) X applied to the
 * kernel Mhat^+ Mhat, with dMhat = -kappa^2 (dD_eo D_oe + D_eo dD_oe):
 *     e_a S = 2 kappa^2 Re[ Y^+ (e_a D) X ],  Y_e = Mhat X_e,
 * so F_a = -e_a S = kappa^2 bc [TA W]_a (force_xy_add with coef kappa^2).
 * The result is ADDED to F (scaled by `scale`). */
void oracle_fermion_force_add(const int L[4], double kappa, const cplx *U, const cplx *Xe,
                              double scale, double *F) {
    long Vh = lat_volume(L) / 2;
    cplx *ye = malloc(sizeof(cplx) * 12 * Vh);
    oracle_mhat(L, kappa, U, Xe, ye, 0);
    force_xy_add(L, U, Xe, ye, scale * kappa * kappa, F);
    free(ye);
}

/* ------------------------------------------------------------------ */
/* clover (Sheikholeslami-Wohlert) term                                */
/* ------------------------------------------------------------------ */
/* The paper claims its integrators for any action; the clover term is the
 * standard O(a)-improvement of the Wilson operator, written here in the
 * hopping normalisation of M = 1 - kappa D:
 *     M = A - kappa D,  A(x) = 1 + i kappa csw sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}(x),
 *     sigma_{mu nu} = (i/2)[g_mu, g_nu],  Fhat_{mu nu} = (Q_{mu nu} - Q_{mu nu}^+) / 8,
 * Q_{mu nu}(x) the sum of the four plaquette leaves at x in the (mu, nu) plane.
 * A(x) is Hermitian and commutes with g5.  Even-odd: det M = det A_oo det Mhat
 * with Mhat = A_ee - kappa^2 D_eo A_oo^-1 D_oe, so the two-flavour action is
 *     S = phi^+ (Mhat^+ Mhat)^-1 phi - 2 sum_{x odd} log det A(x). */

static void sigma_mn(int mu, int nu, cplx s[4][4]) {
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) {
            cplx v = 0;
            for (int k = 0; k < 4; k++) v += GAM[mu][a][k] * GAM[nu][k][b] - GAM[nu][a][k] * GAM[mu][k][b];
            s[a][b] = 0.5 * I * v;
        }
}

/* for tests: sigma_{mu nu} (mu, nu = 0..3) as a 4x4 row-major complex matrix */
void oracle_sigma(int mu, int nu, cplx *out) {
    cplx s[4][4];
    gamma_init();
    sigma_mn(mu, nu, s);
    memcpy(out, s, sizeof s);
}

/* the four leaves in the (mu, nu) plane at x: the same counter-clockwise
 * plaquette loop (+mu before +nu) started at each of its corners, as steps
 * +-1 along mu and +-2 along nu */
static const int LEAF[4][4] = {{1, 2, -1, -2}, {2, -1, -2, 1}, {-1, -2, 1, 2}, {-2, 1, 2, -1}};

static void leaf_steps(int mu, int nu, int l, int st[4]) {
    for (int k = 0; k < 4; k++) {
        int a = LEAF[l][k], d = (a == 1 || a == -1) ? mu : nu;
        st[k] = a > 0 ? d + 1 : -(d + 1);
    }
}

static mat3 clover_Q(const int L[4], const cplx *U, long i, int mu, int nu) {
    mat3 Q = m_zero();
    for (int l = 0; l < 4; l++) {
        int st[4];
        leaf_steps(mu, nu, l, st);
        Q = m_add(Q, path_product(L, U, i, st, 4, NULL, NULL));
    }
    return Q;
}

/* In-place inverse of a 12x12 complex matrix by Gauss-Jordan elimination with
 * partial pivoting; returns log det (complex: the sum of the logs of the
 * pivots, i pi per row exchange). */
static cplx inv12(const cplx *A, cplx *Ainv) {
    cplx a[12][24];
    cplx ld = 0;
    for (int r = 0; r < 12; r++)
        for (int c = 0; c < 24; c++) a[r][c] = c < 12 ? A[r * 12 + c] : (c - 12 == r ? 1.0 : 0.0);
    for (int c = 0; c < 12; c++) {
        int piv = c;
        for (int r = c + 1; r < 12; r++)
            if (cabs(a[r][c]) > cabs(a[piv][c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < 24; k++) { cplx t = a[c][k]; a[c][k] = a[piv][k]; a[piv][k] = t; }
            ld += I * M_PI;
        }
        cplx d = a[c][c];
        ld += clog(d);
        for (int k = 0; k < 24; k++) a[c][k] /= d;
        for (int r = 0; r < 12; r++) {
            if (r == c) continue;
            cplx f = a[r][c];
            if (f == 0) continue;
            for (int k = 0; k < 24; k++) a[r][k] -= f * a[c][k];
        }
    }
    for (int r = 0; r < 12; r++)
        for (int c = 0; c < 12; c++) Ainv[r * 12 + c] = a[r][c + 12];
    return ld;
}

/* A(x), A(x)^-1 and log det A(x) (real part; A is Hermitian) for every site */
static void clover_build(const int L[4], double kappa, double csw, const cplx *U, clover_t *cl, double *logdet) {
    long V = lat_volume(L);
    gamma_init();
    cplx sg[6][4][4];
    int pm[6], pn[6], np = 0;
    for (int mu = 0; mu < 4; mu++)
        for (int nu = mu + 1; nu < 4; nu++) { sigma_mn(mu, nu, sg[np]); pm[np] = mu; pn[np] = nu; np++; }
    cl->csw = csw;
    cl->A = malloc(sizeof(cplx) * 144 * V);
    cl->Ainv = malloc(sizeof(cplx) * 144 * V);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        cplx *A = cl->A + i * 144;
        for (int r = 0; r < 144; r++) A[r] = (r % 13 == 0) ? 1.0 : 0.0;
        for (int q = 0; q < 6; q++) {
            mat3 Q = clover_Q(L, U, i, pm[q], pn[q]);
            mat3 Fh = m_scale(m_add(Q, m_scale(m_dag(Q), -1.0)), 0.125);
            for (int s = 0; s < 4; s++)
                for (int t = 0; t < 4; t++)
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++)
                            A[(s * 3 + a) * 12 + t * 3 + b] += I * kappa * csw * sg[q][s][t] * Fh.m[a][b];
        }
        cplx ld = inv12(A, cl->Ainv + i * 144);
        if (logdet) logdet[i] = creal(ld);
    }
}

static void clover_free(clover_t *cl) {
    if (!cl) return;
    free(cl->A); free(cl->Ainv);
    cl->A = cl->Ainv = NULL;
}

/* for tests: A(x) and A(x)^-1 ([V][12][12], either may be NULL) and the
 * per-site log det A(x); returns -2 sum_{x odd} log det A(x) */
double oracle_clover(const int L[4], double kappa, double csw, const cplx *U, cplx *A, cplx *Ainv, double *logdet) {
    long V = lat_volume(L);
    clover_t cl;
    double *ld = malloc(sizeof(double) * V), s = 0;
    clover_build(L, kappa, csw, U, &cl, ld);
    if (A) memcpy(A, cl.A, sizeof(cplx) * 144 * V);
    if (Ainv) memcpy(Ainv, cl.Ainv, sizeof(cplx) * 144 * V);
    if (logdet) memcpy(logdet, ld, sizeof(double) * V);
    for (long i = 0; i < V; i++)
        if (lat_parity(L, i) == 1) s += -2.0 * ld[i];
    clover_free(&cl);
    free(ld);
    return s;
}

/* full-lattice M = A - kappa D with the clover term (for tests) */
void oracle_clover_wilson(const int L[4], double kappa, double csw, const cplx *U, const cplx *in, cplx *out) {
    long V = lat_volume(L);
    clover_t cl;
    clover_build(L, kappa, csw, U, &cl, NULL);
    oracle_dhop(L, U, in, out);
    for (long i = 0; i < V; i++) {
        cplx t[12];
        site_mul12(cl.A + i * 144, in + i * 12, t);
        for (int r = 0; r < 12; r++) out[i * 12 + r] = t[r] - kappa * out[i * 12 + r];
    }
    clover_free(&cl);
}

void oracle_clover_mhat(const int L[4], double kappa, double csw, const cplx *U, const cplx *in, cplx *out,
                        int dagger) {
    clover_t cl;
    clover_build(L, kappa, csw, U, &cl, NULL);
    mhat_cl(L, kappa, U, &cl, in, out, dagger);
    clover_free(&cl);
}

/* S_F = Re phi^+ X with X = (Mhat^+ Mhat)^-1 phi for the clover Mhat */
double oracle_clover_pf_action(const int L[4], double kappa, double csw, const cplx *U, const cplx *phi,
                               double tol, int maxiter, int *iters) {
    long Vh = lat_volume(L) / 2;
    clover_t cl;
    clover_build(L, kappa, csw, U, &cl, NULL);
    cplx *X = malloc(sizeof(cplx) * 12 * Vh);
    double *h = malloc(sizeof(double) * Vh), s = 0;
    int it = cg_cl(L, kappa, U, &cl, phi, X, tol, maxiter, NULL, 0);
    if (iters) *iters = it;
    pf_density(Vh, phi, X, h);
    for (long k = 0; k < Vh; k++) s += h[k];
    free(X); free(h);
    clover_free(&cl);
    return s;
}

/* Force of sum_x sum_{mu<nu} Re Tr[Q_{mu nu}(x) Kt_{mu nu}(x)] for given
 * per-site, per-plane colour matrices Kt ([V][6], planes in the order
 * (0,1),(0,2),(0,3),(1,2),(1,3),(2,3)): every link of every leaf is
 * differentiated where it stands in the loop.  A forward factor U at
 * position k of the loop f_1 ... f_4 started at x gives
 * e_a = Re Tr[T^a f_k ... f_4 Kt f_1 ... f_(k-1)]; a backward factor U^+
 * (d(U^+) = -U^+ T^a) gives -Re Tr[T^a f_(k+1) ... f_4 Kt f_1 ... f_k].  With
 * Re Tr[T^a W] = -[TA W]_a / 2, F_a = -e_a adds coef [TA W]_a / 2 (forward)
 * or -coef [TA W]_a / 2 (backward). */
static void leaf_force_add(const int L[4], const cplx *U, const mat3 *Kt, double coef, double *F) {
    long V = lat_volume(L);
    for (long i = 0; i < V; i++) {
        int q = 0;
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++, q++) {
                mat3 K = Kt[i * 6 + q];
                for (int l = 0; l < 4; l++) {
                    int st[4];
                    leaf_steps(mu, nu, l, st);
                    mat3 f[4];
                    long lk[4];
                    int dk[4];
                    long y = i;
                    for (int k = 0; k < 4; k++) {
                        int d = abs(st[k]) - 1;
                        if (st[k] > 0) {
                            f[k] = link_get(U, V, d, y);
                            lk[k] = y;
                            y = lat_step(L, y, d, +1);
                        } else {
                            y = lat_step(L, y, d, -1);
                            f[k] = m_dag(link_get(U, V, d, y));
                            lk[k] = y;
                        }
                        dk[k] = d;
                    }
                    for (int k = 0; k < 4; k++) {
                        int fwd = st[k] > 0;
                        int from = fwd ? k : k + 1;   /* W = f_from ... f_4 Kt f_1 ... f_(from-1) */
                        mat3 W = m_unit();
                        for (int j = from; j < 4; j++) W = m_mul(W, f[j]);
                        W = m_mul(W, K);
                        for (int j = 0; j < from; j++) W = m_mul(W, f[j]);
                        double x[8];
                        alg_components(traceless_antiherm(W), x);
                        double sgn = fwd ? 0.5 : -0.5;
                        for (int a = 0; a < 8; a++) F[((long)dk[k] * V + lk[k]) * 8 + a] += coef * sgn * x[a];
                    }
                }
            }
    }
}

/* Kt += (K - K^+) / 8 for K = c * i * Z, where Z_{ba} = sum_{s,t} sigma_{st}
 * Bm[(t,b),(s,a)] for a 12x12 matrix Bm given by its entries */
static void kt_add(const cplx sg[4][4], const cplx *Bm, cplx c, mat3 *Kt) {
    mat3 Z = m_zero();
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            cplx v = 0;
            for (int s = 0; s < 4; s++)
                for (int t = 0; t < 4; t++) v += sg[s][t] * Bm[(t * 3 + b) * 12 + s * 3 + a];
            Z.m[b][a] = v;
        }
    mat3 K = m_scale(Z, c * I);
    *Kt = m_add(*Kt, m_scale(m_add(K, m_scale(m_dag(K), -1.0)), 0.125));
}

/* Forces of the clover action given the solution X_e = (Mhat^+ Mhat)^-1 phi
 * (pf_scale: S_F; det_scale: the -2 log det A_oo term), ADDED to F.  With
 * Ye_given the pseudofermion part is the bilinear -2 Re[Y^+ (e_a Mhat) X] for
 * that Y_e instead (the chi-dependent part of the Hasenbusch ratio term).
 * With Y_e = Mhat X_e, X_o = A_oo^-1 D_oe X_e, Y_o = A_oo^-1 D_eo^+ Y_e:
 *   e_a S_F = -2 Re[Y^+ (e_a Mhat) X]
 *           = 2 kappa^2 Re[Y^+ (e_a D) X]                     (hopping, full X, Y)
 *             - 2 sum_x w_x Re[Y(x)^+ (e_a A(x)) X(x)]        (w = 1 even, kappa^2 odd),
 *   e_a S_det = -2 sum_{x odd} Tr[A(x)^-1 e_a A(x)],
 * and with e_a A = i kappa csw sum sigma (x) e_a Fhat, each clover part is
 * Re Tr[e_a Fhat K] = Re Tr[e_a Q (K - K^+)/8] for a colour matrix K per site
 * and plane (kt_add), whose leaf derivatives leaf_force_add takes. */
static void clover_force_add(const int L[4], double kappa, const cplx *U, const clover_t *cl, const cplx *Xe,
                             const cplx *Ye_given, double pf_scale, double det_scale, double *F) {
    long V = lat_volume(L), Vh = V / 2;
    gamma_init();
    cplx sg[6][4][4];
    int np = 0;
    for (int mu = 0; mu < 4; mu++)
        for (int nu = mu + 1; nu < 4; nu++) sigma_mn(mu, nu, sg[np++]);
    mat3 *Kt = malloc(sizeof(mat3) * 6 * V);
    for (long k = 0; k < 6 * V; k++) Kt[k] = m_zero();
    double kc = kappa * cl->csw;
    if (pf_scale != 0.0 && Xe) {
        cplx *ye = malloc(sizeof(cplx) * 12 * Vh);
        cplx *X = malloc(sizeof(cplx) * 12 * V), *Y = malloc(sizeof(cplx) * 12 * V);
        if (Ye_given) memcpy(ye, Ye_given, sizeof(cplx) * 12 * Vh);
        else mhat_cl(L, kappa, U, cl, Xe, ye, 0);
        full_xy(L, U, Xe, ye, X, Y);
        for (long i = 0; i < V; i++)
            if (lat_parity(L, i) == 1) {
                cplx t[12];
                site_mul12(cl->Ainv + i * 144, X + i * 12, t);
                memcpy(X + i * 12, t, sizeof t);
                site_mul12(cl->Ainv + i * 144, Y + i * 12, t);
                memcpy(Y + i * 12, t, sizeof t);
            }
        bilinear_add(L, U, X, Y, NULL, pf_scale * kappa * kappa, F);
        /* e_a S_F clover part: -2 w Re[Y^+ (i kc sigma (x) e_a Fhat) X]
         * = Re Tr[e_a Fhat (-2 w kc i Z)], Z_{ba} = sum sigma_{st} X_{tb} Y*_{sa} */
        for (long i = 0; i < V; i++) {
            double w = lat_parity(L, i) == 0 ? 1.0 : kappa * kappa;
            cplx Bm[144];
            for (int r = 0; r < 12; r++)
                for (int c = 0; c < 12; c++) Bm[r * 12 + c] = X[i * 12 + r] * conj(Y[i * 12 + c]);
            for (int q = 0; q < 6; q++) kt_add(sg[q], Bm, -2.0 * w * kc * pf_scale, Kt + i * 6 + q);
        }
        free(ye); free(X); free(Y);
    }
    if (det_scale != 0.0) {
        /* e_a S_det = -2 Tr[A^-1 (i kc sigma (x) e_a Fhat)] = Re Tr[e_a Fhat (-2 kc i Z')],
         * Z'_{ba} = sum sigma_{st} Ainv[(t,b),(s,a)] */
        for (long i = 0; i < V; i++)
            if (lat_parity(L, i) == 1)
                for (int q = 0; q < 6; q++) kt_add(sg[q], cl->Ainv + i * 144, -2.0 * kc * det_scale, Kt + i * 6 + q);
    }
    leaf_force_add(L, U, Kt, 1.0, F);
    free(Kt);
}

/* for tests: the clover pseudofermion force (hopping and clover parts) for
 * the solution X_e, scaled by pf_scale, plus the log det force scaled by
 * det_scale, ADDED to F (Xe may be NULL when pf_scale is 0) */
void oracle_clover_force_add(const int L[4], double kappa, double csw, const cplx *U, const cplx *Xe,
                             double pf_scale, double det_scale, double *F) {
    clover_t cl;
    clover_build(L, kappa, csw, U, &cl, NULL);
    clover_force_add(L, kappa, U, &cl, Xe, NULL, pf_scale, det_scale, F);
    clover_free(&cl);
}

/* for tests: X_e = (Mhat^+ Mhat)^-1 phi with the clover Mhat; returns the
 * iteration count or -1 */
int oracle_clover_cg(const int L[4], double kappa, double csw, const cplx *U, const cplx *phi, cplx *x, double tol,
                     int maxiter) {
    clover_t cl;
    clover_build(L, kappa, csw, U, &cl, NULL);
    int it = cg_cl(L, kappa, U, &cl, phi, x, tol, maxiter, NULL, 0);
    clover_free(&cl);
    return it;
}

/* Link field dU_l = V_l U_l, the derivative of exp(t V_l) U_l at t = 0.  The
 * hopping term is linear in every link and in its adjoint, and
 * d(U_l^+) = (V_l U_l)^+, so the hopping term built on dU is the derivative
 * of D along V. */
static void tangent_links(long V, const cplx *U, const mat3 *Vm, cplx *dU) {
    for (int mu = 0; mu < 4; mu++)
        for (long i = 0; i < V; i++) link_put(dU, V, mu, i, m_mul(Vm[(long)mu * V + i], link_get(U, V, mu, i)));
}

/* odd part of D_{oe} applied to an even vector given on the full lattice
 * (even sites set, odd zero): out = (0, D_oe in_e) with the links U */
static void hop_to_odd(const int L[4], const cplx *U, const cplx *in_full, cplx *out_full) {
    oracle_dhop(L, U, in_full, out_full);
    zero_parity(L, out_full, 0);
}

/* derivative of Mhat along V on a compact even vector:
 *   dMhat in_e = -kappa^2 (dD_eo D_oe + D_eo dD_oe) in_e,
 * dD the hopping term on the tangent links dU; dagger != 0 applies
 * dMhat^+ = g5 dMhat g5. */
static void dmhat(const int L[4], double kappa, const cplx *U, const cplx *dU, const cplx *in, cplx *out,
                  int dagger) {
    long V = lat_volume(L), Vh = V / 2;
    cplx *f = malloc(sizeof(cplx) * 12 * V), *g = malloc(sizeof(cplx) * 12 * V);
    cplx *h1 = malloc(sizeof(cplx) * 12 * V), *h2 = malloc(sizeof(cplx) * 12 * V);
    cplx *tmp = malloc(sizeof(cplx) * 12 * Vh), *e1 = malloc(sizeof(cplx) * 12 * Vh);
    memcpy(tmp, in, sizeof(cplx) * 12 * Vh);
    if (dagger) apply_g5(Vh, tmp);
    even_to_full(L, tmp, f);
    hop_to_odd(L, U, f, g);       /* D_oe in */
    oracle_dhop(L, dU, g, h1);    /* even part: dD_eo D_oe in */
    hop_to_odd(L, dU, f, g);      /* dD_oe in */
    oracle_dhop(L, U, g, h2);     /* even part: D_eo dD_oe in */
    full_to_even(L, h1, out);
    full_to_even(L, h2, e1);
    for (long k = 0; k < Vh * 12; k++) out[k] = -kappa * kappa * (out[k] + e1[k]);
    if (dagger) apply_g5(Vh, out);
    free(f); free(g); free(h1); free(h2); free(tmp); free(e1);
}

/* Directional derivative of the pseudofermion force along a field of algebra
 * elements V_l (components v[mu][i][8]):
 *   J_V[F_F] = d/dt F_F(exp(t V) U) at t = 0,
 * the force gradient of Section 4 for S = phi^+ A^-1 phi, A = Mhat^+ Mhat,
 * given X_e = A^-1 phi.  Section 4 writes the force as X^+ e_a(A) X and
 * differentiates it by the Leibniz rule: one derivative of X, which costs
 * the one extra solve
 *     Z = d_V X_e = -A^-1 (d_V A) X_e,
 *     d_V A = dMhat^+ Mhat + Mhat^+ dMhat,
 * (Section 4's Y, whose operator e^j(S) e_j is -d_V for V = F), one
 * derivative of the explicit link dependence, and the derivative of the
 * other X.  Here the force is kept in its hopping-term form
 * kappa^2 bc [TA W(X, Y)]_a with full-lattice X = (X_e, D_oe X_e),
 * Y = (Mhat X_e, D_eo^+ Mhat X_e), so the same three contributions read
 *     J = kappa^2 bc [TA( W(dX, Y) + W(X, dY) + V W(X, Y) )]_a
 * with the full derivatives of the vectors
 *     dX = (Z, dD_oe X_e + D_oe Z),
 *     dY = (dMhat X_e + Mhat Z, g5 dD_oe g5 Y_e + g5 D_oe g5 dY_e)
 * and V W the explicit derivative of e_a D (bilinear_add with Vm).
 * scale * J is ADDED to Jout.  Returns the CG iteration count of the Z
 * solve (-1 on maxiter). */
/* The body of the force gradient above for links U, tangent links dU = V U
 * (Vm the V_l), given X_e: the solve's right-hand side gets extra_rhs added
 * when given (the derivative of a U-dependent source, for S_2 below), and
 * Z = d_V X_e is copied to Zout when given. */
static int pf_tangent_core(const int L[4], double kappa, const cplx *U, const cplx *dU, const mat3 *Vm,
                           const cplx *Xe, const cplx *extra_rhs, double tol, int maxiter, double scale,
                           double *Jout, cplx *Zout) {
    long V = lat_volume(L), Vh = V / 2;
    size_t ne = sizeof(cplx) * 12 * Vh, nf = sizeof(cplx) * 12 * V;
    cplx *Ye = malloc(ne), *a = malloc(ne), *b = malloc(ne), *rhs = malloc(ne), *Z = malloc(ne);
    cplx *dYe = malloc(ne);
    /* Y_e = Mhat X_e;  rhs = -(dMhat^+ Y_e + Mhat^+ dMhat X_e) = -(d_V A) X_e */
    oracle_mhat(L, kappa, U, Xe, Ye, 0);
    dmhat(L, kappa, U, dU, Xe, a, 0);
    oracle_mhat(L, kappa, U, a, b, 1);
    dmhat(L, kappa, U, dU, Ye, rhs, 1);
    for (long k = 0; k < Vh * 12; k++) rhs[k] = -(rhs[k] + b[k]);
    if (extra_rhs)
        for (long k = 0; k < Vh * 12; k++) rhs[k] += extra_rhs[k];
    int it = oracle_cg(L, kappa, U, rhs, Z, tol, maxiter, NULL);
    /* dY_e = dMhat X_e + Mhat Z */
    oracle_mhat(L, kappa, U, Z, b, 0);
    for (long k = 0; k < Vh * 12; k++) dYe[k] = a[k] + b[k];
    /* full vectors */
    cplx *X = malloc(nf), *Y = malloc(nf), *dX = malloc(nf), *dY = malloc(nf);
    cplx *f = malloc(nf), *g = malloc(nf);
    full_xy(L, U, Xe, Ye, X, Y);
    full_xy(L, U, Z, dYe, dX, dY);    /* (Z, D_oe Z) and (dY_e, g5 D_oe g5 dY_e) */
    even_to_full(L, Xe, f);
    hop_to_odd(L, dU, f, g);          /* + dD_oe X_e */
    for (long k = 0; k < V * 12; k++) dX[k] += g[k];
    even_to_full(L, Ye, f);
    apply_g5(V, f);
    hop_to_odd(L, dU, f, g);
    apply_g5(V, g);                   /* + g5 dD_oe g5 Y_e */
    for (long k = 0; k < V * 12; k++) dY[k] += g[k];
    double c = scale * kappa * kappa;
    bilinear_add(L, U, dX, Y, NULL, c, Jout);
    bilinear_add(L, U, X, dY, NULL, c, Jout);
    bilinear_add(L, U, X, Y, Vm, c, Jout);
    if (Zout) memcpy(Zout, Z, ne);
    free(Ye); free(a); free(b); free(rhs); free(Z); free(dYe);
    free(X); free(Y); free(dX); free(dY); free(f); free(g);
    return it;
}

int oracle_fermion_force_tangent_add(const int L[4], double kappa, const cplx *U, const cplx *Xe,
                                     const double *v, double tol, int maxiter, double scale, double *Jout) {
    long V = lat_volume(L);
    mat3 *Vm = malloc(sizeof(mat3) * 4 * V);
    for (long l = 0; l < 4 * V; l++) Vm[l] = alg_from_components(v + l * 8);
    cplx *dU = malloc(sizeof(cplx) * 4 * V * 9);
    tangent_links(V, U, Vm, dU);
    int it = pf_tangent_core(L, kappa, U, dU, Vm, Xe, NULL, tol, maxiter, scale, Jout, NULL);
    free(Vm); free(dU);
    return it;
}

/* Hasenbusch mass preconditioning: S_F = S_1 + S_2 with a heavier kappa2,
 *   S_1 = phi1^+ (Mhat2^+ Mhat2)^-1 phi1                      (Mhat2 at kappa2)
 *   S_2 = chi^+ (Mhat^+ Mhat)^-1 chi,  chi = Mhat2^+ phi2.
 * Heatbath: phi1 = Mhat2^+ eta1, phi2 = Mhat2 (Mhat2^+ Mhat2)^-1 Mhat^+ eta2, so
 * S_1 = eta1^+ eta1 and S_2 = eta2^+ eta2 at the start. */
int oracle_hasen_heatbath(const int L[4], double kappa, double kappa2, const cplx *U, const cplx *eta2,
                          cplx *phi2, double tol, int maxiter) {
    long Vh = lat_volume(L) / 2;
    cplx *a = malloc(sizeof(cplx) * 12 * Vh), *x = malloc(sizeof(cplx) * 12 * Vh);
    oracle_mhat(L, kappa, U, eta2, a, 1);
    int it = oracle_cg(L, kappa2, U, a, x, tol, maxiter, NULL);
    oracle_mhat(L, kappa2, U, x, phi2, 0);
    free(a); free(x);
    return it;
}

/* S_2 value: Re chi^+ X2, X2 = (Mhat^+ Mhat)^-1 chi (returns X2 when asked);
 * start != 0: the solve starts from the X2out given on entry */
static double hasen_action_from(const int L[4], double kappa, double kappa2, const cplx *U, const cplx *phi2,
                                double tol, int maxiter, cplx *X2out, int *iters, int start) {
    long Vh = lat_volume(L) / 2;
    cplx *chi = malloc(sizeof(cplx) * 12 * Vh), *x = malloc(sizeof(cplx) * 12 * Vh);
    oracle_mhat(L, kappa2, U, phi2, chi, 1);
    if (start) memcpy(x, X2out, sizeof(cplx) * 12 * Vh);
    int it = oracle_cg_from(L, kappa, U, chi, x, tol, maxiter, NULL, start);
    if (iters) *iters = it;
    double s = 0;
    for (long k = 0; k < Vh; k++) s += vdot_re(12, chi + k * 12, x + k * 12);
    if (X2out) memcpy(X2out, x, sizeof(cplx) * 12 * Vh);
    free(chi); free(x);
    return s;
}

double oracle_hasen_action(const int L[4], double kappa, double kappa2, const cplx *U, const cplx *phi2,
                           double tol, int maxiter, cplx *X2out, int *iters) {
    return hasen_action_from(L, kappa, kappa2, U, phi2, tol, maxiter, X2out, iters, 0);
}

/* Force of S_2 given X2 = (Mhat^+ Mhat)^-1 Mhat2^+ phi2:
 *   dS_2 = 2 Re[(dMhat2^+ phi2)^+ X2] - X2^+ d(Mhat^+ Mhat) X2
 * The second term is the ordinary pseudofermion force of X2 at kappa; the
 * first is 2 Re[phi2^+ dMhat2 X2] = -2 kappa2^2 Re[Z^+ dD W] with W built from
 * X2 and Z from phi2, i.e. force_xy_add(X2, phi2) with coef -kappa2^2.
 * Added to F, scaled by `scale`. */
void oracle_hasen_force_add(const int L[4], double kappa, double kappa2, const cplx *U, const cplx *phi2,
                            const cplx *X2, double scale, double *F) {
    oracle_fermion_force_add(L, kappa, U, X2, scale, F);
    force_xy_add(L, U, X2, phi2, -scale * kappa2 * kappa2, F);
}

/* Directional derivative along V of the S_2 force above (the force gradient
 * of the Hasenbusch ratio term, Section 4's Leibniz rule with a source that
 * depends on U).  With chi = Mhat2^+ phi2 and X2 = A^-1 chi, A = Mhat^+ Mhat:
 *   d_V X2 = A^-1 (d_V chi - (d_V A) X2),   d_V chi = dMhat2^+ phi2
 * (one solve), the first force term differentiates as the plain
 * pseudofermion force of X2 with that d_V X2, and the second,
 * -kappa2^2 bc TA W(X, Y) with X = (X2, D_oe X2), Y = (phi2, g5 D_oe g5 phi2),
 * by the vectors and the links:
 *   dX = (d_V X2, dD_oe X2 + D_oe d_V X2),  dY = (0, g5 dD_oe g5 phi2).
 * scale * J is ADDED to Jout; returns the solve's iteration count (-1 on
 * maxiter). */
int oracle_hasen_force_tangent_add(const int L[4], double kappa, double kappa2, const cplx *U, const cplx *phi2,
                                   const cplx *X2, const double *v, double tol, int maxiter, double scale,
                                   double *Jout) {
    long V = lat_volume(L), Vh = V / 2;
    size_t ne = sizeof(cplx) * 12 * Vh, nf = sizeof(cplx) * 12 * V;
    mat3 *Vm = malloc(sizeof(mat3) * 4 * V);
    for (long l = 0; l < 4 * V; l++) Vm[l] = alg_from_components(v + l * 8);
    cplx *dU = malloc(sizeof(cplx) * 4 * V * 9);
    tangent_links(V, U, Vm, dU);
    cplx *dchi = malloc(ne), *Z = malloc(ne), *zero = calloc(12 * Vh, sizeof(cplx));
    dmhat(L, kappa2, U, dU, phi2, dchi, 1);
    int it = pf_tangent_core(L, kappa, U, dU, Vm, X2, dchi, tol, maxiter, scale, Jout, Z);
    cplx *X = malloc(nf), *Y = malloc(nf), *dX = malloc(nf), *dY = malloc(nf), *f = malloc(nf), *g = malloc(nf);
    full_xy(L, U, X2, phi2, X, Y);
    full_xy(L, U, Z, zero, dX, dY);   /* (Z, D_oe Z); dY zero so far */
    even_to_full(L, X2, f);
    hop_to_odd(L, dU, f, g);          /* + dD_oe X2 */
    for (long k = 0; k < V * 12; k++) dX[k] += g[k];
    even_to_full(L, phi2, f);
    apply_g5(V, f);
    hop_to_odd(L, dU, f, g);
    apply_g5(V, g);                   /* g5 dD_oe g5 phi2 */
    for (long k = 0; k < V * 12; k++) dY[k] += g[k];
    double c = -scale * kappa2 * kappa2;
    bilinear_add(L, U, dX, Y, NULL, c, Jout);
    bilinear_add(L, U, X, dY, NULL, c, Jout);
    bilinear_add(L, U, X, Y, Vm, c, Jout);
    free(Vm); free(dU); free(dchi); free(Z); free(zero);
    free(X); free(Y); free(dX); free(dY); free(f); free(g);
    return it;
}

/* ------------------------------------------------------------------ */
/* stout smearing of the links the fermions see                       */
/* (Morningstar and Peardon, Phys. Rev. D 69 (2004) 054501)           */
/* ------------------------------------------------------------------ */

/* exp of an n x n complex matrix (row-major) by Taylor series with scaling and
 * squaring, as mat_exp: scaled to Frobenius norm below 1/8, 24 terms. */
static void matn_exp(int n, const cplx *X, cplx *out) {
    cplx *Y = malloc(sizeof(cplx) * n * n), *term = malloc(sizeof(cplx) * n * n);
    cplx *tmp = malloc(sizeof(cplx) * n * n);
    double nrm = 0;
    for (int k = 0; k < n * n; k++) nrm += creal(X[k] * conj(X[k]));
    nrm = sqrt(nrm);
    int s = 0;
    while (nrm > 0.125) { nrm *= 0.5; s++; }
    for (int k = 0; k < n * n; k++) Y[k] = X[k] * ldexp(1.0, -s);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) out[i * n + j] = term[i * n + j] = (i == j);
    for (int m = 1; m <= 24; m++) {
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) {
                cplx a = 0;
                for (int k = 0; k < n; k++) a += term[i * n + k] * Y[k * n + j];
                tmp[i * n + j] = a / m;
            }
        for (int k = 0; k < n * n; k++) { term[k] = tmp[k]; out[k] += tmp[k]; }
    }
    for (int r = 0; r < s; r++) {
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) {
                cplx a = 0;
                for (int k = 0; k < n; k++) a += out[i * n + k] * out[k * n + j];
                tmp[i * n + j] = a;
            }
        memcpy(out, tmp, sizeof(cplx) * n * n);
    }
    free(Y); free(term); free(tmp);
}

/* derivative of exp at A along B: d/dt exp(A + t B) at t = 0, the upper right
 * block of exp([[A, B], [0, A]]) */
static mat3 dexp(mat3 A, mat3 B) {
    cplx N[36], E[36];
    memset(N, 0, sizeof N);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            N[i * 6 + j] = N[(i + 3) * 6 + j + 3] = A.m[i][j];
            N[i * 6 + j + 3] = B.m[i][j];
        }
    matn_exp(6, N, E);
    mat3 D;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) D.m[i][j] = E[i * 6 + j + 3];
    return D;
}

/* The two staples of link (mu, x) in plane nu, as paths from x to x + mu:
 * U_nu(x) U_mu(x+nu) U_nu(x+mu)^+ and U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu). */
static void stout_paths(int mu, int nu, int up[3], int dn[3]) {
    up[0] = nu + 1; up[1] = mu + 1; up[2] = -(nu + 1);
    dn[0] = -(nu + 1); dn[1] = mu + 1; dn[2] = nu + 1;
}

/* C_mu(x) = rho * (sum of its 6 staples); with xi given, *dC its derivative
 * under U_l -> exp(t xi_l) U_l (path_product) */
static mat3 stout_C(const int L[4], double rho, const cplx *U, long i, int mu, const mat3 *xi, mat3 *dC) {
    mat3 C = m_zero(), D = m_zero();
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        int up[3], dn[3];
        stout_paths(mu, nu, up, dn);
        mat3 d1, d2;
        C = m_add(C, path_product(L, U, i, up, 3, xi, xi ? &d1 : NULL));
        C = m_add(C, path_product(L, U, i, dn, 3, xi, xi ? &d2 : NULL));
        if (xi) D = m_add(D, m_add(d1, d2));
    }
    if (dC) *dC = m_scale(D, rho);
    return m_scale(C, rho);
}

/* One stout level: Omega = C U^+, U' = exp(TA(Omega)) U on every link. */
static void stout_level(const int L[4], double rho, const cplx *U, cplx *Up) {
    long V = lat_volume(L);
#pragma omp parallel for collapse(2) schedule(static)
    for (int mu = 0; mu < 4; mu++)
        for (long i = 0; i < V; i++) {
            mat3 u = link_get(U, V, mu, i);
            mat3 Om = m_mul(stout_C(L, rho, U, i, mu, NULL, NULL), m_dag(u));
            link_put(Up, V, mu, i, m_mul(mat_exp(traceless_antiherm(Om)), u));
        }
}

/* n levels of stout smearing with parameter rho (n = 0: a copy) */
void oracle_stout_smear(const int L[4], double rho, int n, const cplx *U, cplx *Us) {
    long V = lat_volume(L);
    memcpy(Us, U, sizeof(cplx) * 4 * V * 9);
    cplx *T = malloc(sizeof(cplx) * 4 * V * 9);
    for (int k = 0; k < n; k++) {
        stout_level(L, rho, Us, T);
        memcpy(Us, T, sizeof(cplx) * 4 * V * 9);
    }
    free(T);
}

/* Tangent of one level: the links move as dU_l = xi_l U_l; the smeared links
 * then move as dU'_l = xi'_l U'_l, with (product rule, then the derivative of
 * exp) dC from the staples, dOmega = dC U^+ - Omega xi, dA = TA(dOmega),
 * dU' = dexp_A(dA) U + exp(A) xi U. */
static void stout_level_jvp(const int L[4], double rho, const cplx *U, const mat3 *xi, mat3 *xip) {
    long V = lat_volume(L);
#pragma omp parallel for collapse(2) schedule(static)
    for (int mu = 0; mu < 4; mu++)
        for (long i = 0; i < V; i++) {
            long l = (long)mu * V + i;
            mat3 u = link_get(U, V, mu, i), dC;
            mat3 C = stout_C(L, rho, U, i, mu, xi, &dC);
            mat3 Om = m_mul(C, m_dag(u));
            mat3 dOm = m_add(m_mul(dC, m_dag(u)), m_scale(m_mul(Om, xi[l]), -1.0));
            mat3 A = traceless_antiherm(Om), dA = traceless_antiherm(dOm);
            mat3 E = mat_exp(A);
            mat3 up = m_mul(E, u);
            mat3 dup = m_add(m_mul(dexp(A, dA), u), m_mul(m_mul(E, xi[l]), u));
            xip[l] = m_mul(dup, m_dag(up));
        }
}

/* Adjoint of one level: given G' per smeared link (su(3), pairing
 * <X, Y> = -2 Re Tr(X Y) = sum_a x_a y_a), G per input link with
 * <G, xi> = <G', xi'> for every xi.  Per link l, with A = TA(Omega), E = exp(A),
 * Gamma = exp(-A) dexp_A(G'_l) (the adjoint of the exp derivative):
 *   G_l += E^+ G'_l E - TA(Gamma Omega),
 * and, with M = rho U_l^+ Gamma, every link k on a staple S = Lf f R of C_l
 * receives TA(U_k R M Lf) when it is a forward factor f = U_k and
 * -TA(R M Lf U_k^+) when it is a backward one f = U_k^+. */
static void stout_level_vjp(const int L[4], double rho, const cplx *U, const mat3 *Gp, mat3 *G) {
    long V = lat_volume(L);
    mat3 *Ms = malloc(sizeof(mat3) * 4 * V);
    /* the per-link terms (independent across links) */
#pragma omp parallel for collapse(2) schedule(static)
    for (int mu = 0; mu < 4; mu++)
        for (long i = 0; i < V; i++) {
            long l = (long)mu * V + i;
            mat3 u = link_get(U, V, mu, i);
            mat3 Om = m_mul(stout_C(L, rho, U, i, mu, NULL, NULL), m_dag(u));
            mat3 A = traceless_antiherm(Om), E = mat_exp(A);
            mat3 Gam = m_mul(mat_exp(m_scale(A, -1.0)), dexp(A, Gp[l]));
            G[l] = m_add(m_mul(m_mul(m_dag(E), Gp[l]), E), m_scale(traceless_antiherm(m_mul(Gam, Om)), -1.0));
            Ms[l] = m_scale(m_mul(m_dag(u), Gam), rho);
        }
    /* the staple terms, scattered to the links of each staple in turn */
    for (int mu = 0; mu < 4; mu++)
        for (long i = 0; i < V; i++) {
            mat3 M = Ms[(long)mu * V + i];
            for (int nu = 0; nu < 4; nu++) {
                if (nu == mu) continue;
                int paths[2][3];
                stout_paths(mu, nu, paths[0], paths[1]);
                for (int w = 0; w < 2; w++) {
                    /* the path's links and their orientation */
                    long site[3];
                    int dir[3], fwd[3];
                    long y = i;
                    for (int k = 0; k < 3; k++) {
                        int st = paths[w][k], d = abs(st) - 1;
                        dir[k] = d; fwd[k] = st > 0;
                        if (st > 0) { site[k] = y; y = lat_step(L, y, d, +1); }
                        else { y = lat_step(L, y, d, -1); site[k] = y; }
                    }
                    mat3 f[3];
                    for (int k = 0; k < 3; k++) {
                        mat3 uk = link_get(U, V, dir[k], site[k]);
                        f[k] = fwd[k] ? uk : m_dag(uk);
                    }
                    for (int k = 0; k < 3; k++) {
                        mat3 Lf = m_unit(), R = m_unit();
                        for (int j = 0; j < k; j++) Lf = m_mul(Lf, f[j]);
                        for (int j = k + 1; j < 3; j++) R = m_mul(R, f[j]);
                        long lk = (long)dir[k] * V + site[k];
                        mat3 uk = link_get(U, V, dir[k], site[k]);
                        mat3 RML = m_mul(m_mul(R, M), Lf);
                        if (fwd[k]) G[lk] = m_add(G[lk], traceless_antiherm(m_mul(uk, RML)));
                        else G[lk] = m_add(G[lk], m_scale(traceless_antiherm(m_mul(RML, m_dag(uk))), -1.0));
                    }
                }
            }
        }
    free(Ms);
}

/* The n levels U_0 = U, U_{k+1} = stout(U_k), stored consecutively in Ul
 * (n + 1 fields); returns Ul. */
static cplx *stout_levels(const int L[4], double rho, int n, const cplx *U) {
    long V = lat_volume(L), sz = 4 * V * 9;
    cplx *Ul = malloc(sizeof(cplx) * sz * (n + 1));
    memcpy(Ul, U, sizeof(cplx) * sz);
    for (int k = 0; k < n; k++) stout_level(L, rho, Ul + k * sz, Ul + (k + 1) * sz);
    return Ul;
}

/* Tangent of n levels: v (components per thin link) -> vout (per smeared link) */
void oracle_stout_jvp(const int L[4], double rho, int n, const cplx *U, const double *v, double *vout) {
    long V = lat_volume(L), sz = 4 * V * 9;
    cplx *Ul = stout_levels(L, rho, n, U);
    mat3 *a = malloc(sizeof(mat3) * 4 * V), *b = malloc(sizeof(mat3) * 4 * V);
    for (long l = 0; l < 4 * V; l++) a[l] = alg_from_components(v + l * 8);
    for (int k = 0; k < n; k++) {
        stout_level_jvp(L, rho, Ul + k * sz, a, b);
        mat3 *t = a; a = b; b = t;
    }
    for (long l = 0; l < 4 * V; l++) alg_components(traceless_antiherm(a[l]), vout + l * 8);
    free(Ul); free(a); free(b);
}

/* Adjoint of n levels: g (components per smeared link) -> gout (per thin link).
 * With g = the force on the smeared links, gout is the force on the thin ones. */
void oracle_stout_vjp(const int L[4], double rho, int n, const cplx *U, const double *g, double *gout) {
    long V = lat_volume(L), sz = 4 * V * 9;
    cplx *Ul = stout_levels(L, rho, n, U);
    mat3 *a = malloc(sizeof(mat3) * 4 * V), *b = malloc(sizeof(mat3) * 4 * V);
    for (long l = 0; l < 4 * V; l++) a[l] = alg_from_components(g + l * 8);
    for (int k = n - 1; k >= 0; k--) {
        stout_level_vjp(L, rho, Ul + k * sz, a, b);
        mat3 *t = a; a = b; b = t;
    }
    for (long l = 0; l < 4 * V; l++) alg_components(a[l], gout + l * 8);
    free(Ul); free(a); free(b);
}

/* ------------------------------------------------------------------ */
/* total force and integrator                                          */
/* ------------------------------------------------------------------ */

typedef struct {
    double beta, kappa, cg_tol;
    int cg_maxiter;
    int fermions;    /* 0: pure gauge */
    int fg_exact;    /* G stages: 0 displacement form, 1 exact form */
    double c1;       /* rectangle coefficient of the gauge action */
    double stout_rho;
    int stout_n;     /* stout levels of the links the fermions see (0: thin links) */
    double csw;      /* clover coefficient of the fermion matrix (0: Wilson) */
} oracle_action;

/* the links the fermion operator sees: a new smeared copy, or NULL for U itself */
static cplx *fermion_links(const int L[4], const oracle_action *act, const cplx *U) {
    if (act->stout_n <= 0) return NULL;
    cplx *Us = malloc(sizeof(cplx) * 4 * lat_volume(L) * 9);
    oracle_stout_smear(L, act->stout_rho, act->stout_n, U, Us);
    return Us;
}

typedef struct {
    long solves, cg_iters, cg_fail;
} oracle_stats;

static void add_solve(oracle_stats *st, const oracle_action *act, int it) {
    st->solves++;
    if (it < 0) { st->cg_fail++; st->cg_iters += act->cg_maxiter; }
    else st->cg_iters += it;
}

/* F = F_G + F_F at U (F_F needs one CG solve, from zero or from X0 when
 * given); the solution X_e is copied to Xout when given */
static void total_force_from(const int L[4], const oracle_action *act, const cplx *U, const cplx *phi,
                             double *F, oracle_stats *st, cplx *Xout, const cplx *X0) {
    oracle_gauge_force(L, act->beta, act->c1, U, F);
    if (!act->fermions) return;
    long V = lat_volume(L), Vh = V / 2;
    cplx *Us = fermion_links(L, act, U);
    const cplx *Uf = Us ? Us : U;
    cplx *X = malloc(sizeof(cplx) * 12 * Vh);
    if (X0) memcpy(X, X0, sizeof(cplx) * 12 * Vh);
    clover_t cl;
    if (act->csw != 0.0) clover_build(L, act->kappa, act->csw, Uf, &cl, NULL);
    const clover_t *clp = act->csw != 0.0 ? &cl : NULL;
    int it = cg_cl(L, act->kappa, Uf, clp, phi, X, act->cg_tol, act->cg_maxiter, NULL, X0 != NULL);
    add_solve(st, act, it);
    /* the force on the links the fermions see; with smearing it is carried
     * back to the thin ones */
    double *Ff = Us ? calloc(4 * V * 8, sizeof(double)) : F;
    if (clp) clover_force_add(L, act->kappa, Uf, clp, X, NULL, 1.0, 1.0, Ff);
    else oracle_fermion_force_add(L, act->kappa, Uf, X, 1.0, Ff);
    if (Us) {
        double *G = malloc(sizeof(double) * 4 * V * 8);
        oracle_stout_vjp(L, act->stout_rho, act->stout_n, U, Ff, G);
        for (long k = 0; k < 4 * V * 8; k++) F[k] += G[k];
        free(Ff); free(G);
    }
    if (clp) clover_free(&cl);
    if (Xout) memcpy(Xout, X, sizeof(cplx) * 12 * Vh);
    free(X); free(Us);
}

static void total_force_x(const int L[4], const oracle_action *act, const cplx *U, const cplx *phi,
                          double *F, oracle_stats *st, cplx *Xout) {
    total_force_from(L, act, U, phi, F, st, Xout, NULL);
}

static void total_force(const int L[4], const oracle_action *act, const cplx *U, const cplx *phi,
                        double *F, oracle_stats *st) {
    total_force_x(L, act, U, phi, F, st, NULL);
}

/* J = J_V[F] = d/dt F(exp(t V) U) at t = 0 for the total force F = F_G + F_F;
 * X_e = A^-1 phi at U (the fermion part costs one more solve) */
static void total_force_tangent(const int L[4], const oracle_action *act, const cplx *U, const cplx *Xe,
                                const double *v, double *J, oracle_stats *st) {
    oracle_gauge_force_tangent(L, act->beta, act->c1, U, v, J);
    if (!act->fermions) return;
    int it = oracle_fermion_force_tangent_add(L, act->kappa, U, Xe, v, act->cg_tol, act->cg_maxiter, 1.0, J);
    add_solve(st, act, it);
}

/* J_V[F] of the total force at U (pure gauge when fermions == 0); stats3 as
 * in oracle_force (two solves with fermions: X, then d_V X) */
void oracle_force_tangent(const int L[4], double beta, double kappa, int fermions, double cg_tol,
                          int cg_maxiter, const cplx *U, const cplx *phi, const double *v, double *J,
                          long *stats3, double c1) {
    oracle_action act = {beta, kappa, cg_tol, cg_maxiter, fermions, 1, c1, 0.0, 0};
    oracle_stats st = {0, 0, 0};
    long V = lat_volume(L), Vh = V / 2;
    cplx *X = fermions ? malloc(sizeof(cplx) * 12 * Vh) : NULL;
    double *F = malloc(sizeof(double) * 4 * V * 8);
    total_force_x(L, &act, U, phi, F, &st, X);
    total_force_tangent(L, &act, U, X, v, J, &st);
    if (stats3) { stats3[0] = st.solves; stats3[1] = st.cg_iters; stats3[2] = st.cg_fail; }
    free(X); free(F);
}

void oracle_force(const int L[4], double beta, double kappa, int fermions, double cg_tol,
                  int cg_maxiter, const cplx *U, const cplx *phi, double *F, long *stats3, double c1,
                  double stout_rho, int stout_n, double csw) {
    oracle_action act = {beta, kappa, cg_tol, cg_maxiter, fermions, 0, c1, stout_rho, stout_n, csw};
    oracle_stats st = {0, 0, 0};
    total_force(L, &act, U, phi, F, &st);
    if (stats3) { stats3[0] = st.solves; stats3[1] = st.cg_iters; stats3[2] = st.cg_fail; }
}

/* One HMC molecular-dynamics trajectory of nsteps steps of size dt = tau/nsteps.
 * The step is given as a table of stages, each (kind, w, xi):
 *   'P': p += w dt F(U)                                      (S-hat flow)
 *   'Q': U <- exp(w dt P) U                                  (T-hat flow)
 *   'G': the combined S-hat and force-gradient flow of Table 1's last row,
 *        exp(w dt S-hat - xi dt^3 C-hat) with C = {S,{S,T}}.  Since C depends
 *        on U only, its flow is a momentum kick by -(-xi dt^3) grad C, which
 *        for C = sum_a (e_a S)^2 is 2 xi dt^3 J_F[F] with
 *        J_F[F] = d/dt F(exp(tF) U); the whole stage is
 *          exact form:        p += w dt F + 2 xi dt^3 J_F[F]
 *          displacement form: U' = exp((2 xi / w) dt^2 F(U)) U,
 *                             p += w dt F(U')   (same to O(dt^5)).
 * With fg_start, the solve of the displaced force F(U') starts from the
 * solution at U (both are functions of the stage's U alone, so the stage
 * stays a momentum kick by a function of U); without it, from zero.
 * Consecutive P stages (the last of one step and the first of the next) are
 * merged into one, so every P stage costs one force evaluation.
 * eta (compact even sites) is the pseudofermion heatbath noise:
 * phi = Mhat^+ eta is formed first and S_F(start) = eta^+ eta.  When
 * phi_in is given instead (eta NULL), phi = phi_in and S_F(start) is measured
 * with a CG solve (used to run a trajectory backwards on the same phi).
 * dH = H(end) - H(start) summed as per-site differences.
 * Returns 0, or -3 when some CG solve hit maxiter. */
int oracle_trajectory(const int L[4], double beta, double kappa, int fermions, double cg_tol,
                      int cg_maxiter, int fg_exact, int nstages, const char *kinds,
                      const double *ws, const double *xis, double tau, int nsteps, cplx *U,
                      double *P, const cplx *eta, const cplx *phi_in, double *dH, long *stats3, int fg_start,
                      double c1, double stout_rho, int stout_n, double csw) {
    oracle_action act = {beta, kappa, cg_tol, cg_maxiter, fermions, fg_exact, c1, stout_rho, stout_n, csw};
    if (fg_exact && fermions && (stout_n > 0 || csw != 0.0)) return -2;
    oracle_stats st = {0, 0, 0};
    long V = lat_volume(L), Vh = V / 2;
    double dt = tau / nsteps;

    /* expand the step table over all steps and merge neighbouring P stages */
    int nmax = nstages * nsteps, n = 0;
    char *K = malloc(nmax);
    double *W = malloc(sizeof(double) * nmax), *XI = malloc(sizeof(double) * nmax);
    for (int s = 0; s < nsteps; s++)
        for (int k = 0; k < nstages; k++) {
            if (kinds[k] == 'P' && n > 0 && K[n - 1] == 'P') { W[n - 1] += ws[k]; continue; }
            K[n] = kinds[k]; W[n] = ws[k]; XI[n] = xis ? xis[k] : 0.0; n++;
        }

    cplx *phi = NULL;
    double *h0 = malloc(sizeof(double) * V), *h1 = malloc(sizeof(double) * V);
    double *tmp = malloc(sizeof(double) * V);
    double *F = malloc(sizeof(double) * 4 * V * 8), *F2 = malloc(sizeof(double) * 4 * V * 8);
    cplx *Ud = malloc(sizeof(cplx) * 4 * V * 9);
    cplx *Xg = fermions ? malloc(sizeof(cplx) * 12 * Vh) : NULL;
    double *hf0 = NULL, *hf1 = NULL;

    /* start Hamiltonian, per site */
    gauge_density(L, beta, c1, U, h0);
    kinetic_density(L, P, tmp);
    for (long i = 0; i < V; i++) h0[i] += tmp[i];
    if (fermions) {
        phi = malloc(sizeof(cplx) * 12 * Vh);
        hf0 = malloc(sizeof(double) * Vh);
        hf1 = malloc(sizeof(double) * Vh);
        cplx *Us = fermion_links(L, &act, U);
        const cplx *Uf = Us ? Us : U;
        clover_t cl;
        const clover_t *clp = NULL;
        if (csw != 0.0) {
            /* the -2 log det A_oo term, per odd site, is part of H */
            double *ld = malloc(sizeof(double) * V);
            clover_build(L, kappa, csw, Uf, &cl, ld);
            clp = &cl;
            for (long i = 0; i < V; i++)
                if (lat_parity(L, i) == 1) h0[i] += -2.0 * ld[i];
            free(ld);
        }
        if (eta) {
            mhat_cl(L, kappa, Uf, clp, eta, phi, 1);
            for (long k = 0; k < Vh; k++) hf0[k] = vdot_re(12, eta + k * 12, eta + k * 12);
        } else {
            cplx *X0 = malloc(sizeof(cplx) * 12 * Vh);
            memcpy(phi, phi_in, sizeof(cplx) * 12 * Vh);
            int it = cg_cl(L, kappa, Uf, clp, phi, X0, cg_tol, cg_maxiter, NULL, 0);
            st.solves++;
            if (it < 0) { st.cg_fail++; st.cg_iters += cg_maxiter; } else st.cg_iters += it;
            pf_density(Vh, phi, X0, hf0);
            free(X0);
        }
        if (clp) clover_free(&cl);
        free(Us);
    }

    for (int s = 0; s < n; s++) {
        double w = W[s];
        if (K[s] == 'P') {
            total_force(L, &act, U, phi, F, &st);
            for (long k = 0; k < 4 * V * 8; k++) P[k] += w * dt * F[k];
        } else if (K[s] == 'Q') {
            oracle_link_update(L, w * dt, P, U);
        } else if (K[s] == 'G') {
            if (fg_exact) {
                total_force_x(L, &act, U, phi, F, &st, Xg);
                total_force_tangent(L, &act, U, Xg, F, F2, &st);
                for (long k = 0; k < 4 * V * 8; k++)
                    P[k] += w * dt * F[k] + 2.0 * XI[s] * dt * dt * dt * F2[k];
            } else {
                total_force_x(L, &act, U, phi, F, &st, Xg);
                memcpy(Ud, U, sizeof(cplx) * 4 * V * 9);
                oracle_link_update(L, 2.0 * XI[s] / w * dt * dt, F, Ud);
                total_force_from(L, &act, Ud, phi, F2, &st, NULL, fg_start ? Xg : NULL);
                for (long k = 0; k < 4 * V * 8; k++) P[k] += w * dt * F2[k];
            }
        }
    }

    gauge_density(L, beta, c1, U, h1);
    kinetic_density(L, P, tmp);
    for (long i = 0; i < V; i++) h1[i] += tmp[i];
    double d = 0;
    for (long i = 0; i < V; i++) d += h1[i] - h0[i];
    int status = 0;
    if (fermions) {
        cplx *X = malloc(sizeof(cplx) * 12 * Vh);
        cplx *Us = fermion_links(L, &act, U);
        const cplx *Uf = Us ? Us : U;
        clover_t cl;
        const clover_t *clp = NULL;
        if (csw != 0.0) {
            double *ld = malloc(sizeof(double) * V);
            clover_build(L, kappa, csw, Uf, &cl, ld);
            clp = &cl;
            for (long i = 0; i < V; i++)
                if (lat_parity(L, i) == 1) d += -2.0 * ld[i];   /* the start's term is in h0 */
            free(ld);
        }
        int it = cg_cl(L, kappa, Uf, clp, phi, X, cg_tol, cg_maxiter, NULL, 0);
        if (clp) clover_free(&cl);
        free(Us);
        st.solves++;
        if (it < 0) { st.cg_fail++; st.cg_iters += cg_maxiter; } else st.cg_iters += it;
        pf_density(Vh, phi, X, hf1);
        for (long k = 0; k < Vh; k++) d += hf1[k] - hf0[k];
        free(X);
    }
    *dH = d;
    if (st.cg_fail) status = -3;
    if (stats3) { stats3[0] = st.solves; stats3[1] = st.cg_iters; stats3[2] = st.cg_fail; }
    free(K); free(W); free(XI); free(h0); free(h1); free(tmp); free(F); free(F2); free(Ud); free(Xg);
    free(phi); free(hf0); free(hf1);
    return status;
}

/* ------------------------------------------------------------------ */
/* nested (multi time scale) integrator with Hasenbusch terms          */
/* ------------------------------------------------------------------ */

#define TERM_GAUGE 1
#define TERM_FERM 2   /* S_F, or S_1 when kappa2 != 0 */
#define TERM_HASEN 4  /* S_2 */

typedef struct {
    const int *L;
    double beta, c1, kappa, kappa2, tol;
    int maxiter, nlevels;
    const int *nstages, *terms, *nsub;
    const char *const *kinds;
    const double *const *ws, *const *xis;
    const cplx *phi1, *phi2;
    cplx *U;
    double *P;
    oracle_stats st;
    int fg_start;        /* displaced solves start from the undisplaced solutions */
    cplx *X1, *X2;       /* the last solutions of the S_F (S_1) and S_2 solves */
    double stout_rho;
    int stout_n;         /* stout levels of the links the fermions see */
    int fg_exact;        /* G stages in the exact form */
    double csw;          /* clover coefficient (no Hasenbusch split with it) */
} nested_run;

/* the links the fermion terms see at W: a new smeared copy, or NULL for W */
static cplx *nested_fermion_links(const nested_run *r, const cplx *W) {
    if (r->stout_n <= 0) return NULL;
    cplx *Ws = malloc(sizeof(cplx) * 4 * lat_volume(r->L) * 9);
    oracle_stout_smear(r->L, r->stout_rho, r->stout_n, W, Ws);
    return Ws;
}

static void count_solve(nested_run *r, int it) {
    r->st.solves++;
    if (it < 0) { r->st.cg_fail++; r->st.cg_iters += r->maxiter; } else r->st.cg_iters += it;
}

/* F = sum of the forces of the selected terms at links W; with from_last the
 * solves start from the last solutions (r->X1, r->X2), which they replace */
static void terms_force(nested_run *r, const cplx *W, int terms, double *F, int from_last) {
    const int *L = r->L;
    long V = lat_volume(L), Vh = V / 2;
    memset(F, 0, sizeof(double) * 4 * V * 8);
    if (terms & TERM_GAUGE) {
        double *g = malloc(sizeof(double) * 4 * V * 8);
        oracle_gauge_force(L, r->beta, r->c1, W, g);
        for (long k = 0; k < 4 * V * 8; k++) F[k] += g[k];
        free(g);
    }
    if (r->kappa == 0.0 || !(terms & (TERM_FERM | TERM_HASEN))) return;
    /* with smearing the fermion forces are taken on the smeared links and
     * carried back to W */
    cplx *Ws = nested_fermion_links(r, W);
    const cplx *Wf = Ws ? Ws : W;
    double *Ff = Ws ? calloc(4 * V * 8, sizeof(double)) : F;
    if (terms & TERM_FERM) {
        double k1 = r->kappa2 != 0.0 ? r->kappa2 : r->kappa;
        if (r->csw != 0.0) {   /* S_F (S_1 at kappa2) and -2 log det A_oo at kappa */
            clover_t cl;
            clover_build(L, k1, r->csw, Wf, &cl, NULL);
            count_solve(r, cg_cl(L, k1, Wf, &cl, r->phi1, r->X1, r->tol, r->maxiter, NULL, from_last));
            clover_force_add(L, k1, Wf, &cl, r->X1, NULL, 1.0, k1 == r->kappa ? 1.0 : 0.0, Ff);
            clover_free(&cl);
            if (k1 != r->kappa) {
                clover_build(L, r->kappa, r->csw, Wf, &cl, NULL);
                clover_force_add(L, r->kappa, Wf, &cl, NULL, NULL, 0.0, 1.0, Ff);
                clover_free(&cl);
            }
        } else {
            count_solve(r, oracle_cg_from(L, k1, Wf, r->phi1, r->X1, r->tol, r->maxiter, NULL, from_last));
            oracle_fermion_force_add(L, k1, Wf, r->X1, 1.0, Ff);
        }
    }
    if ((terms & TERM_HASEN) && r->kappa2 != 0.0 && r->csw != 0.0) {
        /* S_2 = chi^+ (Mhat^+ Mhat)^-1 chi, chi = Mhat2^+ phi2 (clover at kappa2):
         * the ordinary force of X2 at kappa, plus +2 Re[phi2^+ (e_a Mhat2) X2]
         * from chi, i.e. the bilinear (X2, phi2) of Mhat2 at scale -1 */
        clover_t c1l, c2l;
        clover_build(L, r->kappa, r->csw, Wf, &c1l, NULL);
        clover_build(L, r->kappa2, r->csw, Wf, &c2l, NULL);
        cplx *chi = malloc(sizeof(cplx) * 12 * Vh);
        mhat_cl(L, r->kappa2, Wf, &c2l, r->phi2, chi, 1);
        count_solve(r, cg_cl(L, r->kappa, Wf, &c1l, chi, r->X2, r->tol, r->maxiter, NULL, from_last));
        clover_force_add(L, r->kappa, Wf, &c1l, r->X2, NULL, 1.0, 0.0, Ff);
        clover_force_add(L, r->kappa2, Wf, &c2l, r->X2, r->phi2, -1.0, 0.0, Ff);
        free(chi);
        clover_free(&c1l); clover_free(&c2l);
    } else if ((terms & TERM_HASEN) && r->kappa2 != 0.0) {
        int it;
        hasen_action_from(L, r->kappa, r->kappa2, Wf, r->phi2, r->tol, r->maxiter, r->X2, &it, from_last);
        count_solve(r, it);
        oracle_hasen_force_add(L, r->kappa, r->kappa2, Wf, r->phi2, r->X2, 1.0, Ff);
    }
    if (Ws) {
        double *G = malloc(sizeof(double) * 4 * V * 8);
        oracle_stout_vjp(L, r->stout_rho, r->stout_n, W, Ff, G);
        for (long k = 0; k < 4 * V * 8; k++) F[k] += G[k];
        free(G); free(Ff); free(Ws);
    }
    (void)Vh;
}

/* run level l for n steps of size h: the step table repeated n times with
 * neighbouring P stages merged; a Q stage of an outer level runs the next
 * level for w*h in nsub[l+1] steps; the innermost Q stage updates the links */
/* J = J_V[F_terms] at W (the exact form's force gradient): the gauge part,
 * the S_F (or S_1) part and the S_2 part, whose solutions X1, X2 at W the
 * force evaluation just left in r->X1, r->X2 (one more solve each).  Smeared
 * links have no exact form here (oracle_trajectory_nested refuses them). */
static void terms_tangent(nested_run *r, const cplx *W, int terms, const double *v, double *J) {
    const int *L = r->L;
    long V = lat_volume(L);
    memset(J, 0, sizeof(double) * 4 * V * 8);
    if (terms & TERM_GAUGE) oracle_gauge_force_tangent(L, r->beta, r->c1, W, v, J);
    if (r->kappa != 0.0 && (terms & TERM_FERM)) {
        double k1 = r->kappa2 != 0.0 ? r->kappa2 : r->kappa;
        count_solve(r, oracle_fermion_force_tangent_add(L, k1, W, r->X1, v, r->tol, r->maxiter, 1.0, J));
    }
    if (r->kappa2 != 0.0 && (terms & TERM_HASEN))
        count_solve(r, oracle_hasen_force_tangent_add(L, r->kappa, r->kappa2, W, r->phi2, r->X2, v, r->tol,
                                                      r->maxiter, 1.0, J));
}

static void run_level(nested_run *r, int l, int n, double h) {
    const int *L = r->L;
    long V = lat_volume(L);
    int ns = r->nstages[l], tot = ns * n, m = 0;
    char *K = malloc(tot);
    double *Wt = malloc(sizeof(double) * tot), *XI = malloc(sizeof(double) * tot);
    for (int s = 0; s < n; s++)
        for (int k = 0; k < ns; k++) {
            if (r->kinds[l][k] == 'P' && m > 0 && K[m - 1] == 'P') { Wt[m - 1] += r->ws[l][k]; continue; }
            K[m] = r->kinds[l][k]; Wt[m] = r->ws[l][k]; XI[m] = r->xis[l][k]; m++;
        }
    double *F = malloc(sizeof(double) * 4 * V * 8);
    cplx *Ud = malloc(sizeof(cplx) * 4 * V * 9);
    for (int s = 0; s < m; s++) {
        double w = Wt[s];
        if (K[s] == 'P') {
            terms_force(r, r->U, r->terms[l], F, 0);
            for (long k = 0; k < 4 * V * 8; k++) r->P[k] += w * h * F[k];
        } else if (K[s] == 'Q') {
            if (l + 1 < r->nlevels) run_level(r, l + 1, r->nsub[l + 1], w * h / r->nsub[l + 1]);
            else oracle_link_update(L, w * h, r->P, r->U);
        } else if (r->fg_exact) {
            double *J = malloc(sizeof(double) * 4 * V * 8);
            terms_force(r, r->U, r->terms[l], F, 0);
            terms_tangent(r, r->U, r->terms[l], F, J);
            for (long k = 0; k < 4 * V * 8; k++) r->P[k] += w * h * F[k] + 2.0 * XI[s] * h * h * h * J[k];
            free(J);
        } else {
            terms_force(r, r->U, r->terms[l], F, 0);
            memcpy(Ud, r->U, sizeof(cplx) * 4 * V * 9);
            oracle_link_update(L, 2.0 * XI[s] / w * h * h, F, Ud);
            terms_force(r, Ud, r->terms[l], F, r->fg_start);
            for (long k = 0; k < 4 * V * 8; k++) r->P[k] += w * h * F[k];
        }
    }
    free(K); free(Wt); free(XI); free(F); free(Ud);
}

/* Nested trajectory (level 0 outermost, stage tables concatenated in `kinds`,
 * `ws`, `xis` with nstages[l] entries per level).  Fermions: eta1 (S_F or
 * S_1) and eta2 (S_2, when kappa2 != 0) are heatbath noises.  dH as a sum of
 * per-site differences plus the fermion action differences. */
int oracle_trajectory_nested(const int L[4], double beta, double kappa, double kappa2, double cg_tol,
                             int cg_maxiter, int nlevels, const int *nstages, const int *terms, const int *nsub,
                             const char *kinds, const double *ws, const double *xis, double tau, int nsteps,
                             cplx *U, double *P, const cplx *eta1, const cplx *eta2, double *dH, long *stats3,
                             int fg_start, double c1, double stout_rho, int stout_n, int fg_exact, double csw) {
    if (fg_exact && kappa != 0.0 && stout_n > 0) return -2;
    if (kappa != 0.0 && csw != 0.0 && fg_exact) return -2;
    long V = lat_volume(L), Vh = V / 2;
    const char *kp[8];
    const double *wp[8], *xp[8];
    int off = 0;
    for (int l = 0; l < nlevels && l < 8; l++) {
        kp[l] = kinds + off; wp[l] = ws + off; xp[l] = xis + off;
        off += nstages[l];
    }
    nested_run r = {L, beta, c1, kappa, kappa2, cg_tol, cg_maxiter, nlevels, nstages, terms, nsub, kp, wp, xp,
                    NULL, NULL, U, P, {0, 0, 0}, fg_start, NULL, NULL};
    r.X1 = calloc(12 * Vh, sizeof(cplx));
    r.X2 = calloc(12 * Vh, sizeof(cplx));
    r.stout_rho = stout_rho;
    r.stout_n = stout_n;
    r.fg_exact = fg_exact;
    r.csw = csw;
    cplx *phi1 = NULL, *phi2 = NULL;
    double *h0 = malloc(sizeof(double) * V), *h1 = malloc(sizeof(double) * V), *tmp = malloc(sizeof(double) * V);
    gauge_density(L, beta, c1, U, h0);
    kinetic_density(L, P, tmp);
    for (long i = 0; i < V; i++) h0[i] += tmp[i];
    double sf0 = 0.0;
    if (kappa != 0.0) {
        cplx *Us = nested_fermion_links(&r, U);
        const cplx *Uf = Us ? Us : U;
        phi1 = malloc(sizeof(cplx) * 12 * Vh);
        if (csw != 0.0) {
            /* phi1 = Mhat^+ eta1 (Mhat2 with Hasenbusch); -2 log det A_oo at kappa */
            clover_t cl, c2l;
            double *ld = malloc(sizeof(double) * V);
            clover_build(L, kappa, csw, Uf, &cl, ld);
            for (long i = 0; i < V; i++)
                if (lat_parity(L, i) == 1) sf0 += -2.0 * ld[i];
            if (kappa2 != 0.0) {
                /* phi2 = Mhat2 (Mhat2^+ Mhat2)^-1 Mhat^+ eta2 */
                clover_build(L, kappa2, csw, Uf, &c2l, NULL);
                mhat_cl(L, kappa2, Uf, &c2l, eta1, phi1, 1);
                phi2 = malloc(sizeof(cplx) * 12 * Vh);
                cplx *a = malloc(sizeof(cplx) * 12 * Vh), *x = malloc(sizeof(cplx) * 12 * Vh);
                mhat_cl(L, kappa, Uf, &cl, eta2, a, 1);
                count_solve(&r, cg_cl(L, kappa2, Uf, &c2l, a, x, cg_tol, cg_maxiter, NULL, 0));
                mhat_cl(L, kappa2, Uf, &c2l, x, phi2, 0);
                sf0 += vdot_re(12 * Vh, eta2, eta2);
                free(a); free(x);
                clover_free(&c2l);
            } else {
                mhat_cl(L, kappa, Uf, &cl, eta1, phi1, 1);
            }
            clover_free(&cl);
            free(ld);
        } else {
            oracle_pf_heatbath(L, kappa2 != 0.0 ? kappa2 : kappa, Uf, eta1, phi1);
        }
        sf0 += vdot_re(12 * Vh, eta1, eta1);
        if (kappa2 != 0.0 && csw == 0.0) {
            phi2 = malloc(sizeof(cplx) * 12 * Vh);
            count_solve(&r, oracle_hasen_heatbath(L, kappa, kappa2, Uf, eta2, phi2, cg_tol, cg_maxiter));
            sf0 += vdot_re(12 * Vh, eta2, eta2);
        }
        free(Us);
    }
    r.phi1 = phi1;
    r.phi2 = phi2;
    run_level(&r, 0, nsteps, tau / nsteps);
    gauge_density(L, beta, c1, U, h1);
    kinetic_density(L, P, tmp);
    double d = 0;
    for (long i = 0; i < V; i++) d += (h1[i] + tmp[i]) - h0[i];
    if (kappa != 0.0) {
        int it;
        cplx *Us = nested_fermion_links(&r, U);
        const cplx *Uf = Us ? Us : U;
        double s1;
        if (csw != 0.0) {
            double *ld = malloc(sizeof(double) * V);
            clover_t cl, c2l;
            clover_build(L, kappa, csw, Uf, &cl, ld);
            const double k1 = kappa2 != 0.0 ? kappa2 : kappa;
            if (kappa2 != 0.0) clover_build(L, kappa2, csw, Uf, &c2l, NULL);
            const clover_t *c1p = kappa2 != 0.0 ? &c2l : &cl;
            cplx *X = malloc(sizeof(cplx) * 12 * Vh);
            double *hd = malloc(sizeof(double) * Vh);
            it = cg_cl(L, k1, Uf, c1p, phi1, X, cg_tol, cg_maxiter, NULL, 0);
            pf_density(Vh, phi1, X, hd);
            s1 = 0.0;
            for (long k = 0; k < Vh; k++) s1 += hd[k];
            for (long i = 0; i < V; i++)
                if (lat_parity(L, i) == 1) s1 += -2.0 * ld[i];
            if (kappa2 != 0.0) {
                /* S_2 = chi^+ (Mhat^+ Mhat)^-1 chi, chi = Mhat2^+ phi2 */
                count_solve(&r, it);
                cplx *chi = malloc(sizeof(cplx) * 12 * Vh);
                mhat_cl(L, kappa2, Uf, &c2l, phi2, chi, 1);
                it = cg_cl(L, kappa, Uf, &cl, chi, X, cg_tol, cg_maxiter, NULL, 0);
                pf_density(Vh, chi, X, hd);
                for (long k = 0; k < Vh; k++) s1 += hd[k];
                free(chi);
                clover_free(&c2l);
            }
            clover_free(&cl);
            free(ld); free(X); free(hd);
        } else {
            s1 = oracle_pf_action(L, kappa2 != 0.0 ? kappa2 : kappa, Uf, phi1, cg_tol, cg_maxiter, &it);
        }
        count_solve(&r, it);
        if (kappa2 != 0.0 && csw == 0.0) {
            s1 += oracle_hasen_action(L, kappa, kappa2, Uf, phi2, cg_tol, cg_maxiter, NULL, &it);
            count_solve(&r, it);
        }
        d += s1 - sf0;
        free(Us);
    }
    *dH = d;
    if (stats3) { stats3[0] = r.st.solves; stats3[1] = r.st.cg_iters; stats3[2] = r.st.cg_fail; }
    free(phi1); free(phi2); free(h0); free(h1); free(tmp); free(r.X1); free(r.X2);
    return r.st.cg_fail ? -3 : 0;
}

/* Poisson brackets of Section 3 at (U, P):
 *   SST = {S,{S,T}} = sum_{links,a} (e_a S)^2 = sum F_a^2            (Section 4)
 *   TST = {T,{S,T}} = d/dt <p, F(exp(tP) U)> at t = 0, by a central
 *         difference with step h (needs two force evaluations).         */
void oracle_brackets(const int L[4], double beta, double kappa, int fermions, double cg_tol,
                     int cg_maxiter, const cplx *U, const double *P, const cplx *phi, double h,
                     double *SST, double *TST, double c1, double stout_rho, int stout_n, double csw) {
    long V = lat_volume(L), n = 4 * V * 8;
    oracle_action act = {beta, kappa, cg_tol, cg_maxiter, fermions, 0, c1, stout_rho, stout_n, csw};
    oracle_stats st = {0, 0, 0};
    double *F = malloc(sizeof(double) * n);
    cplx *Ud = malloc(sizeof(cplx) * 4 * V * 9);
    total_force(L, &act, U, phi, F, &st);
    double s = 0;
    for (long k = 0; k < n; k++) s += F[k] * F[k];
    *SST = s;
    double fp = 0, fm = 0;
    memcpy(Ud, U, sizeof(cplx) * 4 * V * 9);
    oracle_link_update(L, h, P, Ud);
    total_force(L, &act, Ud, phi, F, &st);
    for (long k = 0; k < n; k++) fp += P[k] * F[k];
    memcpy(Ud, U, sizeof(cplx) * 4 * V * 9);
    oracle_link_update(L, -h, P, Ud);
    total_force(L, &act, Ud, phi, F, &st);
    for (long k = 0; k < n; k++) fm += P[k] * F[k];
    *TST = (fp - fm) / (2.0 * h);
    free(F); free(Ud);
}

/* The four dt^4 brackets of Table 1 that are not identically zero, at
 * (U, P), for the total force (gauge action with rectangle coefficient c1,
 * plus Wilson pseudofermions when fermions != 0), in the paper's nesting:
 *   STSST = {{S,T},{S,{S,T}}},   STTST = {{S,T},{T,{S,T}}},
 *   TTSST = {T,{T,{S,{S,T}}}},   TTTST = {T,{T,{T,{S,T}}}}.
 * With the flows of the integrator's steps as derivations -- L_T W =
 * d/dt W(exp(tP) U, P) (the T-hat flow) and L_S W = d/ds W(U, P + s F(U))
 * (the S-hat flow) -- one has {T, W} = -L_T W, {S, W} = -L_S W, and by the
 * Jacobi identity {{S,T}, W} = L_S L_T W - L_T L_S W.  With
 * J_V = J_V[F] = d/dt F(exp(tV) U) (the exact force gradient) and D_b G =
 * d/dt G(exp(tb) U), every term reduces to force gradients at U and one
 * derivative of J_P along P or along F:
 *   STSST = L_S L_T |F|^2             = 2 <F, J_F>
 *   STTST = [L_S, L_T] <P, J_P>       = <P, D_F J_P> - |J_P|^2 - <P, J_{J_P}>
 *   TTSST = L_T^2 |F|^2               = 2 |J_P|^2 + 2 <F, D_P J_P>
 *   TTTST = L_T^3 <P, F>              = d^2/dt^2 <P, J_P(exp(tP) U)>
 * (<P, F> = -{S,T}; TST = L_T <P, F> = <P, J_P>; in flat space with
 * J_V = -Hess(S) V these are the familiar -2 g.H.g, K[g,P,P] - 2|HP|^2,
 * 2 K[P,P,g] + 2|HP|^2 and -L[P,P,P,P]).  D_F J_P, D_P J_P and the second
 * derivative are central differences with step h (J_P at exp(+-hP) U and
 * exp(+-hF) U).  Also returns SST = |F|^2 and TST = <P, J_P> (exact here).
 * out = {SST, TST, STSST, STTST, TTSST, TTTST}; returns 0, or -3 when a
 * solve hit maxiter. */
static double dotn(const double *a, const double *b, long n) {
    double s = 0;
    for (long k = 0; k < n; k++) s += a[k] * b[k];
    return s;
}

int oracle_brackets4(const int L[4], double beta, double kappa, int fermions, double cg_tol, int cg_maxiter,
                     const cplx *U, const double *P, const cplx *phi, double h, double c1, double *out) {
    long V = lat_volume(L), Vh = V / 2, n = 4 * V * 8, nu = 4 * V * 9;
    oracle_action act = {beta, kappa, cg_tol, cg_maxiter, fermions, 1, c1, 0.0, 0, 0.0};
    oracle_stats st = {0, 0, 0};
    double *F = malloc(sizeof(double) * n), *Fd = malloc(sizeof(double) * n);
    double *JP = malloc(sizeof(double) * n), *JF = malloc(sizeof(double) * n);
    double *JJ = malloc(sizeof(double) * n), *Jd = malloc(sizeof(double) * n);
    cplx *X = fermions ? malloc(sizeof(cplx) * 12 * Vh) : NULL;
    cplx *Xd = fermions ? malloc(sizeof(cplx) * 12 * Vh) : NULL;
    cplx *Ud = malloc(sizeof(cplx) * nu);
    /* at U: F, J_P, J_F, J_{J_P} */
    total_force_x(L, &act, U, phi, F, &st, X);
    total_force_tangent(L, &act, U, X, P, JP, &st);
    total_force_tangent(L, &act, U, X, F, JF, &st);
    total_force_tangent(L, &act, U, X, JP, JJ, &st);
    double sst = dotn(F, F, n), tst = dotn(P, JP, n), jpjp = dotn(JP, JP, n);
    /* J_P at exp(+-hP) U: D_P J_P and <P, J_P(exp(tP) U)> at t = +-h */
    double fp_p = 0, fp_m = 0, kp = 0, km = 0;
    for (int sgn = 1; sgn >= -1; sgn -= 2) {
        memcpy(Ud, U, sizeof(cplx) * nu);
        oracle_link_update(L, sgn * h, P, Ud);
        total_force_x(L, &act, Ud, phi, Fd, &st, Xd);
        total_force_tangent(L, &act, Ud, Xd, P, Jd, &st);
        if (sgn > 0) { fp_p = dotn(F, Jd, n); kp = dotn(P, Jd, n); }
        else { fp_m = dotn(F, Jd, n); km = dotn(P, Jd, n); }
    }
    /* J_P at exp(+-hF) U: D_F J_P */
    double pf_p = 0, pf_m = 0;
    for (int sgn = 1; sgn >= -1; sgn -= 2) {
        memcpy(Ud, U, sizeof(cplx) * nu);
        oracle_link_update(L, sgn * h, F, Ud);
        total_force_x(L, &act, Ud, phi, Fd, &st, Xd);
        total_force_tangent(L, &act, Ud, Xd, P, Jd, &st);
        if (sgn > 0) pf_p = dotn(P, Jd, n);
        else pf_m = dotn(P, Jd, n);
    }
    const double F_DP_JP = (fp_p - fp_m) / (2.0 * h);
    const double P_DF_JP = (pf_p - pf_m) / (2.0 * h);
    out[0] = sst;
    out[1] = tst;
    out[2] = 2.0 * dotn(F, JF, n);
    out[3] = P_DF_JP - jpjp - dotn(P, JJ, n);
    out[4] = 2.0 * jpjp + 2.0 * F_DP_JP;
    out[5] = (kp - 2.0 * tst + km) / (h * h);
    free(F); free(Fd); free(JP); free(JF); free(JJ); free(Jd); free(X); free(Xd); free(Ud);
    return st.cg_fail ? -3 : 0;
}

/* ------------------------------------------------------------------ */
/* Markov chain: counter-based draws and the HMC accept/reject loop    */
/* ------------------------------------------------------------------ */

/* Philox4x32-10, from its definition in Salmon, Moraes, Dror and Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3" (SC11, 2011): the state is a
 * 128-bit counter (four 32-bit words) and a 64-bit key; a round multiplies
 * words 0 and 2 by 0xD2511F53 and 0xCD9E8D57 into 64-bit products, and the new
 * words are (hi(w2 M1) ^ w1 ^ k0, lo(w2 M1), hi(w0 M0) ^ w3 ^ k1, lo(w0 M0));
 * between rounds the key advances by (0x9E3779B9, 0xBB67AE85).  Ten rounds. */
void oracle_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t w[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t a = (uint64_t)w[0] * 0xD2511F53u;
        uint64_t b = (uint64_t)w[2] * 0xCD9E8D57u;
        uint32_t nw[4];
        nw[0] = (uint32_t)(b >> 32) ^ w[1] ^ k0;
        nw[1] = (uint32_t)b;
        nw[2] = (uint32_t)(a >> 32) ^ w[3] ^ k1;
        nw[3] = (uint32_t)a;
        memcpy(w, nw, sizeof w);
    }
    memcpy(out, w, sizeof w);
}

/* uniform in (0, 1): 32 bits of a and the top 20 of b as m, (m + 1/2) 2^-52 */
static double unif52(uint32_t a, uint32_t b) {
    uint64_t m = ((uint64_t)a << 20) | (uint64_t)(b >> 12);
    return ((double)m + 0.5) / 4503599627370496.0;
}

/* Box-Muller pair of the counter (c0, c1, c2, 0) under the seed's key */
static void normal_pair(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, double *z0, double *z1) {
    uint32_t ctr[4] = {c0, c1, c2, 0u}, key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)}, x[4];
    oracle_philox(ctr, key, x);
    double r = sqrt(-2.0 * log(unif52(x[0], x[1])));
    double phase = 6.283185307179586 * unif52(x[2], x[3]);
    *z0 = r * cos(phase);
    *z1 = r * sin(phase);
}

/* The heatbath draws of trajectory traj of the chain `seed` in the user
 * layouts (any of P, eta1, eta2 may be NULL):
 *   P[mu][i][2j + b], b = 0, 1 the pair of counter (4 (mu V + i) + j, traj, 0)
 *   eta[k][e] = (z0 + i z1) / sqrt(2) of counter (12 k + e, traj, 1 | 2)
 * (e = 3 spin + colour, k the k-th even site). */
void oracle_refresh(const int L[4], uint64_t seed, uint32_t traj, double *P, cplx *eta1, cplx *eta2) {
    long V = lat_volume(L), Vh = V / 2;
    if (P)
        for (long l = 0; l < 4 * V; l++)
            for (int j = 0; j < 4; j++)
                normal_pair(seed, (uint32_t)(4 * l + j), traj, 0u, &P[l * 8 + 2 * j], &P[l * 8 + 2 * j + 1]);
    cplx *etas[2] = {eta1, eta2};
    for (int s = 0; s < 2; s++) {
        if (!etas[s]) continue;
        for (long k = 0; k < Vh; k++)
            for (int e = 0; e < 12; e++) {
                double z0, z1;
                normal_pair(seed, (uint32_t)(12 * k + e), traj, (uint32_t)(1 + s), &z0, &z1);
                etas[s][k * 12 + e] = z0 * 0.7071067811865476 + I * (z1 * 0.7071067811865476);
            }
    }
}

/* the Metropolis uniform of trajectory traj: counter (0, traj, 3) */
double oracle_metropolis_uniform(uint64_t seed, uint32_t traj) {
    uint32_t ctr[4] = {0u, traj, 3u, 0u}, key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)}, x[4];
    oracle_philox(ctr, key, x);
    return unif52(x[0], x[1]);
}

/* HMC Markov chain: for t = traj0 .. traj0 + ntraj - 1, draw P and eta for
 * trajectory t, run one trajectory (oracle_trajectory) from the chain's
 * links, accept when metropolis == 0 or u_t < exp(-dH), then reunitarise the
 * chain's links.  U is updated in place; dH, acc, plaq (average plaquette
 * after each trajectory) may be NULL.  Returns 0, or -3 when a solve failed. */
int oracle_hmc_run(const int L[4], double beta, double kappa, int fermions, double cg_tol, int cg_maxiter,
                   int fg_exact, int nstages, const char *kinds, const double *ws, const double *xis, double tau,
                   int nsteps, cplx *U, uint64_t seed, uint32_t traj0, int ntraj, int metropolis, double *dH,
                   int *acc, double *plaq, int fg_start, double c1, double stout_rho, int stout_n) {
    long V = lat_volume(L), Vh = V / 2;
    double *P = malloc(sizeof(double) * 4 * V * 8);
    cplx *Ut = malloc(sizeof(cplx) * 4 * V * 9);
    cplx *eta = fermions ? malloc(sizeof(cplx) * 12 * Vh) : NULL;
    int status = 0;
    for (int k = 0; k < ntraj; k++) {
        uint32_t t = traj0 + (uint32_t)k;
        oracle_refresh(L, seed, t, P, eta, NULL);
        memcpy(Ut, U, sizeof(cplx) * 4 * V * 9);
        double d = 0.0;
        long st3[3];
        int rc = oracle_trajectory(L, beta, kappa, fermions, cg_tol, cg_maxiter, fg_exact, nstages, kinds, ws, xis,
                                   tau, nsteps, Ut, P, eta, NULL, &d, st3, fg_start, c1, stout_rho, stout_n, 0.0);
        if (rc) status = rc;
        int a = !metropolis || oracle_metropolis_uniform(seed, t) < exp(-d);
        if (a) memcpy(U, Ut, sizeof(cplx) * 4 * V * 9);
        oracle_reunitarize(L, U);
        if (dH) dH[k] = d;
        if (acc) acc[k] = a;
        if (plaq) plaq[k] = oracle_plaquette(L, U);
    }
    free(P); free(Ut); free(eta);
    return status;
}
