/*
 * idp_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, scalar FP64 CPU reference of the second-order
 * invariant-domain-preserving Q1 scheme for the compressible Euler equations
 * (Maier & Kronbichler, "Efficient parallel 3D computation of the
 * compressible Euler equations with an invariant-domain preserving
 * second-order finite-element scheme", arXiv:2007.00094).
 *
 * Only the test-suite, the package smoke check and the benchmark's CPU
 * baseline may load this file.  It shares no code with the HIP library: it
 * builds its own sparsity graph, its own quadrature and its own matrices,
 * and evaluates every formula literally in the paper's order and notation,
 * with sequential loops (rows ascending, columns ascending within a row).
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (no FMA contraction).
 * OpenMP may split independent row loops; results do not depend on the
 * thread count (each row has one writer, reductions are min/sequential).
 *
 * Readings of points the paper leaves open (they are also listed in the
 * design notes of the repository):
 *   - low-order and high-order sums use -(f_j - f_i).c_ij; equal to the
 *     paper's -f_j.c_ij because sum_j c_ij = 0 (partition of unity), and it
 *     keeps a uniform state exactly unchanged;
 *   - the indicator sums over every j in I(i) (the j>i restriction of
 *     Alg. 1 applies to d_ij only), D_i sums all d+2 components, and
 *     alpha_i = 0 when D_i = 0;
 *   - [x]_neg = (|x| - x)/2; a negative two-rarefaction numerator is
 *     clamped to zero (vacuum);
 *   - density bounds from the bar states (with U_ii_bar = U_i), entropy
 *     bound from the states U_j, j in I(i) including i;
 *   - limiter candidate of row i from (U_i, P_ij, bounds_i), symmetrised by
 *     min(l_ij, l_ji); exactly two passes; pass 2 uses the rescaled P;
 *   - Alg. 2: t_R := 1, density-max check then density-min check on the
 *     updated t_R, zero density direction gives t_R = 0, clamp to [0,1];
 *     dPsi_L at t_L, dPsi_R at t_R; Alg. 3 with sign = -1, eps = 2^-52,
 *     Lambda clipped at 0, a zero denominator leaves the end point, new
 *     points clamped into the old bracket; for rho(P) < 0 (third derivative
 *     of Psi positive) the two quadratic roots swap roles;
 *     Psi(t) = rho*eps(U+tP) - phi_min rho(U+tP)^(gamma+1);
 *     Newton iterations and tolerance are parameters (2, 1e-10);
 *   - lambda_i = 1/(card I(i) - 1);  m_i = sum_j m_ij;
 *   - tau from stage 1 of SSP-RK3, held fixed; stages 2 and 3 only flag a
 *     violation of tau <= m_i/(-2 d_ii);
 *   - SSP-RK3 in increment form U^n + theta (E(U) - U^n);
 *   - Dirichlet nodes keep their step-initial state after every stage;
 *   - matrices by 3-point tensor Gauss quadrature (exact for Q1 on
 *     multilinear cells);
 *   - the projected state of the wave-speed bound has the internal energy
 *     of U, so p~ = p and c~ = c (exact identity); n_ij = c_ij (1/|c_ij|);
 *   - x^y by one fixed series method (ora_pow), so that an implementation
 *     following the same steps reproduces these results bit for bit.
 * Parity pins: see tests/test_oracle_*.py.  The relaxation of the bounds
 * (optional, off by default) has no formula in the paper; the one used
 * here widens each bound by (m_i/|Omega|)^(1.5/d), and is pinned by the
 * second-order convergence it restores on a smooth vortex, not by a value
 * the paper prints.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_MAXC 5   /* max components d+2 (d <= 3) */

typedef struct {
    int dim, nc;
    double gamma, cfl, newton_tol;
    int passes, newton_max, relax, literal_alg3;
    int limiter_mode;     /* 0 Alg. 2 candidates; 1 l = 1 (the high-order
                           * update, unlimited); 2 l = 0 (the low-order one) */
    int64_t n, nnz;
    int64_t *row_ptr;     /* [n+1] */
    int64_t *col;         /* [nnz], ascending within a row, diagonal incl. */
    int64_t *tpos;        /* [nnz], position of (j,i) for entry (i,j) */
    double *mij;          /* [nnz] consistent mass matrix */
    double *cij;          /* [nnz][dim] */
    double *mi;           /* [n] lumped mass m_i = sum_j m_ij */
    double *lam;          /* [n] 1/(card I(i) - 1) */
    uint8_t *dirichlet;   /* [n] */
    double volume;        /* sum of |T| (det J quadrature) */
    double mass_total;    /* sum_i m_i in ascending node order (= |Omega|) */
    /* work / debug arrays of the last forward-Euler stage */
    double *dij;          /* [nnz] graph viscosity d^L_ij, diagonal d_ii */
    double *alpha;        /* [n] */
    double *R;            /* [n][nc] */
    double *UL;           /* [n][nc] */
    double *bnd;          /* [n][3] rho_min, rho_max, phi_min */
    double *P;            /* [nnz][nc] current limiter directions */
    double *l1, *l2;      /* [nnz] limiter candidates, pass 1 and 2 */
    double *Upass;        /* [n][nc] state after pass 1 */
    double *taui;         /* [n] m_i/(-2 d_ii) */
    double last_tau_bound;  /* min_i taui of the last stage */
} ora_t;

/* ------------------------------------------------------------ x^y */
/* x^y for x > 0 (and 0^y = 0 for y > 0) by one fixed, published method so that every
 * implementation of this scheme that follows the same steps produces the
 * same bits: binary exponent reduction x = m 2^e with m in [sqrt(1/2),
 * sqrt(2)); ln m = 2 atanh(s), s = (m-1)/(m+1), by its odd power series
 * (11 terms, Horner in s^2); ln x = e ln2_hi + (e ln2_lo + ln m) with the
 * two-part ln 2 of Cody and Waite, kept as a two-term sum; z = y ln x as a
 * two-term sum (Dekker product via fma); exp z by z = k ln2 + r,
 * |r| <= ln2/2, and the Taylor series of e^r to degree 14 (Horner), scaled
 * by 2^k.
 * Relative error a few units in the last place (pinned against a
 * 60-digit reference in the tests).  The paper uses a vectorised library
 * pow; it fixes no particular method.                                     */
#define ORA_LN2_HI 6.93147180369123816490e-01
#define ORA_LN2_LO 1.90821492927058770002e-10
#define ORA_INV_LN2 1.44269504088896338700e+00
#define ORA_SQRT_HALF 0.70710678118654752440

static double ora_atanh_c[12];   /* 1/(2k+1), k = 0..11 */
static double ora_inv_fact[15];  /* 1/n!, n = 0..14, by repeated division */
static int ora_pow_ready = 0;

static void ora_pow_init(void)
{
    if (ora_pow_ready) return;
    for (int k = 0; k < 12; ++k) ora_atanh_c[k] = 1.0 / (double)(2 * k + 1);
    ora_inv_fact[0] = 1.0;
    for (int n = 1; n < 15; ++n) ora_inv_fact[n] = ora_inv_fact[n - 1] / (double)n;
    ora_pow_ready = 1;
}

double ora_pow(double x, double y)
{
    ora_pow_init();
    if (x == 0.0 && y > 0.0) return 0.0;
    if (!(x > 0.0) || isinf(x) || isnan(y)) return NAN;
    int e;
    double m = frexp(x, &e);
    if (m < ORA_SQRT_HALF) { m = 2.0 * m; e -= 1; }
    double s = (m - 1.0) / (m + 1.0);
    double s2 = s * s;
    double t = ora_atanh_c[11];
    for (int k = 10; k >= 1; --k) t = t * s2 + ora_atanh_c[k];
    double w = 2.0 * s;
    double lnm = w + w * (s2 * t);
    /* ln x = lh + ll (Fast2Sum: |e ln2_hi| >= |ln m| when e != 0) */
    double de = (double)e;
    double A = de * ORA_LN2_HI;
    double B = de * ORA_LN2_LO + lnm;
    double lh = A + B;
    double ll = (A - lh) + B;
    /* z = y ln x = zh + zl, exact product of y and lh by one fma */
    double zh = y * lh;
    double zl = fma(y, lh, -zh) + y * ll;
    if (zh > 709.78) return INFINITY;
    if (zh < -745.0) return 0.0;
    double k = rint(zh * ORA_INV_LN2);
    double r = ((zh - k * ORA_LN2_HI) - k * ORA_LN2_LO) + zl;
    double p = ora_inv_fact[14];
    for (int n = 13; n >= 0; --n) p = p * r + ora_inv_fact[n];
    return ldexp(p, (int)k);
}

/* ------------------------------------------------------------------ EOS */
/* Section 2: v = m/rho, eps = E - |m|^2/(2 rho) (internal energy per
 * volume), p = (gamma-1) eps, c = sqrt(gamma p/rho), phi = eps rho^-gamma,
 * eta = (rho eps)^(1/(gamma+1)).                                          */

static double ora_internal_energy(const double *U, int dim)
{
    double m2 = 0.0;
    for (int k = 0; k < dim; ++k) m2 += U[1 + k] * U[1 + k];
    return U[dim + 1] - 0.5 * m2 / U[0];
}

double ora_pressure(const double *U, int dim, double gamma)
{
    return (gamma - 1.0) * ora_internal_energy(U, dim);
}

double ora_speed_of_sound(const double *U, int dim, double gamma)
{
    return sqrt(gamma * ora_pressure(U, dim, gamma) / U[0]);
}

/* eq. specific_entropy: phi(U) = eps rho^(-gamma) */
double ora_specific_entropy(const double *U, int dim, double gamma)
{
    return ora_internal_energy(U, dim) * ora_pow(U[0], -gamma);
}

/* Harten-type entropy eta(U) = (rho eps)^(1/(gamma+1)) */
double ora_harten_entropy(const double *U, int dim, double gamma)
{
    return ora_pow(U[0] * ora_internal_energy(U, dim), 1.0 / (gamma + 1.0));
}

/* Section 3.8: eta'(U) = (rho eps)^(-gamma/(gamma+1))/(gamma+1) (E,-m,rho) */
void ora_harten_entropy_derivative(const double *U, int dim, double gamma,
                                   double *out)
{
    double re = U[0] * ora_internal_energy(U, dim);
    double f = ora_pow(re, -gamma / (gamma + 1.0)) / (gamma + 1.0);
    out[0] = f * U[dim + 1];
    for (int k = 0; k < dim; ++k) out[1 + k] = -f * U[1 + k];
    out[dim + 1] = f * U[0];
}

/* eq. flux contracted with a vector c: f(U).c, rows (rho, m, E)
 * f(U) = (m, v (x) m + p I, v (E + p))^T                                 */
static void ora_flux(const double *U, int dim, double gamma, double F[][3])
{
    double rho = U[0], E = U[dim + 1];
    double p = ora_pressure(U, dim, gamma);
    double v[3];
    for (int k = 0; k < dim; ++k) v[k] = U[1 + k] / rho;
    for (int k = 0; k < dim; ++k) F[0][k] = U[1 + k];
    for (int a = 0; a < dim; ++a)
        for (int k = 0; k < dim; ++k)
            F[1 + a][k] = v[k] * U[1 + a] + (a == k ? p : 0.0);
    for (int k = 0; k < dim; ++k) F[dim + 1][k] = v[k] * (E + p);
}

/* (f(U_j) - f(U_i)) . c  ->  out[nc] */
static void ora_flux_diff_dot(const double *Ui, const double *Uj,
                              const double *c, int dim, double gamma,
                              double *out)
{
    double Fi[ORA_MAXC][3], Fj[ORA_MAXC][3];
    ora_flux(Ui, dim, gamma, Fi);
    ora_flux(Uj, dim, gamma, Fj);
    for (int r = 0; r < dim + 2; ++r) {
        double s = 0.0;
        for (int k = 0; k < dim; ++k) s += (Fj[r][k] - Fi[r][k]) * c[k];
        out[r] = s;
    }
}

static double pos_part(double x) { return 0.5 * (fabs(x) + x); }
static double neg_part(double x) { return 0.5 * (fabs(x) - x); }

/* ------------------------------------------------- approximate Riemann */
/* Section 3.7 projected 1D state: rho~ = rho, m~ = n.m, u~ = m~/rho~ and
 * E~ = E - |m - m~ n|^2/(2 rho).  Its internal energy
 * E~ - m~^2/(2 rho) = E - |m|^2/(2 rho) equals that of U (Pythagoras), so
 * p~ = p(U) and c~ = c(U); they are evaluated in that form.             */
typedef struct { double rho, u, p, c; } ora_state1d;

static ora_state1d ora_project(const double *U, const double *n, int dim,
                               double gamma)
{
    ora_state1d s;
    double mt = 0.0;
    for (int k = 0; k < dim; ++k) mt += n[k] * U[1 + k];
    s.rho = U[0];
    s.u = mt / U[0];
    s.p = ora_pressure(U, dim, gamma);
    s.c = ora_speed_of_sound(U, dim, gamma);
    return s;
}

/* f(U, p) of the monotone, concave function psi (Section 3.7) */
static double ora_psi_branch(const ora_state1d *s, double p, double gamma)
{
    if (p >= s->p)
        return sqrt(2.0) * (p - s->p) /
               sqrt(s->rho * ((gamma + 1.0) * p + (gamma - 1.0) * s->p));
    return (ora_pow(p / s->p, (gamma - 1.0) / (2.0 * gamma)) - 1.0) *
           2.0 * s->c / (gamma - 1.0);
}

/* Guaranteed upper bound lambda~_max(n, U_i, U_j); optionally p*. */
double ora_lambda_max(const double *n, const double *Ui, const double *Uj,
                      int dim, double gamma, double *pstar_out)
{
    ora_state1d si = ora_project(Ui, n, dim, gamma);
    ora_state1d sj = ora_project(Uj, n, dim, gamma);
    /* two-rarefaction pressure */
    double num = si.c + sj.c - 0.5 * (gamma - 1.0) * (sj.u - si.u);
    double den = si.c * ora_pow(si.p / sj.p, -(gamma - 1.0) / (2.0 * gamma)) + sj.c;
    double ptilde = sj.p * ora_pow(pos_part(num) / den, 2.0 * gamma / (gamma - 1.0));
    double pmax = si.p > sj.p ? si.p : sj.p;
    double psi = ora_psi_branch(&si, pmax, gamma) +
                 ora_psi_branch(&sj, pmax, gamma) + sj.u - si.u;
    double pstar;
    if (psi < 0.0)
        pstar = ptilde;
    else
        pstar = pmax < ptilde ? pmax : ptilde;
    double f = (gamma + 1.0) / (2.0 * gamma);
    double lam1 = si.u - si.c * sqrt(1.0 + f * pos_part((pstar - si.p) / si.p));
    double lam3 = sj.u + sj.c * sqrt(1.0 + f * pos_part((pstar - sj.p) / sj.p));
    double a = neg_part(lam1), b = pos_part(lam3);
    if (pstar_out) *pstar_out = pstar;
    return a > b ? a : b;
}

/* ------------------------------------------------------------- limiter */
/* Psi(t) = rho eps(U + tP) - phi_min rho(U + tP)^(gamma+1); Psi'(t).     */
static void ora_psi_line(const double *U, const double *P, double t,
                         double phi_min, int dim, double gamma,
                         double *psi, double *dpsi)
{
    double V[ORA_MAXC];
    for (int k = 0; k < dim + 2; ++k) V[k] = U[k] + t * P[k];
    double rho = V[0], E = V[dim + 1];
    double m2 = 0.0, mP = 0.0;
    for (int k = 0; k < dim; ++k) {
        m2 += V[1 + k] * V[1 + k];
        mP += V[1 + k] * P[1 + k];
    }
    double rho_eps = rho * E - 0.5 * m2;
    double rg1 = ora_pow(rho, gamma + 1.0);
    if (psi) *psi = rho_eps - phi_min * rg1;
    if (dpsi)
        *dpsi = P[0] * E + rho * P[dim + 1] - mP -
                phi_min * (gamma + 1.0) * (rg1 / rho) * P[0];
}

/* One step of the quadratic enclosure of Alg. 3.  The bracket [a, b] has
 * Psi(a) = fa >= 0 > Psi(b) = fb and slopes ga, gb.  Divided differences
 * over the width w = b - a (kept positive by 2^-52): p = (fb - fa)/w,
 * ka = (p - ga)/w, kb = (gb - p)/w.  The quadratic through (a, fa, ga) and
 * (b, fb) is fa + ga (t - a) + ka (t - a)^2, the one through (b, fb, gb)
 * and (a, fa) is fb + gb (t - b) + kb (t - b)^2.  Along the line the third
 * derivative of Psi has the sign of -rho(P), so (Hermite remainder) for
 * rho(P) >= 0 the first quadratic stays below Psi on [a, b] and its root
 * is an admissible new a, the root of the second a new b; for rho(P) < 0
 * the roots change roles (unless literal, which keeps the printed
 * assignment).  Each root nearest its expansion point t0 is computed as
 * t0 - 2 f/(g - sqrt(g^2 - 4 f k)); a negative discriminant counts as 0
 * and a zero denominator keeps t0.  The new end points are clamped into
 * [a, b] and kept ordered.                                                */
static void ora_enclosure_step(double *a, double *b, double fa, double fb,
                               double ga, double gb, double rhoP, int literal)
{
    double w_inv = 1.0 / (*b - *a + 0x1p-52);
    double slope = (fb - fa) * w_inv;
    double ka = (slope - ga) * w_inv;
    double kb = (gb - slope) * w_inv;
    double disc_a = ga * ga - 4.0 * fa * ka;
    double disc_b = gb * gb - 4.0 * fb * kb;
    if (disc_a < 0.0) disc_a = 0.0;
    if (disc_b < 0.0) disc_b = 0.0;
    double den_a = ga - sqrt(disc_a);
    double den_b = gb - sqrt(disc_b);
    double root_a = *a, root_b = *b;
    if (den_a != 0.0) root_a = *a - 2.0 * fa / den_a;
    if (den_b != 0.0) root_b = *b - 2.0 * fb / den_b;
    int swap = rhoP < 0.0 && !literal;
    double na = swap ? root_b : root_a;
    double nb = swap ? root_a : root_b;
    if (!(na >= *a)) na = *a;
    if (!(na <= *b)) na = *b;
    if (!(nb <= *b)) nb = *b;
    if (!(nb >= *a)) nb = *a;
    if (nb < na) nb = na;
    *a = na;
    *b = nb;
}

/* Limiter of Section 3.9 (Alg. 2): the largest t in [0, 1] found along
 * U + t P with rho in [rho_min, rho_max] and Psi(t) >= 0.  The density is
 * linear in t: cut t = 1 where it leaves a violated bound (the maximum
 * tested first, then the minimum at the cut value; a zero density
 * direction gives 0) and keep the cut in [0, 1].  Then at most newton_max
 * enclosure steps on [a, b] = [0, cut]: stop with b if Psi(b) >= 0, with a
 * if Psi(a) <= TOL.                                                       */
double ora_limiter(const double *U, const double *P, const double *bounds,
                   int dim, double gamma, int newton_max, double tol,
                   int literal_alg3)
{
    const double rho_min = bounds[0], rho_max = bounds[1], phi_min = bounds[2];
    const double rho0 = U[0], drho = P[0];
    double b = 1.0;
    if (rho0 + b * drho > rho_max)
        b = drho != 0.0 ? fabs(rho_max - rho0) / fabs(drho) : 0.0;
    if (rho0 + b * drho < rho_min)
        b = drho != 0.0 ? fabs(rho_min - rho0) / fabs(drho) : 0.0;
    if (b > 1.0) b = 1.0;
    if (b < 0.0) b = 0.0;
    double a = 0.0;
    for (int step = 0; step < newton_max; ++step) {
        double fb, fa, ga, gb;
        ora_psi_line(U, P, b, phi_min, dim, gamma, &fb, NULL);
        if (fb >= 0.0) return b;
        ora_psi_line(U, P, a, phi_min, dim, gamma, &fa, NULL);
        if (fa <= tol) return a;
        ora_psi_line(U, P, a, phi_min, dim, gamma, NULL, &ga);
        ora_psi_line(U, P, b, phi_min, dim, gamma, NULL, &gb);
        ora_enclosure_step(&a, &b, fa, fb, ga, gb, drho, literal_alg3);
    }
    return a;
}

/* ---------------------------------------------------------- geometry */
/* Q1 basis on the reference cell [0,1]^d, vertex b = bx + 2by + 4bz.    */
static double q1_phi(int b, const double *xi, int dim)
{
    double v = 1.0;
    for (int k = 0; k < dim; ++k)
        v *= ((b >> k) & 1) ? xi[k] : 1.0 - xi[k];
    return v;
}

static void q1_grad(int b, const double *xi, int dim, double *g)
{
    for (int k = 0; k < dim; ++k) {
        double v = ((b >> k) & 1) ? 1.0 : -1.0;
        for (int l = 0; l < dim; ++l)
            if (l != k) v *= ((b >> l) & 1) ? xi[l] : 1.0 - xi[l];
        g[k] = v;
    }
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

static int64_t find_col(const ora_t *o, int64_t i, int64_t j)
{
    int64_t lo = o->row_ptr[i], hi = o->row_ptr[i + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (o->col[mid] == j) return mid;
        if (o->col[mid] < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

void ora_destroy(ora_t *o)
{
    if (!o) return;
    free(o->row_ptr); free(o->col); free(o->tpos); free(o->mij);
    free(o->cij); free(o->mi); free(o->lam); free(o->dirichlet);
    free(o->dij); free(o->alpha); free(o->R); free(o->UL); free(o->bnd);
    free(o->P); free(o->l1); free(o->l2); free(o->Upass); free(o->taui);
    free(o);
}

/* Build the stencil graph I(i) and the matrices m_ij, c_ij, m_i (eq.
 * matrices) from a Q1 mesh.  Returns NULL on allocation failure; *err = -2
 * if some cell has det J <= 0 at a quadrature point.                     */
ora_t *ora_create(int dim, double gamma, double cfl, int passes,
                  int newton_max, double newton_tol, int relax,
                  int64_t n, const double *coords, int64_t ncells,
                  const int64_t *cells, const uint8_t *dirichlet, int *err)
{
    *err = 0;
    if (dim < 2 || dim > 3 || n <= 0 || ncells <= 0) { *err = -1; return NULL; }
    ora_t *o = (ora_t *)calloc(1, sizeof(ora_t));
    if (!o) { *err = -3; return NULL; }
    o->dim = dim; o->nc = dim + 2; o->gamma = gamma; o->cfl = cfl;
    o->passes = passes; o->newton_max = newton_max;
    o->newton_tol = newton_tol; o->relax = relax; o->n = n;
    int nv = 1 << dim;
    for (int64_t t = 0; t < ncells * nv; ++t)
        if (cells[t] < 0 || cells[t] >= n) { *err = -1; ora_destroy(o); return NULL; }
    /* node -> cells */
    int64_t *ncnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t t = 0; t < ncells * nv; ++t) ncnt[cells[t] + 1]++;
    for (int64_t i = 0; i < n; ++i) ncnt[i + 1] += ncnt[i];
    int64_t *nlist = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncells * nv));
    int64_t *fill = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    for (int64_t c = 0; c < ncells; ++c)
        for (int b = 0; b < nv; ++b) {
            int64_t v = cells[c * nv + b];
            nlist[ncnt[v] + fill[v]++] = c;
        }
    /* rows: sorted unique union of the cells' vertices */
    o->row_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t maxcand = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = (ncnt[i + 1] - ncnt[i]) * nv;
        if (k > maxcand) maxcand = k;
    }
    int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)(maxcand + 1));
    for (int64_t pass = 0; pass < 2; ++pass) {
        int64_t nnz = 0;
        for (int64_t i = 0; i < n; ++i) {
            int64_t k = 0;
            for (int64_t q = ncnt[i]; q < ncnt[i + 1]; ++q)
                for (int b = 0; b < nv; ++b) cand[k++] = cells[nlist[q] * nv + b];
            qsort(cand, (size_t)k, sizeof(int64_t), cmp_i64);
            int64_t u = 0;
            for (int64_t q = 0; q < k; ++q)
                if (u == 0 || cand[q] != cand[u - 1]) cand[u++] = cand[q];
            if (pass == 0) o->row_ptr[i + 1] = o->row_ptr[i] + u;
            else for (int64_t q = 0; q < u; ++q) o->col[nnz + q] = cand[q];
            nnz += u;
        }
        if (pass == 0) {
            o->nnz = nnz;
            o->col = (int64_t *)malloc(sizeof(int64_t) * (size_t)nnz);
        }
    }
    free(cand); free(fill);
    int64_t Z = o->nnz;
    o->tpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)Z);
    o->mij = (double *)calloc((size_t)Z, sizeof(double));
    o->cij = (double *)calloc((size_t)Z * dim, sizeof(double));
    o->mi = (double *)calloc((size_t)n, sizeof(double));
    o->lam = (double *)calloc((size_t)n, sizeof(double));
    o->dirichlet = (uint8_t *)calloc((size_t)n, 1);
    o->dij = (double *)calloc((size_t)Z, sizeof(double));
    o->alpha = (double *)calloc((size_t)n, sizeof(double));
    o->R = (double *)calloc((size_t)n * o->nc, sizeof(double));
    o->UL = (double *)calloc((size_t)n * o->nc, sizeof(double));
    o->bnd = (double *)calloc((size_t)n * 3, sizeof(double));
    o->P = (double *)calloc((size_t)Z * o->nc, sizeof(double));
    o->l1 = (double *)calloc((size_t)Z, sizeof(double));
    o->l2 = (double *)calloc((size_t)Z, sizeof(double));
    o->Upass = (double *)calloc((size_t)n * o->nc, sizeof(double));
    o->taui = (double *)calloc((size_t)n, sizeof(double));
    if (!o->tpos || !o->mij || !o->cij || !o->P || !o->taui) {
        free(ncnt); free(nlist); ora_destroy(o); *err = -3; return NULL;
    }
    if (dirichlet) memcpy(o->dirichlet, dirichlet, (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t q = o->row_ptr[i]; q < o->row_ptr[i + 1]; ++q)
            o->tpos[q] = find_col(o, o->col[q], i);
    /* quadrature: 3-point Gauss-Legendre on [0,1] per direction */
    const double gx[3] = {0.5 - 0.5 * sqrt(0.6), 0.5, 0.5 + 0.5 * sqrt(0.6)};
    const double gw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    int nq = dim == 2 ? 9 : 27;
    o->volume = 0.0;
    for (int64_t c = 0; c < ncells; ++c) {
        const int64_t *vx = cells + c * nv;
        double mloc[8][8], cloc[8][8][3];
        memset(mloc, 0, sizeof(mloc));
        memset(cloc, 0, sizeof(cloc));
        for (int q = 0; q < nq; ++q) {
            double xi[3];
            double w = 1.0;
            int qq = q;
            for (int k = 0; k < dim; ++k) {
                xi[k] = gx[qq % 3];
                w *= gw[qq % 3];
                qq /= 3;
            }
            /* J_pk = d x_p / d xi_k */
            double J[3][3] = {{0}};
            double gr[8][3], ph[8];
            for (int b = 0; b < nv; ++b) {
                q1_grad(b, xi, dim, gr[b]);
                ph[b] = q1_phi(b, xi, dim);
                const double *xb = coords + vx[b] * dim;
                for (int p = 0; p < dim; ++p)
                    for (int k = 0; k < dim; ++k) J[p][k] += xb[p] * gr[b][k];
            }
            double det, Jinv[3][3];
            if (dim == 2) {
                det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
                Jinv[0][0] = J[1][1] / det;  Jinv[0][1] = -J[0][1] / det;
                Jinv[1][0] = -J[1][0] / det; Jinv[1][1] = J[0][0] / det;
            } else {
                det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                      J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                      J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                Jinv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
                Jinv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
                Jinv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
                Jinv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
                Jinv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
                Jinv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
                Jinv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
                Jinv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
                Jinv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
            }
            if (!(det > 0.0)) {
                free(ncnt); free(nlist); ora_destroy(o); *err = -2; return NULL;
            }
            double wd = w * det;
            o->volume += wd;
            /* physical gradients: grad phi_b = J^{-T} grad_ref phi_b */
            double gp[8][3];
            for (int b = 0; b < nv; ++b)
                for (int p = 0; p < dim; ++p) {
                    double s = 0.0;
                    for (int k = 0; k < dim; ++k) s += Jinv[k][p] * gr[b][k];
                    gp[b][p] = s;
                }
            for (int a = 0; a < nv; ++a)
                for (int b = 0; b < nv; ++b) {
                    mloc[a][b] += wd * (ph[a] * ph[b]); /* symmetric in a,b */
                    for (int p = 0; p < dim; ++p)
                        cloc[a][b][p] += wd * ph[a] * gp[b][p];
                }
        }
        for (int a = 0; a < nv; ++a)
            for (int b = 0; b < nv; ++b) {
                int64_t pos = find_col(o, vx[a], vx[b]);
                o->mij[pos] += mloc[a][b];
                for (int p = 0; p < dim; ++p)
                    o->cij[pos * dim + p] += cloc[a][b][p];
            }
    }
    free(ncnt); free(nlist);
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t q = o->row_ptr[i]; q < o->row_ptr[i + 1]; ++q) s += o->mij[q];
        o->mi[i] = s;
        o->lam[i] = 1.0 / (double)(o->row_ptr[i + 1] - o->row_ptr[i] - 1);
    }
    o->mass_total = 0.0;
    for (int64_t i = 0; i < n; ++i) o->mass_total += o->mi[i];
    return o;
}

/* ------------------------------------------------- forward Euler stage */
/* Whether a pair's coefficients are opposite: c_ij + c_ji is the boundary
 * integral of phi_i phi_j n (zero whenever i or j is an interior node),
 * so the test separates pairs where it vanishes, whose assembled sum is
 * rounding noise, from boundary pairs, where it is of the size of c_ij:
 * sum_k |c_ij,k + c_ji,k| <= 2^-36 sum_k (|c_ij,k| + |c_ji,k|).          */
static int ora_mirror_pair(const double *cij, const double *cji, int dim)
{
    double s = 0.0, m = 0.0;
    for (int k = 0; k < dim; ++k) {
        s += fabs(cij[k] + cji[k]);
        m += fabs(cij[k]) + fabs(cji[k]);
    }
    return s <= 0x1p-36 * m;
}

static void stage_viscosity(ora_t *o, const double *U)
{
    const int dim = o->dim, nc = o->nc;
    const double g = o->gamma;
    /* Steps 1 and 2 of Alg. 1: d_ij for j != i (both orientations, the
     * larger wins; one where they mirror each other), d_ii = -sum,
     * alpha_i, tau_i = m_i/(-2 d_ii).                                     */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < o->n; ++i) {
        const double *Ui = U + i * nc;
        double dsum = 0.0;
        int64_t diag_pos = -1;
        for (int64_t q = o->row_ptr[i]; q < o->row_ptr[i + 1]; ++q) {
            int64_t j = o->col[q];
            if (j == i) { diag_pos = q; continue; }
            const double *Uj = U + j * nc;
            const double *cij = o->cij + q * dim;
            const double *cji = o->cij + o->tpos[q] * dim;
            double nij[3], nji[3], aij = 0.0, aji = 0.0;
            for (int k = 0; k < dim; ++k) { aij += cij[k] * cij[k]; aji += cji[k] * cji[k]; }
            aij = sqrt(aij); aji = sqrt(aji);
            double t1 = 0.0, t2 = 0.0;
            if (ora_mirror_pair(cij, cji, dim)) {
                /* c_ji = -c_ij: the problem (n_ji, U_j, U_i) mirrors
                 * (n_ij, U_i, U_j) and has the same bound; the pair's
                 * lower node id gives the orientation evaluated.          */
                const double *ca = i < j ? cij : cji;
                const double *Ua = i < j ? Ui : Uj, *Ub = i < j ? Uj : Ui;
                const double a = i < j ? aij : aji;
                if (a > 0.0) {
                    double inv = 1.0 / a;
                    for (int k = 0; k < dim; ++k) nij[k] = ca[k] * inv;
                    t1 = ora_lambda_max(nij, Ua, Ub, dim, g, NULL) * a;
                }
            } else {
                if (aij > 0.0) {
                    double inv = 1.0 / aij;
                    for (int k = 0; k < dim; ++k) nij[k] = cij[k] * inv;
                    t1 = ora_lambda_max(nij, Ui, Uj, dim, g, NULL) * aij;
                }
                if (aji > 0.0) {
                    double inv = 1.0 / aji;
                    for (int k = 0; k < dim; ++k) nji[k] = cji[k] * inv;
                    t2 = ora_lambda_max(nji, Uj, Ui, dim, g, NULL) * aji;
                }
            }
            double d = t1 > t2 ? t1 : t2;
            o->dij[q] = d;
            dsum += d;
        }
        o->dij[diag_pos] = -dsum;
        o->taui[i] = o->mi[i] / (-2.0 * o->dij[diag_pos]);

        /* Section 3.8 indicator over all j in I(i) */
        double eta_i = ora_harten_entropy(Ui, dim, g);
        double etap[ORA_MAXC];
        ora_harten_entropy_derivative(Ui, dim, g, etap);
        double er_i = eta_i / Ui[0];
        double a = 0.0, b[ORA_MAXC] = {0};
        for (int64_t q = o->row_ptr[i]; q < o->row_ptr[i + 1]; ++q) {
            int64_t j = o->col[q];
            const double *Uj = U + j * nc;
            const double *cij = o->cij + q * dim;
            double er_j = ora_harten_entropy(Uj, dim, g) / Uj[0];
            double mc = 0.0;
            for (int k = 0; k < dim; ++k) mc += Uj[1 + k] * cij[k];
            a += (er_j - er_i) * mc;
            double fd[ORA_MAXC];
            ora_flux_diff_dot(Ui, Uj, cij, dim, g, fd);
            for (int r = 0; r < nc; ++r) b[r] += fd[r];
        }
        double etab = 0.0;
        for (int r = 0; r < nc; ++r) etab += etap[r] * b[r];
        double N = fabs(a - etab + er_i * b[0]);
        double D = fabs(a);
        for (int r = 0; r < nc; ++r)
            D += fabs(etap[r] - (r == 0 ? er_i : 0.0)) * fabs(b[r]);
        o->alpha[i] = D > 0.0 ? N / D : 0.0;
    }
    double tmin = INFINITY;
    for (int64_t i = 0; i < o->n; ++i)
        if (o->taui[i] < tmin) tmin = o->taui[i];
    o->last_tau_bound = tmin;
}

/* Step 3: R_i, U^L_i, bounds.  Step 4: P_ij and l1_ij.  Steps 5, 6: two
 * limiter passes.  Output E(U) into Uout.                                */
static void stage_update(ora_t *o, const double *U, double tau, double *Uout)
{
    const int dim = o->dim, nc = o->nc;
    const double g = o->gamma;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < o->n; ++i) {
        const double *Ui = U + i * nc;
        double R[ORA_MAXC] = {0}, L[ORA_MAXC] = {0};
        double rho_min = Ui[0], rho_max = Ui[0];
        double phi_min = ora_specific_entropy(Ui, dim, g);
        for (int64_t q = o->row_ptr[i]; q < o->row_ptr[i + 1]; ++q) {
            int64_t j = o->col[q];
            if (j == i) continue;
            const double *Uj = U + j * nc;
            const double *cij = o->cij + q * dim;
            double dL = o->dij[q];
            double dH = dL * (o->alpha[i] + o->alpha[j]) / 2.0;
            double fd[ORA_MAXC];
            ora_flux_diff_dot(Ui, Uj, cij, dim, g, fd);
            for (int r = 0; r < nc; ++r) {
                R[r] += -fd[r] + dH * (Uj[r] - Ui[r]);
                L[r] += -fd[r] + dL * (Uj[r] - Ui[r]);
            }
            /* bar state density, eq. def-ubar */
            double rbar = 0.5 * (Ui[0] + Uj[0]);
            if (dL > 0.0) rbar -= fd[0] / (2.0 * dL);
            if (rbar < rho_min) rho_min = rbar;
            if (rbar > rho_max) rho_max = rbar;
            double phj = ora_specific_entropy(Uj, dim, g);
            if (phj < phi_min) phi_min = phj;
        }
        if (o->relax) {
            /* Relaxation of the bounds (remark of Section 3.9; the paper
             * gives no formula): widen them by r_i = (m_i/|Omega|)^(1.5/d),
             * |Omega| = sum_i m_i.  Pinned by the second-order convergence
             * it restores on a smooth vortex.                            */
            double r = ora_pow(o->mi[i] / o->mass_total, 1.5 / (double)dim);
            rho_min *= (1.0 - r);
            rho_max *= (1.0 + r);
            phi_min *= (1.0 - r);
        }
        for (int r = 0; r < nc; ++r) {
            o->R[i * nc + r] = R[r];
            o->UL[i * nc + r] = Ui[r] + tau / o->mi[i] * L[r];
        }
        o->bnd[i * 3 + 0] = rho_min;
        o->bnd[i * 3 + 1] = rho_max;
        o->bnd[i * 3 + 2] = phi_min;
    }
    /* Step 4: P_ij (eq. def-p) and the pass-1 candidates l_ij */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < o->n; ++i) {
        const double *Ui = U + i * nc;
        const double *Ri = o->R + i * nc;
        double coef = tau / (o->lam[i] * o->mi[i]);
        for (int64_t q = o->row_ptr[i]; q < o->row_ptr[i + 1]; ++q) {
            int64_t j = o->col[q];
            double *P = o->P + q * nc;
            if (j == i) {
                for (int r = 0; r < nc; ++r) P[r] = 0.0;
                o->l1[q] = 1.0;
                continue;
            }
            const double *Uj = U + j * nc;
            const double *Rj = o->R + j * nc;
            double dL = o->dij[q];
            double dH = dL * (o->alpha[i] + o->alpha[j]) / 2.0;
            double bij = -o->mij[q] / o->mi[j];
            double bji = -o->mij[q] / o->mi[i];
            for (int r = 0; r < nc; ++r)
                P[r] = coef * (bij * Rj[r] - bji * Ri[r] + (dH - dL) * (Uj[r] - Ui[r]));
            o->l1[q] = o->limiter_mode == 1 ? 1.0
                     : o->limiter_mode == 2 ? 0.0
                     : ora_limiter(o->UL + i * nc, P, o->bnd + i * 3, dim, g,
                                   o->newton_max, o->newton_tol, o->literal_alg3);
        }
    }
    /* Step 5: pass 1 with min(l_ij, l_ji); rescale P; candidates l2 */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < o->n; ++i) {
        double V[ORA_MAXC];
        for (int r = 0; r < nc; ++r) V[r] = o->UL[i * nc + r];
        for (int64_t q = o->row_ptr[i]; q < o->row_ptr[i + 1]; ++q) {
            if (o->col[q] == i) continue;
            double lij = o->l1[q], lji = o->l1[o->tpos[q]];
            double l = lij < lji ? lij : lji;
            for (int r = 0; r < nc; ++r) V[r] += o->lam[i] * l * o->P[q * nc + r];
        }
        for (int r = 0; r < nc; ++r) o->Upass[i * nc + r] = V[r];
    }
    if (o->passes >= 2) {
        /* candidates l2 from the pass-1 state and the rescaled direction
         * (1 - min(l1_ij, l1_ji)) P_ij                                     */
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < o->n; ++i)
            for (int64_t q = o->row_ptr[i]; q < o->row_ptr[i + 1]; ++q) {
                if (o->col[q] == i) { o->l2[q] = 1.0; continue; }
                double lij = o->l1[q], lji = o->l1[o->tpos[q]];
                double l = lij < lji ? lij : lji;
                double P2[ORA_MAXC];
                for (int r = 0; r < nc; ++r) P2[r] = (1.0 - l) * o->P[q * nc + r];
                o->l2[q] = o->limiter_mode == 1 ? 1.0
                         : o->limiter_mode == 2 ? 0.0
                         : ora_limiter(o->Upass + i * nc, P2, o->bnd + i * 3,
                                       dim, g, o->newton_max, o->newton_tol,
                                       o->literal_alg3);
            }
        /* Step 6: final pass with min(l2_ij, l2_ji) */
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < o->n; ++i) {
            double V[ORA_MAXC];
            for (int r = 0; r < nc; ++r) V[r] = o->Upass[i * nc + r];
            for (int64_t q = o->row_ptr[i]; q < o->row_ptr[i + 1]; ++q) {
                if (o->col[q] == i) continue;
                double a1 = o->l1[q], b1 = o->l1[o->tpos[q]];
                double s1 = a1 < b1 ? a1 : b1;
                double a2 = o->l2[q], b2 = o->l2[o->tpos[q]];
                double s2 = a2 < b2 ? a2 : b2;
                for (int r = 0; r < nc; ++r) {
                    double P2 = (1.0 - s1) * o->P[q * nc + r];
                    V[r] += o->lam[i] * s2 * P2;
                }
            }
            for (int r = 0; r < nc; ++r) Uout[i * nc + r] = V[r];
        }
    } else {
        memcpy(Uout, o->Upass, sizeof(double) * (size_t)(o->n * nc));
    }
}

/* tau_n = c_cfl min_i m_i/(-2 d_ii) for the state U. */
double ora_max_dt(ora_t *o, const double *U)
{
    stage_viscosity(o, U);
    return o->cfl * o->last_tau_bound;
}

/* One forward-Euler stage E(U) with limiting (Alg. 1), step size tau.
 * Returns 1 if tau exceeds min_i m_i/(-2 d_ii) of this stage, else 0.    */
int ora_euler_stage(ora_t *o, const double *U, double tau, double *Uout)
{
    stage_viscosity(o, U);
    stage_update(o, U, tau, Uout);
    return tau > o->last_tau_bound ? 1 : 0;
}

/* One SSP-RK3 step (eq. ssprk3) in increment form, Dirichlet nodes hold
 * their step-initial value after every stage.  dt <= 0: tau from stage 1
 * (c_cfl times the bound).  Returns 0, -6 if a given dt exceeds the stage-1
 * bound, or +1 if tau exceeded the bound of stage 2 or 3.                 */
int ora_step(ora_t *o, double *U, double dt, double *dt_used)
{
    const int nc = o->nc;
    const int64_t len = o->n * nc;
    double *U0 = (double *)malloc(sizeof(double) * (size_t)len);
    double *U1 = (double *)malloc(sizeof(double) * (size_t)len);
    double *E = (double *)malloc(sizeof(double) * (size_t)len);
    if (!U0 || !U1 || !E) { free(U0); free(U1); free(E); return -3; }
    memcpy(U0, U, sizeof(double) * (size_t)len);
    int warn = 0;
    /* stage 1 */
    stage_viscosity(o, U0);
    double tau = dt > 0.0 ? dt : o->cfl * o->last_tau_bound;
    if (dt > 0.0 && dt > o->last_tau_bound) {
        free(U0); free(U1); free(E);
        return -6;
    }
    stage_update(o, U0, tau, U1);
    for (int64_t i = 0; i < o->n; ++i)
        if (o->dirichlet[i])
            for (int r = 0; r < nc; ++r) U1[i * nc + r] = U0[i * nc + r];
    /* stage 2: U2 = U^n + 1/4 (E(U1) - U^n) */
    warn |= ora_euler_stage(o, U1, tau, E);
    for (int64_t k = 0; k < len; ++k) U1[k] = U0[k] + 0.25 * (E[k] - U0[k]);
    for (int64_t i = 0; i < o->n; ++i)
        if (o->dirichlet[i])
            for (int r = 0; r < nc; ++r) U1[i * nc + r] = U0[i * nc + r];
    /* stage 3: U^{n+1} = U^n + 2/3 (E(U2) - U^n) */
    warn |= ora_euler_stage(o, U1, tau, E);
    for (int64_t k = 0; k < len; ++k) U[k] = U0[k] + (2.0 / 3.0) * (E[k] - U0[k]);
    for (int64_t i = 0; i < o->n; ++i)
        if (o->dirichlet[i])
            for (int r = 0; r < nc; ++r) U[i * nc + r] = U0[i * nc + r];
    free(U0); free(U1); free(E);
    if (dt_used) *dt_used = tau;
    return warn ? 1 : 0;
}

/* ------------------------------------------------------------ access */
int64_t ora_n(const ora_t *o) { return o->n; }
int64_t ora_nnz(const ora_t *o) { return o->nnz; }
double ora_volume(const ora_t *o) { return o->volume; }
void ora_set_literal_alg3(ora_t *o, int v) { o->literal_alg3 = v; }
/* 0: the limiter of Alg. 2; 1: every l_ij = 1, so E(U) is the high-order
 * update U^H of eq. high-order-final (no limiting); 2: every l_ij = 0, so
 * E(U) is the low-order update U^L of eq. low-order.  Accuracy studies only. */
void ora_set_limiter_mode(ora_t *o, int mode) { o->limiter_mode = mode; }

int ora_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* what: 0 row_ptr(i64,n+1) 1 col(i64) 2 tpos(i64) 3 m_ij 4 c_ij 5 m_i
 *       6 lambda_i 7 d_ij 8 alpha 9 R 10 U^L 11 bounds 12 P (pass 1)
 *       13 l1 14 l2 15 U after pass 1 16 tau_i                             */
const void *ora_array(const ora_t *o, int what)
{
    switch (what) {
    case 0: return o->row_ptr;
    case 1: return o->col;
    case 2: return o->tpos;
    case 3: return o->mij;
    case 4: return o->cij;
    case 5: return o->mi;
    case 6: return o->lam;
    case 7: return o->dij;
    case 8: return o->alpha;
    case 9: return o->R;
    case 10: return o->UL;
    case 11: return o->bnd;
    case 12: return o->P;
    case 13: return o->l1;
    case 14: return o->l2;
    case 15: return o->Upass;
    case 16: return o->taui;
    default: return NULL;
    }
}
