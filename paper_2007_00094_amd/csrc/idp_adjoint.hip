// Hand-written adjoint (vector-Jacobian product) of one limited
// forward-Euler stage E(U) with a fixed tau, for gfx950.
//
// Given the cotangent Eb of the stage output and the stage's intermediates
// (recomputed by the forward sweeps just before), the sweeps below run the
// stage backwards: pass 2, limiter pass 2, pass 1, limiter pass 1 and the
// directions P_ij (eq. def-p), the low-order update with its bounds, the
// indicator alpha_i (Section 3.8), the graph viscosity (Section 3.7) and the
// node quantities of Section 2.  Where the forward takes a max, a min, a
// clamp or a branch, the derivative follows the branch the forward took
// (at an exact tie: the branch its comparison picks); the limiter's Newton
// iterations (Alg. 2/3) are differentiated as unrolled.
//
// No atomics: every kernel writes its contributions to per-entry slots it
// alone owns (a pair thread owns the entries (i,j) and (j,i)); nodes sum
// the slots of their row, and of their transposed entries, in row order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adjoint.h"
#include "idp_device.h"
#include "kernels.h"
#include "sweep_common.h"

namespace idp {

__device__ __forceinline__ double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }
__device__ __forceinline__ double dpos(double x) { return 0.5 * (sgn(x) + 1.0); }   // d pos/dx
__device__ __forceinline__ double dneg(double x) { return 0.5 * (sgn(x) - 1.0); }   // d neg/dx

// ------------------------------------------------------- node cotangents
// Cotangents of a node's state and of the derived quantities of step 0.
template <int D>
struct NodeCot {
    double U[D + 2];
    double p, c, er, phi;
    double v[D];
    double etap[D + 2];
};

template <int D>
__device__ __forceinline__ void cot_zero(NodeCot<D> &b)
{
#pragma unroll
    for (int r = 0; r < D + 2; ++r) { b.U[r] = 0.0; b.etap[r] = 0.0; }
#pragma unroll
    for (int k = 0; k < D; ++k) b.v[k] = 0.0;
    b.p = b.c = b.er = b.phi = 0.0;
}

// F = f(U) (NC x D), from U, v = m/rho and p: adds F's cotangent Fb.
template <int D>
__device__ __forceinline__ void flux_vjp(const double *U, const double *v, double p,
                                         const double Fb[D + 2][D], NodeCot<D> &b)
{
    const double E = U[D + 1];
#pragma unroll
    for (int k = 0; k < D; ++k) b.U[1 + k] += Fb[0][k];
#pragma unroll
    for (int a = 0; a < D; ++a) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            b.v[k] += Fb[1 + a][k] * U[1 + a];
            b.U[1 + a] += Fb[1 + a][k] * v[k];
        }
        b.p += Fb[1 + a][a];
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        b.v[k] += Fb[D + 1][k] * (E + p);
        b.U[D + 1] += Fb[D + 1][k] * v[k];
        b.p += Fb[D + 1][k] * v[k];
    }
}

// Section 2: v = m/rho, eps = E - |m|^2/(2 rho), p = (g-1) eps,
// c = sqrt(g p/rho), eta/rho with eta = (rho eps)^(1/(g+1)), phi = eps
// rho^-g, eta' = (rho eps)^(-g/(g+1))/(g+1) (E, -m, rho).  Adds dU to Ub.
template <int D>
__device__ __forceinline__ void node_vjp(const double *U, double p, double c, double er,
                                         double phi, double g, const NodeCot<D> &b,
                                         bool with_etap, double *Ub)
{
    const double rho = U[0], E = U[D + 1];
    double m2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) m2 += U[1 + k] * U[1 + k];
    const double eps = E - 0.5 * m2 / rho;
    double rb = b.U[0], Eb = b.U[D + 1], mb[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        mb[k] = b.U[1 + k] + b.v[k] / rho;
        rb -= b.v[k] * U[1 + k] / (rho * rho);
    }
    double pb = b.p, epsb = 0.0, reb = 0.0;
    if (b.c != 0.0 && c > 0.0) {
        const double qb = b.c / (2.0 * c);       // c = sqrt(q), q = g p/rho
        pb += qb * g / rho;
        rb -= qb * g * p / (rho * rho);
    }
    const double re = rho * eps;
    if (b.er != 0.0) {
        const double eta = er * rho;
        rb -= b.er * er / rho;
        reb += (b.er / rho) * eta / ((g + 1.0) * re);
    }
    if (b.phi != 0.0) {
        epsb += b.phi * phi / eps;
        rb -= b.phi * g * phi / rho;
    }
    if (with_etap) {
        const double fac = fpow(re, -g / (g + 1.0)) / (g + 1.0);
        Eb += fac * b.etap[0];
        double facb = b.etap[0] * E + b.etap[D + 1] * rho;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            mb[k] -= fac * b.etap[1 + k];
            facb -= b.etap[1 + k] * U[1 + k];
        }
        rb += fac * b.etap[D + 1];
        reb += facb * (-g / (g + 1.0)) * fac / re;
    }
    rb += reb * eps;
    epsb += reb * rho;
    epsb += (g - 1.0) * pb;
    Eb += epsb;
#pragma unroll
    for (int k = 0; k < D; ++k) mb[k] -= epsb * U[1 + k] / rho;
    rb += epsb * 0.5 * m2 / (rho * rho);
    Ub[0] += rb;
#pragma unroll
    for (int k = 0; k < D; ++k) Ub[1 + k] += mb[k];
    Ub[D + 1] += Eb;
}

// ------------------------------------------------ wave-speed bound VJP
// Adjoint of lambda_max (Section 3.7) for lambda's cotangent lb; adds the
// cotangents of (U, p, c) of the two states to bi, bj.
template <int D>
__device__ __forceinline__ void lambda_vjp(const double *n, const double *Ui, double pi,
                                           double ci, const double *Uj, double pj, double cj,
                                           const GasC &G, double lb, NodeCot<D> &bi,
                                           NodeCot<D> &bj)
{
    const double g = G.g;
    double mti = 0.0, mtj = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) mti += n[k] * Ui[1 + k];
#pragma unroll
    for (int k = 0; k < D; ++k) mtj += n[k] * Uj[1 + k];
    const double ui = mti / Ui[0];
    const double uj = mtj / Uj[0];
    const double num = ci + cj - G.half_gm1 * (uj - ui);
    const double r = pi / pj;
    const double Y = fpow(r, G.e_den);
    const double den = ci * Y + cj;
    const double Q = pos_part(num) / den;
    const double X = fpow(Q, G.e_p);
    const double ptilde = pj * X;
    const double pmax = pi > pj ? pi : pj;
    const double psi = psi_branch<D>(Ui[0], pi, ci, pmax, g) +
                       psi_branch<D>(Uj[0], pj, cj, pmax, g) + uj - ui;
    int sel;   // 0: ptilde, 1: pmax
    double pstar;
    if (psi < 0.0) { pstar = ptilde; sel = 0; }
    else if (pmax < ptilde) { pstar = pmax; sel = 1; }
    else { pstar = ptilde; sel = 0; }
    const double f = G.f;
    const double z1 = (pstar - pi) / pi, z3 = (pstar - pj) / pj;
    const double S1 = sqrt(1.0 + f * pos_part(z1));
    const double S3 = sqrt(1.0 + f * pos_part(z3));
    const double lam1 = ui - ci * S1;
    const double lam3 = uj + cj * S3;
    const double a = neg_part(lam1), b = pos_part(lam3);
    double ab = 0.0, bb = 0.0;
    if (a > b) ab = lb; else bb = lb;
    const double lam1b = ab * dneg(lam1), lam3b = bb * dpos(lam3);
    double uib = lam1b, ujb = lam3b, cib = -S1 * lam1b, cjb = S3 * lam3b;
    double pib = 0.0, pjb = 0.0, pstarb = 0.0;
    const double z1b = (-ci * lam1b) * f * dpos(z1) / (2.0 * S1);
    const double z3b = (cj * lam3b) * f * dpos(z3) / (2.0 * S3);
    pstarb += z1b / pi + z3b / pj;
    pib -= z1b * pstar / (pi * pi);
    pjb -= z3b * pstar / (pj * pj);
    double ptb = 0.0;
    if (sel == 0) ptb = pstarb;
    else {
        if (pi > pj) pib += pstarb; else pjb += pstarb;
    }
    pjb += X * ptb;
    const double Xb = pj * ptb;
    const double Qb = Q > 0.0 ? Xb * G.e_p * X / Q : 0.0;
    const double numb = Qb * dpos(num) / den;
    const double denb = -Qb * pos_part(num) / (den * den);
    cib += numb;
    cjb += numb;
    ujb -= G.half_gm1 * numb;
    uib += G.half_gm1 * numb;
    cib += Y * denb;
    cjb += denb;
    const double Yb = ci * denb;
    const double rb = Yb * G.e_den * Y / r;
    pib += rb / pj;
    pjb -= rb * pi / (pj * pj);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        bi.U[1 + k] += uib / Ui[0] * n[k];
        bj.U[1 + k] += ujb / Uj[0] * n[k];
    }
    bi.U[0] -= uib * ui / Ui[0];
    bj.U[0] -= ujb * uj / Uj[0];
    bi.p += pib;
    bi.c += cib;
    bj.p += pjb;
    bj.c += cjb;
}

// ---------------------------------------------------------- limiter VJP
// Psi(t) = rho eps(V) - phi_min rho^(g+1) on V = U + t P and Psi'(t), with
// the point kept for the backward (the forward's arithmetic, in its order).
template <int D>
struct PsiPt {
    double V[D + 2];
    double rg1, psi, dpsi;
};

template <int D>
__device__ __forceinline__ void psi_eval(const double *U, const double *P, double t,
                                         double phimin, double g, PsiPt<D> &o)
{
#pragma unroll
    for (int k = 0; k < D + 2; ++k) o.V[k] = U[k] + t * P[k];
    const double rho = o.V[0], E = o.V[D + 1];
    double m2 = 0.0, mP = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        m2 += o.V[1 + k] * o.V[1 + k];
        mP += o.V[1 + k] * P[1 + k];
    }
    const double rho_eps = rho * E - 0.5 * m2;
    o.rg1 = fpow(rho, g + 1.0);
    o.psi = rho_eps - phimin * o.rg1;
    o.dpsi = P[0] * E + rho * P[D + 1] - mP - phimin * (g + 1.0) * (o.rg1 / rho) * P[0];
}

// Psi(t) and Psi'(t) backwards at a kept point: adds to Ub, Pb, tb, phib.
template <int D>
__device__ __forceinline__ void psi_adj(const PsiPt<D> &o, const double *P, double t,
                                        double phimin, double g, double psib, double dpsib,
                                        double *Ub, double *Pb, double &tb, double &phib)
{
    constexpr int NC = D + 2;
    const double rho = o.V[0], E = o.V[D + 1];
    const double rg1 = o.rg1;
    const double q = rg1 / rho;                      // rho^g
    double Vb[NC];
    Vb[0] = psib * (E - phimin * (g + 1.0) * q) +
            dpsib * (P[D + 1] - phimin * (g + 1.0) * P[0] * g * q / rho);
    Vb[D + 1] = psib * rho + dpsib * P[0];
#pragma unroll
    for (int k = 0; k < D; ++k) Vb[1 + k] = -psib * o.V[1 + k] - dpsib * P[1 + k];
    phib += -psib * rg1 - dpsib * (g + 1.0) * q * P[0];
    Pb[0] += dpsib * (E - phimin * (g + 1.0) * q);
    Pb[D + 1] += dpsib * rho;
#pragma unroll
    for (int k = 0; k < D; ++k) Pb[1 + k] -= dpsib * o.V[1 + k];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        Ub[k] += Vb[k];
        Pb[k] += t * Vb[k];
        tb += Vb[k] * P[k];
    }
}

// Alg. 3 step backwards: given (nlb, nrb) of the new bracket, adds the
// cotangents of tL, tR, psiL, psiR, dpsiL, dpsiR.
__device__ __forceinline__ void newton_vjp(double tL, double tR, double psiL, double psiR,
                                           double dpsiL, double dpsiR, double rhoP,
                                           double nlb, double nrb, double &tLb, double &tRb,
                                           double &psiLb, double &psiRb, double &dpsiLb,
                                           double &dpsiRb)
{
    const double eps = 2.220446049250313e-16;
    const double scaling = 1.0 / (tR - tL + eps);
    const double d11 = dpsiL, d22 = dpsiR;
    const double d12 = (psiR - psiL) * scaling;
    const double d112 = (d12 - d11) * scaling;
    const double d122 = (d22 - d12) * scaling;
    double LL = dpsiL * dpsiL - 4.0 * psiL * d112;
    double LR = dpsiR * dpsiR - 4.0 * psiR * d122;
    const bool LLneg = LL < 0.0, LRneg = LR < 0.0;
    if (LLneg) LL = 0.0;
    if (LRneg) LR = 0.0;
    const double sL = sqrt(LL), sR = sqrt(LR);
    const double denL = dpsiL - sL, denR = dpsiR - sR;
    const double rootL = denL != 0.0 ? tL - 2.0 * psiL / denL : tL;
    const double rootR = denR != 0.0 ? tR - 2.0 * psiR / denR : tR;
    const bool up = rhoP >= 0.0;
    double nl0 = up ? rootL : rootR, nr0 = up ? rootR : rootL;
    // forward clamps, recorded
    const bool cl1 = !(nl0 >= tL);
    double nl1 = cl1 ? tL : nl0;
    const bool cl2 = !(nl1 <= tR);
    double nl2 = cl2 ? tR : nl1;
    const bool cr1 = !(nr0 <= tR);
    double nr1 = cr1 ? tR : nr0;
    const bool cr2 = !(nr1 >= tL);
    double nr2 = cr2 ? tL : nr1;
    const bool cfin = nr2 < nl2;
    (void)nl2;
    (void)nr2;
    // backwards
    double nl2b = nlb, nr2b = 0.0;
    if (cfin) nl2b += nrb; else nr2b = nrb;
    double nr1b = 0.0;
    if (cr2) tLb += nr2b; else nr1b = nr2b;
    double nr0b = 0.0;
    if (cr1) tRb += nr1b; else nr0b = nr1b;
    double nl1b = 0.0;
    if (cl2) tRb += nl2b; else nl1b = nl2b;
    double nl0b = 0.0;
    if (cl1) tLb += nl1b; else nl0b = nl1b;
    const double rootLb = up ? nl0b : nr0b;
    const double rootRb = up ? nr0b : nl0b;
    double denLb = 0.0, denRb = 0.0;
    if (denL != 0.0) {
        tLb += rootLb;
        psiLb += -2.0 / denL * rootLb;
        denLb += 2.0 * psiL / (denL * denL) * rootLb;
    } else {
        tLb += rootLb;
    }
    if (denR != 0.0) {
        tRb += rootRb;
        psiRb += -2.0 / denR * rootRb;
        denRb += 2.0 * psiR / (denR * denR) * rootRb;
    } else {
        tRb += rootRb;
    }
    dpsiLb += denLb;
    dpsiRb += denRb;
    const double LLb = (!LLneg && sL > 0.0) ? -denLb / (2.0 * sL) : 0.0;
    const double LRb = (!LRneg && sR > 0.0) ? -denRb / (2.0 * sR) : 0.0;
    dpsiLb += 2.0 * dpsiL * LLb;
    psiLb += -4.0 * d112 * LLb;
    double d112b = -4.0 * psiL * LLb;
    dpsiRb += 2.0 * dpsiR * LRb;
    psiRb += -4.0 * d122 * LRb;
    double d122b = -4.0 * psiR * LRb;
    double d12b = 0.0, d11b = 0.0, d22b = 0.0, scb = 0.0;
    d22b += scaling * d122b;
    d12b -= scaling * d122b;
    scb += (d22 - d12) * d122b;
    d12b += scaling * d112b;
    d11b -= scaling * d112b;
    scb += (d12 - d11) * d112b;
    psiRb += scaling * d12b;
    psiLb -= scaling * d12b;
    scb += (psiR - psiL) * d12b;
    dpsiLb += d11b;
    dpsiRb += d22b;
    tRb += -scaling * scaling * scb;
    tLb += scaling * scaling * scb;
}

// Alg. 2 backwards for the result's cotangent tb: adds to Ub, Pb and
// bb = (rho_min, rho_max, phi_min) cotangents.
//
// A direction whose largest component is below 2^-40 of the largest
// component of the state it starts from is rounding noise (a region that
// is uniform up to rounding): the limiter's branches on it are decided by
// rounding, and the derivative of the coefficient there (up to |P|/|P_rho|
// times that of P where a density bound cuts the step) describes the
// rounding, not the method.  For such a direction the coefficient is taken
// as locally constant (no contribution here); the coefficient still
// multiplies the direction's own cotangent in the passes.
constexpr int kAdjNewtonMax = 8;
constexpr double kNoiseDirection = 0x1p-40;

// NMAX: the compile-time bound of newton_max; at NMAX <= 2 the loops unroll
// and the recorded brackets stay in registers.
template <int D, int NMAX>
__device__ __forceinline__ void limiter_vjp(const double *U, const double *P, double rmin,
                                            double rmax, double phimin, double g,
                                            int newton_max, double tol, double tb,
                                            double *Ub, double *Pb, double *bb)
{
    {
        double pm = 0.0, um = 0.0;
#pragma unroll
        for (int r = 0; r < D + 2; ++r) {
            pm = fmax(pm, fabs(P[r]));
            um = fmax(um, fabs(U[r]));
        }
        if (pm <= kNoiseDirection * um) return;
    }
    const double rhoU = U[0], rhoP = P[0];
    // density bounds, recorded
    double tR = 1.0;
    const bool A = rhoU + tR * rhoP > rmax;
    if (A) tR = rhoP != 0.0 ? fabs(rmax - rhoU) / fabs(rhoP) : 0.0;
    const bool B = rhoU + tR * rhoP < rmin;
    if (B) tR = rhoP != 0.0 ? fabs(rmin - rhoU) / fabs(rhoP) : 0.0;
    const bool c1 = tR > 1.0;
    if (c1) tR = 1.0;
    const bool c0 = tR < 0.0;
    if (c0) tR = 0.0;
    // Newton iterations: the brackets recorded, Psi recomputed backwards
    constexpr int kUnroll = NMAX <= 2 ? NMAX : 1;   // loop unroll count
    double tLs[NMAX + 1], tRs[NMAX + 1];
    double tL = 0.0;
    int steps = 0, brk = 0;   // brk: 0 none, 1 psiR >= 0 (t = tR), 2 psiL <= tol (t = tL)
#pragma unroll kUnroll
    for (int it = 0; it < NMAX; ++it) {
        if (it >= newton_max) break;
        tLs[it] = tL;
        tRs[it] = tR;
        double psiR, dpsiR;
        psi_line<D>(U, P, tR, phimin, g, psiR, dpsiR);
        if (psiR >= 0.0) { brk = 1; break; }
        double psiL, dpsiL;
        psi_line<D>(U, P, tL, phimin, g, psiL, dpsiL);
        if (psiL <= tol) { brk = 2; break; }
        enclose_step(tL, tR, psiL, psiR, dpsiL, dpsiR, rhoP);
        ++steps;
    }
    // backwards: cotangents of (tL, tR) at the start of iteration `steps`
    double tLb = 0.0, tRb = 0.0, phib = 0.0;
    if (brk == 1) tRb = tb; else tLb = tb;
#pragma unroll kUnroll
    for (int it = NMAX - 1; it >= 0; --it) {
        if (it >= steps) continue;
        PsiPt<D> R, Lp;
        psi_eval<D>(U, P, tRs[it], phimin, g, R);
        psi_eval<D>(U, P, tLs[it], phimin, g, Lp);
        double ntLb = 0.0, ntRb = 0.0, psiLb = 0.0, psiRb = 0.0, dpsiLb = 0.0, dpsiRb = 0.0;
        newton_vjp(tLs[it], tRs[it], Lp.psi, R.psi, Lp.dpsi, R.dpsi, rhoP, tLb, tRb, ntLb, ntRb,
                   psiLb, psiRb, dpsiLb, dpsiRb);
        psi_adj<D>(R, P, tRs[it], phimin, g, psiRb, dpsiRb, Ub, Pb, ntRb, phib);
        psi_adj<D>(Lp, P, tLs[it], phimin, g, psiLb, dpsiLb, Ub, Pb, ntLb, phib);
        tLb = ntLb;
        tRb = ntRb;
    }
    // tL at iteration 0 is the constant 0; tR went through the bounds
    bb[2] += phib;
    if (c1 || c0) return;
    if (B) {
        if (rhoP != 0.0) {
            const double aP = fabs(rhoP);
            const double num = fabs(rmin - rhoU);
            const double s = sgn(rmin - rhoU);
            bb[0] += tRb * s / aP;
            Ub[0] -= tRb * s / aP;
            Pb[0] -= tRb * num * sgn(rhoP) / (aP * aP);
        }
        return;
    }
    if (A && rhoP != 0.0) {
        const double aP = fabs(rhoP);
        const double num = fabs(rmax - rhoU);
        const double s = sgn(rmax - rhoU);
        bb[1] += tRb * s / aP;
        Ub[0] -= tRb * s / aP;
        Pb[0] -= tRb * num * sgn(rhoP) / (aP * aP);
    }
}

// ------------------------------------------------------------- kernels
// Every sweep is a wavefront sweep (rows: one slice per wavefront; pairs:
// one pair per lane) whose node records come through cooperative gathers,
// and whose per-entry records leave through cooperative scatters.

// Bits of the neighbour ids in a node record: slot 14 holds (min, max),
// slot 15 the phi_min neighbour; -1: the node itself.
__device__ __forceinline__ double pack_ids(int a, int b)
{
    return __longlong_as_double((long long)((unsigned long long)(unsigned)a |
                                            ((unsigned long long)(unsigned)b << 32)));
}
__device__ __forceinline__ int id_lo(double v)
{
    return int((unsigned)((unsigned long long)__double_as_longlong(v) & 0xffffffffull));
}
__device__ __forceinline__ int id_hi(double v)
{
    return int((unsigned)((unsigned long long)__double_as_longlong(v) >> 32));
}

// A pair's limiter record, if the active candidate's cotangents are not
// all zero: stored at Lim[p]; returns p, else -1.
template <int D>
__device__ __forceinline__ int put_lim(double *Lim, int64_t p, bool valid, const double *Ub,
                                       const double *bb)
{
    constexpr int NC = D + 2;
    bool nz = false;
#pragma unroll
    for (int r = 0; r < NC; ++r) nz = nz || Ub[r] != 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) nz = nz || bb[q] != 0.0;
    if (!valid || !nz) return -1;
    double *o = Lim + p * kLimS;
#pragma unroll
    for (int r = 0; r < NC; ++r) o[r] = Ub[r];
#pragma unroll
    for (int q = 0; q < 3; ++q) o[NC + q] = bb[q];
    return int(p);
}

// pass 2 and its limiter backwards (pair).  E_i = U_i' + sum_j lambda_i
// s2_ij (1 - s1_ij) P_ij gives s2's cotangent; the candidate that set
// s2 = min(l_ij, l_ji) is run backwards (Alg. 2/3 on the line U_a' + t
// (1 - s1) P_a): its state and bounds cotangents go to the pair's limiter
// record (indexed from the entry of its row), the direction's to the pair.
template <int D, int NMAX>
__global__ void __launch_bounds__(kBlock) k_adj_lim2(StageArgs P, AdjArgs A)
{
    WAVE_LDS(Chunks<D>::packB)
    static_assert(kTile_ > 0 && Chunks<D>::packB >= kQS / 2 && Chunks<D>::packB >= Chunks<D>::rowB, "tile fits every record");
    WAVE_PAIR_SETUP(P, PAIR_INDEX(P), P.npairs)
    constexpr int NC = D + 2, NU = (NC + 1) / 2;
    using CH = Chunks<D>;
    const double dL = P.dp[pq_], m = P.mp[pq_], s1 = P.l1p[pq_];
    const bool iside = P.side2[pq_] != 0;
    double Pij[NC], Pji[NC];
    {
        NodeB<D> Bi, Bj;
        gather_b<D>(P.packB, i, lw, Bi);
        gather_b<D>(P.packB, j, lw, Bj);
        direction<D>(Bi, Bj, Bi.coef, dL, m, Pij);
        direction<D>(Bj, Bi, Bj.coef, dL, m, Pji);
    }
    double sb;
    {
        double Ei[2 * NU], Ej[2 * NU];
        gather<NU>(A.Ebp, kEbS, i, lw, Ei);
        gather<NU>(A.Ebp, kEbS, j, lw, Ej);
        double EPi = 0.0, EPj = 0.0;
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            EPi += Ei[r] * Pij[r];
            EPj += Ej[r] * Pji[r];
        }
        sb = (1.0 - s1) * (P.lam[i] * EPi + P.lam[j] * EPj);
    }
    // the candidate that set s2: row a's pass-1 state, bounds, direction
    const int a_ = iside ? i : j;
    double Wa[2 * CH::rowB], Ua[2 * NU], Qa[NC];
    gather<CH::rowB>(P.rowB, kRowB, a_, lw, Wa);
    gather<NU>(P.upass, kRowU, a_, lw, Ua);
#pragma unroll
    for (int r = 0; r < NC; ++r) Qa[r] = (1.0 - s1) * (iside ? Pij[r] : Pji[r]);
    double Ub[NC], Qb[NC], bb[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < NC; ++r) { Ub[r] = 0.0; Qb[r] = 0.0; }
    if (valid_ && sb != 0.0)
        limiter_vjp<D, NMAX>(Ua, Qa, Wa[NC], Wa[NC + 1], Wa[NC + 2], P.gamma, P.newton_max, P.tol, sb,
                       Ub, Qb, bb);
    double rq[kQS];
#pragma unroll
    for (int r = 0; r < kQS; ++r) rq[r] = r < NC ? Qb[r] : 0.0;
    scatter<kQS / 2>(A.Qb, kQS, valid_ ? int(p_) : -1, lw, rq);
    const int rec = put_lim<D>(A.Lim, p_, valid_, Ub, bb);
    if (valid_) {
        A.lim2e[e] = iside ? rec : -1;
        A.lim2e[t] = iside ? -1 : rec;
    }
}

// pass 1 backwards (row): U_i' = E_i's cotangent plus the pass-2 limiter
// records of the row's pairs; the bounds' cotangents so far.
template <int D>
__global__ void __launch_bounds__(kBlock) k_adj_pass1(StageArgs P, AdjArgs A)
{
    WAVE_ROW_SETUP(P, ROW_SLICE(P), P.nslices)
    (void)inst_;   // one instance: adjoints run on single meshes
    constexpr int NC = D + 2;
    const int dk = valid_ ? P.diag_k[r_] : -1;
    double u[NC], bnd[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < NC; ++r) u[r] = A.Ebp[int64_t(i) * kEbS + r];
    if (P.passes >= 2) {
        for (int k = 0; k < Lmax_; ++k) {
            const int64_t e = ENTRY(k);
            const bool act = k < L && k != dk;
            const int q_ = act ? A.lim2e[e] : -1;
            if (q_ < 0) continue;
            const double *rec = A.Lim + int64_t(q_) * kLimS;
#pragma unroll
            for (int r = 0; r < NC; ++r) u[r] += rec[r];
#pragma unroll
            for (int q = 0; q < 3; ++q) bnd[q] += rec[NC + q];
        }
    }
    if (!valid_) return;
    double *o = A.Upb + int64_t(i) * kUpS;
#pragma unroll
    for (int r = 0; r < NC; ++r) o[r] = u[r];
#pragma unroll
    for (int q = 0; q < 3; ++q) o[NC + q] = bnd[q];
}

// the directions P_ij, P_ji (eq. def-p) and the pass-1 limiter backwards
// (pair).  P_ij's cotangent gathers pass 2 (lambda_i s2 (1 - s1) Eb_i), the
// pass-2 limiter ((1 - s1) Q if row i set s2) and pass 1 (lambda_i s1 U_i'
// bar); s1's cotangent likewise.  The candidate that set s1 is run
// backwards.  Both directions then reduce to Z = coef_j Pb_ji - coef_i
// Pb_ij: R_i gains b_ji Z, U_i gains (d^H - d^L) Z, R_j and U_j the same
// with -Z and b_ij; alpha_i and alpha_j each gain -Z.(U_j - U_i) d^L/2.
template <int D, int NMAX>
__global__ void __launch_bounds__(kBlock, 2) k_adj_lim1(StageArgs P, AdjArgs A)
{
    WAVE_LDS(Chunks<D>::packB)
    static_assert(kTile_ > 0 && Chunks<D>::packB >= kZS / 2 && Chunks<D>::packB >= kQS / 2, "tile fits every record");
    WAVE_PAIR_SETUP(P, PAIR_INDEX(P), P.npairs)
    constexpr int NC = D + 2, NU = (NC + 1) / 2;
    using CH = Chunks<D>;
    const bool two = P.passes >= 2;
    const double dL = P.dp[pq_], m = P.mp[pq_], s1 = P.l1p[pq_];
    const double s2 = two ? P.l2[e] : 0.0;
    const bool side1 = P.side1[pq_] != 0;
    const bool side2 = two ? P.side2[pq_] != 0 : true;
    const double li = P.lam[i], lj = P.lam[j];
    double Pij[NC], Pji[NC], dU[NC], ci, cj, asum;
    {
        NodeB<D> Bi, Bj;
        gather_b<D>(P.packB, i, lw, Bi);
        gather_b<D>(P.packB, j, lw, Bj);
        direction<D>(Bi, Bj, Bi.coef, dL, m, Pij);
        direction<D>(Bj, Bi, Bj.coef, dL, m, Pji);
#pragma unroll
        for (int r = 0; r < NC; ++r) dU[r] = Bj.U[r] - Bi.U[r];
        ci = Bi.coef;
        cj = Bj.coef;
        asum = Bi.alpha + Bj.alpha;
    }
    // P's cotangents and s1's from pass 2, the pass-2 limiter and pass 1;
    // Z without the pass-1 limiter's share
    double Z[NC], sb;
    {
        double Ei[2 * NU], Ej[2 * NU], Vi[2 * NU], Vj[2 * NU], Qr[kQS];
        gather<NU>(A.Ebp, kEbS, i, lw, Ei);
        gather<NU>(A.Ebp, kEbS, j, lw, Ej);
        gather<NU>(A.Upb, kUpS, i, lw, Vi);
        gather<NU>(A.Upb, kUpS, j, lw, Vj);
        if (two) {
            gather<kQS / 2>(A.Qb, kQS, valid_ ? int(p_) : -1, lw, Qr);
        } else {
#pragma unroll
            for (int r = 0; r < kQS; ++r) Qr[r] = 0.0;
        }
        double EPi = 0.0, EPj = 0.0, VPi = 0.0, VPj = 0.0, QP = 0.0;
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            EPi += Ei[r] * Pij[r];
            EPj += Ej[r] * Pji[r];
            VPi += Vi[r] * Pij[r];
            VPj += Vj[r] * Pji[r];
            QP += Qr[r] * (side2 ? Pij[r] : Pji[r]);
            const double q = (1.0 - s1) * Qr[r];
            const double Pbi = li * s2 * (1.0 - s1) * Ei[r] + li * s1 * Vi[r] + (side2 ? q : 0.0);
            const double Pbj = lj * s2 * (1.0 - s1) * Ej[r] + lj * s1 * Vj[r] + (side2 ? 0.0 : q);
            Z[r] = cj * Pbj - ci * Pbi;
        }
        sb = -s2 * (li * EPi + lj * EPj) - QP + li * VPi + lj * VPj;
    }
    // the candidate that set s1: row a's U^L, bounds, direction
    const int a_ = side1 ? i : j;
    double Wa[2 * CH::rowB], Pa[NC];
    gather<CH::rowB>(P.rowB, kRowB, a_, lw, Wa);
#pragma unroll
    for (int r = 0; r < NC; ++r) Pa[r] = side1 ? Pij[r] : Pji[r];
    double ULb[NC], Pab[NC], bb[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < NC; ++r) { ULb[r] = 0.0; Pab[r] = 0.0; }
    if (valid_ && sb != 0.0)
        limiter_vjp<D, NMAX>(Wa, Pa, Wa[NC], Wa[NC + 1], Wa[NC + 2], P.gamma, P.newton_max, P.tol, sb,
                       ULb, Pab, bb);
    const double ca = side1 ? -ci : cj;
    double kb = 0.0;
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        Z[r] += ca * Pab[r];
        kb -= Z[r] * dU[r];
    }
    const double dH = dL * asum / 2.0;
    const int rec = put_lim<D>(A.Lim, p_, valid_, ULb, bb);
    double re[kZS], rt[kZS];
#pragma unroll
    for (int r = 0; r < kZS; ++r) { re[r] = 0.0; rt[r] = 0.0; }
#pragma unroll
    for (int r = 0; r < NC; ++r) { re[r] = Z[r]; rt[r] = -Z[r]; }
    re[5] = rt[5] = kb * dL / 2.0;
    re[6] = rt[6] = dH - dL;
    re[7] = __longlong_as_double((long long)(side1 ? rec : -1));
    rt[7] = __longlong_as_double((long long)(side1 ? -1 : rec));
    scatter<kZS / 2>(A.C, kZS, valid_ ? int(e) : -1, lw, re);
    scatter<kZS / 2>(A.C, kZS, valid_ ? int(t) : -1, lw, rt);
    if (valid_) A.dLb[p_] = kb * (asum / 2.0 - 1.0);
}

// low-order update, bar states and bounds backwards (row).  The row's
// records give the totals of U^L_i's, the bounds', R_i's cotangents; then
// Lw_i = sum_j (-(f_j - f_i).c_ij + d_ij (U_j - U_i)) and R_i (with d^H)
// run backwards for what belongs to node i itself: U_i's own part, d_ij's
// share of row i (db4, per entry), alpha_i's own share.  The neighbours'
// shares are pulled by the neighbours from the node record.
template <int D>
__global__ void __launch_bounds__(kBlock, 3) k_adj_low(StageArgs P, AdjArgs A)
{
    WAVE_LDS(kNS / 2)
    static_assert(kTile_ > 0 && kNS / 2 >= kZS / 2, "tile fits every record");
    WAVE_ROW_SETUP(P, ROW_SLICE(P), P.nslices)
    (void)inst_;   // one instance: adjoints run on single meshes
    constexpr int NC = D + 2, NU = (NC + 1) / 2;
    const double g = P.gamma;
    const int dk = valid_ ? P.diag_k[r_] : -1;
    NodeA<D> Ai;
    load_a<D>(P.packA + int64_t(i) * kPack, Ai);
    const double al_i = P.packA[int64_t(i) * kPack + kPackAlpha];
    const double mi = P.mi[i];
    double ULb[NC], bnd[3], Rb[NC], Ud[NC], alb = 0.0;
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        ULb[r] = A.Upb[int64_t(i) * kUpS + r];
        Rb[r] = 0.0;
        Ud[r] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) bnd[q] = A.Upb[int64_t(i) * kUpS + NC + q];
    for (int k = 0; k < Lmax_; ++k) {
        const int64_t e = ENTRY(k);
        const bool act = k < L && k != dk;
        double rec[kZS];
        gather<kZS / 2>(A.C, kZS, act ? int(e) : -1, lw, rec);
        if (!act) continue;
        const double b = -P.mij[e] / mi;
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            Rb[r] += b * rec[r];
            Ud[r] += rec[6] * rec[r];
        }
        alb += rec[5];
        const int q_ = int(__double_as_longlong(rec[7]));
        if (q_ >= 0) {
            const double *lr = A.Lim + int64_t(q_) * kLimS;
#pragma unroll
            for (int r = 0; r < NC; ++r) ULb[r] += lr[r];
#pragma unroll
            for (int q = 0; q < 3; ++q) bnd[q] += lr[NC + q];
        }
    }
    double Lwb[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) Lwb[r] = A.tau / mi * ULb[r];
    const int ak = valid_ ? P.argk[i] : 0xFFFFFF;
    const int kmin = ak & 255, kmax = (ak >> 8) & 255, kphi = (ak >> 16) & 255;
    int idmin = -1, idmax = -1, idphi = -1;
    double Uo[NC], Sc[D], Fb0[D];
#pragma unroll
    for (int r = 0; r < NC; ++r) Uo[r] = 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q) { Sc[q] = 0.0; Fb0[q] = 0.0; }
    int jn = Lmax_ > 0 ? P.scol[ENTRY(0)] : 0;
    for (int k = 0; k < Lmax_; ++k) {
        const int64_t e = ENTRY(k);
        const int j = jn;
        if (k + 1 < Lmax_) jn = P.scol[ENTRY(k + 1)];
        const bool act = k < L && k != dk;
        double rec[2 * (NU + 1)];
        gather_tail<NU + 1, kPackAlpha / 2>(P.packA, kPack, act ? j : -1, lw, rec);
        if (!act) continue;
        const double al_j = rec[2 * NU];
        double c[D];
        load_c<D>(P, e, c);
        const double dL = P.d[e];
        const double dH = dL * (al_i + al_j) / 2.0;
        double dLb = 0.0, dHb = 0.0;
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            const double dU = rec[r] - Ai.U[r];
            dHb += Rb[r] * dU;
            dLb += Lwb[r] * dU;
            Uo[r] -= dL * Lwb[r] + dH * Rb[r];
        }
        dLb += dHb * (al_i + al_j) / 2.0;
        alb += dHb * dL / 2.0;
#pragma unroll
        for (int q = 0; q < D; ++q) Sc[q] += c[q];
        double rb = 0.0;
        if (k == kmin) { rb += bnd[0]; idmin = j; }
        if (k == kmax) { rb += bnd[1]; idmax = j; }
        if (k == kphi) idphi = j;
        if (rb != 0.0) {
            Uo[0] += 0.5 * rb;
            if (dL > 0.0) {
                double fd0 = 0.0;
#pragma unroll
                for (int q = 0; q < D; ++q) fd0 += (rec[1 + q] - Ai.U[1 + q]) * c[q];
#pragma unroll
                for (int q = 0; q < D; ++q) Fb0[q] += rb / (2.0 * dL) * c[q];
                dLb += rb * fd0 / (2.0 * dL * dL);
            }
        }
        A.db4[e] = dLb;
    }
    if (kmin == 255) Uo[0] += bnd[0];
    if (kmax == 255) Uo[0] += bnd[1];
    NodeCot<D> ci;
    cot_zero<D>(ci);
    if (kphi == 255) ci.phi = bnd[2];
    double Fb[NC][D];
#pragma unroll
    for (int r = 0; r < NC; ++r)
#pragma unroll
        for (int q = 0; q < D; ++q) Fb[r][q] = (Lwb[r] + Rb[r]) * Sc[q];
#pragma unroll
    for (int q = 0; q < D; ++q) Fb[0][q] += Fb0[q];
    flux_vjp<D>(Ai.U, Ai.v, Ai.p, Fb, ci);
    double Up[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) Up[r] = ULb[r] + Ud[r] + Uo[r];
    node_vjp<D>(Ai.U, Ai.p, Ai.c, Ai.er, Ai.phi, g, ci, false, Up);
    double nr[kNS];
#pragma unroll
    for (int r = 0; r < kNS; ++r) nr[r] = 0.0;
#pragma unroll
    for (int r = 0; r < NC; ++r) { nr[r] = Lwb[r]; nr[5 + r] = Rb[r]; }
#pragma unroll
    for (int q = 0; q < 3; ++q) nr[10 + q] = bnd[q];
    nr[13] = al_i;
    nr[14] = pack_ids(idmin, idmax);
    nr[15] = pack_ids(idphi, -1);
    scatter<kNS / 2>(A.Nrec, kNS, valid_ ? i : -1, lw, nr);
    if (!valid_) return;
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        A.Up4[int64_t(i) * NC + r] = Up[r];
        A.ULt[int64_t(i) * NC + r] = ULb[r];
        A.Rt[int64_t(i) * NC + r] = Rb[r];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) A.bndt[int64_t(i) * 3 + q] = bnd[q];
    A.alb[i] = alb;
}

// indicator alpha_i (Section 3.8) backwards, with what the neighbours' low
// order owes node i (row).  alpha_i's total cotangent adds the neighbours'
// R_j shares; the indicator's sums a_i and b_i are recomputed as the
// forward does and run backwards.  U_i's part: the indicator's own terms
// and, from each neighbour j's record, d_ij Lw_j + d^H R_j bar, the flux
// terms through c_ji, and the bar-state and phi terms where node i set a
// bound of row j.
template <int D>
__global__ void __launch_bounds__(kBlock) k_adj_alpha(StageArgs P, AdjArgs A)
{
    WAVE_LDS(kNS / 2)
    static_assert(kTile_ > 0 && kNS / 2 >= kIS / 2, "tile fits every record");
    WAVE_ROW_SETUP(P, ROW_SLICE(P), P.nslices)
    (void)inst_;   // one instance: adjoints run on single meshes
    constexpr int NC = D + 2;
    constexpr int NCH = kDiagChunks<D>;   // U, p, c, eta/rho (v recomputed)
    const double g = P.gamma;
    const int dk = valid_ ? P.diag_k[r_] : -1;
    NodeA<D> Ai;
    load_a<D>(P.packA + int64_t(i) * kPack, Ai);
    const double al_i = P.packA[int64_t(i) * kPack + kPackAlpha];
    double Fi[NC][D];
    flux<D>(Ai.U, Ai.v, Ai.p, Fi);
    double a = 0.0, b[NC], MC = 0.0, Sc[D], alb = valid_ ? A.alb[i] : 0.0;
    double Fb[NC][D], Up[NC];
    NodeCot<D> ci;
    cot_zero<D>(ci);
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        b[r] = 0.0;
        Up[r] = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) Fb[r][q] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < D; ++q) Sc[q] = 0.0;
    int jn = Lmax_ > 0 ? P.scol[ENTRY(0)] : 0;
    for (int k = 0; k < Lmax_; ++k) {
        const int64_t e = ENTRY(k);
        const int j = jn;
        if (k + 1 < Lmax_) jn = P.scol[ENTRY(k + 1)];
        const bool in = k < L;
        const bool act = in && k != dk;
        double ra[2 * NCH], rn[kNS];
        gather<NCH>(P.packA, kPack, in ? j : -1, lw, ra);
        gather<kNS / 2>(A.Nrec, kNS, act ? j : -1, lw, rn);
        if (!in) continue;
        NodeA<D> Aj;
        load_a_fwd<D>(ra, Aj);
        double c[D];
        load_c<D>(P, e, c);
        double mc = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) mc += Aj.U[1 + q] * c[q];
        a += (Aj.er - Ai.er) * mc;
        double Fj[NC][D], fd[NC];
        flux<D>(Aj.U, Aj.v, Aj.p, Fj);
        flux_diff_dot<D>(Fi, Fj, c, fd);
#pragma unroll
        for (int r = 0; r < NC; ++r) b[r] += fd[r];
        if (!act) continue;
        MC += mc;
#pragma unroll
        for (int q = 0; q < D; ++q) Sc[q] += c[q];
        // neighbour j's low order: Lw_j, R_j with d_ji = d_ij, c_ji
        const double dL = P.d[e];
        const double al_j = rn[13];
        double ct[D];
        ct[0] = P.ct0[e];
        ct[1] = P.ct1[e];
        if (D == 3) ct[D - 1] = P.ct2[e];
        const double dH = dL * (al_j + al_i) / 2.0;
        double rdu = 0.0;
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            rdu += rn[5 + r] * (Ai.U[r] - Aj.U[r]);
            Up[r] += dL * rn[r] + dH * rn[5 + r];
#pragma unroll
            for (int q = 0; q < D; ++q) Fb[r][q] -= (rn[r] + rn[5 + r]) * ct[q];
        }
        alb += rdu * dL / 2.0;
        double rb = 0.0;
        if (id_lo(rn[14]) == i) rb += rn[10];
        if (id_hi(rn[14]) == i) rb += rn[11];
        if (rb != 0.0) {
            Up[0] += 0.5 * rb;
            if (dL > 0.0) {
#pragma unroll
                for (int q = 0; q < D; ++q) Fb[0][q] -= rb / (2.0 * dL) * ct[q];
            }
        }
        if (id_lo(rn[15]) == i) ci.phi += rn[12];
    }
    // alpha_i = |X| / Dn with X = a - eta'(U_i).b + (eta/rho)_i b_rho
    double etap[NC];
    harten_entropy_derivative<D>(Ai.U, g, etap);
    double etab = 0.0;
#pragma unroll
    for (int r = 0; r < NC; ++r) etab += etap[r] * b[r];
    const double X = a - etab + Ai.er * b[0];
    const double N = fabs(X);
    double Dn = fabs(a);
#pragma unroll
    for (int r = 0; r < NC; ++r) Dn += fabs(etap[r] - (r == 0 ? Ai.er : 0.0)) * fabs(b[r]);
    double ab = 0.0, bb[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) bb[r] = 0.0;
    if (alb != 0.0 && Dn > 0.0) {
        const double Nb = alb / Dn;
        const double Dnb = -alb * N / (Dn * Dn);
        const double Xb = Nb * sgn(X);
        ab += Xb;
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            ci.etap[r] -= Xb * b[r];
            bb[r] -= Xb * etap[r];
        }
        ci.er += Xb * b[0];
        bb[0] += Xb * Ai.er;
        ab += Dnb * sgn(a);
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            const double Y = etap[r] - (r == 0 ? Ai.er : 0.0);
            const double Yb = Dnb * sgn(Y) * fabs(b[r]);
            ci.etap[r] += Yb;
            if (r == 0) ci.er -= Yb;
            bb[r] += Dnb * fabs(Y) * sgn(b[r]);
        }
    }
    // the indicator's own terms: a_i through eta/rho_i, b_i through f(U_i)
    ci.er -= ab * MC;
#pragma unroll
    for (int r = 0; r < NC; ++r)
#pragma unroll
        for (int q = 0; q < D; ++q) Fb[r][q] -= bb[r] * Sc[q];
    flux_vjp<D>(Ai.U, Ai.v, Ai.p, Fb, ci);
    node_vjp<D>(Ai.U, Ai.p, Ai.c, Ai.er, Ai.phi, g, ci, true, Up);
    double ir[kIS];
#pragma unroll
    for (int r = 0; r < kIS; ++r) ir[r] = 0.0;
    ir[0] = ab;
#pragma unroll
    for (int r = 0; r < NC; ++r) ir[1 + r] = bb[r];
    ir[6] = Ai.er;
    scatter<kIS / 2>(A.Irec, kIS, valid_ ? i : -1, lw, ir);
    if (!valid_) return;
#pragma unroll
    for (int r = 0; r < NC; ++r) A.Up6[int64_t(i) * NC + r] = Up[r];
    A.alt[i] = alb;
}

// graph viscosity backwards (pair): d_ij's total cotangent (the
// directions', rows i's and j's low order) through the orientation that
// set the max (recorded by the forward) to both states.
template <int D>
__global__ void __launch_bounds__(kBlock) k_adj_dpair(StageArgs P, AdjArgs A)
{
    constexpr int NC = D + 2;
    constexpr int NCH = (NC + 3) / 2;   // U, p, c
    WAVE_LDS(NCH)
    static_assert(kTile_ >= kC5S / 2, "tile fits every record");
    WAVE_PAIR_SETUP(P, PAIR_INDEX(P), P.npairs)
    double Ai[2 * NCH], Aj[2 * NCH];
    gather<NCH>(P.packA, kPack, i, lw, Ai);
    gather<NCH>(P.packA, kPack, j, lw, Aj);
    const double db = A.dLb[pq_] + A.db4[e] + A.db4[t];
    double Ubi[kC5S], Ubj[kC5S];
#pragma unroll
    for (int r = 0; r < kC5S; ++r) { Ubi[r] = 0.0; Ubj[r] = 0.0; }
    if (valid_ && db != 0.0) {
        // orientation i -> j: n_ij = c_ij/|c_ij|; j -> i: c_ji (stored at (i, j))
        const bool fwd = P.sided[pq_] != 0;
        double c[D];
        if (fwd) {
            load_c<D>(P, e, c);
        } else {
            c[0] = P.ct0[e];
            c[1] = P.ct1[e];
            if (D == 3) c[D - 1] = P.ct2[e];
        }
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) a += c[q] * c[q];
        a = sqrt(a);
        if (a > 0.0) {
            const double inv = 1.0 / a;
            double nn[D];
#pragma unroll
            for (int q = 0; q < D; ++q) nn[q] = c[q] * inv;
            const double *Aa = fwd ? Ai : Aj, *Ab = fwd ? Aj : Ai;
            NodeCot<D> ba, bb;
            cot_zero<D>(ba);
            cot_zero<D>(bb);
            lambda_vjp<D>(nn, Aa, Aa[NC], Aa[NC + 1], Ab, Ab[NC], Ab[NC + 1], P.gas, db * a, ba,
                          bb);
            double *Ua = fwd ? Ubi : Ubj, *Uo = fwd ? Ubj : Ubi;
            node_vjp<D>(Aa, Aa[NC], Aa[NC + 1], 0.0, 0.0, P.gamma, ba, false, Ua);
            node_vjp<D>(Ab, Ab[NC], Ab[NC + 1], 0.0, 0.0, P.gamma, bb, false, Uo);
        }
    }
    scatter<kC5S / 2>(A.C, kC5S, valid_ ? int(e) : -1, lw, Ubi);
    scatter<kC5S / 2>(A.C, kC5S, valid_ ? int(t) : -1, lw, Ubj);
    if (valid_) A.dLb[p_] = db;
}

// the node's cotangent (row): its low-order and indicator parts, the graph
// viscosity's entry records, and what the neighbours' indicators owe it
// (a_j through eta/rho_i and m_i, b_j through f(U_i), both along c_ji).
template <int D>
__global__ void __launch_bounds__(kBlock) k_adj_final(StageArgs P, AdjArgs A)
{
    WAVE_LDS(kIS / 2)
    static_assert(kTile_ > 0 && kIS / 2 >= kC5S / 2, "tile fits every record");
    WAVE_ROW_SETUP(P, ROW_SLICE(P), P.nslices)
    (void)inst_;   // one instance: adjoints run on single meshes
    constexpr int NC = D + 2;
    const int dk = valid_ ? P.diag_k[r_] : -1;
    NodeA<D> Ai;
    load_a<D>(P.packA + int64_t(i) * kPack, Ai);
    double U[NC], Fb[NC][D];
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        U[r] = A.Up4[int64_t(i) * NC + r] + A.Up6[int64_t(i) * NC + r];
#pragma unroll
        for (int q = 0; q < D; ++q) Fb[r][q] = 0.0;
    }
    NodeCot<D> ci;
    cot_zero<D>(ci);
    int jn = Lmax_ > 0 ? P.scol[ENTRY(0)] : 0;
    for (int k = 0; k < Lmax_; ++k) {
        const int64_t e = ENTRY(k);
        const int j = jn;
        if (k + 1 < Lmax_) jn = P.scol[ENTRY(k + 1)];
        const bool act = k < L && k != dk;
        double r5[kC5S], ri[kIS];
        gather<kC5S / 2>(A.C, kC5S, act ? int(e) : -1, lw, r5);
        gather<kIS / 2>(A.Irec, kIS, act ? j : -1, lw, ri);
        if (!act) continue;
        double ct[D];
        ct[0] = P.ct0[e];
        ct[1] = P.ct1[e];
        if (D == 3) ct[D - 1] = P.ct2[e];
        double mc = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) mc += Ai.U[1 + q] * ct[q];
        ci.er += ri[0] * mc;
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            U[r] += r5[r];
#pragma unroll
            for (int q = 0; q < D; ++q) Fb[r][q] += ri[1 + r] * ct[q];
        }
#pragma unroll
        for (int q = 0; q < D; ++q) U[1 + q] += ri[0] * (Ai.er - ri[6]) * ct[q];
    }
    flux_vjp<D>(Ai.U, Ai.v, Ai.p, Fb, ci);
    node_vjp<D>(Ai.U, Ai.p, Ai.c, Ai.er, Ai.phi, P.gamma, ci, false, U);
    if (!valid_) return;
#pragma unroll
    for (int r = 0; r < NC; ++r) A.Ub[int64_t(i) * NC + r] = U[r];
}

// U's cotangent layout [n][nc] -> [n][kEbS]
__global__ void k_adj_pad(int64_t n, int nc, const double *in, double *out)
{
    const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (q >= n * nc) return;
    out[(q / nc) * kEbS + q % nc] = in[q];
}

// SSP-RK3 and the held nodes backwards, per node (stage k of a step):
// out = hold ? U0 : U0 + theta (E - U0) with theta = 1 (stage 1: out = E),
// 1/4, 2/3.  Eb = theta * outb off the held nodes (layout [n][kEbS]); U0's
// cotangent gains (1 - theta) outb (all of outb on a held node).
__global__ void k_adj_ssp(int64_t n, int nc, const uint8_t *hold, const double *outb,
                          double theta, double *Eb, double *U0b, int first)
{
    const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (q >= n * nc) return;
    const bool h = hold && hold[q / nc];
    const double o = outb[q];
    Eb[(q / nc) * kEbS + q % nc] = h ? 0.0 : theta * o;
    const double add = h ? o : (1.0 - theta) * o;
    U0b[q] = first ? add : U0b[q] + add;
}

__global__ void k_adj_add(int64_t n, const double *x, double *y)
{
    const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (q < n) y[q] += x[q];
}

// ------------------------------------------------------------ launches
// row and pair sweeps use the XCD renumbering: per * 8 and pper * 8 blocks
static inline int rows_grid(const StageArgs &P) { return P.per * kXcd; }
static inline int pairs_grid(const StageArgs &P) { return P.pper * kXcd; }

#define ADJ_LAUNCH(K, grid)                                                              \
    do {                                                                                 \
        if (grid > 0) {                                                                  \
            if (P.dim == 2)                                                              \
                hipLaunchKernelGGL(K<2>, dim3(grid), dim3(kBlock), 0, st, P, A);         \
            else                                                                         \
                hipLaunchKernelGGL(K<3>, dim3(grid), dim3(kBlock), 0, st, P, A);         \
        }                                                                                \
    } while (0)

// the limiter VJPs by the compile-time bound of newton_max
#define ADJ_LAUNCH_N(K, grid)                                                            \
    do {                                                                                 \
        if (grid > 0) {                                                                  \
            const bool small = P.newton_max <= 2;                                        \
            if (P.dim == 2 && small)                                                     \
                hipLaunchKernelGGL((K<2, 2>), dim3(grid), dim3(kBlock), 0, st, P, A);    \
            else if (P.dim == 2)                                                         \
                hipLaunchKernelGGL((K<2, kAdjNewtonMax>), dim3(grid), dim3(kBlock), 0, st, P, A); \
            else if (small)                                                              \
                hipLaunchKernelGGL((K<3, 2>), dim3(grid), dim3(kBlock), 0, st, P, A);    \
            else                                                                         \
                hipLaunchKernelGGL((K<3, kAdjNewtonMax>), dim3(grid), dim3(kBlock), 0, st, P, A); \
        }                                                                                \
    } while (0)

void launch_stage_vjp(const StageArgs &P, const AdjArgs &A, hipStream_t st)
{
    if (P.passes >= 2) ADJ_LAUNCH_N(k_adj_lim2, pairs_grid(P));
    ADJ_LAUNCH(k_adj_pass1, rows_grid(P));
    ADJ_LAUNCH_N(k_adj_lim1, pairs_grid(P));
    ADJ_LAUNCH(k_adj_low, rows_grid(P));
    ADJ_LAUNCH(k_adj_alpha, rows_grid(P));
    ADJ_LAUNCH(k_adj_dpair, pairs_grid(P));
    ADJ_LAUNCH(k_adj_final, rows_grid(P));
}

static inline int flat_grid(int64_t m) { return int((m + kBlock - 1) / kBlock); }

void launch_adj_pad(hipStream_t st, int64_t n, int nc, const double *in, double *out)
{
    if (n > 0) hipLaunchKernelGGL(k_adj_pad, dim3(flat_grid(n * nc)), dim3(kBlock), 0, st, n, nc, in, out);
}

void launch_adj_ssp(hipStream_t st, int64_t n, int nc, const uint8_t *hold, const double *outb,
                    double theta, double *Eb, double *U0b, int first)
{
    if (n > 0)
        hipLaunchKernelGGL(k_adj_ssp, dim3(flat_grid(n * nc)), dim3(kBlock), 0, st, n, nc, hold,
                           outb, theta, Eb, U0b, first);
}

void launch_adj_add(hipStream_t st, int64_t n, const double *x, double *y)
{
    if (n > 0) hipLaunchKernelGGL(k_adj_add, dim3(flat_grid(n)), dim3(kBlock), 0, st, n, x, y);
}

}  // namespace idp
