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
// Psi(t) and Psi'(t) backwards: adds to Ub, Pb, tb, phib.
template <int D>
__device__ __forceinline__ void psi_vjp(const double *U, const double *P, double t,
                                        double phimin, double g, double psib, double dpsib,
                                        double *Ub, double *Pb, double &tb, double &phib)
{
    constexpr int NC = D + 2;
    double V[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) V[k] = U[k] + t * P[k];
    const double rho = V[0], E = V[D + 1];
    const double rg1 = fpow(rho, g + 1.0);
    const double q = rg1 / rho;                      // rho^g
    double Vb[NC];
    Vb[0] = psib * (E - phimin * (g + 1.0) * q) +
            dpsib * (P[D + 1] - phimin * (g + 1.0) * P[0] * g * q / rho);
    Vb[D + 1] = psib * rho + dpsib * P[0];
#pragma unroll
    for (int k = 0; k < D; ++k) Vb[1 + k] = -psib * V[1 + k] - dpsib * P[1 + k];
    phib += -psib * rg1 - dpsib * (g + 1.0) * q * P[0];
    Pb[0] += dpsib * (E - phimin * (g + 1.0) * q);
    Pb[D + 1] += dpsib * rho;
#pragma unroll
    for (int k = 0; k < D; ++k) Pb[1 + k] -= dpsib * V[1 + k];
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
constexpr int kAdjNewtonMax = 8;

template <int D>
__device__ __forceinline__ void limiter_vjp(const double *U, const double *P, double rmin,
                                            double rmax, double phimin, double g,
                                            int newton_max, double tol, double tb,
                                            double *Ub, double *Pb, double *bb)
{
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
    // Newton iterations, recorded
    double tLs[kAdjNewtonMax + 1], tRs[kAdjNewtonMax + 1];
    double pL[kAdjNewtonMax], pR[kAdjNewtonMax], dL[kAdjNewtonMax], dR[kAdjNewtonMax];
    double tL = 0.0;
    int steps = 0, brk = 0;   // brk: 0 none, 1 psiR >= 0 (t = tR), 2 psiL <= tol (t = tL)
    for (int it = 0; it < newton_max; ++it) {
        tLs[it] = tL;
        tRs[it] = tR;
        double psiR, dpsiR;
        psi_line<D>(U, P, tR, phimin, g, psiR, dpsiR);
        if (psiR >= 0.0) { brk = 1; break; }
        double psiL, dpsiL;
        psi_line<D>(U, P, tL, phimin, g, psiL, dpsiL);
        if (psiL <= tol) { brk = 2; break; }
        pL[it] = psiL;
        pR[it] = psiR;
        dL[it] = dpsiL;
        dR[it] = dpsiR;
        quadratic_newton(tL, tR, psiL, psiR, dpsiL, dpsiR, rhoP);
        ++steps;
    }
    tLs[steps] = tL;
    tRs[steps] = tR;
    // backwards: cotangents of (tL, tR) at the start of iteration `steps`
    double tLb = 0.0, tRb = 0.0, phib = 0.0;
    if (brk == 1) tRb = tb; else tLb = tb;
    for (int it = steps - 1; it >= 0; --it) {
        double ntLb = 0.0, ntRb = 0.0, psiLb = 0.0, psiRb = 0.0, dpsiLb = 0.0, dpsiRb = 0.0;
        newton_vjp(tLs[it], tRs[it], pL[it], pR[it], dL[it], dR[it], rhoP, tLb, tRb, ntLb, ntRb,
                   psiLb, psiRb, dpsiLb, dpsiRb);
        psi_vjp<D>(U, P, tRs[it], phimin, g, psiRb, dpsiRb, Ub, Pb, ntRb, phib);
        psi_vjp<D>(U, P, tLs[it], phimin, g, psiLb, dpsiLb, Ub, Pb, ntLb, phib);
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

// direction P_ij (eq. def-p) backwards for P's cotangent Pbar; adds R and
// U cotangents of both rows, alpha cotangents and returns dL's.
template <int D>
__device__ __forceinline__ double direction_vjp(const NodeB<D> &Bi, const NodeB<D> &Bj,
                                                double coef, double dL, double mij,
                                                const double *Pbar, double *Rbi, double *Rbj,
                                                double *Ubi, double *Ubj, double &albi,
                                                double &albj)
{
    const double dH = dL * (Bi.alpha + Bj.alpha) / 2.0;
    const double bij = -mij / Bj.m;
    const double bji = -mij / Bi.m;
    const double k = dH - dL;
    double kb = 0.0;
#pragma unroll
    for (int r = 0; r < D + 2; ++r) {
        const double w = coef * Pbar[r];
        Rbj[r] += bij * w;
        Rbi[r] -= bji * w;
        Ubj[r] += k * w;
        Ubi[r] -= k * w;
        kb += w * (Bj.U[r] - Bi.U[r]);
    }
    albi += kb * dL / 2.0;
    albj += kb * dL / 2.0;
    return kb * ((Bi.alpha + Bj.alpha) / 2.0 - 1.0);
}

// ------------------------------------------------------------- kernels
#define ADJ_PAIR_SETUP(P)                                                    \
    const int64_t p_ = int64_t(blockIdx.x) * kBlock + threadIdx.x;           \
    if (p_ >= P.npairs) return;                                              \
    const int64_t e = P.pair_e[p_];                                          \
    const int64_t t = P.pair_t[p_];                                          \
    const int i = P.pair_i[p_];                                              \
    const int j = P.pair_j[p_];

template <int D> constexpr int kNodeSlot = D + 5;   // nc + 3 bounds per entry

// pass 2 backwards (row): Up's cotangent = Eb; s2, s1 and P cotangents per entry
template <int D>
__global__ void __launch_bounds__(kBlock) k_adj_pass2(StageArgs P, AdjArgs A)
{
    ROW_SETUP(P)
    constexpr int NC = D + 2;
    NodeB<D> Bi;
    load_b<D>(P.packB + int64_t(i) * kPack, Bi);
    double Eb[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        Eb[r] = A.Eb[int64_t(i) * NC + r];
        A.Upb[int64_t(i) * NC + r] = Eb[r];
    }
    const double lam = P.lam[i];
    const double coef = A.tau / (lam * Bi.m);
    for (int k = 0; k < L; ++k) {
        const int64_t e = ENTRY(k);
        const int j = P.scol[e];
        double *Pb = A.Pb + e * NC;
        if (j == i || P.passes < 2) {
            A.sb1[e] = 0.0;
            A.sb2[e] = 0.0;
#pragma unroll
            for (int r = 0; r < NC; ++r) Pb[r] = 0.0;
            continue;
        }
        const double s1 = P.l1[e], s2 = P.l2[e];
        NodeB<D> Bj;
        load_b<D>(P.packB + int64_t(j) * kPack, Bj);
        double Pd[NC];
        direction<D>(Bi, Bj, coef, P.d[e], P.mij[e], Pd);
        double EP = 0.0;
#pragma unroll
        for (int r = 0; r < NC; ++r) EP += Eb[r] * Pd[r];
        A.sb2[e] = lam * (1.0 - s1) * EP;
        A.sb1[e] = -lam * s2 * EP;
#pragma unroll
        for (int r = 0; r < NC; ++r) Pb[r] = lam * s2 * (1.0 - s1) * Eb[r];
    }
}

// limiter pass 2 backwards (pair): the active candidate of min(l_ij, l_ji)
template <int D>
__global__ void __launch_bounds__(kBlock) k_adj_lim2(StageArgs P, AdjArgs A)
{
    ADJ_PAIR_SETUP(P)
    constexpr int NC = D + 2, NS = kNodeSlot<D>;
    NodeB<D> Bi, Bj;
    load_b<D>(P.packB + int64_t(i) * kPack, Bi);
    load_b<D>(P.packB + int64_t(j) * kPack, Bj);
    const double *Wi = P.rowB + int64_t(i) * kRowB, *Wj = P.rowB + int64_t(j) * kRowB;
    const double *Ui = P.upass + int64_t(i) * kRowU, *Uj = P.upass + int64_t(j) * kRowU;
    const double dL = P.dp[p_], m = P.mp[p_], s1 = P.l1p[p_];
    double Pij[NC], Pji[NC], Qij[NC], Qji[NC];
    direction<D>(Bi, Bj, Bi.coef, dL, m, Pij);
    direction<D>(Bj, Bi, Bj.coef, dL, m, Pji);
#pragma unroll
    for (int r = 0; r < NC; ++r) { Qij[r] = (1.0 - s1) * Pij[r]; Qji[r] = (1.0 - s1) * Pji[r]; }
    double Uc[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) Uc[r] = Ui[r];
    const double lij = row_limiter<D>(Uc, Wi, Qij, P);
#pragma unroll
    for (int r = 0; r < NC; ++r) Uc[r] = Uj[r];
    const double lji = row_limiter<D>(Uc, Wj, Qji, P);
    const double sb = A.sb2[e] + A.sb2[t];
    double *ce = A.cnode + e * NS, *ct = A.cnode + t * NS;
#pragma unroll
    for (int r = 0; r < NS; ++r) { ce[r] = 0.0; ct[r] = 0.0; }
    const bool iside = lij < lji;
    const double *Ua = iside ? Ui : Uj;
    const double *Wa = iside ? Wi : Wj;
    const double *Qa = iside ? Qij : Qji;
    const double *Pa = iside ? Pij : Pji;
    double *ca = iside ? ce : ct;
    const int64_t ea = iside ? e : t;
    double Ub[NC], Qb[NC], bb[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < NC; ++r) { Ub[r] = 0.0; Qb[r] = 0.0; Uc[r] = Ua[r]; }
    limiter_vjp<D>(Uc, Qa, Wa[NC], Wa[NC + 1], Wa[NC + 2], P.gamma, P.newton_max, P.tol, sb, Ub,
                   Qb, bb);
    double QP = 0.0;
    double *Pb = A.Pb + ea * NC;
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        ca[r] = Ub[r];
        Pb[r] += (1.0 - s1) * Qb[r];
        QP += Qb[r] * Pa[r];
    }
    ca[NC] = bb[0];
    ca[NC + 1] = bb[1];
    ca[NC + 2] = bb[2];
    A.sb1[ea] -= QP;
}

// pass 1 backwards (row): Up's total cotangent (= U^L's), bounds' so far
template <int D>
__global__ void __launch_bounds__(kBlock) k_adj_pass1(StageArgs P, AdjArgs A)
{
    ROW_SETUP(P)
    constexpr int NC = D + 2, NS = kNodeSlot<D>;
    double Upb[NC], bnd[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < NC; ++r) Upb[r] = A.Upb[int64_t(i) * NC + r];
    if (P.passes >= 2) {
        for (int k = 0; k < L; ++k) {
            const int64_t e = ENTRY(k);
            if (P.scol[e] == i) continue;
            const double *c = A.cnode + e * NS;
#pragma unroll
            for (int r = 0; r < NC; ++r) Upb[r] += c[r];
            bnd[0] += c[NC];
            bnd[1] += c[NC + 1];
            bnd[2] += c[NC + 2];
        }
    }
#pragma unroll
    for (int r = 0; r < NC; ++r) A.Upb[int64_t(i) * NC + r] = Upb[r];
    A.bndb[int64_t(i) * 3 + 0] = bnd[0];
    A.bndb[int64_t(i) * 3 + 1] = bnd[1];
    A.bndb[int64_t(i) * 3 + 2] = bnd[2];
    NodeB<D> Bi;
    load_b<D>(P.packB + int64_t(i) * kPack, Bi);
    const double lam = P.lam[i];
    const double coef = A.tau / (lam * Bi.m);
    for (int k = 0; k < L; ++k) {
        const int64_t e = ENTRY(k);
        const int j = P.scol[e];
        if (j == i) continue;
        NodeB<D> Bj;
        load_b<D>(P.packB + int64_t(j) * kPack, Bj);
        double Pd[NC];
        direction<D>(Bi, Bj, coef, P.d[e], P.mij[e], Pd);
        const double s1 = P.l1[e];
        double UP = 0.0;
        double *Pb = A.Pb + e * NC;
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            UP += Upb[r] * Pd[r];
            Pb[r] += lam * s1 * Upb[r];
        }
        A.sb1[e] += lam * UP;
    }
}

// limiter pass 1 and the directions backwards (pair)
template <int D>
__global__ void __launch_bounds__(kBlock) k_adj_lim1(StageArgs P, AdjArgs A)
{
    ADJ_PAIR_SETUP(P)
    constexpr int NC = D + 2, NS = kNodeSlot<D>;
    NodeB<D> Bi, Bj;
    load_b<D>(P.packB + int64_t(i) * kPack, Bi);
    load_b<D>(P.packB + int64_t(j) * kPack, Bj);
    const double *Wi = P.rowB + int64_t(i) * kRowB, *Wj = P.rowB + int64_t(j) * kRowB;
    const double dL = P.dp[p_], m = P.mp[p_];
    double Pij[NC], Pji[NC], Uc[NC];
    direction<D>(Bi, Bj, Bi.coef, dL, m, Pij);
    direction<D>(Bj, Bi, Bj.coef, dL, m, Pji);
#pragma unroll
    for (int r = 0; r < NC; ++r) Uc[r] = Wi[r];
    const double lij = row_limiter<D>(Uc, Wi, Pij, P);
#pragma unroll
    for (int r = 0; r < NC; ++r) Uc[r] = Wj[r];
    const double lji = row_limiter<D>(Uc, Wj, Pji, P);
    const double sb = A.sb1[e] + A.sb1[t];
    double *ce = A.cnode + e * NS, *ct = A.cnode + t * NS;
#pragma unroll
    for (int r = 0; r < NS; ++r) { ce[r] = 0.0; ct[r] = 0.0; }
    const bool iside = lij < lji;
    const double *Wa = iside ? Wi : Wj;
    const double *Pa = iside ? Pij : Pji;
    double *ca = iside ? ce : ct;
    double Ub[NC], Pab[NC], bb[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < NC; ++r) { Ub[r] = 0.0; Pab[r] = 0.0; Uc[r] = Wa[r]; }
    limiter_vjp<D>(Uc, Pa, Wa[NC], Wa[NC + 1], Wa[NC + 2], P.gamma, P.newton_max, P.tol, sb, Ub,
                   Pab, bb);
#pragma unroll
    for (int r = 0; r < NC; ++r) ca[r] = Ub[r];
    ca[NC] = bb[0];
    ca[NC + 1] = bb[1];
    ca[NC + 2] = bb[2];
    // total P cotangents of both directions
    double Pbij[NC], Pbji[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        Pbij[r] = A.Pb[e * NC + r] + (iside ? Pab[r] : 0.0);
        Pbji[r] = A.Pb[t * NC + r] + (iside ? 0.0 : Pab[r]);
        A.Pb[e * NC + r] = Pbij[r];   // totals (kept for inspection)
        A.Pb[t * NC + r] = Pbji[r];
    }
    double Rbi[NC], Rbj[NC], Ubi[NC], Ubj[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) { Rbi[r] = Rbj[r] = Ubi[r] = Ubj[r] = 0.0; }
    double albi = 0.0, albj = 0.0;
    double dLb = direction_vjp<D>(Bi, Bj, Bi.coef, dL, m, Pbij, Rbi, Rbj, Ubi, Ubj, albi, albj);
    dLb += direction_vjp<D>(Bj, Bi, Bj.coef, dL, m, Pbji, Rbj, Rbi, Ubj, Ubi, albj, albi);
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        A.cR[e * NC + r] = Rbi[r];
        A.cR[t * NC + r] = Rbj[r];
        A.cU[e * NC + r] = Ubi[r];
        A.cU[t * NC + r] = Ubj[r];
    }
    A.cal[e] = albi;
    A.cal[t] = albj;
    A.dbp[p_] = dLb;
}

// low-order update, bar states and bounds backwards (row)
template <int D>
__global__ void __launch_bounds__(kBlock) k_adj_low(StageArgs P, AdjArgs A)
{
    ROW_SETUP(P)
    constexpr int NC = D + 2, NS = kNodeSlot<D>;
    const double g = P.gamma;
    NodeA<D> Ai;
    load_a<D>(P.packA + int64_t(i) * kPack, Ai);
    const double alpha_i = P.alpha[i];
    const double mi = P.mi[i];
    // cotangents of R_i, U^L_i and the bounds of row i
    double Rb[NC], ULb[NC], bnd[3];
#pragma unroll
    for (int r = 0; r < NC; ++r) { Rb[r] = 0.0; ULb[r] = A.Upb[int64_t(i) * NC + r]; }
#pragma unroll
    for (int q = 0; q < 3; ++q) bnd[q] = A.bndb[int64_t(i) * 3 + q];
    double Fi[NC][D];
    flux<D>(Ai.U, Ai.v, Ai.p, Fi);
    // forward pass over the row: the entries that set the bounds
    double rho_min = Ai.U[0], rho_max = Ai.U[0], phi_min = Ai.phi;
    int kmin = -1, kmax = -1, kphi = -1;
    for (int k = 0; k < L; ++k) {
        const int64_t e = ENTRY(k);
        const int j = P.scol[e];
        if (j == i) continue;
        const double *cn = A.cnode + e * NS;
        const double *cr = A.cR + e * NC;
#pragma unroll
        for (int r = 0; r < NC; ++r) { ULb[r] += cn[r]; Rb[r] += cr[r]; }
        bnd[0] += cn[NC];
        bnd[1] += cn[NC + 1];
        bnd[2] += cn[NC + 2];
        NodeA<D> Aj;
        load_a<D>(P.packA + int64_t(j) * kPack, Aj);
        double c[D];
        load_c<D>(P, e, c);
        const double dL = P.d[e];
        double Fj[NC][D], fd[NC];
        flux<D>(Aj.U, Aj.v, Aj.p, Fj);
        flux_diff_dot<D>(Fi, Fj, c, fd);
        double rbar = 0.5 * (Ai.U[0] + Aj.U[0]);
        if (dL > 0.0) rbar -= fd[0] / (2.0 * dL);
        if (rbar < rho_min) { rho_min = rbar; kmin = k; }
        if (rbar > rho_max) { rho_max = rbar; kmax = k; }
        if (Aj.phi < phi_min) { phi_min = Aj.phi; kphi = k; }
    }
    double Lwb[NC], Ubi[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        Lwb[r] = A.tau / mi * ULb[r];
        Ubi[r] = ULb[r];
        A.ULt[int64_t(i) * NC + r] = ULb[r];
        A.Rt[int64_t(i) * NC + r] = Rb[r];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) A.bndt[int64_t(i) * 3 + q] = bnd[q];
    double Fbi[NC][D];
#pragma unroll
    for (int r = 0; r < NC; ++r)
#pragma unroll
        for (int q = 0; q < D; ++q) Fbi[r][q] = 0.0;
    double albi = 0.0;
    for (int k = 0; k < L; ++k) {
        const int64_t e = ENTRY(k);
        const int j = P.scol[e];
        double *cuj = A.cUj + e * NC;
        if (j == i) {
#pragma unroll
            for (int r = 0; r < NC; ++r) cuj[r] = 0.0;
            A.calj[e] = 0.0;
            A.db3[e] = 0.0;
            continue;
        }
        NodeA<D> Aj;
        load_a<D>(P.packA + int64_t(j) * kPack, Aj);
        const double alpha_j = P.packA[int64_t(j) * kPack + kPackAlpha];
        double c[D];
        load_c<D>(P, e, c);
        const double dL = P.d[e];
        const double dH = dL * (alpha_i + alpha_j) / 2.0;
        double Fj[NC][D], fd[NC];
        flux<D>(Aj.U, Aj.v, Aj.p, Fj);
        flux_diff_dot<D>(Fi, Fj, c, fd);
        double fdb[NC], Ujb[NC];
        double dHb = 0.0, dLb = 0.0;
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            const double dU = Aj.U[r] - Ai.U[r];
            fdb[r] = -Lwb[r] - Rb[r];
            dHb += Rb[r] * dU;
            dLb += Lwb[r] * dU;
            Ujb[r] = dL * Lwb[r] + dH * Rb[r];
            Ubi[r] -= Ujb[r];
        }
        dLb += dHb * (alpha_i + alpha_j) / 2.0;
        albi += dHb * dL / 2.0;
        const double albj = dHb * dL / 2.0;
        double rb = 0.0;
        if (k == kmin) rb += bnd[0];
        if (k == kmax) rb += bnd[1];
        if (rb != 0.0) {
            Ubi[0] += 0.5 * rb;
            Ujb[0] += 0.5 * rb;
            if (dL > 0.0) {
                fdb[0] -= rb / (2.0 * dL);
                dLb += rb * fd[0] / (2.0 * dL * dL);
            }
        }
        NodeCot<D> cj;
        cot_zero<D>(cj);
        if (k == kphi) cj.phi = bnd[2];
        double Fbj[NC][D];
#pragma unroll
        for (int r = 0; r < NC; ++r)
#pragma unroll
            for (int q = 0; q < D; ++q) {
                Fbj[r][q] = fdb[r] * c[q];
                Fbi[r][q] -= fdb[r] * c[q];
            }
        flux_vjp<D>(Aj.U, Aj.v, Aj.p, Fbj, cj);
        node_vjp<D>(Aj.U, Aj.p, Aj.c, Aj.er, Aj.phi, g, cj, false, Ujb);
#pragma unroll
        for (int r = 0; r < NC; ++r) cuj[r] = Ujb[r];
        A.calj[e] = albj;
        A.db3[e] = dLb;
    }
    if (kmin < 0) Ubi[0] += bnd[0];
    if (kmax < 0) Ubi[0] += bnd[1];
    NodeCot<D> ci;
    cot_zero<D>(ci);
    if (kphi < 0) ci.phi = bnd[2];
    flux_vjp<D>(Ai.U, Ai.v, Ai.p, Fbi, ci);
    node_vjp<D>(Ai.U, Ai.p, Ai.c, Ai.er, Ai.phi, g, ci, false, Ubi);
#pragma unroll
    for (int r = 0; r < NC; ++r) A.Ub3[int64_t(i) * NC + r] = Ubi[r];
    A.alb[i] = albi;
}

// indicator alpha_i backwards (row)
template <int D>
__global__ void __launch_bounds__(kBlock) k_adj_alpha(StageArgs P, AdjArgs A)
{
    ROW_SETUP(P)
    constexpr int NC = D + 2;
    const double g = P.gamma;
    double alb = A.alb[i];
    for (int k = 0; k < L; ++k) {
        const int64_t e = ENTRY(k);
        if (P.scol[e] == i) continue;
        alb += A.cal[e] + A.calj[P.stpos[e]];
    }
    A.alt[i] = alb;
    double Ubi[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) Ubi[r] = 0.0;
    NodeA<D> Ai;
    load_a<D>(P.packA + int64_t(i) * kPack, Ai);
    double Fi[NC][D];
    flux<D>(Ai.U, Ai.v, Ai.p, Fi);
    double a = 0.0, b[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) b[r] = 0.0;
    for (int k = 0; k < L; ++k) {
        const int64_t e = ENTRY(k);
        const int j = P.scol[e];
        NodeA<D> Aj;
        load_a<D>(P.packA + int64_t(j) * kPack, Aj);
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
    }
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
    NodeCot<D> ci;
    cot_zero<D>(ci);
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
    double Fbi[NC][D];
#pragma unroll
    for (int r = 0; r < NC; ++r)
#pragma unroll
        for (int q = 0; q < D; ++q) Fbi[r][q] = 0.0;
    for (int k = 0; k < L; ++k) {
        const int64_t e = ENTRY(k);
        const int j = P.scol[e];
        double *cuj = A.cUj2 + e * NC;
        double Ujb[NC];
#pragma unroll
        for (int r = 0; r < NC; ++r) Ujb[r] = 0.0;
        {
            NodeA<D> Aj;
            load_a<D>(P.packA + int64_t(j) * kPack, Aj);
            double c[D];
            load_c<D>(P, e, c);
            double mc = 0.0;
#pragma unroll
            for (int q = 0; q < D; ++q) mc += Aj.U[1 + q] * c[q];
            NodeCot<D> cj;
            cot_zero<D>(cj);
            cj.er = ab * mc;
            ci.er -= ab * mc;
#pragma unroll
            for (int q = 0; q < D; ++q) cj.U[1 + q] += ab * (Aj.er - Ai.er) * c[q];
            double Fbj[NC][D];
#pragma unroll
            for (int r = 0; r < NC; ++r)
#pragma unroll
                for (int q = 0; q < D; ++q) {
                    Fbj[r][q] = bb[r] * c[q];
                    Fbi[r][q] -= bb[r] * c[q];
                }
            flux_vjp<D>(Aj.U, Aj.v, Aj.p, Fbj, cj);
            node_vjp<D>(Aj.U, Aj.p, Aj.c, Aj.er, Aj.phi, g, cj, false, Ujb);
        }
        if (j == i) {
#pragma unroll
            for (int r = 0; r < NC; ++r) { Ubi[r] += Ujb[r]; cuj[r] = 0.0; }
        } else {
#pragma unroll
            for (int r = 0; r < NC; ++r) cuj[r] = Ujb[r];
        }
    }
    flux_vjp<D>(Ai.U, Ai.v, Ai.p, Fbi, ci);
    node_vjp<D>(Ai.U, Ai.p, Ai.c, Ai.er, Ai.phi, g, ci, true, Ubi);
#pragma unroll
    for (int r = 0; r < NC; ++r) A.Ub2[int64_t(i) * NC + r] = Ubi[r];
}

// graph viscosity backwards (pair): the active orientation of the max
template <int D>
__global__ void __launch_bounds__(kBlock) k_adj_dpair(StageArgs P, AdjArgs A)
{
    ADJ_PAIR_SETUP(P)
    constexpr int NC = D + 2;
    const double db = A.dbp[p_] + A.db3[e] + A.db3[t];
    A.dbp[p_] = db;
    if (db == 0.0) return;
    NodeA<D> Ai, Aj;
    load_a<D>(P.packA + int64_t(i) * kPack, Ai);
    load_a<D>(P.packA + int64_t(j) * kPack, Aj);
    double c[D], ct[D];
    load_c<D>(P, e, c);
    ct[0] = P.ct0[e];
    ct[1] = P.ct1[e];
    if (D == 3) ct[D - 1] = P.ct2[e];
    double aij = 0.0, aji = 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
        aij += c[q] * c[q];
        aji += ct[q] * ct[q];
    }
    aij = sqrt(aij);
    aji = sqrt(aji);
    double nij[D], nji[D], t1 = 0.0, t2 = 0.0;
    if (aij > 0.0) {
        const double inv = 1.0 / aij;
#pragma unroll
        for (int q = 0; q < D; ++q) nij[q] = c[q] * inv;
        t1 = lambda_max<D>(nij, Ai.U, Ai.p, Ai.c, Aj.U, Aj.p, Aj.c, P.gas) * aij;
    }
    if (aji > 0.0) {
        const double inv = 1.0 / aji;
#pragma unroll
        for (int q = 0; q < D; ++q) nji[q] = ct[q] * inv;
        t2 = lambda_max<D>(nji, Aj.U, Aj.p, Aj.c, Ai.U, Ai.p, Ai.c, P.gas) * aji;
    }
    NodeCot<D> bi, bj;
    cot_zero<D>(bi);
    cot_zero<D>(bj);
    if (t1 > t2) {
        if (aij > 0.0)
            lambda_vjp<D>(nij, Ai.U, Ai.p, Ai.c, Aj.U, Aj.p, Aj.c, P.gas, db * aij, bi, bj);
    } else if (aji > 0.0) {
        lambda_vjp<D>(nji, Aj.U, Aj.p, Aj.c, Ai.U, Ai.p, Ai.c, P.gas, db * aji, bj, bi);
    }
    double Ubi[NC], Ubj[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) { Ubi[r] = 0.0; Ubj[r] = 0.0; }
    node_vjp<D>(Ai.U, Ai.p, Ai.c, Ai.er, Ai.phi, P.gamma, bi, false, Ubi);
    node_vjp<D>(Aj.U, Aj.p, Aj.c, Aj.er, Aj.phi, P.gamma, bj, false, Ubj);
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        A.cU[e * NC + r] += Ubi[r];
        A.cU[t * NC + r] += Ubj[r];
    }
}

// the node's cotangent: its own parts and its entries' and transposed
// entries' slots, in row order
template <int D>
__global__ void __launch_bounds__(kBlock) k_adj_final(StageArgs P, AdjArgs A)
{
    ROW_SETUP(P)
    constexpr int NC = D + 2;
    double Ub[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r)
        Ub[r] = A.Ub3[int64_t(i) * NC + r] + A.Ub2[int64_t(i) * NC + r];
    for (int k = 0; k < L; ++k) {
        const int64_t e = ENTRY(k);
        if (P.scol[e] == i) continue;
        const int64_t t = P.stpos[e];
#pragma unroll
        for (int r = 0; r < NC; ++r)
            Ub[r] += A.cU[e * NC + r] + A.cUj[t * NC + r] + A.cUj2[t * NC + r];
    }
#pragma unroll
    for (int r = 0; r < NC; ++r) A.Ub[int64_t(i) * NC + r] = Ub[r];
}

// SSP-RK3 and the held nodes backwards, per node (stage k of a step):
// out = hold ? U0 : U0 + theta (E - U0) with theta = 1 (stage 1: out = E),
// 1/4, 2/3.  Eb = theta * outb off the held nodes; U0's cotangent gains
// (1 - theta) outb (all of outb on a held node).
__global__ void k_adj_ssp(int64_t n, int nc, const uint8_t *hold, const double *outb,
                          double theta, double *Eb, double *U0b, int first)
{
    const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (q >= n * nc) return;
    const bool h = hold && hold[q / nc];
    const double o = outb[q];
    Eb[q] = h ? 0.0 : theta * o;
    const double add = h ? o : (1.0 - theta) * o;
    U0b[q] = first ? add : U0b[q] + add;
}

__global__ void k_adj_add(int64_t n, const double *x, double *y)
{
    const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (q < n) y[q] += x[q];
}

// ------------------------------------------------------------ launches
// row kernels use the XCD renumbering of ROW_SETUP: per * 8 blocks
static inline int rows_grid(const StageArgs &P) { return P.per * kXcd; }
static inline int pairs_grid(const StageArgs &P) { return int((P.npairs + kBlock - 1) / kBlock); }

#define ADJ_LAUNCH(K, grid)                                                              \
    do {                                                                                 \
        if (grid > 0) {                                                                  \
            if (P.dim == 2)                                                              \
                hipLaunchKernelGGL(K<2>, dim3(grid), dim3(kBlock), 0, st, P, A);         \
            else                                                                         \
                hipLaunchKernelGGL(K<3>, dim3(grid), dim3(kBlock), 0, st, P, A);         \
        }                                                                                \
    } while (0)

void launch_stage_vjp(const StageArgs &P, const AdjArgs &A, hipStream_t st)
{
    ADJ_LAUNCH(k_adj_pass2, rows_grid(P));
    if (P.passes >= 2) ADJ_LAUNCH(k_adj_lim2, pairs_grid(P));
    ADJ_LAUNCH(k_adj_pass1, rows_grid(P));
    ADJ_LAUNCH(k_adj_lim1, pairs_grid(P));
    ADJ_LAUNCH(k_adj_low, rows_grid(P));
    ADJ_LAUNCH(k_adj_alpha, rows_grid(P));
    ADJ_LAUNCH(k_adj_dpair, pairs_grid(P));
    ADJ_LAUNCH(k_adj_final, rows_grid(P));
}

void launch_adj_ssp(hipStream_t st, int64_t n, int nc, const uint8_t *hold, const double *outb,
                    double theta, double *Eb, double *U0b, int first)
{
    const int64_t m = n * nc;
    hipLaunchKernelGGL(k_adj_ssp, dim3(int((m + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, n, nc,
                       hold, outb, theta, Eb, U0b, first);
}

void launch_adj_add(hipStream_t st, int64_t n, const double *x, double *y)
{
    hipLaunchKernelGGL(k_adj_add, dim3(int((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, n, x,
                       y);
}

}  // namespace idp
