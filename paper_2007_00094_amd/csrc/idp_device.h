// Device arithmetic of the IDP Q1 Euler scheme (arXiv:2007.00094), FP64.
//
// Every routine evaluates its formula in a fixed operation order with IEEE
// add/sub/mul/div/sqrt only (the library is compiled without FMA
// contraction); together with the fixed-method power below this makes the
// results reproducible bit for bit by any implementation that follows the
// same steps on an IEEE machine.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace idp {

// ------------------------------------------------------------ x^y
// Fixed method, x > 0 (0^y = 0 for y > 0): x = m 2^e with m in
// [sqrt(1/2), sqrt(2)); ln m = 2 atanh s, s = (m-1)/(m+1), odd series to
// s^23 by Horner in s^2; ln x = e ln2_hi + (e ln2_lo + ln m) kept as a
// two-term sum; y ln x as a two-term sum (exact product via fma);
// exp by z = k ln2 + r (Cody-Waite two-part ln 2) and the Taylor series of
// e^r to degree 14, scaled by 2^k.  A few ulp relative error.
constexpr double kLn2Hi = 6.93147180369123816490e-01;
constexpr double kLn2Lo = 1.90821492927058770002e-10;
constexpr double kInvLn2 = 1.44269504088896338700e+00;
constexpr double kSqrtHalf = 0.70710678118654752440;

constexpr double atanh_coef_(int k) { return 1.0 / double(2 * k + 1); }
constexpr double inv_fact_(int n) { return n == 0 ? 1.0 : inv_fact_(n - 1) / double(n); }
// compile-time constants: 1/(2k+1) and 1/n! (the latter by repeated division)
template <int K> struct AtanhC { static constexpr double v = atanh_coef_(K); };
template <int N> struct InvF { static constexpr double v = inv_fact_(N); };

__device__ __forceinline__ double fpow(double x, double y)
{
    if (x == 0.0 && y > 0.0) return 0.0;
    if (!(x > 0.0) || isinf(x) || isnan(y)) return __builtin_nan("");
    // frexp: x = m 2^e, m in [1/2, 1) (exact)
    double m = __builtin_amdgcn_frexp_mant(x);
    int e = __builtin_amdgcn_frexp_exp(x);
    if (m < kSqrtHalf) { m = 2.0 * m; e -= 1; }
    const double s = (m - 1.0) / (m + 1.0);
    const double s2 = s * s;
    double t = AtanhC<11>::v;
    t = t * s2 + AtanhC<10>::v;
    t = t * s2 + AtanhC<9>::v;
    t = t * s2 + AtanhC<8>::v;
    t = t * s2 + AtanhC<7>::v;
    t = t * s2 + AtanhC<6>::v;
    t = t * s2 + AtanhC<5>::v;
    t = t * s2 + AtanhC<4>::v;
    t = t * s2 + AtanhC<3>::v;
    t = t * s2 + AtanhC<2>::v;
    t = t * s2 + AtanhC<1>::v;
    const double w = 2.0 * s;
    const double lnm = w + w * (s2 * t);
    const double de = double(e);
    const double A = de * kLn2Hi;
    const double B = de * kLn2Lo + lnm;
    const double lh = A + B;
    const double ll = (A - lh) + B;
    const double zh = y * lh;
    const double zl = fma(y, lh, -zh) + y * ll;
    if (zh > 709.78) return __builtin_inf();
    if (zh < -745.0) return 0.0;
    const double k = rint(zh * kInvLn2);
    const double r = ((zh - k * kLn2Hi) - k * kLn2Lo) + zl;
    double p = InvF<14>::v;
    p = p * r + InvF<13>::v;
    p = p * r + InvF<12>::v;
    p = p * r + InvF<11>::v;
    p = p * r + InvF<10>::v;
    p = p * r + InvF<9>::v;
    p = p * r + InvF<8>::v;
    p = p * r + InvF<7>::v;
    p = p * r + InvF<6>::v;
    p = p * r + InvF<5>::v;
    p = p * r + InvF<4>::v;
    p = p * r + InvF<3>::v;
    p = p * r + InvF<2>::v;
    p = p * r + InvF<1>::v;
    p = p * r + InvF<0>::v;
    return __builtin_amdgcn_ldexp(p, int(k));
}

// ------------------------------------------------------------- EOS
// Section 2 (ideal gas): eps = E - |m|^2/(2 rho), p = (gamma-1) eps,
// c = sqrt(gamma p / rho), phi = eps rho^-gamma, eta = (rho eps)^(1/(g+1)).
template <int D>
__device__ __forceinline__ double internal_energy(const double *U)
{
    double m2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) m2 += U[1 + k] * U[1 + k];
    return U[D + 1] - 0.5 * m2 / U[0];
}

template <int D>
__device__ __forceinline__ double pressure(const double *U, double g)
{
    return (g - 1.0) * internal_energy<D>(U);
}

template <int D>
__device__ __forceinline__ double speed_of_sound(const double *U, double g)
{
    return sqrt(g * pressure<D>(U, g) / U[0]);
}

template <int D>
__device__ __forceinline__ double specific_entropy(const double *U, double g)
{
    return internal_energy<D>(U) * fpow(U[0], -g);
}

template <int D>
__device__ __forceinline__ double harten_entropy(const double *U, double g)
{
    return fpow(U[0] * internal_energy<D>(U), 1.0 / (g + 1.0));
}

// Section 3.8: eta'(U) = (rho eps)^(-g/(g+1))/(g+1) (E, -m, rho)
template <int D>
__device__ __forceinline__ void harten_entropy_derivative(const double *U, double g,
                                                          double *out)
{
    const double re = U[0] * internal_energy<D>(U);
    const double f = fpow(re, -g / (g + 1.0)) / (g + 1.0);
    out[0] = f * U[D + 1];
#pragma unroll
    for (int k = 0; k < D; ++k) out[1 + k] = -f * U[1 + k];
    out[D + 1] = f * U[0];
}

__device__ __forceinline__ double pos_part(double x) { return 0.5 * (fabs(x) + x); }
__device__ __forceinline__ double neg_part(double x) { return 0.5 * (fabs(x) - x); }

// eq. flux contracted: F[r][k] of f(U) = (m, v (x) m + p I, v (E + p))^T,
// from U, v = m/rho and p given.
template <int D>
__device__ __forceinline__ void flux(const double *U, const double *v, double p,
                                     double F[D + 2][D])
{
    const double E = U[D + 1];
#pragma unroll
    for (int k = 0; k < D; ++k) F[0][k] = U[1 + k];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int k = 0; k < D; ++k) F[1 + a][k] = v[k] * U[1 + a] + (a == k ? p : 0.0);
#pragma unroll
    for (int k = 0; k < D; ++k) F[D + 1][k] = v[k] * (E + p);
}

// out = (f(U_j) - f(U_i)) . c
template <int D>
__device__ __forceinline__ void flux_diff_dot(const double Fi[D + 2][D],
                                              const double Fj[D + 2][D],
                                              const double *c, double *out)
{
#pragma unroll
    for (int r = 0; r < D + 2; ++r) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s += (Fj[r][k] - Fi[r][k]) * c[k];
        out[r] = s;
    }
}

// ------------------------------------------------- wave-speed bound
// Section 3.7.  A state enters as (rho, m, p, c); the projected 1D state
// has rho~ = rho, u~ = (n.m)/rho and the internal energy of U, hence
// p~ = p and c~ = c.
template <int D>
__device__ __forceinline__ double psi_branch(double rho, double ps, double cs, double p,
                                             double g)
{
    if (p >= ps)
        return 1.4142135623730951 * (p - ps) /
               sqrt(rho * ((g + 1.0) * p + (g - 1.0) * ps));
    return (fpow(p / ps, (g - 1.0) / (2.0 * g)) - 1.0) * 2.0 * cs / (g - 1.0);
}

// Constants of the bound that depend on gamma only, evaluated once per
// launch with exactly the expressions the formula uses.
struct GasC {
    double g;
    double half_gm1;   // (g - 1)/2 as 0.5 * (g - 1)
    double e_den;      // -(g - 1)/(2 g)
    double e_p;        // 2 g/(g - 1)
    double f;          // (g + 1)/(2 g)
};

__host__ __device__ inline GasC make_gas(double g)
{
    GasC G;
    G.g = g;
    G.half_gm1 = 0.5 * (g - 1.0);
    G.e_den = -(g - 1.0) / (2.0 * g);
    G.e_p = 2.0 * g / (g - 1.0);
    G.f = (g + 1.0) / (2.0 * g);
    return G;
}

// psi_branch(rho_i, p_i, c_i, p_max) + psi_branch(rho_j, p_j, c_j, p_max),
// p_max = max(p_i, p_j): the same for both orientations of a pair (the sum
// commutes), so a pair evaluates it once.  The state whose pressure is
// p_max contributes exactly +0 (its shock branch has p - p_s = 0 over a
// positive root), and x + 0 = x for the other term (never -0), so only the
// other state's term is evaluated.
template <int D>
__device__ __forceinline__ double psi_sum(double rhoi, double pi, double ci, double rhoj,
                                          double pj, double cj, const GasC &G)
{
    const bool jlow = pi > pj;
    const double pmax = jlow ? pi : pj;
    const double rho = jlow ? rhoj : rhoi, ps = jlow ? pj : pi, cs = jlow ? cj : ci;
    return psi_branch<D>(rho, ps, cs, pmax, G.g);
}

// The guaranteed upper bound on the maximum wave speed of the 1D Riemann
// problem along n between U_i (left) and U_j (right) (Section 3.7): the
// pressure bound is the two-rarefaction pressure p~, capped at p_max when
// psi(p_max) >= 0 (then p* <= p_max); then the extreme speeds of the 1-wave
// and 3-wave at that pressure.  S is psi_sum of the pair (psi(p_max)
// without its u_j - u_i term).
template <int D>
__device__ __forceinline__ double lambda_max_s(const double *n, const double *Ui, double pi,
                                               double ci, const double *Uj, double pj,
                                               double cj, double S, const GasC &G)
{
    double mti = 0.0, mtj = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) mti += n[k] * Ui[1 + k];
#pragma unroll
    for (int k = 0; k < D; ++k) mtj += n[k] * Uj[1 + k];
    const double ui = mti / Ui[0];
    const double uj = mtj / Uj[0];
    const double num = ci + cj - G.half_gm1 * (uj - ui);
    const double den = ci * fpow(pi / pj, G.e_den) + cj;
    const double ptilde = pj * fpow(pos_part(num) / den, G.e_p);
    const double pmax = pi > pj ? pi : pj;
    const double psi = S + uj - ui;
    double pstar;
    if (psi < 0.0)
        pstar = ptilde;
    else
        pstar = pmax < ptilde ? pmax : ptilde;
    const double lam1 = ui - ci * sqrt(1.0 + G.f * pos_part((pstar - pi) / pi));
    const double lam3 = uj + cj * sqrt(1.0 + G.f * pos_part((pstar - pj) / pj));
    const double a = neg_part(lam1), b = pos_part(lam3);
    return a > b ? a : b;
}

// ------------------------------------------------------------ limiter
// Psi(t) = rho eps(U + tP) - phi_min rho(U + tP)^(g+1) and Psi'(t).
template <int D>
__device__ __forceinline__ void psi_line(const double *U, const double *P, double t,
                                         double phi_min, double g, double &psi,
                                         double &dpsi)
{
    double V[D + 2];
#pragma unroll
    for (int k = 0; k < D + 2; ++k) V[k] = U[k] + t * P[k];
    const double rho = V[0], E = V[D + 1];
    double m2 = 0.0, mP = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        m2 += V[1 + k] * V[1 + k];
        mP += V[1 + k] * P[1 + k];
    }
    const double rho_eps = rho * E - 0.5 * m2;
    const double rg1 = fpow(rho, g + 1.0);
    psi = rho_eps - phi_min * rg1;
    dpsi = P[0] * E + rho * P[D + 1] - mP - phi_min * (g + 1.0) * (rg1 / rho) * P[0];
}

// Alg. 3 with sign = -1, eps = 2^-52; Lambda clipped at 0; a zero
// denominator leaves the end point; new points clamped into the old
// bracket; for rho(P) < 0 (third derivative of Psi positive) the q_R root
// bounds from below and the q_L root from above.
__device__ __forceinline__ void quadratic_newton(double &tL, double &tR, double psiL,
                                                 double psiR, double dpsiL,
                                                 double dpsiR, double rhoP)
{
    const double eps = 2.220446049250313e-16;
    const double sign = -1.0;
    const double scaling = 1.0 / (tR - tL + eps);
    const double d11 = dpsiL;
    const double d12 = (psiR - psiL) * scaling;
    const double d22 = dpsiR;
    const double d112 = (d12 - d11) * scaling;
    const double d122 = (d22 - d12) * scaling;
    double LL = dpsiL * dpsiL - 4.0 * psiL * d112;
    double LR = dpsiR * dpsiR - 4.0 * psiR * d122;
    if (LL < 0.0) LL = 0.0;
    if (LR < 0.0) LR = 0.0;
    const double denL = dpsiL + sign * sqrt(LL);
    const double denR = dpsiR + sign * sqrt(LR);
    const double rootL = denL != 0.0 ? tL - 2.0 * psiL / denL : tL;
    const double rootR = denR != 0.0 ? tR - 2.0 * psiR / denR : tR;
    double nl, nr;
    if (rhoP >= 0.0) { nl = rootL; nr = rootR; }
    else { nl = rootR; nr = rootL; }
    if (!(nl >= tL)) nl = tL;
    if (!(nl <= tR)) nl = tR;
    if (!(nr <= tR)) nr = tR;
    if (!(nr >= tL)) nr = tL;
    if (nr < nl) nr = nl;
    tL = nl;
    tR = nr;
}

// Alg. 2: largest admissible t in [0,1] found for U + t P under the
// bounds (rho_min, rho_max, phi_min).
template <int D>
__device__ __forceinline__ double limiter(const double *U, const double *P,
                                          double rho_min, double rho_max,
                                          double phi_min, double g, int newton_max,
                                          double tol)
{
    const double rhoU = U[0], rhoP = P[0];
    double tL = 0.0, tR = 1.0;
    if (rhoU + tR * rhoP > rho_max)
        tR = rhoP != 0.0 ? fabs(rho_max - rhoU) / fabs(rhoP) : 0.0;
    if (rhoU + tR * rhoP < rho_min)
        tR = rhoP != 0.0 ? fabs(rho_min - rhoU) / fabs(rhoP) : 0.0;
    if (tR > 1.0) tR = 1.0;
    if (tR < 0.0) tR = 0.0;
    for (int it = 0; it < newton_max; ++it) {
        double psiR, dpsiR;
        psi_line<D>(U, P, tR, phi_min, g, psiR, dpsiR);
        if (psiR >= 0.0) { tL = tR; break; }
        double psiL, dpsiL;
        psi_line<D>(U, P, tL, phi_min, g, psiL, dpsiL);
        if (psiL <= tol) break;
        quadratic_newton(tL, tR, psiL, psiR, dpsiL, dpsiR, rhoP);
    }
    return tL;
}

}  // namespace idp
