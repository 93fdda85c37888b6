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
// other state's term is evaluated.  TR: *code receives 1 if p_i > p_j.
template <int D, bool TR = false>
__device__ __forceinline__ double psi_sum(double rhoi, double pi, double ci, double rhoj,
                                          double pj, double cj, const GasC &G,
                                          unsigned *code = nullptr)
{
    const bool jlow = pi > pj;
    const double pmax = jlow ? pi : pj;
    const double rho = jlow ? rhoj : rhoi, ps = jlow ? pj : pi, cs = jlow ? cj : ci;
    if constexpr (TR) *code = jlow ? 1u : 0u;
    return psi_branch<D>(rho, ps, cs, pmax, G.g);
}

// Decision bits of one wave-speed bound (decision traces): which branch
// each comparison, clamp and max of the bound took.
enum : unsigned {
    kLamPsiNeg = 1u,       // psi(p_max) < 0: p* = p~
    kLamCapped = 2u,       // p_max < p~ (p* = p_max when psi(p_max) >= 0)
    kLamNumPos = 4u,       // the two-rarefaction numerator is positive
    kLamShock1 = 8u,       // p* > p_i: the 1-wave speed grows
    kLamShock3 = 16u,      // p* > p_j: the 3-wave speed grows
    kLamWave1 = 32u        // [lambda_1]_neg > [lambda_3]_pos
};

// The guaranteed upper bound on the maximum wave speed of the 1D Riemann
// problem along n between U_i (left) and U_j (right) (Section 3.7): the
// pressure bound is the two-rarefaction pressure p~, capped at p_max when
// psi(p_max) >= 0 (then p* <= p_max); then the extreme speeds of the 1-wave
// and 3-wave at that pressure.  S is psi_sum of the pair (psi(p_max)
// without its u_j - u_i term).  TR: *code receives the kLam* bits.
template <int D, bool TR = false>
__device__ __forceinline__ double lambda_max_s(const double *n, const double *Ui, double pi,
                                               double ci, const double *Uj, double pj,
                                               double cj, double S, const GasC &G,
                                               unsigned *code = nullptr)
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
    const double gi = (pstar - pi) / pi, gj = (pstar - pj) / pj;
    const double lam1 = ui - ci * sqrt(1.0 + G.f * pos_part(gi));
    const double lam3 = uj + cj * sqrt(1.0 + G.f * pos_part(gj));
    const double a = neg_part(lam1), b = pos_part(lam3);
    if constexpr (TR)
        *code = (psi < 0.0 ? kLamPsiNeg : 0u) | (pmax < ptilde ? kLamCapped : 0u) |
                (num > 0.0 ? kLamNumPos : 0u) | (gi > 0.0 ? kLamShock1 : 0u) |
                (gj > 0.0 ? kLamShock3 : 0u) | (a > b ? kLamWave1 : 0u);
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

// Decision bits of one limiter evaluation (decision traces).
enum : unsigned {
    kLimRhoMax = 1u,       // the step was cut where rho reaches rho_max
    kLimRhoMin = 2u,       // ... where rho reaches rho_min
    kLimClamp = 4u,        // the cut step fell outside [0, 1]
    kLimStepShift = 3,     // bits 3-4: enclosure steps taken (saturating at 3)
    kLimExitHi = 32u,      // the search ended with Psi(hi) >= 0 (hi accepted)
    kLimExitLo = 64u,      // ... with Psi(lo) <= TOL (lo accepted)
    kLimGuard = 128u       // a safeguard of an enclosure step acted
};

// One step of the quadratic enclosure of Alg. 3 on the bracket [lo, hi],
// where Psi(lo) = f_lo >= 0 > Psi(hi) = f_hi, with slopes s_lo, s_hi.  With
// the divided differences D1 = (f_hi - f_lo)/w over the width w (w kept
// above zero by 2^-52), k_lo = (D1 - s_lo)/w and k_hi = (s_hi - D1)/w, the
// quadratics q_lo(t) = f_lo + s_lo (t - lo) + k_lo (t - lo)^2 and
// q_hi(t) = f_hi + s_hi (t - hi) + k_hi (t - hi)^2 interpolate Psi and its
// slope at one end and Psi at the other.  Along the line the third
// derivative of Psi is -phi_min (gamma+1) gamma (gamma-1) rho^(gamma-2)
// rho(P)^3, so by the Hermite remainder q_lo lies below Psi on the bracket
// when rho(P) >= 0: its root is a safe new lo and the root of q_hi a new
// hi; for rho(P) < 0 the two swap.  A root is taken next to its expansion
// point in the cancellation-free form t0 - 2 f/(s - sqrt(s^2 - 4 f k)),
// with the discriminant clipped at 0 and a vanishing denominator leaving
// t0; the new points are kept inside [lo, hi] and in order.  TR: kLimGuard
// into *code when a clip, a vanishing denominator or a clamp acted.
template <bool TR = false>
__device__ __forceinline__ void enclose_step(double &lo, double &hi, double f_lo, double f_hi,
                                             double s_lo, double s_hi, double rhoP,
                                             unsigned *code = nullptr)
{
    const double inv_w = 1.0 / (hi - lo + 0x1p-52);
    const double D1 = (f_hi - f_lo) * inv_w;
    const double k_lo = (D1 - s_lo) * inv_w;
    const double k_hi = (s_hi - D1) * inv_w;
    double disc_lo = s_lo * s_lo - 4.0 * f_lo * k_lo;
    double disc_hi = s_hi * s_hi - 4.0 * f_hi * k_hi;
    bool guard = disc_lo < 0.0 || disc_hi < 0.0;
    if (disc_lo < 0.0) disc_lo = 0.0;
    if (disc_hi < 0.0) disc_hi = 0.0;
    const double den_lo = s_lo - sqrt(disc_lo);
    const double den_hi = s_hi - sqrt(disc_hi);
    guard = guard || den_lo == 0.0 || den_hi == 0.0;
    const double root_lo = den_lo != 0.0 ? lo - 2.0 * f_lo / den_lo : lo;
    const double root_hi = den_hi != 0.0 ? hi - 2.0 * f_hi / den_hi : hi;
    double new_lo = rhoP >= 0.0 ? root_lo : root_hi;
    double new_hi = rhoP >= 0.0 ? root_hi : root_lo;
    const double in_lo = new_lo, in_hi = new_hi;
    if (!(new_lo >= lo)) new_lo = lo;
    if (!(new_lo <= hi)) new_lo = hi;
    if (!(new_hi <= hi)) new_hi = hi;
    if (!(new_hi >= lo)) new_hi = lo;
    if (new_hi < new_lo) new_hi = new_lo;
    if constexpr (TR)
        if (guard || !(new_lo == in_lo) || !(new_hi == in_hi)) *code |= kLimGuard;
    lo = new_lo;
    hi = new_hi;
}

// Limiter of Section 3.9 (Alg. 2): the largest step t in [0, 1] found along
// V(t) = U + t P that keeps rho(V) in [rho_min, rho_max] and
// Psi(t) = rho eps(V) - phi_min rho(V)^(gamma+1) >= 0.  The density is
// linear in t: the full step is cut where it crosses a violated bound (a
// zero density direction cannot cross: step 0), then kept in [0, 1].  Psi is
// concave along the line and Psi(0) >= 0: a bracket [lo, hi] = [0, cut]
// shrinks by enclosure steps, at most newton_max, and the search ends when
// hi is admissible (returned) or Psi(lo) <= TOL (lo returned).  TR: the
// kLim* bits into *code.
template <int D, bool TR = false>
__device__ __forceinline__ double limiter(const double *U, const double *P,
                                          double rho_min, double rho_max,
                                          double phi_min, double g, int newton_max,
                                          double tol, unsigned *code = nullptr)
{
    const double r0 = U[0], dr = P[0];
    unsigned bits = 0;
    double hi = 1.0;
    if (r0 + hi * dr > rho_max) {
        hi = dr != 0.0 ? fabs(rho_max - r0) / fabs(dr) : 0.0;
        bits |= kLimRhoMax;
    }
    if (r0 + hi * dr < rho_min) {
        hi = dr != 0.0 ? fabs(rho_min - r0) / fabs(dr) : 0.0;
        bits |= kLimRhoMin;
    }
    if (hi > 1.0 || hi < 0.0) bits |= kLimClamp;
    if (hi > 1.0) hi = 1.0;
    if (hi < 0.0) hi = 0.0;
    double lo = 0.0;
    int steps = 0;
    for (int it = 0; it < newton_max; ++it) {
        double f_hi, s_hi;
        psi_line<D>(U, P, hi, phi_min, g, f_hi, s_hi);
        if (f_hi >= 0.0) {
            lo = hi;
            bits |= kLimExitHi;
            break;
        }
        double f_lo, s_lo;
        psi_line<D>(U, P, lo, phi_min, g, f_lo, s_lo);
        if (f_lo <= tol) {
            bits |= kLimExitLo;
            break;
        }
        enclose_step<TR>(lo, hi, f_lo, f_hi, s_lo, s_hi, dr, &bits);
        ++steps;
    }
    if constexpr (TR) *code = bits | (unsigned(steps < 3 ? steps : 3) << kLimStepShift);
    return lo;
}

}  // namespace idp
