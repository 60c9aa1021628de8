// Projected Fermi-Dirac equilibrium on the energy elements (Sec. 3.5.2, Eq.
// fermiDiracProjection) with the bound-enforcing limiter, evaluated by the
// lanes of a wave that own one node each (elements = adjacent lane pairs).
//
// For an element K = [lo, hi] with Legendre-Gauss nodes e1 < e2 and Lagrange
// basis l_1, l_2, the projection D~ solves M D~ = b with the eps^2-weighted
// mass matrix M (host-inverted per element) and b_a = int_K l_a eps^2 f.  Since
// l_a eps^2 is a combination of eps^2 and eps^3, b follows from the moments
// F_k = int_K eps^k f (k = 2, 3); the complement 1 - D~ from the moments of
// 1 - f.  The moments are taken on the parts of K on either side of the
// chemical potential mu, each from the function that is small there (f above
// mu, 1 - f below), the other as the polynomial moment minus it:
//   - parts narrower than 1.5 T: 8-point Gauss-Legendre (f is analytic within
//     pi T of the real axis, so the rule is at rounding level);
//   - wider parts: differences of tail integrals in closed form,
//       int_x^inf eps^k f = T sum_j k!/(k-j)! x^(k-j) T^j F_j(z),
//       int_-inf^x eps^k (1 - f) = T sum_j k!/(k-j)! x^(k-j) (-T)^j F_j(z),
//     z = exp(-|x - mu| / T), F_j(z) = -Li_(j+1)(-z) = sum_m>=1 (-1)^(m+1)
//     z^m / m^(j+1), summed by the alternating-series acceleration of Cohen,
//     Rodriguez Villegas and Zagier (their Algorithm 1, 22 terms: relative
//     error below 4 (3 + sqrt 8)^-22 < 1e-16 for every z in [0, 1]).
// The two lanes of an element split the work (four Gauss points or one tail
// endpoint each) and add partner values by DPP, outside divergent code.
//
// Limiter (Zhang & Shu): D = Dbar + theta (D~ - Dbar) with Dbar = F_2 /
// int_K eps^2 and the largest theta in [0, 1] that keeps D >= D_min and
// 1 - D >= 1 - D_max at both nodes and both element edges; an element whose
// average itself lies outside takes the bound.
#pragma once

#include "nmc_wave.h"

namespace nmc {
namespace fdp {

constexpr int kTerms = 22;

// CVZ weights w_k (sum_k w_k a_k ~ sum_k (-1)^k a_k), computed at compile time
struct Cvz {
  double w[kTerms];
  constexpr Cvz() : w() {
    double d = 1.0;
    for (int i = 0; i < kTerms; ++i) d *= 3.0 + 2.8284271247461900976;  // (3 + sqrt 8)^n
    d = 0.5 * (d + 1.0 / d);
    double b = -1.0, c = -d;
    for (int k = 0; k < kTerms; ++k) {
      c = b - c;
      w[k] = c / d;
      b = (double)(k + kTerms) * (double)(k - kTerms) * b / ((k + 0.5) * (k + 1.0));
    }
  }
};
constexpr Cvz kCvz{};

// tail-integral coefficients: F_j(z) = sum_k c_j[k] z^(k+1), c_j[k] = w_k / (k+1)^(j+1)
struct TailCoef {
  double c[4][kTerms];
  constexpr TailCoef() : c() {
    for (int k = 0; k < kTerms; ++k) {
      double r = kCvz.w[k];
      for (int j = 0; j < 4; ++j) {
        r /= (double)(k + 1);
        c[j][k] = r;
      }
    }
  }
};
constexpr TailCoef kTail{};

// 8-point Gauss-Legendre rule on (-1, 1), nodes ascending
constexpr double kGx[8] = {-0.96028985649753623168, -0.79666647741362673959, -0.52553240991632898582,
                           -0.18343464249564980494, 0.18343464249564980494,  0.52553240991632898582,
                           0.79666647741362673959,  0.96028985649753623168};
constexpr double kGw[8] = {0.10122853629037625915, 0.22238103445337447054, 0.31370664587788728734,
                           0.36268378337836198297, 0.36268378337836198297, 0.31370664587788728734,
                           0.22238103445337447054, 0.10122853629037625915};

// Tail integrals at x for k = 2, 3: sgn = +1 gives int_x^inf eps^k f, sgn = -1
// gives int_-inf^x eps^k (1 - f).  |x - mu| / T is the distance from mu.
__device__ __forceinline__ void tails(double x, double mu, double T, double sgn, double& t2, double& t3) {
  const double z = exp(-fabs(x - mu) / T);
  double F0 = 0.0, F1 = 0.0, F2 = 0.0, F3 = 0.0, zp = 1.0;
#pragma unroll
  for (int k = 0; k < kTerms; ++k) {
    zp *= z;
    F0 = __builtin_fma(kTail.c[0][k], zp, F0);
    F1 = __builtin_fma(kTail.c[1][k], zp, F1);
    F2 = __builtin_fma(kTail.c[2][k], zp, F2);
    F3 = __builtin_fma(kTail.c[3][k], zp, F3);
  }
  const double s = sgn * T;
  t2 = T * (x * x * F0 + 2.0 * x * s * F1 + 2.0 * s * s * F2);
  t3 = T * (x * x * x * F0 + 3.0 * x * x * s * F1 + 6.0 * x * s * s * F2 + 6.0 * s * s * s * F3);
}

// This lane's share of the moments (k = 2, 3) over [a, b] of f (above = true,
// the part lies above mu) or of 1 - f (below mu); the partner lane of the
// element holds the rest.  side = 0 or 1 within the element.
__device__ __forceinline__ void part_share(double a, double b, double mu, double T, bool above, int side, double& m2,
                                           double& m3) {
  m2 = m3 = 0.0;
  if (!(b > a)) return;
  if (b - a <= 1.5 * T) {
    const double c = 0.5 * (a + b), r = 0.5 * (b - a);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int g = 4 * side + i;
      const double e = __builtin_fma(r, kGx[g], c);
      const double x = (e - mu) / T;
      // f above mu, 1 - f below: exp(-|x|) / (1 + exp(-|x|)) in both
      const double ex = exp(-fabs(x));
      const double v = ex / (1.0 + ex);
      const double w = r * kGw[g] * e * e * v;
      m2 += w;
      m3 += w * e;
    }
  } else {
    double t2, t3;
    const double x = side ? b : a;
    tails(x, mu, T, above ? 1.0 : -1.0, t2, t3);
    // f: int_a^b = G(a) - G(b); 1 - f: int_a^b = H(b) - H(a)
    const double sg = (above == (side == 0)) ? 1.0 : -1.0;
    m2 = sg * t2;
    m3 = sg * t3;
  }
}

// Projected, limited equilibrium D and complement C = 1 - D of one species at
// the lane's node q (0..nq-1, elements = lane pairs 2e, 2e + 1), for a
// chemical potential mu and temperature T uniform over the lane's element.
// Every lane of the wave calls it (the partner exchange is a quad_perm DPP).
__device__ __forceinline__ void projected_node(const DevModel* __restrict__ mg, int q, double T, double mu,
                                               double& D, double& C) {
  const int side = q & 1;
  const double lo = mg->pelo[q], hi = mg->pehi[q];
  // parts of the element above and below mu
  const double aA = fmax(lo, mu), bB = fmin(hi, mu);
  double sA2, sA3, sB2, sB3;
  part_share(aA, hi, mu, T, true, side, sA2, sA3);
  part_share(lo, bB, mu, T, false, side, sB2, sB3);
  sA2 += dpp<0xB1>(sA2);  // quad_perm [1,0,3,2]: the element's partner lane
  sA3 += dpp<0xB1>(sA3);
  sB2 += dpp<0xB1>(sB2);
  sB3 += dpp<0xB1>(sB3);
  // polynomial moments of the two parts
  const double pA2 = hi > aA ? (hi * hi * hi - aA * aA * aA) / 3.0 : 0.0;
  const double pA3 = hi > aA ? (hi * hi * hi * hi - aA * aA * aA * aA) / 4.0 : 0.0;
  const double pB2 = bB > lo ? (bB * bB * bB - lo * lo * lo) / 3.0 : 0.0;
  const double pB3 = bB > lo ? (bB * bB * bB * bB - lo * lo * lo * lo) / 4.0 : 0.0;
  const double F2 = sA2 + (pB2 - sB2), F3 = sA3 + (pB3 - sB3);
  const double C2 = (pA2 - sA2) + sB2, C3 = (pA3 - sA3) + sB3;
  // b_a = int l_a eps^2 g with l_a eps^2 = u_a eps^3 + v_a eps^2 (host tables)
  const double u1 = mg->pl[q][0], v1 = mg->pl[q][1], u2 = mg->pl[q][2], v2 = mg->pl[q][3];
  const double bf1 = u1 * F3 + v1 * F2, bf2 = u2 * F3 + v2 * F2;
  const double bc1 = u1 * C3 + v1 * C2, bc2 = u2 * C3 + v2 * C2;
  // row of the inverse mass matrix for this node
  const double r0 = mg->pinv[q][0], r1 = mg->pinv[q][1];
  const double dt = r0 * bf1 + r1 * bf2, ct = r0 * bc1 + r1 * bc2;
  const double rm0 = mg->prm0[q];
  const double dbar = F2 * rm0, cbar = C2 * rm0;
  // values at the nodes and the element edges (l_own at lo and hi from the host)
  const double llo = mg->pedge[q][0], lhi = mg->pedge[q][1];
  const double dt_p = dpp<0xB1>(dt), ct_p = dpp<0xB1>(ct);
  const double dlo = __builtin_fma(dt, llo, dpp<0xB1>(dt * llo));
  const double dhi = __builtin_fma(dt, lhi, dpp<0xB1>(dt * lhi));
  const double clo = __builtin_fma(ct, llo, dpp<0xB1>(ct * llo));
  const double chi = __builtin_fma(ct, lhi, dpp<0xB1>(ct * lhi));
  const double mD = fmin(fmin(dt, dt_p), fmin(dlo, dhi));
  const double mC = fmin(fmin(ct, ct_p), fmin(clo, chi));
  const double dmin = mg->deq_min, cmin = mg->ceq_min;
  if (dbar < dmin) {
    D = dmin;
    C = 1.0 - dmin;
  } else if (cbar < cmin) {
    D = 1.0 - cmin;
    C = cmin;
  } else {
    double th = 1.0;
    if (mD < dmin) th = fmin(th, (dbar - dmin) / (dbar - mD));
    if (mC < cmin) th = fmin(th, (cbar - cmin) / (cbar - mC));
    D = __builtin_fma(th, dt - dbar, dbar);
    C = __builtin_fma(th, ct - cbar, cbar);
  }
}

}  // namespace fdp
}  // namespace nmc
