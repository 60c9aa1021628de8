// Minerbo closure of the O(v) two-moment model (Eqs. eddingtonFactorMinerbo,
// eddingtonTensor), shared by the O(v) solve and the primitive recovery.
#pragma once

#include "nmc_wave.h"

namespace nmc {

// Minerbo closure at one node: v.I and (v^i K_ij)_j with K_ij = k_ij D,
// k_ij = ((1 - psi) delta_ij + (3 psi - 1) n_i n_j) / 2, n = I / |I|, psi the
// polynomial Eddington factor of the flux factor h = |I| / D, taken as 0
// without flux and limited to [0, 1] (1 when D <= 0 carries a flux).
// The closure from |I| (Imag); rinv() gives 1 / |I| (0 without flux).
template <class RInv>
__device__ __forceinline__ void closure_from_norm(double D, const double (&I)[3], const double (&v)[3], double Imag,
                                                  RInv&& rinv, double& vI, double (&vK)[3]) {
  double h = 0.0;
  // Imag < D keeps D normal where its reciprocal is taken (a nonzero Imag is
  // at least ~1e-162: its components' squares underflow below that)
  if (Imag > 0.0) h = Imag < D ? Imag * rcp_nr(D) : 1.0;
  const double psi = 1.0 / 3.0 + (2.0 / 15.0) * (3.0 - h + 3.0 * h * h) * h * h;
  const double a = 0.5 * (1.0 - psi), b = 0.5 * (3.0 * psi - 1.0);
  const double rI = rinv();
  const double n0 = I[0] * rI, n1 = I[1] * rI, n2 = I[2] * rI;
  const double bvn = b * (v[0] * n0 + v[1] * n1 + v[2] * n2);
  vI = v[0] * I[0] + v[1] * I[1] + v[2] * I[2];
  vK[0] = D * (a * v[0] + bvn * n0);
  vK[1] = D * (a * v[1] + bvn * n1);
  vK[2] = D * (a * v[2] + bvn * n2);
}

__device__ __forceinline__ void closure_terms(double D, const double (&I)[3], const double (&v)[3], double& vI,
                                              double (&vK)[3]) {
  const double Imag = sqrt(I[0] * I[0] + I[1] * I[1] + I[2] * I[2]);
  closure_from_norm(D, I, v, Imag, [&] { return Imag > 0.0 ? rcp_nr(Imag) : 0.0; }, vI, vK);
}

// The same for moments of order one (a flux whose squared norm is at least
// 2^-1000, else the square root above): |I| and 1 / |I| from one reciprocal
// square root estimate y of s = |I|^2, refined by two coupled Newton steps on
// (g, h) -> (sqrt(s), 1 / (2 sqrt(s))) and a last correction of g.
__device__ __forceinline__ void closure_terms_unit(double D, const double (&I)[3], const double (&v)[3], double& vI,
                                                   double (&vK)[3]) {
  const double s = I[0] * I[0] + I[1] * I[1] + I[2] * I[2];
  double Imag, rI;
  if (s >= 0x1p-1000 && s <= 0x1p+1000) {
    const double y = __builtin_amdgcn_rsq(s);
    double g = s * y, hh = 0.5 * y;
    double e = __builtin_fma(-g, hh, 0.5);
    g = __builtin_fma(g, e, g);
    hh = __builtin_fma(hh, e, hh);
    e = __builtin_fma(-g, hh, 0.5);
    g = __builtin_fma(g, e, g);
    hh = __builtin_fma(hh, e, hh);
    Imag = __builtin_fma(__builtin_fma(-g, g, s), hh, g);
    rI = 2.0 * hh;
  } else {
    Imag = sqrt(s);
    rI = Imag > 0.0 ? rcp_nr(Imag) : 0.0;
  }
  closure_from_norm(D, I, v, Imag, [&] { return rI; }, vI, vK);
}

// Linear-order collision terms of one species at one node (Eqs.
// zerothMomentCollisionTerm_NES/_Pair, firstMomentCollisionTerm_NES/_Pair):
// with P = L_in - L_pro and R = L_out - L_ann (vectors over i),
//   number equation: (R - P).I
//   flux equation j: P_j / 3 + (K (R - P))_j,  K = D ((1 - psi) 1 + (3 psi - 1) n n) / 2
// (the Minerbo tensor of the node, as in closure_terms)
__device__ __forceinline__ void phi1_collision(double D, const double (&I)[3], const double (&P)[3],
                                               const double (&R)[3], double& c0, double (&c1)[3]) {
  const double Imag = sqrt(I[0] * I[0] + I[1] * I[1] + I[2] * I[2]);
  double h = 0.0;
  if (Imag > 0.0) h = Imag < D ? Imag * rcp_nr(D) : 1.0;
  const double psi = 1.0 / 3.0 + (2.0 / 15.0) * (3.0 - h + 3.0 * h * h) * h * h;
  const double a = 0.5 * (1.0 - psi), b = 0.5 * (3.0 * psi - 1.0);
  const double rI = Imag > 0.0 ? rcp_nr(Imag) : 0.0;
  const double n0 = I[0] * rI, n1 = I[1] * rI, n2 = I[2] * rI;
  const double d0 = R[0] - P[0], d1 = R[1] - P[1], d2 = R[2] - P[2];
  const double bnd = b * (n0 * d0 + n1 * d1 + n2 * d2);
  c0 = d0 * I[0] + d1 * I[1] + d2 * I[2];
  c1[0] = P[0] * (1.0 / 3.0) + D * (a * d0 + bnd * n0);
  c1[1] = P[1] * (1.0 / 3.0) + D * (a * d1 + bnd * n1);
  c1[2] = P[2] * (1.0 / 3.0) + D * (a * d2 + bnd * n2);
}

}  // namespace nmc
