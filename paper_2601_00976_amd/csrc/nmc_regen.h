// Energy-coupling rates of one kernel row regenerated from per-node exponent
// splits (Eqs. nesRatesNodal, pairRatesNodal), over 16 of the 32 columns.
// Shared by the one-point-per-wavefront solvers; L is their LDS layout (it
// provides the split factors E, the model table m, the amplitudes An, Ap and
// the broadcast vectors X = W e D and Y = W e (1 - D)).
#pragma once

#include "nmc_wave.h"

namespace nmc {

// Rates of row q over columns j0 .. j0 + 15 (partial sums); KM = 2 takes the
// pair factors b from Bq, KM = 1 recomputes them:
// eta = Phi_in W D_s + Phi_pro W (1 - D_sbar),
// chi = eta + Phi_out W (1 - D_s) + Phi_ann W D_sbar
template <int NS, int KM, class L>
__device__ __forceinline__ void regen_rates_half(const L& S, int q, int j0, const double (&Bq)[KM == 2 ? 16 : 1],
                                                 double (&eta)[NS], double (&chi)[NS]) {
  const SplitExp& E = S.E;
  const double Gq = E.G[q], eq = S.m.eps[q];
  const double Aeq = S.An * eq, Apq = S.Ap * eq;
  double etaN[NS], outN[NS], annP[NS], etaP[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) etaN[t] = outN[t] = annP[t] = etaP[t] = 0.0;
  // columns are read in 16-byte pairs (one ds_read_b128 per array and
  // pair, addressed from a single per-half base)
  const double2* __restrict__ G2 = reinterpret_cast<const double2*>(&E.G[j0]);
#pragma unroll(KM == 2 ? 8 : 2)
  for (int jp = 0; jp < 8; ++jp) {
    const double2 g2 = G2[jp];
    double2 x2[NS], y2[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      x2[t] = reinterpret_cast<const double2*>(&S.X[t][j0])[jp];
      y2[t] = reinterpret_cast<const double2*>(&S.Y[t][j0])[jp];
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int jj = 2 * jp + e, j = j0 + jj;
      const double Gj = e ? g2.y : g2.x;
      const bool up = j > q;  // q is the lower node of the pair
      double b;
      if constexpr (KM == 2) {
        b = Bq[jj];
      } else {
        const double Pq = E.P2[q], Rq = E.R2[q], Pj = E.P2[j], Rj = E.R2[j];
        const int nq = E.n2[q], nj = E.n2[j];
        b = ldexp(up ? Pq * Rj : Pj * Rq, up ? nq - nj : nj - nq);
      }
      // kernel entries without the factor A e_q e_j: e_j rides on the
      // broadcast vectors X, Y and A e_q is applied to the row sums
      const double b2 = b * b, b3 = b2 * b;
      const double fin = up ? b : b3, fout = up ? b3 : b;
      // G of the higher node of the pair is the smaller one (G falls with
      // energy and the nodes are in increasing energy)
      const double fann = b2, fpro = fmin(Gj, Gq);
      double x[NS], y[NS];
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        x[t] = e ? x2[t].y : x2[t].x;
        y[t] = e ? y2[t].y : y2[t].x;
      }
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int tb = pair_partner<NS>(t);
        etaN[t] = __builtin_fma(fin, x[t], etaN[t]);
        outN[t] = __builtin_fma(fout, y[t], outN[t]);
        annP[t] = __builtin_fma(fann, x[tb], annP[t]);
        etaP[t] = __builtin_fma(fpro, y[tb], etaP[t]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    eta[t] = __builtin_fma(Aeq, etaN[t], Apq * etaP[t]);
    chi[t] = __builtin_fma(Aeq, etaN[t] + outN[t], Apq * (etaP[t] + annP[t]));
  }
}

}  // namespace nmc
