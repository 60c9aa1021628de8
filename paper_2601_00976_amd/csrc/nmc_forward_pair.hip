// Forward kernel of the implicit coupling solve for 32 energy nodes, two
// points per wavefront (CDNA4).
//
// Same algorithm as the one-point kernels (Algorithm neutrinoMatterCoupling,
// Sec. 3.5.3), different work decomposition.  Lane = 32 h + q: half h of the
// wave solves point 2u + h of pair u, and lane q of the half owns D_s[q] and
// I_s[q] of every species.  Every per-point step that a one-point kernel
// issues for a whole wave (equation of state, opacities, Anderson solves,
// convergence tests, matter update) serves two points here, and each lane
// contracts all 32 columns of its row:
//   - once per outer iteration the lanes of a point fill a 32 x 32 LDS tile
//     with its pair factors b(q, j) = exp(-|e_q - e_j| / (2T)), signed by
//     orientation (+b where j > q, -b otherwise), each unordered pair by one
//     lane, and every lane reads its row back into VGPRs (the tile shares
//     LDS with the Anderson history, which is dead between inner loops);
//   - in every inner iteration the vectors W e D and W e (1 - D) of the point
//     are redistributed with v_permlane16_swap, so that each 16-lane row
//     holds one half of its point's vector, and every FMA takes its column
//     through a DPP row_newbcast operand (v_fmac_f64_dpp): the contraction
//     reads no LDS (the moments and G_j come by broadcast from registers);
//   - per column, with s the signed factor and c = s^3 (same sign),
//     max(s, -c) and max(c, -s) are the Phi_in and Phi_out entries (b and
//     b^3 in one order or the other) without compares or selects;
//     Phi_ann = s^2 and Phi_pro = min(G_j, G_q) (G falls with energy), all
//     without their common factor A e_q e_j.
// The row sums take their factors A e_q in the Q step.
//
// Both halves run one instruction stream.  A half whose point has finished
// (or which has no point, past the end of an odd batch) keeps computing with
// its state frozen, so no barrier or cross-lane step is ever in divergent
// control flow; every per-point decision is a per-lane value that is uniform
// within its half.
#include "nmc_fdproj.h"
#include "nmc_pair.h"

namespace nmc {
namespace {

using namespace pairk;

template <int NS>
struct PairLds {
  ModelLds m;
  SplitExp E[2];                   // per point: exponent splits at its current temperature
  union {
    struct {
      double hist[4][2 * NS][kLanes];  // Anderson history per lane and owned moment: Q_prev, F_prev, dQ_old, dF_old
      double fac[2][NS][kLanes];       // projected equilibrium: 1 / sqrt(o) and o per species (o = D / (1 - D))
    };
    double tile[2][NQP][NQP];        // per point, signed pair factors: [j][q] = +b if j > q, else -b
  } u;
  struct Pt {                      // per-point state of the outer (matter) loop
    double y[2], oq[2], of[2], odq[2], odf[2];
    double r3, K, An, Ap;
    double ye_st, e_st, chi0, T_fix, mu_fix;
  } pt[2];
};

// PROJ: the equilibrium is the projected, limited Fermi-Dirac distribution of
// every species (Eq. fermiDiracProjection), and the kernels take their
// detailed-balance factors from its odds o = D / (1 - D) (Eqs.
// detailedBalanceNES, detailedBalancePair): g = sqrt(o) and h = o of each
// species replace exp(-e / (2T)) and exp(-e / T) of the pointwise form.  The
// limiter bounds o, so the symmetric core serves every temperature.
template <int NS, bool COUPLED, bool PROJ>
struct PairSolver {
  static constexpr int NQ = NQP;

  // settle() is called once the pair's inputs are loaded (work-queue hook)
  template <class Settle>
  __device__ static void solve(const FwdArgs& a, int64_t u, PairLds<NS>& S, Settle&& settle) {
    const_ptr<DevModel> md = scalar_ptr(a.mdl);
    const ModelLds& mt = S.m;
    const int lane = threadIdx.x;
    const int h = lane >> 5, q0 = lane & 31;
    const double dtau = a.dtau;
    // point of this half; past the end of an odd batch the half mirrors its
    // neighbour and stores nothing
    const int64_t p_raw = 2 * u + h;
    const bool has_point = p_raw < a.P;
    const int64_t p = has_point ? p_raw : p_raw - 1;
    const int64_t base = p * (int64_t)(NS * NQ);
    const double rho = a.rho11[p];
    const bool fixedT = a.prm.fixed_matter && a.T_fixed;
    typename PairLds<NS>::Pt& pt = S.pt[h];
    // ||D_c^[k,1]||_W^2 of the current inner loop for this lane's species
    // class c (spread_conv_sums; zero beyond NS), in a register
    const int cls = spread_class(lane);
    double dref = 0.0;

    double Dst[NS], Ist[NS], D[NS], I[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int64_t o = base + md->ext[t] * NQ + q0;
      Dst[t] = D[t] = a.D0[o];
      Ist[t] = I[t] = a.I0[o];
    }
    settle();

    // coupling disabled at low density (Sec. 7.2): the state passes through
    const bool skip = rho < md->rho11_min;

    pt.r3 = cbrt(rho);
    pt.K = md->kcoup / rho;
    pt.An = (md->flags & NMC_NES) ? mt.theta[NQ] * rho : 0.0;
    pt.Ap = (md->flags & NMC_PAIR) ? mt.theta[NQ + 1] * rho : 0.0;
    pt.ye_st = pt.y[0] = a.ye0[p];
    pt.e_st = pt.y[1] = a.e0[p];
    pt.chi0 = a.chi0 ? a.chi0[p] : md->chi_ref * rho;
    if (fixedT) pt.T_fix = a.T_fixed[p];
    if (a.prm.fixed_matter && a.mu_fixed) pt.mu_fix = a.mu_fixed[p];
#pragma unroll
    for (int i = 0; i < 2; ++i) pt.oq[i] = pt.of[i] = pt.odq[i] = pt.odf[i] = 0.0;
    {
      const double w2q = mt.w2[q0];
      double v[2 * ((NS + 1) / 2)], s[2 * ((NS + 1) / 2)];
#pragma unroll
      for (int t = 0; t < 2 * ((NS + 1) / 2); ++t) v[t] = t < NS ? w2q * D[t < NS ? t : 0] * D[t < NS ? t : 0] : 0.0;
      half_own_sums<(NS + 1) / 2>(v, s);
      dref = class_pick<NS>(s, cls);
    }

    int status = NMC_STATUS_OK;
    bool fatal = false, inner_failed = false, outer_conv = false;
    bool run = !skip;  // this half's point is still iterating the outer loop
    int k_done = 0, total_inner = 0;
    double T_last = 0.0;  // temperature of the last outer iteration this half ran

    for (int k = 1; k <= a.prm.max_outer && __builtin_amdgcn_ballot_w64(run) != 0; ++k) {
      const_ptr<DevModel> md = scalar_ptr(a.mdl);
      const int q = opaque(q0);
      if (run) k_done = k;
      // ---- ComputeOpacities(y^[k]) --------------------------------------
      const double r3 = pt.r3;
      const double y0 = pt.y[0], y1 = pt.y[1];
      // reciprocals by refined estimates (no IEEE division): the EOS is
      // evaluated per lane once per outer iteration
      const double T = fixedT ? pt.T_fix
                              : (y1 - md->eos_b * ye43(y0) * r3) * rcp_nr(md->eos_a * (1.0 + y0));
      const double mu = (a.prm.fixed_matter && a.mu_fixed)
                            ? pt.mu_fix
                            : md->mu_a * (y0 - md->mu_ye0) * r3 + md->mu_b * log_pos(T * md->inv_mu_t0);
      if (run && (!(T > 0.0) || !(y0 >= 0.0) || !isfinite(T) || !isfinite(mu))) {
        status = NMC_STATUS_EOS_DOMAIN;
        fatal = true;
        run = false;
      }
      T_last = run ? T : T_last;
      // a finished half keeps a harmless temperature
      const double Tu = run ? T : 1.0, muu = run ? mu : 0.0;
      const double invT = rcp_nr(Tu);
      // the exponent split of this lane's node (pair factors below), issued
      // here so that it overlaps the equilibrium's exponentials
      const double epsq = mt.eps[q];
      const ExpSplit xs = exp_split(epsq, invT);
      double baseD[NS], den0D[NS];
      // projected equilibrium and its complement at node q (every lane, both
      // halves: the element partner exchange is a DPP)
      double pD[PROJ ? NS : 1], pC[PROJ ? NS : 1];
      if constexpr (PROJ) {
#pragma unroll
        for (int t = 0; t < NS; ++t) fdp::projected_node(a.mdl, q, Tu, md->imusign[t] * muu, pD[t], pC[t]);
      }
      double dsig = 0.0;  // dtau sigma: 1 + dtau kappa = 1 + dtau chi + dsig
      {
        const double shape = pt.chi0 * mt.shape[q];
        const double sig = (md->flags & NMC_ISO) ? md->sigma_ratio * shape : 0.0;
        const double emab_q = (md->flags & NMC_EMAB) ? mt.theta[q] * shape : 0.0;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const double chia = md->iemab[t] * emab_q;
          double deq = 0.0;
          if constexpr (PROJ) {
            deq = pD[t];
          } else if (!(NS == 3 && t == 2)) {
            // three species are nu_e, anti-nu_e, nu_x in this order, and
            // nu_x has no emission or absorption (chia = 0): no equilibrium
            const double x = (epsq - md->imusign[t] * muu) * invT;
            const double ex = exp(-fabs(x));
            const double r = rcp_nr(1.0 + ex);
            deq = x > 0.0 ? ex * r : r;
          }
          baseD[t] = Dst[t] + dtau * (chia * deq);
          den0D[t] = 1.0 + dtau * chia;
        }
        dsig = dtau * sig;
      }
      // Pair factors of this lane's row, j = 0..31.  Symmetric form (sym):
      // B2(q, j) = b^2 = exp(-|e_q - e_j| / T), the core shared by all four
      // kernels: with g = exp(-e / (2T)) and h = g^2,
      //   Phi_in[q][j] = A e e' B2 g_q / g_j,  Phi_out[q][j] = A e e' B2 g_j / g_q,
      //   Phi_ann = A' e e' B2,  Phi_pro = A' e e' B2 h_q h_j,
      // so 1 / g_j and g_j ride on the contracted vectors and g_q, 1 / g_q on
      // the row sums, each scaled by 2^-+c (c centres the point's exponents,
      // so both stay in range while the grid spans at most kSymBits powers of
      // two in g, T above ~0.12 MeV).  Otherwise (colder points) the signed
      // orientation form: +b(q, j) for j > q (q the lower node), -b(q, j)
      // otherwise, every entry a product of factors <= 1.
      // Where the grid spans at most kDirectBits powers of two in g (T above
      // ~0.22 MeV) every lane forms its whole row from the point's scaled h
      // and 1 / h, broadcast from registers (direct_row_regs); otherwise the
      // lanes fill the point's LDS tile, each unordered pair once, and read
      // their rows back.
      double B[COUPLED ? NQ : 1];
      double hq = 0.0;  // exp(-e_q / T)
      double gq = 1.0, rgq = 1.0;  // g_q 2^c and 2^-c / g_q (symmetric form)
      bool sym = false;  // wave-uniform
      if constexpr (COUPLED) {
        SplitExp& E = S.E[h];
        E.P2[q] = xs.P;
        E.R2[q] = xs.R;
        E.n2[q] = xs.n;
        hq = ldexp(xs.R * xs.R, -2 * xs.n);  // 2^(-2x) = exp(-e / T)
        __syncthreads();
        // g = 2^-x with x = n + f increasing along the grid
        const int nlo = E.n2[0], nhi = E.n2[NQ - 1];
        const int c = (nlo + nhi) >> 1;
        const bool direct = __builtin_amdgcn_readfirstlane((uint32_t)(
                                __builtin_amdgcn_ballot_w64(run && nhi - nlo > kDirectBits) == 0)) != 0;
        if constexpr (PROJ) {
          sym = true;
        } else {
          sym = __builtin_amdgcn_readfirstlane(
                    (uint32_t)(__builtin_amdgcn_ballot_w64(run && nhi - nlo > kSymBits) == 0)) != 0;
          gq = sym ? ldexp(xs.R, c - xs.n) : 1.0;
          rgq = sym ? ldexp(xs.P, xs.n - c) : 1.0;
        }
        if (direct) {
          const double gt = PROJ ? ldexp(xs.R, c - xs.n) : gq;
          const double rgt = PROJ ? ldexp(xs.P, xs.n - c) : rgq;
          const double ht = gt * gt, rht = rgt * rgt;
          direct_row_regs(ht, rht, B);
        } else {
          // pair factors of the point, each unordered pair (q, q + d mod 32)
          // once: d = 1..15 by every lane, d = 16 by lanes q < 16
          double (*T)[NQ] = S.u.tile[h];
          if (sym) {
            pair_tile_rows<true>(&T[0][0], E.P2, E.R2, E.n2, q, xs.P, xs.R, xs.n);
            T[q][q] = 1.0;
          } else {
            pair_tile_rows<false>(&T[0][0], E.P2, E.R2, E.n2, q, xs.P, xs.R, xs.n);
            T[q][q] = -1.0;
          }
          __syncthreads();
          // row q of the lane: element [j][q] (consecutive lanes, consecutive words)
#pragma unroll
          for (int j = 0; j < NQ; ++j) B[j] = T[j][q];
          __syncthreads();
        }
        if constexpr (PROJ) {
          // the tile is consumed: its space holds the lane's factors
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            const double o = pD[t] / pC[t];
            S.u.fac[0][t][lane] = 1.0 / sqrt(o);
            S.u.fac[1][t][lane] = o;
          }
        }
      }

      // ---- inner loop over moments at fixed matter ------------------------
      const double w2q = mt.w2[q], w2eq = w2q * epsq;
      const double Aeq = pt.An * epsq, Apq = pt.Ap * epsq, Apqh = Apq * hq;

      double G11 = 0.0;
      // the reference norm of this inner loop (constant within the loop: a
      // converged loop sets the next loop's and ends)
      const double dref0 = dref;
      const bool ran = run;  // this half runs this outer iteration
      bool act = run;        // this half is still iterating the inner loop
      bool cvd = false;      // this half's inner loop converged
      int l_done = 0;
      for (int l = 1; l <= a.prm.max_inner && __builtin_amdgcn_ballot_w64(act) != 0; ++l) {
        if (act) l_done = l;
        double etaN[NS], outN[NS], annP[NS], etaP[NS];
#pragma unroll
        for (int t = 0; t < NS; ++t) etaN[t] = outN[t] = annP[t] = etaP[t] = 0.0;
        if constexpr (COUPLED) {
          // the pair factors are re-read per iteration: the per-column
          // products are not hoisted out of the inner loop (they would need
          // four times the registers)
#pragma unroll
          for (int j = 0; j < NQ; ++j) asm volatile("" : "+v"(B[j]));
          if (sym) {
            // W e D / g, g W e (1 - D), W e D and h W e (1 - D) of the point
            // (g scaled by 2^c), each 16-lane row holding the half
            // [16 R, 16 R + 16) of the nodes in [.][R][.]
            double AR[2][NS], BR[2][NS], CR[2][NS], DR[2][NS];
#pragma unroll
            for (int t = 0; t < NS; ++t) {
              double rg = rgq, g = gq, hh = hq;
              if constexpr (PROJ) {
                rg = S.u.fac[0][t][lane];
                hh = S.u.fac[1][t][lane];
                g = hh * rg;
              }
              const double xv = w2eq * D[t], yv = w2eq - xv;
              swap16(xv * rg, AR[0][t], AR[1][t]);
              swap16(yv * g, BR[0][t], BR[1][t]);
              swap16(xv, CR[0][t], CR[1][t]);
              swap16(hh * yv, DR[0][t], DR[1][t]);
            }
            static_for<0, NQ / 4>([&](auto jj) __attribute__((always_inline)) {
              constexpr int j = 4 * decltype(jj)::value;
              ColSym<NS>::template run<j % 16>(etaN, outN, annP, etaP, AR[j / 16], BR[j / 16], CR[j / 16],
                                               DR[j / 16], B[j], B[j + 1], B[j + 2], B[j + 3]);
            });
          } else {
            // W e D, W e (1 - D) and h W e (1 - D) of the point, each 16-lane
            // row holding the half [16 R, 16 R + 16) of the nodes in XR[.][R],
            // YR[.][R], HR[.][R]
            double XR[2][NS], YR[2][NS], HR[2][NS];
#pragma unroll
            for (int t = 0; t < NS; ++t) {
              const double xv = w2eq * D[t], yv = w2eq - xv;
              swap16(xv, XR[0][t], XR[1][t]);
              swap16(yv, YR[0][t], YR[1][t]);
              swap16(hq * yv, HR[0][t], HR[1][t]);
            }
            static_for<0, NQ / 2>([&](auto jj) __attribute__((always_inline)) {
              constexpr int j0 = 2 * decltype(jj)::value;
              static_for<0, 2>([&](auto ee) __attribute__((always_inline)) {
                constexpr int j = j0 + decltype(ee)::value;
                // with s = +-b and c = s^3 = +-b^3 (the same sign): max(s, -c)
                // is b where s > 0 and b^3 where s < 0, i.e. Phi_in, and
                // max(c, -s) is Phi_out (scaled entries), without compares or
                // selects; Phi_ann = b^2 serves the pair production term as
                // well (detailed balance: Phi_pro = Phi_ann h_q h_j)
                const double sb = B[j], b2 = sb * sb, c3 = sb * b2;
                ColFmac<NS>::template run<j % 16>(etaN, outN, annP, etaP, XR[j / 16], YR[j / 16], HR[j / 16],
                                                  max_neg_f64(sb, c3), max_neg_f64(c3, sb), b2);
              });
            });
          }
        }
        // Q and residual of both owned moments x = (D_t, I_t); the row sums
        // take their factors A e_q here, and one reciprocal of the product of
        // the two denominators serves both
        double Qx[2 * NS], Fx[2 * NS];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          double ag = Aeq * gq, arg = Aeq * rgq, aph = Apqh;
          if constexpr (PROJ && COUPLED) {
            const double rg = S.u.fac[0][t][lane], hh = S.u.fac[1][t][lane];
            ag = Aeq * (hh * rg);
            arg = Aeq * rg;
            aph = Apq * hh;
          }
          const double eta = __builtin_fma(ag, etaN[t], aph * etaP[t]);
          const double chi = __builtin_fma(arg, outN[t], __builtin_fma(Apq, annP[t], eta));
          const double dD = __builtin_fma(dtau, chi, den0D[t]), dI = dD + dsig;
          const double r = rcp_nr(dD * dI);
          Qx[t] = __builtin_fma(dtau, eta, baseD[t]) * (r * dI);
          Qx[NS + t] = Ist[t] * (r * dD);
          Fx[t] = Qx[t] - D[t];
          Fx[NS + t] = Qx[NS + t] - I[t];
        }
        // Anderson step over min(l, M_inner) residuals (difference form)
        const int mem = l < a.prm.m_inner ? l : a.prm.m_inner;
        double Xn[2 * NS];
        if (mem == 1) {
          // the older difference column is weighted zero at the second
          // iterate: clear it, so that no stale LDS word (a NaN pattern left
          // by another point or kernel) enters that product
#pragma unroll
          for (int x = 0; x < 2 * NS; ++x) {
            Xn[x] = Qx[x];
            S.u.hist[2][x][lane] = 0.0;
            S.u.hist[3][x][lane] = 0.0;
          }
        } else {
          double dQ2[2 * NS], dF2[2 * NS];
          double v4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int x = 0; x < 2 * NS; ++x) {
            dQ2[x] = Qx[x] - S.u.hist[0][x][lane];
            dF2[x] = Fx[x] - S.u.hist[1][x][lane];
            const double dF1 = S.u.hist[3][x][lane];
            v4[0] += dF1 * dF2[x];
            v4[1] += dF2[x] * dF2[x];
            v4[2] += dF1 * Fx[x];
            v4[3] += dF2[x] * Fx[x];
          }
          double gs[4];
          half_sums4(v4, gs);
          double g1, g2;
          anderson2(mem == 3, G11, gs[0], gs[1], gs[2], gs[3], g1, g2);
#pragma unroll
          for (int x = 0; x < 2 * NS; ++x) {
            Xn[x] = Qx[x] - g2 * dQ2[x] - g1 * S.u.hist[2][x][lane];
            S.u.hist[2][x][lane] = dQ2[x];
            S.u.hist[3][x][lane] = dF2[x];
          }
          G11 = gs[1];
        }
#pragma unroll
        for (int x = 0; x < 2 * NS; ++x) {
          S.u.hist[0][x][lane] = Qx[x];
          S.u.hist[1][x][lane] = Fx[x];
        }
        bool bad = false;
#pragma unroll
        for (int x = 0; x < 2 * NS; ++x) bad |= !isfinite(Xn[x]);
        if (half_any(bad) && act) {
          status = NMC_STATUS_NONFINITE;
          fatal = true;
          act = run = false;
        }
        // Algorithm innerConverged (weighted per species, reference guarded
        // by the new norm), compared squared
        {
          // the sums are spread over the half (lane class c holds species c,
          // spread_conv_sums); the half has converged when every lane passes
          double vm[2][NS], vn[NS];
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            const double dd = Xn[t] - D[t], di = Xn[NS + t] - I[t];
            vm[0][t] = w2q * dd * dd;
            vm[1][t] = w2q * di * di;
            vn[t] = w2q * Xn[t] * Xn[t];
          }
          double dm2[1], dn2;
          spread_conv_sums<NS, 2>(vm, vn, dm2, dn2);
          const double dref2 = dref0 > dn2 ? dref0 : dn2;
          const bool conv = !half_any(!(dm2[0] <= a.tol_inner2 * dref2));
          // ||D^[k,*]|| is the reference of the next inner loop
          dref = (act && conv) ? dn2 : dref;
          if (act) {
#pragma unroll
            for (int t = 0; t < NS; ++t) {
              D[t] = Xn[t];
              I[t] = Xn[NS + t];
            }
            if (conv) {
              cvd = true;
              act = false;
            }
          }
        }
      }
      if (ran) total_inner += l_done;
      if (run && !cvd) inner_failed = true;
      // the sums of the matter right-hand side (Eq. implicitFluidNodal at
      // v = 0) and, where a running point's inner loop failed, the reference
      // norms of its next inner loop (the norm of the current moments) in one
      // reduction.  A converged loop took its reference from the convergence
      // test's norm of the same moments (the same sum in another fixed order).
      double yq0, yq1;
      {
        const double w3 = mt.w3[q];
        double m0 = 0.0, m1 = 0.0;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const double dd = D[t] - Dst[t];
          m0 += md->ig[t] * w2q * dd;
          m1 += md->imult[t] * w3 * dd;
        }
        if (__builtin_amdgcn_ballot_w64(run && !cvd) != 0) {
          constexpr int KR = (NS + 3) / 2;
          double v[2 * KR], s[2 * KR];
#pragma unroll
          for (int t = 0; t < NS; ++t) v[t] = w2q * D[t] * D[t];
          v[NS] = m0;
          v[NS + 1] = m1;
#pragma unroll
          for (int t = NS + 2; t < 2 * KR; ++t) v[t] = 0.0;
          half_own_sums<KR>(v, s);
          dref = (run && !cvd) ? class_pick<NS>(s, cls) : dref;
          yq0 = pt.ye_st - pt.K * s[NS];
          yq1 = pt.e_st - pt.K * s[NS + 1];
        } else {
          double v[2] = {m0, m1}, s[2];
          half_own_sums<1>(v, s);
          yq0 = pt.ye_st - pt.K * s[0];
          yq1 = pt.e_st - pt.K * s[1];
        }
      }
      if (a.prm.fixed_matter) {
        if (run) outer_conv = true;
        run = false;
      }
      if (run) {
        const double f0 = yq0 - pt.y[0], f1 = yq1 - pt.y[1];
        const int omem = k < a.prm.m_outer ? k : a.prm.m_outer;
        double yn0, yn1;
        if (omem == 1) {
          yn0 = yq0;
          yn1 = yq1;
        } else {
          const double dq20 = yq0 - pt.oq[0], dq21 = yq1 - pt.oq[1];
          const double df20 = f0 - pt.of[0], df21 = f1 - pt.of[1];
          const double odf0 = pt.odf[0], odf1 = pt.odf[1];
          const double G22 = df20 * df20 + df21 * df21, b2 = df20 * f0 + df21 * f1;
          const double G11o = odf0 * odf0 + odf1 * odf1;
          const double G12 = odf0 * df20 + odf1 * df21, b1 = odf0 * f0 + odf1 * f1;
          double g1, g2;
          anderson2(omem == 3, G11o, G12, G22, b1, b2, g1, g2);
          yn0 = yq0 - g2 * dq20 - g1 * pt.odq[0];
          yn1 = yq1 - g2 * dq21 - g1 * pt.odq[1];
          pt.odq[0] = dq20;
          pt.odq[1] = dq21;
          pt.odf[0] = df20;
          pt.odf[1] = df21;
        }
        pt.oq[0] = yq0;
        pt.oq[1] = yq1;
        pt.of[0] = f0;
        pt.of[1] = f1;
        if (!isfinite(yn0) || !isfinite(yn1)) {
          status = NMC_STATUS_NONFINITE;
          fatal = true;
          run = false;
        } else {
          // Algorithm outerConverged: componentwise against y*
          const bool oc = fabs(yn0 - pt.y[0]) <= a.prm.tol_outer * fabs(pt.ye_st) &&
                          fabs(yn1 - pt.y[1]) <= a.prm.tol_outer * fabs(pt.e_st);
          pt.y[0] = yn0;
          pt.y[1] = yn1;
          if (oc) {
            outer_conv = true;
            run = false;
          }
        }
      }
    }
    if (!skip && !fatal) {
      if (!outer_conv) status = NMC_STATUS_MAX_OUTER;
      else if (inner_failed) status = NMC_STATUS_MAX_INNER;
    }

    // ---- outputs --------------------------------------------------------
    const double ye_st = pt.ye_st, e_st = pt.e_st;
    double ye_out = ye_st, e_out = e_st, T_out = T_last;
    {
      const double w2 = mt.w2[q0], w3 = mt.w3[q0];
      double mv[2] = {0.0, 0.0}, s[2];
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const double dd = D[t] - Dst[t];
        mv[0] += md->ig[t] * w2 * dd;
        mv[1] += md->imult[t] * w3 * dd;
      }
      half_own_sums<1>(mv, s);
      if (skip) {
        T_out = fixedT ? pt.T_fix : (e_st - md->eos_b * ye43(ye_st) * pt.r3) / (md->eos_a * (1.0 + ye_st));
      } else if (!a.prm.fixed_matter) {
        ye_out = ye_st - pt.K * s[0];
        e_out = e_st - pt.K * s[1];
        T_out = (e_out - md->eos_b * ye43(ye_out) * pt.r3) / (md->eos_a * (1.0 + ye_out));
      } else if (status == NMC_STATUS_EOS_DOMAIN) {
        T_out = fixedT ? pt.T_fix : (e_st - md->eos_b * ye43(ye_st) * pt.r3) / (md->eos_a * (1.0 + ye_st));
      }
    }
    if (has_point) {
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int64_t o = base + md->ext[t] * NQ + q0;
        a.D[o] = D[t];
        a.I[o] = I[t];
      }
      if (q0 == 0) {
        a.ye[p] = ye_out;
        a.e[p] = e_out;
        a.T[p] = T_out;
        a.n_outer[p] = skip ? 0 : k_done;
        a.n_inner[p] = total_inner;
        a.status[p] = status;
      }
    }
    __syncthreads();
  }
};

template <int NS, bool COUPLED, bool PROJ>
__global__ __launch_bounds__(kLanes, 2) void fwd_pair_kernel(FwdArgs a) {
  __shared__ PairLds<NS> S;
  load_model(a.mdl, a.theta, S.m);
  const int64_t pairs = (a.P + 1) / 2;
  if (a.queue) {
    WorkQueue wq(a.queue, pairs, a.chunk);
    for (int64_t g; (g = wq.next()) >= 0;) {
      const int64_t b0 = uniform64(g * a.chunk);
      const int64_t end = uniform64(b0 + a.chunk < pairs ? b0 + a.chunk : pairs);
      for (int64_t u = b0; u < end; ++u) PairSolver<NS, COUPLED, PROJ>::solve(a, u, S, [&] { wq.settle(); });
    }
  } else {
    const int64_t b0 = (int64_t)blockIdx.x * a.chunk;
    const int64_t end = b0 + a.chunk < pairs ? b0 + a.chunk : pairs;
    for (int64_t u = b0; u < end; ++u) PairSolver<NS, COUPLED, PROJ>::solve(a, u, S, [] {});
  }
}

template <int NS, bool COUPLED, bool PROJ>
hipError_t launch_pair_t(const FwdArgs& a, const nmc_launch& L, int num_cu, hipStream_t s) {
  auto kern = fwd_pair_kernel<NS, COUPLED, PROJ>;
  const int64_t pairs = (a.P + 1) / 2;
  const int64_t need = (pairs + a.chunk - 1) / a.chunk;
  int64_t grid;
  if (a.queue) {
    int bpc = L.blocks_per_cu;
    if (bpc <= 0) {
      static int occ = 0;
      if (occ <= 0) {
        int o = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, kern, kLanes, 0) != hipSuccess || o <= 0) o = 8;
        // the query under-reports resident one-wave work-groups; a surplus is
        // harmless (late work-groups find the queue drained and exit)
        occ = o < 16 ? 16 : o;
      }
      bpc = occ;
    }
    grid = (int64_t)bpc * num_cu;
    if (grid > need) grid = need;
  } else {
    grid = need;
  }
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kLanes), 0, s, a);
  return hipGetLastError();
}

template <bool PROJ>
hipError_t launch_pair_p(const FwdArgs& a, int ns, bool coupled, const nmc_launch& L, int num_cu, hipStream_t s) {
  if (coupled) {
    switch (ns) {
      case 1: return launch_pair_t<1, true, PROJ>(a, L, num_cu, s);
      case 2: return launch_pair_t<2, true, PROJ>(a, L, num_cu, s);
      case 3: return launch_pair_t<3, true, PROJ>(a, L, num_cu, s);
    }
  } else {
    switch (ns) {
      case 1: return launch_pair_t<1, false, PROJ>(a, L, num_cu, s);
      case 2: return launch_pair_t<2, false, PROJ>(a, L, num_cu, s);
      case 3: return launch_pair_t<3, false, PROJ>(a, L, num_cu, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_forward_pair(const FwdArgs& a, int ns, bool coupled, bool proj, const nmc_launch& L, int num_cu,
                               hipStream_t s) {
  return proj ? launch_pair_p<true>(a, ns, coupled, L, num_cu, s) : launch_pair_p<false>(a, ns, coupled, L, num_cu, s);
}

}  // namespace nmc
