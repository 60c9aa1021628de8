// Forward kernels of the implicit neutrino-matter coupling solve on CDNA4,
// 32 energy nodes, one point per wavefront (kernel_store WAVE, REGEN,
// REGISTERS; the default is the two-points-per-wave kernel of
// nmc_forward_pair.hip, dispatched from launch_forward below).
//
// One 64-lane wavefront solves one spatial point at a time (Algorithm
// neutrinoMatterCoupling, Sec. 3.5.3); spatial points are independent because
// the nodal DG collocation decouples them (Sec. 3.1.2).
//
// Lane layout: lane = 32 h + q.
//   h = 0 ("number lanes"): own the number moments D_s[q] of every species;
//   h = 1 ("flux lanes"):   own the flux moments I_s[q].
// Both halves of row q cooperate on the energy-coupling rates of node q
// (Eqs. nesRatesNodal, pairRatesNodal), in one of three modes (KM):
//   KM = 2 (WAVE) / 1 (REGEN): the two halves take columns 0..15 / 16..31 of the
//     four kernel matrices, regenerate the entries from per-node exponent
//     splits (KM = 2 keeps the lane's pair factors b in VGPRs across the inner
//     loop) without their common factor A e_q e_j, contract them against
//     W e D and W e (1 - D) broadcast from LDS and scale the row sums by
//     A e_q; the half sums combine with v_permlane32_swap.
//   KM = 0: number lanes hold rows q of Phi_in and Phi_ann, flux lanes rows q
//     of Phi_out and Phi_pro in VGPRs (assembled once per outer iteration in
//     an LDS tile); the moment vectors are replicated per 16-lane DPP row with
//     v_permlane16_swap and broadcast into v_fmac_f64_dpp row_newbcast FMAs.
// Anderson inner products and weighted norms are register reductions; the
// Anderson history and the per-point uniform state live in LDS.
#include "nmc_regen.h"

namespace nmc {
namespace {

// Per-wave LDS scratch of the point solver: per-lane arrays, reduction
// staging, and the uniform per-point state of the outer (matter) loop, kept
// here so that it does not occupy VGPRs across the inner loop.
template <int NS, int KM>
struct WaveLds {
  ModelLds m;
  double mst[KM == 0 ? NS : 1][kLanes];  // owned moment of the old state (D* or I*); in VGPRs when KM >= 1
  double base[NS][kLanes];  // D* + dtau chi^EmAb D_eq (number lanes) or I* (flux lanes)
  double den0[NS][kLanes];  // 1 + dtau chi^EmAb (number lanes) or 1 + dtau (chi^EmAb + sigma^Iso)
  union {
    struct {
      double hist[4][NS][kLanes];                     // Anderson history: Q_prev, F_prev, dQ_old, dF_old
      double red[KM == 0 ? 2 * NS * kLanes : 1];      // reduction staging (KM = 0)
      double redout[KM == 0 ? 16 : 1];
    } it;                                             // live during an inner loop
    double tile[KM == 0 ? 32 * kTileStride : 1];      // kernel-row assembly (KM = 0), live while building
  } u;
  SplitExp E;                  // per-node factors of the current temperature
  alignas(16) double X[KM >= 1 ? NS : 1][32];  // W e D of the current iterate (KM >= 1)
  alignas(16) double Y[KM >= 1 ? NS : 1][32];  // W e (1 - D) of the current iterate (KM >= 1)
  // uniform per-point state
  double dref[NS];                      // ||D_s^[k,1]||_W^2 of the current inner loop
  double y[2];                          // matter iterate (Ye, e)
  double oq[2], of[2], odq[2], odf[2];  // outer Anderson history
  double T_last, r3, K, An, Ap;
  // per-point inputs read in every outer iteration, staged once per point
  double ye_st, e_st, chi0, T_fix, mu_fix;
};

// KM = 0: kernel rows built once per outer iteration and held in VGPRs,
// contracted with DPP broadcasts.  KM = 1: kernel entries regenerated in
// every inner iteration from the per-node exponent splits, the two lane
// halves taking columns 0..15 and 16..31 of the same rows.  KM = 2: as KM = 1,
// with the lane's 16 factors b computed once per outer iteration and kept in
// VGPRs (the default).
template <int NS, int NQ, bool COUPLED, int KM>
struct PointSolver {
  static_assert(NQ == 32, "lane layout is for 32 energy nodes");

  // KM = 1 / 2: rates of row q over columns j0 .. j0 + 15 (partial sums)
  __device__ __forceinline__ static void regen_rates(const WaveLds<NS, KM>& S, int q, int j0,
                                                     const double (&Bq)[KM == 2 ? 16 : 1], double (&eta)[NS],
                                                     double (&chi)[NS]) {
    regen_rates_half<NS, KM>(S, q, j0, Bq, eta, chi);
  }

  // Energy-coupling contraction: a1[t] = sum_j M1[j] X_t[j], a2[t] = sum_j M2[j] X_t[j]
  // where X_t = W D_t on number lanes and W (1 - D_t) on flux lanes.  Column
  // j of the vector lives in lane (j mod 16) of every 16-lane row of
  // XR[t][j / 16]; v_fmac_f64_dpp with row_newbcast broadcasts it into the
  // FMA, so no separate move is issued.
  __device__ __forceinline__ static void contract(const double (&M1)[NQ], const double (&M2)[NQ],
                                                  const double (&XR)[NS][2], double (&a1)[NS], double (&a2)[NS]) {
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      a1[t] = 0.0;
      a2[t] = 0.0;
    }
    asm volatile("s_nop 4" ::);  // DPP after a possible EXEC write
    static_for<0, NQ / 4>([&](auto bb) {
      constexpr int B = decltype(bb)::value, C = (4 * B) / 16, L0 = (4 * B) % 16, j = 4 * B;
      double x[NS];
#pragma unroll
      for (int t = 0; t < NS; ++t) x[t] = XR[t][C];
      Fmac4<NS>::template run<L0>(a1, a2, x, M1[j], M1[j + 1], M1[j + 2], M1[j + 3], M2[j], M2[j + 1], M2[j + 2],
                                  M2[j + 3]);
    });
  }

  // per-half sums (lanes 0..31, lanes 32..63) of V lane values, every lane
  // gets both: through LDS (KM = 0) or register permutations (KM = 1)
  template <int V>
  __device__ __forceinline__ static void hsum(const double (&v)[V], double (&s0)[V], double (&s1)[V],
                                              WaveLds<NS, KM>& S) {
    if constexpr (KM == 0) {
      half_sums<V>(v, s0, s1, S.u.it.red, S.u.it.redout);
    } else {
      constexpr int K = (V + 1) / 2;
      double w[2 * K], a0[2 * K], a1[2 * K];
#pragma unroll
      for (int i = 0; i < 2 * K; ++i) w[i] = i < V ? v[i < V ? i : 0] : 0.0;
      half_sums_reg<K>(w, a0, a1);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        s0[i] = a0[i];
        s1[i] = a1[i];
      }
    }
  }

  // Kernel rows at temperature T, assembled in the LDS tile three times:
  // Phi_in (number lanes load row q, flux lanes column q = row q of
  // Phi_out), Phi_ann (number lanes load row q), Phi_pro (flux lanes load
  // row q).
  __device__ __forceinline__ static void build_rows(int h, int q, double invT, double An, double Ap, WaveLds<NS, KM>& S,
                                                    double (&M1)[NQ], double (&M2)[NQ]) {
    constexpr int ST = kTileStride;
    double* T0 = S.u.tile;
    split_exp_prepare(S.m, invT, S.E);
    fill_tile<kTilePhiIn>(S.m, S.E, An, h, q, T0);
    __syncthreads();
    {
      const int step = h ? ST : 1;
      const double* p = T0 + (h ? q : q * ST);
#pragma unroll
      for (int j = 0; j < NQ; ++j) M1[j] = p[j * step];
    }
    __syncthreads();
    fill_tile<kTilePhiAnn>(S.m, S.E, Ap, h, q, T0);
    __syncthreads();
    if (h == 0) {
      const double* p = T0 + q * ST;
#pragma unroll
      for (int j = 0; j < NQ; ++j) M2[j] = p[j];
    }
    __syncthreads();
    fill_tile<kTilePhiPro>(S.m, S.E, Ap, h, q, T0);
    __syncthreads();
    if (h != 0) {
      const double* p = T0 + q * ST;
#pragma unroll
      for (int j = 0; j < NQ; ++j) M2[j] = p[j];
    }
    __syncthreads();
  }

  // settle() is called once the point's inputs are loaded (work-queue hook)
  template <class Settle>
  __device__ static void solve(const FwdArgs& a, int64_t p, WaveLds<NS, KM>& S, Settle&& settle) {
    const_ptr<DevModel> md = scalar_ptr(a.mdl);
    const ModelLds& mt = S.m;
    const int lane = threadIdx.x;
    const int h0 = lane >> 5;  // 0: number lanes, 1: flux lanes
    const int q0 = lane & 31;
    const int h = h0, q = q0;
    const double dtau = a.dtau;
    const int64_t base = p * (int64_t)(NS * NQ);

    const double rho = a.rho11[p];
    const bool fixedT = a.prm.fixed_matter && a.T_fixed;

    // the moment a lane owns: D* on number lanes, I* on flux lanes; D* on
    // every lane (flux lanes form W (1 - D) from it)
    // (both loads in every lane: the two lanes of node q read the same
    // elements, so the wave still fetches each line once, and no load waits
    // behind a branch)
    double M[NS], Dcur[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int64_t o = base + md->ext[t] * NQ + q;
      const double dv = a.D0[o], iv = a.I0[o];
      Dcur[t] = dv;
      M[t] = h ? iv : dv;
    }

    settle();
    if (rho < md->rho11_min) {
      // coupling disabled at low density (Sec. 7.2): pass the state through
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        if (h == 0) a.D[base + md->ext[t] * NQ + q] = M[t];
        else a.I[base + md->ext[t] * NQ + q] = M[t];
      }
      if (lane == 0) {
        const double ye_st = a.ye0[p], e_st = a.e0[p];
        a.ye[p] = ye_st;
        a.e[p] = e_st;
        a.T[p] = fixedT ? a.T_fixed[p]
                        : (e_st - md->eos_b * ye43(ye_st) * cbrt(rho)) / (md->eos_a * (1.0 + ye_st));
        a.n_outer[p] = 0;
        a.n_inner[p] = 0;
        a.status[p] = NMC_STATUS_OK;
      }
      return;
    }
    double MstR[KM >= 1 ? NS : 1];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      if constexpr (KM == 0) S.mst[t][lane] = M[t];
      else MstR[t] = M[t];
    }
    auto mst = [&](int t) -> double {
      if constexpr (KM == 0) return S.mst[t][lane];
      else return MstR[t];
    };

    // point constants: rho^(1/3), coupling K, kernel amplitudes
    S.r3 = cbrt(rho);
    S.K = md->kcoup / rho;
    S.An = (md->flags & NMC_NES) ? mt.theta[NQ] * rho : 0.0;
    S.Ap = (md->flags & NMC_PAIR) ? mt.theta[NQ + 1] * rho : 0.0;

    // ||D_s||_W^2 of the initial moments (reference of the first inner loop)
    {
      const double w2q = mt.w2[q];
      double v[NS], s0[NS], s1[NS];
#pragma unroll
      for (int t = 0; t < NS; ++t) v[t] = h ? 0.0 : w2q * Dcur[t] * Dcur[t];
      hsum<NS>(v, s0, s1, S);
#pragma unroll
      for (int t = 0; t < NS; ++t) S.dref[t] = s0[t];
    }
    S.ye_st = S.y[0] = a.ye0[p];
    S.e_st = S.y[1] = a.e0[p];
    S.chi0 = a.chi0 ? a.chi0[p] : md->chi_ref * rho;
    if (fixedT) S.T_fix = a.T_fixed[p];
    if (a.prm.fixed_matter && a.mu_fixed) S.mu_fix = a.mu_fixed[p];
#pragma unroll
    for (int i = 0; i < 2; ++i) S.oq[i] = S.of[i] = S.odq[i] = S.odf[i] = 0.0;
    S.T_last = 0.0;

    int status = NMC_STATUS_OK;
    bool fatal = false, inner_failed = false, outer_conv = false;
    int k, total_inner = 0;

    double M1[KM == 0 ? NQ : 1], M2[KM == 0 ? NQ : 1];
    for (k = 1; k <= a.prm.max_outer; ++k) {
      // per-iteration opaque copies keep lane invariants from being hoisted
      // out of this loop (and spilled)
      const_ptr<DevModel> md = scalar_ptr(a.mdl);
      const int q = opaque(q0), h = opaque(h0);
      // ---- ComputeOpacities(y^[k]) --------------------------------------
      const double r3 = S.r3;
      const double y0 = S.y[0], y1 = S.y[1];
      const double T = fixedT ? S.T_fix : (y1 - md->eos_b * ye43(y0) * r3) / (md->eos_a * (1.0 + y0));
      const double mu = (a.prm.fixed_matter && a.mu_fixed)
                            ? S.mu_fix
                            : md->mu_a * (y0 - md->mu_ye0) * r3 + md->mu_b * log(T / md->mu_t0);
      if (!(T > 0.0) || !(y0 >= 0.0) || !isfinite(T) || !isfinite(mu)) {
        status = NMC_STATUS_EOS_DOMAIN;
        fatal = true;
        break;
      }
      S.T_last = T;
      const double invT = 1.0 / T;

      // Eq. emissivityEmAbNodal with the nodal Fermi-Dirac equilibrium: the
      // number lanes need chi^EmAb D_eq and chi^EmAb, the flux lanes
      // chi^EmAb + sigma^Iso (transport opacity, Eq. transportOpacityNodal).
      // chi^EmAb = theta_q chi0 shape_q (electron flavours), sigma^Iso =
      // sigma_ratio chi0 shape_q.  Stored as the constant parts of the
      // numerator and denominator of Q.
      {
        const double chi0 = S.chi0;
        const double shape = chi0 * mt.shape[q];
        const double sig = (md->flags & NMC_ISO) ? md->sigma_ratio * shape : 0.0;
        const double emab_q = (md->flags & NMC_EMAB) ? mt.theta[q] * shape : 0.0;
        const double epsq = mt.eps[q];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const double chia = md->iemab[t] * emab_q;
          const double x = (epsq - md->imusign[t] * mu) * invT;
          const double ex = exp(-fabs(x));
          const double r = rcp_nr(1.0 + ex);
          const double deq = x > 0.0 ? ex * r : r;
          S.base[t][lane] = h ? mst(t) : mst(t) + dtau * (chia * deq);
          S.den0[t][lane] = 1.0 + dtau * (h ? chia + sig : chia);
        }
      }

      // kernel rows in registers: number lanes Phi_in[q][:], Phi_ann[q][:];
      // flux lanes Phi_out[q][:], Phi_pro[q][:]
      double Bq[KM == 2 ? 16 : 1];
      if constexpr (COUPLED) {
        if constexpr (KM == 0) build_rows(h, q, invT, S.An, S.Ap, S, M1, M2);
        else split_exp_prepare(S.m, invT, S.E);
        if constexpr (KM == 2) {
          // b of this lane's 16 columns, kept in VGPRs for the inner loop
          const double Pq = S.E.P2[q], Rq = S.E.R2[q];
          const int nq = S.E.n2[q];
#pragma unroll
          for (int jj = 0; jj < 16; ++jj) {
            const int j = 16 * h + jj;
            const bool up = j > q;
            Bq[jj] = ldexp(up ? Pq * S.E.R2[j] : S.E.P2[j] * Rq, up ? nq - S.E.n2[j] : S.E.n2[j] - nq);
          }
        }
      }

      // ---- inner loop over moments at fixed matter (M^[k,1] = M^[k-1,*]) --
      const double w2q = mt.w2[q], w2eq = w2q * mt.eps[q];
      const double xa = h ? -w2q : w2q, xb = h ? w2q : 0.0;  // X = xa D + xb
      const double dth = h ? 0.0 : dtau;
      double G11 = 0.0;
      bool conv = false;
      int l;
      for (l = 1; l <= a.prm.max_inner; ++l) {
        // ComputeRates(M^[k,l])
        double eta_c[NS], chi_c[NS];
        if constexpr (COUPLED && KM >= 1) {
          if (h == 0) {
#pragma unroll
            for (int t = 0; t < NS; ++t) {
              S.X[t][q] = w2eq * Dcur[t];
              S.Y[t][q] = __builtin_fma(-w2eq, Dcur[t], w2eq);
            }
          }
          __syncthreads();
          double e_p[NS], c_p[NS];
          regen_rates(S, q, 16 * h, Bq, e_p, c_p);
          __syncthreads();
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            eta_c[t] = sum_halves(e_p[t]);
            chi_c[t] = sum_halves(c_p[t]);
          }
        } else if constexpr (COUPLED) {
          double XR[NS][2];
#pragma unroll
          for (int t = 0; t < NS; ++t) swap16(__builtin_fma(xa, Dcur[t], xb), XR[t][0], XR[t][1]);
          double a1[NS], a2[NS];
          contract(M1, M2, XR, a1, a2);
          // number lanes: a1 = eta^NES, a2 = Phi_ann W D (per partner);
          // flux lanes: a1 = Phi_out W (1 - D), a2 = eta^Pair (per partner)
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const double pa = a2[pair_partner<NS>(s)];
            const double u = h ? pa : a1[s];
            const double v = a1[s] + pa;
            eta_c[s] = sum_halves(u);  // eta^NES + eta^Pair
            chi_c[s] = sum_halves(v);  // chi^NES + chi^Pair
          }
        } else {
#pragma unroll
          for (int s = 0; s < NS; ++s) eta_c[s] = chi_c[s] = 0.0;
        }

        // moment right-hand side Q (Eq. implicitMomentsNodal, lambda = 1) and residual
        double Q[NS], F[NS];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const double num = __builtin_fma(dth, eta_c[t], S.base[t][lane]);
          const double den = __builtin_fma(dtau, chi_c[t], S.den0[t][lane]);
          Q[t] = num * rcp_nr(den);
          F[t] = Q[t] - M[t];
        }

        // Anderson step over the last min(l, M_inner) residuals, as two
        // difference columns (the older one weighted zero when absent)
        const int mem = l < a.prm.m_inner ? l : a.prm.m_inner;
        double Mnew[NS];
        if (mem == 1) {
          // clear the older difference column (weighted zero at the second
          // iterate), so that no stale LDS word enters that product
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            Mnew[t] = Q[t];
            S.u.it.hist[2][t][lane] = 0.0;
            S.u.it.hist[3][t][lane] = 0.0;
          }
        } else {
          const double use1 = (mem == 3) ? 1.0 : 0.0;
          double dQ2[NS], dF2[NS];
          double v4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            dQ2[t] = Q[t] - S.u.it.hist[0][t][lane];
            dF2[t] = F[t] - S.u.it.hist[1][t][lane];
            const double dF1 = use1 * S.u.it.hist[3][t][lane];
            v4[0] += dF1 * dF2[t];
            v4[1] += dF2[t] * dF2[t];
            v4[2] += dF1 * F[t];
            v4[3] += dF2[t] * F[t];
          }
          double gs[4];
          wave_sums4(v4, gs);
          const double G12 = gs[0], G22 = gs[1];
          const double b1 = gs[2], b2 = gs[3];
          double g1, g2;
          anderson2(mem == 3, G11, G12, G22, b1, b2, g1, g2);
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            Mnew[t] = Q[t] - g2 * dQ2[t] - g1 * S.u.it.hist[2][t][lane];
            S.u.it.hist[2][t][lane] = dQ2[t];
            S.u.it.hist[3][t][lane] = dF2[t];
          }
          G11 = G22;
        }
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          S.u.it.hist[0][t][lane] = Q[t];
          S.u.it.hist[1][t][lane] = F[t];
        }

        bool bad = false;
#pragma unroll
        for (int t = 0; t < NS; ++t) bad |= !isfinite(Mnew[t]);
        if (wave_any(bad)) {
          status = NMC_STATUS_NONFINITE;
          fatal = true;
          break;
        }

        // Algorithm innerConverged (weighted per species, reference guarded
        // by the new norm): sqrt(max(S_D, S_I)) <= tol max(||D^[k,1]||,
        // ||D^[k,l+1]||), compared squared
        {
          double v[2 * NS], s0[2 * NS], s1[2 * NS];
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            const double d = Mnew[t] - M[t];
            v[t] = w2q * d * d;
            v[NS + t] = h ? 0.0 : w2q * Mnew[t] * Mnew[t];
          }
          half_sums_reg<NS>(v, s0, s1);
          conv = true;
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            const double sd = s0[t], si = s1[t];
            const double dm2 = sd > si ? sd : si;
            const double dn2 = s0[NS + t];
            const double d0 = S.dref[t];
            const double dref2 = d0 > dn2 ? d0 : dn2;
            if (!(dm2 <= a.tol_inner2 * dref2)) conv = false;
          }
          if (conv) {
            // ||D^[k,*]|| is the reference of the next inner loop
#pragma unroll
            for (int t = 0; t < NS; ++t) S.dref[t] = s0[NS + t];
          }
        }
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          M[t] = Mnew[t];
          double f, s;
          swap32(M[t], f, s);  // number moments of lanes 0..31 to both halves
          Dcur[t] = f;
        }
        if (conv) break;
      }
      total_inner += (l > a.prm.max_inner ? a.prm.max_inner : l);
      if (fatal) break;
      if (!conv) {
        inner_failed = true;
        // reference for the next loop: the norm of the current moments
        double v[NS], s0[NS], s1[NS];
#pragma unroll
        for (int t = 0; t < NS; ++t) v[t] = h ? 0.0 : w2q * M[t] * M[t];
        hsum<NS>(v, s0, s1, S);
#pragma unroll
        for (int t = 0; t < NS; ++t) S.dref[t] = s0[t];
      }
      if (a.prm.fixed_matter) {
        outer_conv = true;
        break;
      }

      // ---- matter right-hand side (Eq. implicitFluidNodal at v = 0) -------
      double yq0, yq1;
      {
        const double w3 = mt.w3[q];
        double mv[2] = {0.0, 0.0}, s0[2], s1[2];
        if (h == 0) {
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            const double dd = M[t] - mst(t);
            mv[0] += md->ig[t] * w2q * dd;
            mv[1] += md->imult[t] * w3 * dd;
          }
        }
        hsum<2>(mv, s0, s1, S);
        yq0 = S.ye_st - S.K * s0[0];
        yq1 = S.e_st - S.K * s0[1];
      }
      const double f0 = yq0 - S.y[0], f1 = yq1 - S.y[1];

      // outer Anderson step on (Ye, e), same least-squares rule
      const int omem = k < a.prm.m_outer ? k : a.prm.m_outer;
      double yn0, yn1;
      if (omem == 1) {
        yn0 = yq0;
        yn1 = yq1;
      } else {
        const double dq20 = yq0 - S.oq[0], dq21 = yq1 - S.oq[1];
        const double df20 = f0 - S.of[0], df21 = f1 - S.of[1];
        const double odf0 = S.odf[0], odf1 = S.odf[1];
        const double G22 = df20 * df20 + df21 * df21, b2 = df20 * f0 + df21 * f1;
        const double G11o = odf0 * odf0 + odf1 * odf1;
        const double G12 = odf0 * df20 + odf1 * df21, b1 = odf0 * f0 + odf1 * f1;
        double g1, g2;
        anderson2(omem == 3, G11o, G12, G22, b1, b2, g1, g2);
        yn0 = yq0 - g2 * dq20 - g1 * S.odq[0];
        yn1 = yq1 - g2 * dq21 - g1 * S.odq[1];
        S.odq[0] = dq20;
        S.odq[1] = dq21;
        S.odf[0] = df20;
        S.odf[1] = df21;
      }
      S.oq[0] = yq0;
      S.oq[1] = yq1;
      S.of[0] = f0;
      S.of[1] = f1;
      if (!isfinite(yn0) || !isfinite(yn1)) {
        status = NMC_STATUS_NONFINITE;
        fatal = true;
        break;
      }
      // Algorithm outerConverged: componentwise against y*
      const bool oc = fabs(yn0 - S.y[0]) <= a.prm.tol_outer * fabs(S.ye_st) &&
                      fabs(yn1 - S.y[1]) <= a.prm.tol_outer * fabs(S.e_st);
      S.y[0] = yn0;
      S.y[1] = yn1;
      if (oc) {
        outer_conv = true;
        break;
      }
    }
    if (k > a.prm.max_outer) k = a.prm.max_outer;
    if (!fatal) {
      if (!outer_conv) status = NMC_STATUS_MAX_OUTER;
      else if (inner_failed) status = NMC_STATUS_MAX_INNER;
    }

    // ---- outputs --------------------------------------------------------
    const double ye_st = S.ye_st, e_st = S.e_st;
    double ye_out = ye_st, e_out = e_st, T_out = S.T_last;
    if (!a.prm.fixed_matter) {
      // final matter state from the final moments (exact lepton-number and
      // energy balance)
      const double w2 = mt.w2[q], w3 = mt.w3[q];
      double mv[2] = {0.0, 0.0}, s0[2], s1[2];
      if (h == 0) {
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const double dd = M[t] - mst(t);
          mv[0] += md->ig[t] * w2 * dd;
          mv[1] += md->imult[t] * w3 * dd;
        }
      }
      hsum<2>(mv, s0, s1, S);
      ye_out = ye_st - S.K * s0[0];
      e_out = e_st - S.K * s0[1];
      T_out = (e_out - md->eos_b * ye43(ye_out) * S.r3) / (md->eos_a * (1.0 + ye_out));
    } else if (status == NMC_STATUS_EOS_DOMAIN) {
      T_out = fixedT ? S.T_fix : (e_st - md->eos_b * ye43(ye_st) * S.r3) / (md->eos_a * (1.0 + ye_st));
    }
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      if (h == 0) a.D[base + md->ext[t] * NQ + q] = M[t];
      else a.I[base + md->ext[t] * NQ + q] = M[t];
    }
    if (lane == 0) {
      a.ye[p] = ye_out;
      a.e[p] = e_out;
      a.T[p] = T_out;
      a.n_outer[p] = k;
      a.n_inner[p] = total_inner;
      a.status[p] = status;
    }
  }
};

template <int NS, int NQ, bool COUPLED, int KM>
__global__ __launch_bounds__(kLanes, KM == 1 ? 3 : 2) void fwd_kernel(FwdArgs a) {
  __shared__ WaveLds<NS, KM> S;
  load_model(a.mdl, a.theta, S.m);
  if (a.queue) {
    WorkQueue wq(a.queue, a.P, a.chunk);
    for (int64_t g; (g = wq.next()) >= 0;) {
      const int64_t b0 = uniform64(g * a.chunk);
      const int64_t end = uniform64(b0 + a.chunk < a.P ? b0 + a.chunk : a.P);
      for (int64_t p = b0; p < end; ++p) PointSolver<NS, NQ, COUPLED, KM>::solve(a, p, S, [&] { wq.settle(); });
    }
  } else {
    const int64_t b0 = (int64_t)blockIdx.x * a.chunk;
    const int64_t end = b0 + a.chunk < a.P ? b0 + a.chunk : a.P;
    for (int64_t p = b0; p < end; ++p) PointSolver<NS, NQ, COUPLED, KM>::solve(a, p, S, [] {});
  }
}

__global__ void reset_counter_kernel(int* c) {
  if (threadIdx.x < kQueues) c[threadIdx.x * kQueueStride] = 0;
}

template <int NS, int NQ, bool COUPLED, int KM>
hipError_t launch_fwd_t(const FwdArgs& a, const nmc_launch& L, int num_cu, hipStream_t s) {
  auto kern = fwd_kernel<NS, NQ, COUPLED, KM>;
  int64_t grid;
  if (a.queue) {
    int bpc = L.blocks_per_cu;
    if (bpc <= 0) {
      // occupancy of this kernel variant, queried once per process
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
    const int64_t need = (a.P + a.chunk - 1) / a.chunk;
    if (grid > need) grid = need;
  } else {
    grid = (a.P + a.chunk - 1) / a.chunk;
  }
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kLanes), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_reset_counter(int* counter, hipStream_t s) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, counter);
  return hipGetLastError();
}

hipError_t launch_forward(const FwdArgs& a, int nq, int ns, bool coupled, bool proj, const nmc_launch& L,
                          int num_cu, hipStream_t s) {
  if (nq == 32) {
    if (L.kernel_store == NMC_KERNELS_ON_CHIP || L.kernel_store == NMC_KERNELS_PAIRED)
      return launch_forward_pair(a, ns, coupled, proj, L, num_cu, s);
    if (proj) return hipErrorInvalidValue;
    if (coupled && L.kernel_store == NMC_KERNELS_REGEN) {
      switch (ns) {
        case 1: return launch_fwd_t<1, 32, true, 1>(a, L, num_cu, s);
        case 2: return launch_fwd_t<2, 32, true, 1>(a, L, num_cu, s);
        case 3: return launch_fwd_t<3, 32, true, 1>(a, L, num_cu, s);
      }
    } else if (coupled && L.kernel_store != NMC_KERNELS_REGISTERS) {
      switch (ns) {
        case 1: return launch_fwd_t<1, 32, true, 2>(a, L, num_cu, s);
        case 2: return launch_fwd_t<2, 32, true, 2>(a, L, num_cu, s);
        case 3: return launch_fwd_t<3, 32, true, 2>(a, L, num_cu, s);
      }
    } else if (coupled) {
      switch (ns) {
        case 1: return launch_fwd_t<1, 32, true, 0>(a, L, num_cu, s);
        case 2: return launch_fwd_t<2, 32, true, 0>(a, L, num_cu, s);
        case 3: return launch_fwd_t<3, 32, true, 0>(a, L, num_cu, s);
      }
    } else {
      switch (ns) {
        case 1: return launch_fwd_t<1, 32, false, 0>(a, L, num_cu, s);
        case 2: return launch_fwd_t<2, 32, false, 0>(a, L, num_cu, s);
        case 3: return launch_fwd_t<3, 32, false, 0>(a, L, num_cu, s);
      }
    }
  }
  if (nq == 64 && !proj) return launch_forward64(a, ns, coupled, L, num_cu, s);
  return hipErrorInvalidValue;
}

}  // namespace nmc
