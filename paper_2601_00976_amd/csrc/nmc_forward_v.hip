// Forward kernel of the implicit neutrino-matter coupling solve with a
// nonzero fluid velocity (the O(v/c) two-moment model), 32 energy nodes, one
// point per wavefront.
//
// Moment equations: Eqs. implicitNumberNodal / implicitNumberFluxNodal with
// all velocity terms, iterated in the fixed-point form of Eq.
// implicitMomentsNodal with lambda = 1 / (1 + |v|); the flux equation is
// closed with the Minerbo Eddington tensor (Eqs. eddingtonFactorMinerbo,
// eddingtonTensor).  Matter: Eq. implicitFluidNodal with the Eulerian
// lepton number, energy and momentum of Eqs. eulerianNumberLG,
// eulerianEnergyLG, eulerianMomentumLG, y = (Ye, ef, v_1, v_2, v_3) with ef
// the specific fluid energy (internal plus kinetic) per baryon.  The
// collision rates depend on the number moments only and are computed as in
// the static one-point-per-wavefront kernel (entries regenerated from the
// per-node exponent splits, the lane's 16 pair factors kept in VGPRs).
//
// Lane layout: lane = 32 h + q.  Every node carries four moments per species
// (D, I_1, I_2, I_3); lane h = 0 owns (D, I_1) and lane h = 1 owns (I_2, I_3)
// of node q, so both halves carry the same Anderson work.  Two
// v_permlane32_swap per species give every lane the full moment vector of
// its node, which the closure and the velocity terms need.
#include "nmc_closure.h"
#include "nmc_regen.h"

namespace nmc {
namespace {

constexpr double kMuC2 = 931.49410242;  // atomic mass unit rest energy [MeV]

template <int NS, bool PHI1>
struct VLds {
  ModelLds m;
  double cst[NS][2][kLanes];      // owned moment of the old conserved state: N* or G*_j
  double base[NS][2][kLanes];     // lambda (N* + dtau chi^EmAb D_eq), or lambda G*_j
  double den0[NS][2][kLanes];     // 1 + lambda dtau chi^EmAb, or 1 + lambda dtau (chi^EmAb + sigma^Iso)
  double hist[4][NS][2][kLanes];  // Anderson history: Q_prev, F_prev, dQ_old, dF_old
  SplitExp E;                     // per-node factors of the current temperature
  alignas(16) double X[NS][32];   // W e D of the current iterate
  alignas(16) double Y[NS][32];   // W e (1 - D) of the current iterate
  alignas(16) double XI[PHI1 ? NS : 1][3][32];  // W e I_i of the current iterate (linear-order kernels)
  // uniform per-point state
  double dref[NS];
  double y[5];      // matter iterate (Ye, ef, v_1, v_2, v_3)
  double yst[5];    // old matter state y*
  double yused[5];  // matter iterate of the last inner loop
  double X0[5];     // Eulerian (N, E, F_1, F_2, F_3) of the old state
  double oq[5], of[5], odq[5], odf[5];  // outer Anderson history
  double T_last, r3, K, An, Ap, chi0;
};

// Linear-order kernel integrals of one kernel row over columns j0 .. j0 + 15
// (partial sums), flux component i: with the isotropic kernels' entries
// regenerated as in regen_rates_half (without their factor A e_q e_j),
//   Lin[s]  += Phi_in  W e I_s,i     Lout[s] += Phi_out W e I_s,i
//   Lpro[s] += Phi_pro W e I_sbar,i  Lann[s] += Phi_ann W e I_sbar,i
// (Eqs. linearCorrectionsNES, linearCorrectionsPair; Phi_1 = phi1 Phi_0, the
// fractions and A e_q are applied by the caller)
template <int NS, class L>
__device__ __forceinline__ void phi1_half(const L& S, int q, int j0, const double (&Bq)[16], int i,
                                          double (&Lin)[NS], double (&Lout)[NS], double (&Lpro)[NS],
                                          double (&Lann)[NS]) {
  const SplitExp& E = S.E;
  const double Gq = E.G[q];
#pragma unroll
  for (int t = 0; t < NS; ++t) Lin[t] = Lout[t] = Lpro[t] = Lann[t] = 0.0;
#pragma unroll 4
  for (int jj = 0; jj < 16; ++jj) {
    const int j = j0 + jj;
    const bool up = j > q;
    const double b = Bq[jj], b2 = b * b, b3 = b2 * b;
    const double fin = up ? b : b3, fout = up ? b3 : b;
    const double fann = b2, fpro = fmin(E.G[j], Gq);
    double x[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) x[t] = S.XI[t][i][j];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int tb = pair_partner<NS>(t);
      Lin[t] = __builtin_fma(fin, x[t], Lin[t]);
      Lout[t] = __builtin_fma(fout, x[t], Lout[t]);
      Lpro[t] = __builtin_fma(fpro, x[tb], Lpro[t]);
      Lann[t] = __builtin_fma(fann, x[tb], Lann[t]);
    }
  }
}

template <int NS, bool COUPLED, bool PHI1>
struct PointSolverV {
  static constexpr int NQ = 32;
  // the lane's 16 pair factors are kept in VGPRs across the inner loop (2);
  // recomputing them from the per-node splits in every inner iteration (1)
  // frees the registers the three-species kernel spills but measured slower
  static constexpr int KMV = 2;

  // lane contributions (number lanes only) to the Eulerian integrals
  // (N, E, F_1, F_2, F_3) of the moments (Df, If) at velocity v; per-half
  // sums, the number-lane half in s0
  __device__ __forceinline__ static void eulerian(const_ptr<DevModel> md, const ModelLds& mt, int h, int q,
                                                  const double (&Df)[NS], const double (&If)[NS][3],
                                                  const double (&v)[3], double (&X)[5]) {
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (h == 0) {
      const double w2 = mt.w2[q], w3 = mt.w3[q];
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        double vI, vK[3];
        closure_terms(Df[t], If[t], v, vI, vK);
        acc[0] += md->ig[t] * w2 * (Df[t] + vI);
        acc[1] += md->imult[t] * w3 * (Df[t] + 2.0 * vI);
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[2 + j] += md->imult[t] * w3 * (If[t][j] + v[j] * Df[t] + vK[j]);
      }
    }
    double s0[6], s1[6];
    half_sums_reg<3>(acc, s0, s1);
#pragma unroll
    for (int i = 0; i < 5; ++i) X[i] = s0[i];
  }

  // matter right-hand side q(M, y) (Eq. implicitFluidNodal)
  __device__ __forceinline__ static void matter_rhs(const VLds<NS, PHI1>& S, const double (&X)[5], double (&yq)[5]) {
    yq[0] = S.yst[0] - S.K * (X[0] - S.X0[0]);
    yq[1] = S.yst[1] - S.K * (X[1] - S.X0[1]);
    const double Kv = S.K * (1.0 / kMuC2);
#pragma unroll
    for (int j = 0; j < 3; ++j) yq[2 + j] = S.yst[2 + j] - Kv * (X[2 + j] - S.X0[2 + j]);
  }

  // temperature of the EOS at the internal energy ef - m_u c^2 |v|^2 / 2
  __device__ __forceinline__ static double temperature(const_ptr<DevModel> md, const double* y, double r3) {
    const double v2 = y[2] * y[2] + y[3] * y[3] + y[4] * y[4];
    const double e = y[1] - 0.5 * kMuC2 * v2;
    return (e - md->eos_b * ye43(y[0]) * r3) / (md->eos_a * (1.0 + y[0]));
  }

  // full moment vector of node q from the owned pairs: lanes h = 0 own
  // (D, I_1), lanes h = 1 own (I_2, I_3)
  __device__ __forceinline__ static void exchange(const double (&u)[NS][2], double (&Df)[NS], double (&If)[NS][3]) {
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      double a0, b0, a1, b1;
      swap32(u[t][0], a0, b0);
      swap32(u[t][1], a1, b1);
      Df[t] = a0;
      If[t][0] = a1;
      If[t][1] = b0;
      If[t][2] = b1;
    }
  }

  template <class Settle>
  __device__ static void solve(const FwdVArgs& a, int64_t p, VLds<NS, PHI1>& S, Settle&& settle) {
    const_ptr<DevModel> md = scalar_ptr(a.mdl);
    const ModelLds& mt = S.m;
    const int lane = threadIdx.x;
    const int h0 = lane >> 5, q0 = lane & 31;
    const int h = h0, q = q0;
    const double dtau = a.dtau;
    const int64_t baseD = p * (int64_t)(NS * NQ), baseI = p * (int64_t)(NS * 3 * NQ);
    const double rho = a.rho11[p];

    // the node's old moments (every lane loads all four of its node)
    double Df[NS], If[NS][3];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int ex = md->ext[t];
      Df[t] = a.D0[baseD + ex * NQ + q];
#pragma unroll
      for (int j = 0; j < 3; ++j) If[t][j] = a.I0[baseI + (ex * 3 + j) * NQ + q];
    }
    double yst[5];
    yst[0] = a.ye0[p];
    yst[1] = a.ef0[p];
#pragma unroll
    for (int j = 0; j < 3; ++j) yst[2 + j] = a.v0[3 * p + j];
    settle();

    // owned moments: slot c holds moment 2 h + c of (D, I_1, I_2, I_3)
    double u[NS][2];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      u[t][0] = h ? If[t][1] : Df[t];
      u[t][1] = h ? If[t][2] : If[t][0];
    }
    auto store_moments = [&](const double (&w)[NS][2]) {
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int ex = md->ext[t];
        if (h == 0) {
          a.D[baseD + ex * NQ + q] = w[t][0];
          a.I[baseI + (ex * 3 + 0) * NQ + q] = w[t][1];
        } else {
          a.I[baseI + (ex * 3 + 1) * NQ + q] = w[t][0];
          a.I[baseI + (ex * 3 + 2) * NQ + q] = w[t][1];
        }
      }
    };

    if (rho < md->rho11_min) {
      // coupling disabled at low density (Sec. 7.2): pass the state through
      store_moments(u);
      if (lane == 0) {
        a.ye[p] = yst[0];
        a.ef[p] = yst[1];
#pragma unroll
        for (int j = 0; j < 3; ++j) a.v[3 * p + j] = yst[2 + j];
        a.T[p] = temperature(md, yst, cbrt(rho));
        a.n_outer[p] = 0;
        a.n_inner[p] = 0;
        a.status[p] = NMC_STATUS_OK;
      }
      return;
    }

    S.r3 = cbrt(rho);
    S.K = md->kcoup / rho;
    S.An = (md->flags & NMC_NES) ? mt.theta[NQ] * rho : 0.0;
    S.Ap = (md->flags & NMC_PAIR) ? mt.theta[NQ + 1] * rho : 0.0;
    S.chi0 = a.chi0 ? a.chi0[p] : md->chi_ref * rho;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      S.yst[i] = S.y[i] = S.yused[i] = yst[i];
      S.oq[i] = S.of[i] = S.odq[i] = S.odf[i] = 0.0;
    }
    S.T_last = temperature(md, yst, S.r3);

    // old conserved moments N* = D* + v*.I*, G*_j = I*_j + v*^i K*_ij (Eq.
    // numberDensityEulerian and the left-hand sides of Eqs.
    // implicitNumberNodal, implicitNumberFluxNodal at the old state), and the
    // old Eulerian integrals
    {
      const double vs[3] = {yst[2], yst[3], yst[4]};
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        double vI, vK[3];
        closure_terms(Df[t], If[t], vs, vI, vK);
        const double Nst = Df[t] + vI;
        const double G0 = If[t][0] + vK[0], G1 = If[t][1] + vK[1], G2 = If[t][2] + vK[2];
        S.cst[t][0][lane] = h ? G1 : Nst;
        S.cst[t][1][lane] = h ? G2 : G0;
      }
      double X0[5];
      eulerian(md, mt, h, q, Df, If, vs, X0);
#pragma unroll
      for (int i = 0; i < 5; ++i) S.X0[i] = X0[i];
      // ||D_s||_W^2 of the initial moments
      const double w2q = mt.w2[q];
      double vv[2 * ((NS + 1) / 2)], s0[2 * ((NS + 1) / 2)], s1[2 * ((NS + 1) / 2)];
#pragma unroll
      for (int i = 0; i < 2 * ((NS + 1) / 2); ++i) vv[i] = (i < NS && h == 0) ? w2q * Df[i < NS ? i : 0] * Df[i < NS ? i : 0] : 0.0;
      half_sums_reg<(NS + 1) / 2>(vv, s0, s1);
#pragma unroll
      for (int t = 0; t < NS; ++t) S.dref[t] = s0[t];
    }

    int status = NMC_STATUS_OK;
    bool fatal = false, inner_failed = false, outer_conv = false;
    int k, total_inner = 0;
    for (k = 1; k <= a.prm.max_outer; ++k) {
      const_ptr<DevModel> md = scalar_ptr(a.mdl);
      const int q = opaque(q0), h = opaque(h0);
      // ---- ComputeOpacities(y^[k]) --------------------------------------
      const double v[3] = {S.y[2], S.y[3], S.y[4]};
      const double vmag = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      // step-size parameter of the fixed-point form
      const double lam = 1.0 / (1.0 + vmag);
      const double T = temperature(md, a.prm.fixed_matter ? S.yst : S.y, S.r3);
      const double y0 = S.y[0];
      const double mu = md->mu_a * (y0 - md->mu_ye0) * S.r3 + md->mu_b * log(T / md->mu_t0);
      if (!(T > 0.0) || !(y0 >= 0.0) || !isfinite(T) || !isfinite(mu)) {
        status = NMC_STATUS_EOS_DOMAIN;
        fatal = true;
        break;
      }
      S.T_last = T;
#pragma unroll
      for (int i = 0; i < 5; ++i) S.yused[i] = S.y[i];
      const double invT = 1.0 / T;
      {
        const double shape = S.chi0 * mt.shape[q];
        const double sig = (md->flags & NMC_ISO) ? md->sigma_ratio * shape : 0.0;
        const double emab_q = (md->flags & NMC_EMAB) ? mt.theta[q] * shape : 0.0;
        const double epsq = mt.eps[q];
        const double ldt = lam * dtau;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const double chia = md->iemab[t] * emab_q;
          const double x = (epsq - md->imusign[t] * mu) * invT;
          const double ex = exp(-fabs(x));
          const double r = rcp_nr(1.0 + ex);
          const double deq = x > 0.0 ? ex * r : r;
          // slot 0: D (h = 0) or I_2 (h = 1); slot 1: I_1 or I_3
          S.base[t][0][lane] = h ? lam * S.cst[t][0][lane] : lam * (S.cst[t][0][lane] + dtau * (chia * deq));
          S.den0[t][0][lane] = 1.0 + ldt * (h ? chia + sig : chia);
          S.base[t][1][lane] = lam * S.cst[t][1][lane];
          S.den0[t][1][lane] = 1.0 + ldt * (chia + sig);
        }
      }
      double Bq[KMV == 2 ? 16 : 1];
      if constexpr (COUPLED) split_exp_prepare(S.m, invT, S.E);
      if constexpr (COUPLED && KMV == 2) {
        const double Pq = S.E.P2[q], Rq = S.E.R2[q];
        const int nq = S.E.n2[q];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
          const int j = 16 * h + jj;
          const bool up = j > q;
          Bq[jj] = ldexp(up ? Pq * S.E.R2[j] : S.E.P2[j] * Rq, up ? nq - S.E.n2[j] : S.E.n2[j] - nq);
        }
      }

      // ---- inner loop over moments at fixed matter (M^[k,1] = M^[k-1,*]) --
      const double w2q = mt.w2[q], w2eq = w2q * mt.eps[q];
      const double oml = 1.0 - lam, ldt = lam * dtau;
      // velocity component and flux-direction index of each owned flux slot
      double G11 = 0.0;
      bool conv = false;
      int l;
      for (l = 1; l <= a.prm.max_inner; ++l) {
        double eta_c[NS], chi_c[NS];
        if constexpr (COUPLED) {
          if (h == 0) {
#pragma unroll
            for (int t = 0; t < NS; ++t) {
              S.X[t][q] = w2eq * Df[t];
              S.Y[t][q] = __builtin_fma(-w2eq, Df[t], w2eq);
            }
          }
          __syncthreads();
          double e_p[NS], c_p[NS];
          regen_rates_half<NS, KMV>(S, q, 16 * h, Bq, e_p, c_p);
          __syncthreads();
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            eta_c[t] = sum_halves(e_p[t]);
            chi_c[t] = sum_halves(c_p[t]);
          }
        } else {
#pragma unroll
          for (int t = 0; t < NS; ++t) eta_c[t] = chi_c[t] = 0.0;
        }

        // linear-order corrections at the current iterate, added to the
        // right-hand sides like the emissivity: c_own[t][c] for the owned
        // moment c of species t (number equation, or flux component)
        double c_own[NS][2];
#pragma unroll
        for (int t = 0; t < NS; ++t) c_own[t][0] = c_own[t][1] = 0.0;
        if constexpr (PHI1) {
          if (h == 0) {
#pragma unroll
            for (int t = 0; t < NS; ++t)
#pragma unroll
              for (int i = 0; i < 3; ++i) S.XI[t][i][q] = w2eq * If[t][i];
          }
          __syncthreads();
          const double rN = md->phi1_nes * S.An * mt.eps[q], rP = md->phi1_pair * S.Ap * mt.eps[q];
          double P[NS][3], R[NS][3];
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            double Lin[NS], Lout[NS], Lpro[NS], Lann[NS];
            phi1_half<NS>(S, q, 16 * h, Bq, i, Lin, Lout, Lpro, Lann);
#pragma unroll
            for (int t = 0; t < NS; ++t) {
              P[t][i] = sum_halves(__builtin_fma(rN, Lin[t], -rP * Lpro[t]));
              R[t][i] = sum_halves(__builtin_fma(rN, Lout[t], -rP * Lann[t]));
            }
          }
          __syncthreads();
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            double c0, c1[3];
            phi1_collision(Df[t], If[t], P[t], R[t], c0, c1);
            c_own[t][0] = h ? c1[1] : c0;
            c_own[t][1] = h ? c1[2] : c1[0];
          }
        }

        // moment right-hand side Q (Eq. implicitMomentsNodal) and residual:
        // Q_D = ((1 - lam) D - lam v.I + lam (N* + dtau (eta + c))) / (1 + lam dtau chi),
        // Q_Ij = ((1 - lam) I_j - lam v^i K_ij + lam (G*_j + dtau c_j)) / (1 + lam dtau kappa)
        double Q[NS][2], F[NS][2];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          double vI, vK[3];
          closure_terms(Df[t], If[t], v, vI, vK);
          const double V0 = h ? vK[1] : vI, V1 = h ? vK[2] : vK[0];
          const double ex0 = h ? 0.0 : ldt * eta_c[t];
          double n0 = __builtin_fma(oml, u[t][0], S.base[t][0][lane]) - lam * V0 + ex0;
          double n1 = __builtin_fma(oml, u[t][1], S.base[t][1][lane]) - lam * V1;
          if constexpr (PHI1) {
            n0 = __builtin_fma(ldt, c_own[t][0], n0);
            n1 = __builtin_fma(ldt, c_own[t][1], n1);
          }
          const double d0 = __builtin_fma(ldt, chi_c[t], S.den0[t][0][lane]);
          const double d1 = __builtin_fma(ldt, chi_c[t], S.den0[t][1][lane]);
          Q[t][0] = n0 * rcp_nr(d0);
          Q[t][1] = n1 * rcp_nr(d1);
          F[t][0] = Q[t][0] - u[t][0];
          F[t][1] = Q[t][1] - u[t][1];
        }

        // Anderson step over the last min(l, M_inner) residuals (two
        // difference columns, the older one weighted zero when absent)
        const int mem = l < a.prm.m_inner ? l : a.prm.m_inner;
        double Mn[NS][2];
        if (mem == 1) {
          // clear the older difference column (weighted zero at the second
          // iterate), so that no stale LDS word enters that product
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            Mn[t][0] = Q[t][0];
            Mn[t][1] = Q[t][1];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              S.hist[2][t][c][lane] = 0.0;
              S.hist[3][t][c][lane] = 0.0;
            }
          }
        } else {
          const double use1 = (mem == 3) ? 1.0 : 0.0;
          double dQ2[NS][2], dF2[NS][2];
          double v4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int t = 0; t < NS; ++t)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              dQ2[t][c] = Q[t][c] - S.hist[0][t][c][lane];
              dF2[t][c] = F[t][c] - S.hist[1][t][c][lane];
              const double dF1 = use1 * S.hist[3][t][c][lane];
              v4[0] += dF1 * dF2[t][c];
              v4[1] += dF2[t][c] * dF2[t][c];
              v4[2] += dF1 * F[t][c];
              v4[3] += dF2[t][c] * F[t][c];
            }
          double gs[4];
          wave_sums4(v4, gs);
          double g1, g2;
          anderson2(mem == 3, G11, gs[0], gs[1], gs[2], gs[3], g1, g2);
#pragma unroll
          for (int t = 0; t < NS; ++t)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              Mn[t][c] = Q[t][c] - g2 * dQ2[t][c] - g1 * S.hist[2][t][c][lane];
              S.hist[2][t][c][lane] = dQ2[t][c];
              S.hist[3][t][c][lane] = dF2[t][c];
            }
          G11 = gs[1];
        }
#pragma unroll
        for (int t = 0; t < NS; ++t)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            S.hist[0][t][c][lane] = Q[t][c];
            S.hist[1][t][c][lane] = F[t][c];
          }

        bool bad = false;
#pragma unroll
        for (int t = 0; t < NS; ++t) bad |= !isfinite(Mn[t][0]) || !isfinite(Mn[t][1]);
        if (wave_any(bad)) {
          status = NMC_STATUS_NONFINITE;
          fatal = true;
          break;
        }

        // Algorithm innerConverged over the four moments of each species:
        // sqrt(max_m sum_q W dM_m^2) <= tol max(||D^[k,1]||, ||D^[k,l+1]||)
        {
          constexpr int KR = (3 * NS + 1) / 2;
          double vv[2 * KR], s0[2 * KR], s1[2 * KR];
#pragma unroll
          for (int i = 0; i < 2 * KR; ++i) vv[i] = 0.0;
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            const double d0 = Mn[t][0] - u[t][0], d1 = Mn[t][1] - u[t][1];
            vv[t] = w2q * d0 * d0;
            vv[NS + t] = w2q * d1 * d1;
            vv[2 * NS + t] = h ? 0.0 : w2q * Mn[t][0] * Mn[t][0];
          }
          half_sums_reg<KR>(vv, s0, s1);
          conv = true;
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            const double m01 = s0[t] > s0[NS + t] ? s0[t] : s0[NS + t];
            const double m23 = s1[t] > s1[NS + t] ? s1[t] : s1[NS + t];
            const double dm2 = m01 > m23 ? m01 : m23;
            const double dn2 = s0[2 * NS + t];
            const double dref2 = S.dref[t] > dn2 ? S.dref[t] : dn2;
            if (!(dm2 <= a.tol_inner2 * dref2)) conv = false;
          }
          if (conv) {
#pragma unroll
            for (int t = 0; t < NS; ++t) S.dref[t] = s0[2 * NS + t];
          }
        }
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          u[t][0] = Mn[t][0];
          u[t][1] = Mn[t][1];
        }
        exchange(u, Df, If);
        if (conv) break;
      }
      total_inner += (l > a.prm.max_inner ? a.prm.max_inner : l);
      if (fatal) break;
      if (!conv) {
        inner_failed = true;
        // reference of the next inner loop: the norm of the current moments
        double vv[2 * ((NS + 1) / 2)], s0[2 * ((NS + 1) / 2)], s1[2 * ((NS + 1) / 2)];
#pragma unroll
        for (int i = 0; i < 2 * ((NS + 1) / 2); ++i) vv[i] = (i < NS && h == 0) ? w2q * Df[i < NS ? i : 0] * Df[i < NS ? i : 0] : 0.0;
        half_sums_reg<(NS + 1) / 2>(vv, s0, s1);
#pragma unroll
        for (int t = 0; t < NS; ++t) S.dref[t] = s0[t];
      }
      if (a.prm.fixed_matter) {
        outer_conv = true;
        break;
      }

      // ---- matter right-hand side, residual, outer Anderson step on y ------
      double X[5], yq[5], f[5];
      eulerian(md, mt, h, q, Df, If, v, X);
      matter_rhs(S, X, yq);
#pragma unroll
      for (int i = 0; i < 5; ++i) f[i] = yq[i] - S.y[i];
      const int omem = k < a.prm.m_outer ? k : a.prm.m_outer;
      double yn[5];
      if (omem == 1) {
#pragma unroll
        for (int i = 0; i < 5; ++i) yn[i] = yq[i];
      } else {
        double dq2[5], df2[5];
        double G22 = 0.0, b2 = 0.0, G11o = 0.0, G12 = 0.0, b1 = 0.0;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          dq2[i] = yq[i] - S.oq[i];
          df2[i] = f[i] - S.of[i];
          const double o = S.odf[i];
          G22 += df2[i] * df2[i];
          b2 += df2[i] * f[i];
          G11o += o * o;
          G12 += o * df2[i];
          b1 += o * f[i];
        }
        double g1, g2;
        anderson2(omem == 3, G11o, G12, G22, b1, b2, g1, g2);
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          yn[i] = yq[i] - g2 * dq2[i] - g1 * S.odq[i];
          S.odq[i] = dq2[i];
          S.odf[i] = df2[i];
        }
      }
      bool finite = true;
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        S.oq[i] = yq[i];
        S.of[i] = f[i];
        finite = finite && isfinite(yn[i]);
      }
      if (!finite) {
        status = NMC_STATUS_NONFINITE;
        fatal = true;
        break;
      }
      // Algorithm outerConverged: Ye and ef against y* componentwise, each
      // velocity component against the speed max(|v*|, |v^[k+1]|)
      const double vst = sqrt(S.yst[2] * S.yst[2] + S.yst[3] * S.yst[3] + S.yst[4] * S.yst[4]);
      const double vnw = sqrt(yn[2] * yn[2] + yn[3] * yn[3] + yn[4] * yn[4]);
      const double vref = vst > vnw ? vst : vnw;
      bool oc = fabs(yn[0] - S.y[0]) <= a.prm.tol_outer * fabs(S.yst[0]) &&
                fabs(yn[1] - S.y[1]) <= a.prm.tol_outer * fabs(S.yst[1]);
#pragma unroll
      for (int j = 0; j < 3; ++j) oc = oc && fabs(yn[2 + j] - S.y[2 + j]) <= a.prm.tol_outer * vref;
#pragma unroll
      for (int i = 0; i < 5; ++i) S.y[i] = yn[i];
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
    double yout[5], T_out;
    if (a.prm.fixed_matter) {
#pragma unroll
      for (int i = 0; i < 5; ++i) yout[i] = S.yst[i];
      T_out = S.T_last;
    } else {
      // matter right-hand side at the final moments and the matter iterate
      // they were solved at
      const double vu[3] = {S.yused[2], S.yused[3], S.yused[4]};
      double X[5];
      eulerian(md, mt, h, q, Df, If, vu, X);
      matter_rhs(S, X, yout);
      T_out = temperature(md, yout, S.r3);
    }
    store_moments(u);
    if (lane == 0) {
      a.ye[p] = yout[0];
      a.ef[p] = yout[1];
#pragma unroll
      for (int j = 0; j < 3; ++j) a.v[3 * p + j] = yout[2 + j];
      a.T[p] = T_out;
      a.n_outer[p] = k;
      a.n_inner[p] = total_inner;
      a.status[p] = status;
    }
  }
};

template <int NS, bool COUPLED, bool PHI1>
__global__ __launch_bounds__(kLanes, 2) void fwd_v_kernel(FwdVArgs a) {
  __shared__ VLds<NS, PHI1> S;
  load_model(a.mdl, a.theta, S.m);
  if (a.queue) {
    WorkQueue wq(a.queue, a.P, a.chunk);
    for (int64_t g; (g = wq.next()) >= 0;) {
      const int64_t b0 = uniform64(g * a.chunk);
      const int64_t end = uniform64(b0 + a.chunk < a.P ? b0 + a.chunk : a.P);
      for (int64_t p = b0; p < end; ++p) PointSolverV<NS, COUPLED, PHI1>::solve(a, p, S, [&] { wq.settle(); });
    }
  } else {
    const int64_t b0 = (int64_t)blockIdx.x * a.chunk;
    const int64_t end = b0 + a.chunk < a.P ? b0 + a.chunk : a.P;
    for (int64_t p = b0; p < end; ++p) PointSolverV<NS, COUPLED, PHI1>::solve(a, p, S, [] {});
  }
}

template <int NS, bool COUPLED, bool PHI1 = false>
hipError_t launch_v_t(const FwdVArgs& a, const nmc_launch& L, int num_cu, hipStream_t s) {
  auto kern = fwd_v_kernel<NS, COUPLED, PHI1>;
  int64_t grid;
  if (a.queue) {
    int bpc = L.blocks_per_cu;
    if (bpc <= 0) {
      static int occ = 0;
      if (occ <= 0) {
        int o = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, kern, kLanes, 0) != hipSuccess || o <= 0) o = 8;
        occ = o;
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

hipError_t launch_forward_v(const FwdVArgs& a, int ns, bool coupled, bool phi1, const nmc_launch& L, int num_cu,
                            hipStream_t s) {
  if (phi1) {
    switch (ns) {
      case 1: return launch_v_t<1, true, true>(a, L, num_cu, s);
      case 2: return launch_v_t<2, true, true>(a, L, num_cu, s);
      case 3: return launch_v_t<3, true, true>(a, L, num_cu, s);
    }
  } else if (coupled) {
    switch (ns) {
      case 1: return launch_v_t<1, true>(a, L, num_cu, s);
      case 2: return launch_v_t<2, true>(a, L, num_cu, s);
      case 3: return launch_v_t<3, true>(a, L, num_cu, s);
    }
  } else {
    switch (ns) {
      case 1: return launch_v_t<1, false>(a, L, num_cu, s);
      case 2: return launch_v_t<2, false>(a, L, num_cu, s);
      case 3: return launch_v_t<3, false>(a, L, num_cu, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace nmc
