// Forward kernel of the implicit coupling solve with a nonzero fluid velocity
// (the O(v/c) two-moment model), 32 energy nodes, two points per wavefront
// (CDNA4).
//
// Same equations and iteration as the one-point O(v) kernel: Eqs.
// implicitNumberNodal / implicitNumberFluxNodal in the fixed-point form of
// Eq. implicitMomentsNodal with lambda = 1 / (1 + |v|), the Minerbo closure
// (Eqs. eddingtonFactorMinerbo, eddingtonTensor), Eq. implicitFluidNodal
// with the Eulerian integrals of Eqs. eulerianNumberLG, eulerianEnergyLG,
// eulerianMomentumLG, Algorithm neutrinoMatterCoupling around them.  Work
// decomposition of the static two-point kernel: lane = 32 h + q, half h
// solves point 2u + h, and lane q of the half owns all four moments (D, I_1,
// I_2, I_3) of node q of every species, so the closure and the velocity terms
// of a node are lane-local.  The collision rates depend on the number moments
// only and are contracted as in the static kernel (symmetric b^2 core with
// the columns broadcast by DPP, or the signed orientation form for very cold
// points).  The Anderson history of the 4 NS owned moments lives in
// registers in the coupled kernel (one wave per SIMD leaves them to spare),
// otherwise in LDS, sharing its space with the pair-factor tile, which is dead
// during the inner loop.  PHI1: the linear-order corrections (Eqs.
// zerothMomentCollisionTerm_NES/_Pair, firstMomentCollisionTerm_NES/_Pair with
// Eqs. linearCorrectionsNES/Pair, Phi_1 = r Phi_0 per process), contracted
// against each flux component on the same core as the isotropic rates.
#include "nmc_closure.h"
#include "nmc_pair.h"

namespace nmc {
namespace {

using namespace pairk;

constexpr double kMuC2v = 931.49410242;  // atomic mass unit rest energy [MeV]

template <int NS>
struct VPairLds {
  ModelLds m;
  SplitExp E[2];  // per point: exponent splits at its current temperature
  union {
    double hist[4][4 * NS][kLanes];  // Anderson history per owned moment: Q_prev, F_prev, dQ_old, dF_old
    double tile[2][NQP][NQP];        // per point, pair factors (see the static two-point kernel)
  } u;
  struct Pt {  // per-point state of the outer (matter) loop
    double dref[NS];  // ||D_s^[k,1]||_W^2 of the current inner loop
    double y[5], yst[5], yused[5], X0[5];  // matter iterate, old state, iterate of the last inner loop, old integrals
    double oq[5], of[5], odq[5], odf[5];   // outer Anderson history
    double T_last, r3, K, An, Ap, chi0;
  } pt[2];
};

// temperature of the EOS at the internal energy ef - m_u c^2 |v|^2 / 2
__device__ __forceinline__ double temperature_v(const_ptr<DevModel> md, const double* y, double r3) {
  const double v2 = y[2] * y[2] + y[3] * y[3] + y[4] * y[4];
  const double e = y[1] - 0.5 * kMuC2v * v2;
  return (e - md->eos_b * ye43(y[0]) * r3) * rcp_nr(md->eos_a * (1.0 + y[0]));
}

// The lane's contributions to the Eulerian integrals (N, E, F_1, F_2, F_3) of
// its node's moments at velocity v
template <int NS>
__device__ __forceinline__ void eulerian_node(const_ptr<DevModel> md, double w2, double w3, const double (&D)[NS],
                                              const double (&I)[NS][3], const double (&v)[3], double (&acc)[5]) {
#pragma unroll
  for (int i = 0; i < 5; ++i) acc[i] = 0.0;
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    double vI, vK[3];
    closure_terms(D[t], I[t], v, vI, vK);
    acc[0] += md->ig[t] * w2 * (D[t] + vI);
    acc[1] += md->imult[t] * w3 * (D[t] + 2.0 * vI);
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[2 + j] += md->imult[t] * w3 * (I[t][j] + v[j] * D[t] + vK[j]);
  }
}

// Eulerian integrals (N, E, F_1, F_2, F_3) of the half's point, in every lane
// of the half; one reduction shape for every caller, so that equal moments
// give bitwise equal integrals
template <int NS>
__device__ __forceinline__ void eulerian_point(const_ptr<DevModel> md, double w2, double w3, const double (&D)[NS],
                                               const double (&I)[NS][3], const double (&v)[3], double (&X)[5]) {
  double acc[5], s[6];
  eulerian_node<NS>(md, w2, w3, D, I, v, acc);
  const double vv[6] = {acc[0], acc[1], acc[2], acc[3], acc[4], 0.0};
  half_own_sums<3>(vv, s);
#pragma unroll
  for (int i = 0; i < 5; ++i) X[i] = s[i];
}

// ||D_s||_W^2 of the half's point per species, in every lane of the half
template <int NS>
__device__ __forceinline__ void dnorms(double w2, const double (&D)[NS], double (&n)[NS]) {
  constexpr int K = (NS + 1) / 2;
  double vv[2 * K], s[2 * K];
#pragma unroll
  for (int i = 0; i < 2 * K; ++i) vv[i] = i < NS ? w2 * D[i < NS ? i : 0] * D[i < NS ? i : 0] : 0.0;
  half_own_sums<K>(vv, s);
#pragma unroll
  for (int t = 0; t < NS; ++t) n[t] = s[t];
}

template <int NS, bool COUPLED, bool PHI1>
struct VPairSolver {
  static constexpr int NQ = NQP;
  static constexpr int NM = 4 * NS;            // owned moments per lane
  // the inner Anderson history in registers (the coupled isotropic kernel
  // runs one wave per SIMD and has the registers to spare); otherwise in LDS
  static constexpr bool HREG = COUPLED && !PHI1;

  // matter right-hand side q(M, y) of Eq. implicitFluidNodal from the
  // integrals X of the current moments
  __device__ __forceinline__ static void matter_rhs(const typename VPairLds<NS>::Pt& pt, const double (&X)[5],
                                                    double (&yq)[5]) {
    yq[0] = pt.yst[0] - pt.K * (X[0] - pt.X0[0]);
    yq[1] = pt.yst[1] - pt.K * (X[1] - pt.X0[1]);
    const double Kv = pt.K * (1.0 / kMuC2v);
#pragma unroll
    for (int j = 0; j < 3; ++j) yq[2 + j] = pt.yst[2 + j] - Kv * (X[2 + j] - pt.X0[2 + j]);
  }

  // Phi_1 contraction of flux component x_t = W e I_t,i (one component, all
  // species) on the row B of pair factors: L_in, L_out (own species), L_ann,
  // L_pro (partner species) at node q.  Symmetric core: the g and h factors
  // ride on the vectors and the row sums as in the isotropic rates; the
  // orientation form carries the entries directly.
  __device__ __forceinline__ static void phi1_pass(bool sym, const double (&B)[NQ], const double (&x)[NS], double gq,
                                                   double rgq, double hq, double (&Lin)[NS], double (&Lout)[NS],
                                                   double (&Lann)[NS], double (&Lpro)[NS]) {
    double eN[NS], oN[NS], aP[NS], eP[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) eN[t] = oN[t] = aP[t] = eP[t] = 0.0;
    if (sym) {
      double AR[2][NS], BR[2][NS], CR[2][NS], DR[2][NS];
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        swap16(x[t] * rgq, AR[0][t], AR[1][t]);
        swap16(x[t] * gq, BR[0][t], BR[1][t]);
        swap16(x[t], CR[0][t], CR[1][t]);
        swap16(hq * x[t], DR[0][t], DR[1][t]);
      }
      static_for<0, NQ / 4>([&](auto jj) __attribute__((always_inline)) {
        constexpr int j = 4 * decltype(jj)::value;
        ColSym<NS>::template run<j % 16>(eN, oN, aP, eP, AR[j / 16], BR[j / 16], CR[j / 16], DR[j / 16], B[j],
                                         B[j + 1], B[j + 2], B[j + 3]);
      });
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        Lin[t] = gq * eN[t];
        Lout[t] = rgq * oN[t];
      }
    } else {
      double XR[2][NS], HR[2][NS];
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        swap16(x[t], XR[0][t], XR[1][t]);
        swap16(hq * x[t], HR[0][t], HR[1][t]);
      }
      static_for<0, NQ>([&](auto jj) __attribute__((always_inline)) {
        constexpr int j = decltype(jj)::value;
        const double sb = B[j], b2 = sb * sb, c3 = sb * b2;
        ColFmac<NS>::template run<j % 16>(eN, oN, aP, eP, XR[j / 16], XR[j / 16], HR[j / 16],
                                          max_neg_f64(sb, c3), max_neg_f64(c3, sb), b2);
      });
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        Lin[t] = eN[t];
        Lout[t] = oN[t];
      }
    }
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      Lann[t] = aP[t];
      Lpro[t] = hq * eP[t];
    }
  }

  template <class Settle>
  __device__ static void solve(const FwdVArgs& a, int64_t u, VPairLds<NS>& S, Settle&& settle) {
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
    const int64_t baseD = p * (int64_t)(NS * NQ), baseI = p * (int64_t)(NS * 3 * NQ);
    const double rho = a.rho11[p];
    typename VPairLds<NS>::Pt& pt = S.pt[h];

    double D[NS], I[NS][3];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int ex = md->ext[t];
      D[t] = a.D0[baseD + ex * NQ + q0];
#pragma unroll
      for (int j = 0; j < 3; ++j) I[t][j] = a.I0[baseI + (ex * 3 + j) * NQ + q0];
    }
    double yst[5];
    yst[0] = a.ye0[p];
    yst[1] = a.ef0[p];
#pragma unroll
    for (int j = 0; j < 3; ++j) yst[2 + j] = a.v0[3 * p + j];
    settle();

    // coupling disabled at low density (Sec. 7.2): the state passes through
    const bool skip = rho < md->rho11_min;
    pt.r3 = cbrt(rho);
    pt.K = md->kcoup / rho;
    pt.An = (md->flags & NMC_NES) ? mt.theta[NQ] * rho : 0.0;
    pt.Ap = (md->flags & NMC_PAIR) ? mt.theta[NQ + 1] * rho : 0.0;
    pt.chi0 = a.chi0 ? a.chi0[p] : md->chi_ref * rho;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      pt.yst[i] = pt.y[i] = pt.yused[i] = yst[i];
      pt.oq[i] = pt.of[i] = pt.odq[i] = pt.odf[i] = 0.0;
    }
    pt.T_last = temperature_v(md, yst, pt.r3);

    // old conserved moments N* = D* + v*.I*, G*_j = I*_j + v*^i K*_ij (the
    // left-hand sides of Eqs. implicitNumberNodal, implicitNumberFluxNodal at
    // the old state), the old Eulerian integrals and ||D*_s||_W^2
    double Nst[NS], Gst[NS][3];
    {
      const double vs[3] = {yst[2], yst[3], yst[4]};
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        double vI, vK[3];
        closure_terms(D[t], I[t], vs, vI, vK);
        Nst[t] = D[t] + vI;
#pragma unroll
        for (int j = 0; j < 3; ++j) Gst[t][j] = I[t][j] + vK[j];
      }
      double X0[5], n0[NS];
      eulerian_point<NS>(md, mt.w2[q0], mt.w3[q0], D, I, vs, X0);
      dnorms<NS>(mt.w2[q0], D, n0);
#pragma unroll
      for (int t = 0; t < NS; ++t) pt.dref[t] = n0[t];
#pragma unroll
      for (int i = 0; i < 5; ++i) pt.X0[i] = X0[i];
    }

    int status = NMC_STATUS_OK;
    bool fatal = false, inner_failed = false, outer_conv = false;
    bool run = !skip;  // this half's point is still iterating the outer loop
    int k_done = 0, total_inner = 0;

    for (int k = 1; k <= a.prm.max_outer && __builtin_amdgcn_ballot_w64(run) != 0; ++k) {
      const_ptr<DevModel> md = scalar_ptr(a.mdl);
      const int q = opaque(q0);
      if (run) k_done = k;
      // ---- ComputeOpacities(y^[k]) --------------------------------------
      const double v[3] = {pt.y[2], pt.y[3], pt.y[4]};
      const double lam = rcp_nr(1.0 + sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
      const double T = temperature_v(md, a.prm.fixed_matter ? pt.yst : pt.y, pt.r3);
      const double y0 = pt.y[0];
      const double mu = md->mu_a * (y0 - md->mu_ye0) * pt.r3 + md->mu_b * log_pos(T * md->inv_mu_t0);
      if (run && (!(T > 0.0) || !(y0 >= 0.0) || !isfinite(T) || !isfinite(mu))) {
        status = NMC_STATUS_EOS_DOMAIN;
        fatal = true;
        run = false;
      }
      if (run) {
        pt.T_last = T;
#pragma unroll
        for (int i = 0; i < 5; ++i) pt.yused[i] = pt.y[i];
      }
      // a finished half keeps a harmless temperature
      const double Tu = run ? T : 1.0, muu = run ? mu : 0.0;
      const double invT = rcp_nr(Tu);
      const double ldt = lam * dtau, oml = 1.0 - lam;
      const double epsq = mt.eps[q];
      // per species: lam (N* + dtau chi^EmAb D_eq), 1 + lam dtau chi^EmAb and
      // 1 + lam dtau (chi^EmAb + sigma)
      double baseD[NS], denD[NS], denI[NS];
      {
        const double shape = pt.chi0 * mt.shape[q];
        const double sig = (md->flags & NMC_ISO) ? md->sigma_ratio * shape : 0.0;
        const double emab_q = (md->flags & NMC_EMAB) ? mt.theta[q] * shape : 0.0;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const double chia = md->iemab[t] * emab_q;
          double deq = 0.0;
          if (!(NS == 3 && t == 2)) {
            // three species are nu_e, anti-nu_e, nu_x in this order, and
            // nu_x has no emission or absorption (chia = 0): no equilibrium
            const double x = (epsq - md->imusign[t] * muu) * invT;
            const double ex = exp(-fabs(x));
            const double r = rcp_nr(1.0 + ex);
            deq = x > 0.0 ? ex * r : r;
          }
          baseD[t] = lam * (Nst[t] + dtau * (chia * deq));
          denD[t] = 1.0 + ldt * chia;
          denI[t] = 1.0 + ldt * (chia + sig);
        }
      }
      // pair factors of this lane's row (as in the static two-point kernel)
      double B[COUPLED ? NQ : 1];
      double hq = 0.0;
      double gq = 1.0, rgq = 1.0;
      bool sym = false;  // wave-uniform
      if constexpr (COUPLED) {
        SplitExp& E = S.E[h];
        const ExpSplit xs = exp_split(epsq, invT);
        E.P2[q] = xs.P;
        E.R2[q] = xs.R;
        E.n2[q] = xs.n;
        hq = ldexp(xs.R * xs.R, -2 * xs.n);  // exp(-e / T)
        __syncthreads();
        const int nlo = E.n2[0], nhi = E.n2[NQ - 1];
        const int c = (nlo + nhi) >> 1;
        sym = __builtin_amdgcn_readfirstlane(
                  (uint32_t)(__builtin_amdgcn_ballot_w64(run && nhi - nlo > kSymBits) == 0)) != 0;
        const bool direct = __builtin_amdgcn_readfirstlane((uint32_t)(
                                __builtin_amdgcn_ballot_w64(run && nhi - nlo > kDirectBits) == 0)) != 0;
        gq = sym ? ldexp(xs.R, c - xs.n) : 1.0;
        rgq = sym ? ldexp(xs.P, xs.n - c) : 1.0;
        if (direct) {
          // rows of the symmetric core from the point's scaled h, broadcast
          // from registers
          direct_row_regs(gq * gq, rgq * rgq, B);
        } else {
          double (*Tt)[NQ] = S.u.tile[h];
          if (sym) {
            pair_tile_rows<true>(&Tt[0][0], E.P2, E.R2, E.n2, q, xs.P, xs.R, xs.n);
            Tt[q][q] = 1.0;
          } else {
            pair_tile_rows<false>(&Tt[0][0], E.P2, E.R2, E.n2, q, xs.P, xs.R, xs.n);
            Tt[q][q] = -1.0;
          }
          __syncthreads();
#pragma unroll
          for (int j = 0; j < NQ; ++j) B[j] = Tt[j][q];
          __syncthreads();
        }
      }

      // ---- inner loop over moments at fixed matter (M^[k,1] = M^[k-1,*]) --
      const double w2q = mt.w2[q], w2eq = w2q * epsq;
      const double Aeq = pt.An * epsq, Apq = pt.Ap * epsq, Apqh = Apq * hq;

      double G11 = 0.0;
      double H[4][NM];  // Q_prev, F_prev, dQ_old, dF_old per owned moment (HREG)
      const bool ran = run;
      bool act = run;
      bool cvd = false;
      int l_done = 0;
      for (int l = 1; l <= a.prm.max_inner && __builtin_amdgcn_ballot_w64(act) != 0; ++l) {
        if (act) l_done = l;
        double etaN[NS], outN[NS], annP[NS], etaP[NS];
#pragma unroll
        for (int t = 0; t < NS; ++t) etaN[t] = outN[t] = annP[t] = etaP[t] = 0.0;
        if constexpr (COUPLED) {
#pragma unroll
          for (int j = 0; j < NQ; ++j) asm volatile("" : "+v"(B[j]));
          if (sym) {
            double AR[2][NS], BR[2][NS], CR[2][NS], DR[2][NS];
#pragma unroll
            for (int t = 0; t < NS; ++t) {
              const double xv = w2eq * D[t], yv = w2eq - xv;
              swap16(xv * rgq, AR[0][t], AR[1][t]);
              swap16(yv * gq, BR[0][t], BR[1][t]);
              swap16(xv, CR[0][t], CR[1][t]);
              swap16(hq * yv, DR[0][t], DR[1][t]);
            }
            static_for<0, NQ / 4>([&](auto jj) __attribute__((always_inline)) {
              constexpr int j = 4 * decltype(jj)::value;
              ColSym<NS>::template run<j % 16>(etaN, outN, annP, etaP, AR[j / 16], BR[j / 16], CR[j / 16],
                                               DR[j / 16], B[j], B[j + 1], B[j + 2], B[j + 3]);
            });
          } else {
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
                const double sb = B[j], b2 = sb * sb, c3 = sb * b2;
                ColFmac<NS>::template run<j % 16>(etaN, outN, annP, etaP, XR[j / 16], YR[j / 16], HR[j / 16],
                                                  max_neg_f64(sb, c3), max_neg_f64(c3, sb), b2);
              });
            });
          }
        }
        // linear-order corrections at the current iterate (PHI1): with
        // P = r_N L_in - r_P L_pro and R = r_N L_out - r_P L_ann per flux
        // component, the number equation gains (R - P).I and flux component j
        // P_j / 3 + (K (R - P))_j (phi1_collision), added like the emissivity
        double cN[PHI1 ? NS : 1], cI[PHI1 ? NS : 1][3];
        if constexpr (PHI1) {
          double Pc[NS][3], Rc[NS][3];
          const double rN = md->phi1_nes * Aeq, rP = md->phi1_pair * Apq;
          static_for<0, 3>([&](auto ii) __attribute__((always_inline)) {
            constexpr int i = decltype(ii)::value;
            double x[NS], Lin[NS], Lout[NS], Lann[NS], Lpro[NS];
#pragma unroll
            for (int t = 0; t < NS; ++t) x[t] = w2eq * I[t][i];
            phi1_pass(sym, B, x, gq, rgq, hq, Lin, Lout, Lann, Lpro);
#pragma unroll
            for (int t = 0; t < NS; ++t) {
              Pc[t][i] = __builtin_fma(rN, Lin[t], -rP * Lpro[t]);
              Rc[t][i] = __builtin_fma(rN, Lout[t], -rP * Lann[t]);
            }
          });
#pragma unroll
          for (int t = 0; t < NS; ++t) phi1_collision(D[t], I[t], Pc[t], Rc[t], cN[t], cI[t]);
        }
        // Q and residual of the owned moments (Eq. implicitMomentsNodal):
        //   Q_D  = ((1 - lam) D - lam v.I + lam (N* + dtau (eta + c))) / (1 + lam dtau chi)
        //   Q_Ij = ((1 - lam) I_j - lam v^i K_ij + lam (G*_j + dtau c_j)) / (1 + lam dtau kappa)
        // (c, c_j the linear-order terms, zero without PHI1); one reciprocal
        // of the product of the two denominators serves both
        double Qx[NM];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const double eta = __builtin_fma(Aeq * gq, etaN[t], Apqh * etaP[t]);
          const double chi = __builtin_fma(Aeq * rgq, outN[t], __builtin_fma(Apq, annP[t], eta));
          double vI, vK[3];
          closure_terms(D[t], I[t], v, vI, vK);
          const double dD = __builtin_fma(ldt, chi, denD[t]), dI = __builtin_fma(ldt, chi, denI[t]);
          const double r = rcp_nr(dD * dI);
          double nD = __builtin_fma(oml, D[t], baseD[t]) - lam * vI + ldt * eta;
          if constexpr (PHI1) nD = __builtin_fma(ldt, cN[t], nD);
          Qx[4 * t] = nD * (r * dI);
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            double nI = __builtin_fma(oml, I[t][j], lam * Gst[t][j]) - lam * vK[j];
            if constexpr (PHI1) nI = __builtin_fma(ldt, cI[t][j], nI);
            Qx[4 * t + 1 + j] = nI * (r * dD);
          }
        }
        // the current iterate in moment order, and the residual F = Q - M
        auto cur = [&](int x) { return (x & 3) == 0 ? D[x >> 2] : I[x >> 2][(x & 3) - 1]; };
        // Anderson step over min(l, M_inner) residuals (difference form)
        const int mem = l < a.prm.m_inner ? l : a.prm.m_inner;
        double Xn[NM];
        if constexpr (HREG) {
          // history in registers
          if (mem == 1) {
            // the older difference column is weighted zero at the second
            // iterate: clear it, so that no stale value enters that product
#pragma unroll
            for (int x = 0; x < NM; ++x) {
              Xn[x] = Qx[x];
              H[2][x] = 0.0;
              H[3][x] = 0.0;
            }
          } else {
            double v4[4] = {0.0, 0.0, 0.0, 0.0}, dF2[NM];
#pragma unroll
            for (int x = 0; x < NM; ++x) {
              const double Fx = Qx[x] - cur(x);
              dF2[x] = Fx - H[1][x];
              const double dF1 = H[3][x];
              v4[0] += dF1 * dF2[x];
              v4[1] += dF2[x] * dF2[x];
              v4[2] += dF1 * Fx;
              v4[3] += dF2[x] * Fx;
            }
            double gs[4];
            half_sums4(v4, gs);
            double g1, g2;
            anderson2(mem == 3, G11, gs[0], gs[1], gs[2], gs[3], g1, g2);
#pragma unroll
            for (int x = 0; x < NM; ++x) {
              const double dQ2 = Qx[x] - H[0][x];
              Xn[x] = Qx[x] - g2 * dQ2 - g1 * H[2][x];
              H[2][x] = dQ2;
              H[3][x] = dF2[x];
            }
            G11 = gs[1];
          }
#pragma unroll
          for (int x = 0; x < NM; ++x) {
            H[1][x] = Qx[x] - cur(x);
            H[0][x] = Qx[x];
          }
        } else {
          if (mem == 1) {
            // the older difference column is weighted zero at the second
            // iterate: clear it, so that no stale LDS word enters that product
#pragma unroll
            for (int x = 0; x < NM; ++x) {
              Xn[x] = Qx[x];
              S.u.hist[2][x][lane] = 0.0;
              S.u.hist[3][x][lane] = 0.0;
            }
          } else {
            // two passes over the owned moments: the Gram sums, then the step
            // (the differences are formed again from LDS rather than held)
            double v4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int x = 0; x < NM; ++x) {
              const double Fx = Qx[x] - cur(x);
              const double dF2 = Fx - S.u.hist[1][x][lane];
              const double dF1 = S.u.hist[3][x][lane];
              v4[0] += dF1 * dF2;
              v4[1] += dF2 * dF2;
              v4[2] += dF1 * Fx;
              v4[3] += dF2 * Fx;
            }
            double gs[4];
            half_sums4(v4, gs);
            double g1, g2;
            anderson2(mem == 3, G11, gs[0], gs[1], gs[2], gs[3], g1, g2);
#pragma unroll
            for (int x = 0; x < NM; ++x) {
              const double dQ2 = Qx[x] - S.u.hist[0][x][lane];
              const double dF2 = (Qx[x] - cur(x)) - S.u.hist[1][x][lane];
              Xn[x] = Qx[x] - g2 * dQ2 - g1 * S.u.hist[2][x][lane];
              S.u.hist[2][x][lane] = dQ2;
              S.u.hist[3][x][lane] = dF2;
            }
            G11 = gs[1];
          }
#pragma unroll
          for (int x = 0; x < NM; ++x) {
            S.u.hist[0][x][lane] = Qx[x];
            S.u.hist[1][x][lane] = Qx[x] - cur(x);
          }
        }
        bool bad = false;
#pragma unroll
        for (int x = 0; x < NM; ++x) bad |= !isfinite(Xn[x]);
        if (half_any(bad) && act) {
          status = NMC_STATUS_NONFINITE;
          fatal = true;
          act = run = false;
        }
        // Algorithm innerConverged over the four moments of each species:
        // max_m sum_q W dM_m^2 <= tol^2 max(||D^[k,1]||^2, ||D^[k,l+1]||^2)
        {
          // the sums are spread over the half (lane class c holds species c,
          // spread_conv_sums); the half has converged when every lane passes
          double vm[4][NS], vn[NS];
#pragma unroll
          for (int t = 0; t < NS; ++t) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              const double d = Xn[4 * t + m] - cur(4 * t + m);
              vm[m][t] = w2q * d * d;
            }
            vn[t] = w2q * Xn[4 * t] * Xn[4 * t];
          }
          double dm2[2], dn2;
          spread_conv_sums<NS, 4>(vm, vn, dm2, dn2);
          const int cls = spread_class(lane);
          const double d0 = cls < NS ? pt.dref[cls < NS ? cls : 0] : 0.0;
          const double tr2 = a.tol_inner2 * (d0 > dn2 ? d0 : dn2);
          const bool conv = !half_any(!(dm2[0] <= tr2 && dm2[1] <= tr2));
          // ||D^[k,*]|| is the reference of the next inner loop
          if (act && conv && cls < NS) pt.dref[cls < NS ? cls : 0] = dn2;
          if (act) {
#pragma unroll
            for (int t = 0; t < NS; ++t) {
              D[t] = Xn[4 * t];
#pragma unroll
              for (int j = 0; j < 3; ++j) I[t][j] = Xn[4 * t + 1 + j];
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
      // the reference norms of the next inner loop (after a failed loop: the
      // norm of the current moments) and the Eulerian integrals of the
      // current moments at the matter iterate, in one reduction
      double X[5];
      {
        double nrm[NS];
        dnorms<NS>(w2q, D, nrm);
        if (run && !cvd) {
#pragma unroll
          for (int t = 0; t < NS; ++t) pt.dref[t] = nrm[t];
        }
        eulerian_point<NS>(md, w2q, mt.w3[q], D, I, v, X);
      }
      if (a.prm.fixed_matter) {
        if (run) outer_conv = true;
        run = false;
      }
      if (run) {
        // ---- matter right-hand side, residual, outer Anderson step on y ----
        double yq[5], f[5], yn[5];
        matter_rhs(pt, X, yq);
#pragma unroll
        for (int i = 0; i < 5; ++i) f[i] = yq[i] - pt.y[i];
        const int omem = k < a.prm.m_outer ? k : a.prm.m_outer;
        if (omem == 1) {
#pragma unroll
          for (int i = 0; i < 5; ++i) yn[i] = yq[i];
        } else {
          double dq2[5], df2[5];
          double G22 = 0.0, b2 = 0.0, G11o = 0.0, G12 = 0.0, b1 = 0.0;
#pragma unroll
          for (int i = 0; i < 5; ++i) {
            dq2[i] = yq[i] - pt.oq[i];
            df2[i] = f[i] - pt.of[i];
            const double o = pt.odf[i];
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
            yn[i] = yq[i] - g2 * dq2[i] - g1 * pt.odq[i];
            pt.odq[i] = dq2[i];
            pt.odf[i] = df2[i];
          }
        }
        bool finite = true;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          pt.oq[i] = yq[i];
          pt.of[i] = f[i];
          finite = finite && isfinite(yn[i]);
        }
        if (!finite) {
          status = NMC_STATUS_NONFINITE;
          fatal = true;
          run = false;
        } else {
          // Algorithm outerConverged: Ye and ef against y* componentwise, each
          // velocity component against the speed max(|v*|, |v^[k+1]|)
          const double vst = sqrt(pt.yst[2] * pt.yst[2] + pt.yst[3] * pt.yst[3] + pt.yst[4] * pt.yst[4]);
          const double vnw = sqrt(yn[2] * yn[2] + yn[3] * yn[3] + yn[4] * yn[4]);
          const double vref = vst > vnw ? vst : vnw;
          bool oc = fabs(yn[0] - pt.y[0]) <= a.prm.tol_outer * fabs(pt.yst[0]) &&
                    fabs(yn[1] - pt.y[1]) <= a.prm.tol_outer * fabs(pt.yst[1]);
#pragma unroll
          for (int j = 0; j < 3; ++j) oc = oc && fabs(yn[2 + j] - pt.y[2 + j]) <= a.prm.tol_outer * vref;
#pragma unroll
          for (int i = 0; i < 5; ++i) pt.y[i] = yn[i];
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
    // matter right-hand side at the final moments and the matter iterate they
    // were solved at (every lane of both halves takes part in the reduction)
    double yout[5];
    {
      const double vu[3] = {pt.yused[2], pt.yused[3], pt.yused[4]};
      double X[5];
      eulerian_point<NS>(md, mt.w2[q0], mt.w3[q0], D, I, vu, X);
      matter_rhs(pt, X, yout);
    }
    double T_out;
    if (skip) {
#pragma unroll
      for (int i = 0; i < 5; ++i) yout[i] = pt.yst[i];
      T_out = temperature_v(md, pt.yst, pt.r3);
    } else if (a.prm.fixed_matter) {
#pragma unroll
      for (int i = 0; i < 5; ++i) yout[i] = pt.yst[i];
      T_out = pt.T_last;
    } else {
      T_out = temperature_v(md, yout, pt.r3);
    }
    if (has_point) {
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int ex = md->ext[t];
        a.D[baseD + ex * NQ + q0] = D[t];
#pragma unroll
        for (int j = 0; j < 3; ++j) a.I[baseI + (ex * 3 + j) * NQ + q0] = I[t][j];
      }
      if (q0 == 0) {
        a.ye[p] = yout[0];
        a.ef[p] = yout[1];
#pragma unroll
        for (int j = 0; j < 3; ++j) a.v[3 * p + j] = yout[2 + j];
        a.T[p] = T_out;
        a.n_outer[p] = skip ? 0 : k_done;
        a.n_inner[p] = total_inner;
        a.status[p] = status;
      }
    }
    __syncthreads();
  }
};

template <int NS, bool COUPLED, bool PHI1>
__global__ __launch_bounds__(kLanes, COUPLED ? 1 : 2) void fwd_vpair_kernel(FwdVArgs a) {
  __shared__ VPairLds<NS> S;
  load_model(a.mdl, a.theta, S.m);
  const int64_t pairs = (a.P + 1) / 2;
  if (a.queue) {
    WorkQueue wq(a.queue, pairs, a.chunk);
    for (int64_t g; (g = wq.next()) >= 0;) {
      const int64_t b0 = uniform64(g * a.chunk);
      const int64_t end = uniform64(b0 + a.chunk < pairs ? b0 + a.chunk : pairs);
      for (int64_t u = b0; u < end; ++u) VPairSolver<NS, COUPLED, PHI1>::solve(a, u, S, [&] { wq.settle(); });
    }
  } else {
    const int64_t b0 = (int64_t)blockIdx.x * a.chunk;
    const int64_t end = b0 + a.chunk < pairs ? b0 + a.chunk : pairs;
    for (int64_t u = b0; u < end; ++u) VPairSolver<NS, COUPLED, PHI1>::solve(a, u, S, [] {});
  }
}

template <int NS, bool COUPLED, bool PHI1>
hipError_t launch_vpair_t(const FwdVArgs& a, const nmc_launch& L, int num_cu, hipStream_t s) {
  auto kern = fwd_vpair_kernel<NS, COUPLED, PHI1>;
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
        occ = o;
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

}  // namespace

hipError_t launch_forward_vpair(const FwdVArgs& a, int ns, bool coupled, bool phi1, const nmc_launch& L,
                                int num_cu, hipStream_t s) {
  if (coupled && phi1) {
    switch (ns) {
      case 1: return launch_vpair_t<1, true, true>(a, L, num_cu, s);
      case 2: return launch_vpair_t<2, true, true>(a, L, num_cu, s);
      case 3: return launch_vpair_t<3, true, true>(a, L, num_cu, s);
    }
  } else if (coupled) {
    switch (ns) {
      case 1: return launch_vpair_t<1, true, false>(a, L, num_cu, s);
      case 2: return launch_vpair_t<2, true, false>(a, L, num_cu, s);
      case 3: return launch_vpair_t<3, true, false>(a, L, num_cu, s);
    }
  } else {
    switch (ns) {
      case 1: return launch_vpair_t<1, false, false>(a, L, num_cu, s);
      case 2: return launch_vpair_t<2, false, false>(a, L, num_cu, s);
      case 3: return launch_vpair_t<3, false, false>(a, L, num_cu, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace nmc
