// Forward kernel of the implicit neutrino-matter coupling solve on CDNA4.
//
// One 64-lane wavefront solves one spatial point at a time (Algorithm
// neutrinoMatterCoupling, Sec. 3.5.3); spatial points are independent because
// the nodal DG collocation decouples them (Sec. 3.1.2).
//
// Lane layout for 32 energy nodes: lane = 32 h + q.
//   h = 0 ("number lanes"): own the number moments D_s[q] of every species and
//          hold row q of Phi_in and Phi_ann in VGPRs;
//   h = 1 ("flux lanes"):   own the flux moments I_s[q] and hold row q of
//          Phi_out and Phi_pro.
// The energy-coupling rates (Eqs. nesRatesNodal, pairRatesNodal) are two
// stacked (64 x 32) x (32 x ns) products per inner iteration:
//   [Phi_in ; Phi_out] rows x (W D | W (1 - D))  and  [Phi_ann ; Phi_pro] x (same).
// The moment vectors W D (number lanes' rows) and W (1 - D) (flux lanes' rows)
// are kept replicated per 16-lane DPP row and broadcast into the FMAs with
// DPP row_newbcast, so the kernel rows never leave the register file and no
// LDS traffic is spent on the contraction.  Half-wave partial rates are
// combined with v_permlane32_swap; moment vectors are redistributed with
// v_permlane16_swap.  Weighted norms and Anderson inner products are reduced
// through LDS.
#include <type_traits>
#include <utility>

#include "nmc_internal.h"

namespace nmc {
namespace {

constexpr int kLanes = 64;

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  return __builtin_amdgcn_update_dpp(0.0, x, CTRL, 0xF, 0xF, false);
}

// broadcast lane I of every 16-lane row to the whole row (row_newbcast:I);
// every lane is written, so no "old" operand is needed
template <int I>
__device__ __forceinline__ double row_bcast(double x) {
  const long v = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(long, x), 0x150 + I, 0xF, 0xF, false);
  return __builtin_bit_cast(double, v);
}

__device__ __forceinline__ uint32_t lo32(double x) { return (uint32_t)__builtin_bit_cast(uint64_t, x); }
__device__ __forceinline__ uint32_t hi32(double x) { return (uint32_t)(__builtin_bit_cast(uint64_t, x) >> 32); }
__device__ __forceinline__ double mk64(uint32_t lo, uint32_t hi) {
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// v_permlane16_swap(v, v): first = rows (0,0,2,2) of v, second = rows (1,1,3,3)
__device__ __forceinline__ void swap16(double v, double& first, double& second) {
  auto a = __builtin_amdgcn_permlane16_swap(lo32(v), lo32(v), false, false);
  auto b = __builtin_amdgcn_permlane16_swap(hi32(v), hi32(v), false, false);
  first = mk64(a[0], b[0]);
  second = mk64(a[1], b[1]);
}

// v_permlane32_swap(v, v): first = lanes 0..31 of v in both halves, second = lanes 32..63
__device__ __forceinline__ void swap32(double v, double& first, double& second) {
  auto a = __builtin_amdgcn_permlane32_swap(lo32(v), lo32(v), false, false);
  auto b = __builtin_amdgcn_permlane32_swap(hi32(v), hi32(v), false, false);
  first = mk64(a[0], b[0]);
  second = mk64(a[1], b[1]);
}

// lower-half value + upper-half value, identical bits in every lane
__device__ __forceinline__ double sum_halves(double v) {
  double f, s;
  swap32(v, f, s);
  return f + s;
}

// Per-half sums of V lane values through LDS: s0[k] = sum over lanes 0..31,
// s1[k] = sum over lanes 32..63.  Fixed summation order (deterministic).
template <int V>
__device__ __forceinline__ void half_sums(const double (&v)[V], double (&s0)[V], double (&s1)[V], double* red,
                                          double* redout) {
  static_assert(2 * V <= 16, "at most 16 sums");
  const int l = threadIdx.x;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < V; ++k) red[k * kLanes + l] = v[k];
  __syncthreads();
  const int sidx = l >> 2, r = l & 3;
  double acc = 0.0;
  if (sidx < 2 * V) {
    const int hh = sidx / V, k = sidx - hh * V;
    const double* b = red + k * kLanes + hh * 32 + r * 8;
    acc = ((b[0] + b[1]) + (b[2] + b[3])) + ((b[4] + b[5]) + (b[6] + b[7]));
  }
  acc += dpp<0xB1>(acc);  // quad_perm [1,0,3,2]
  acc += dpp<0x4E>(acc);  // quad_perm [2,3,0,1]
  if (r == 0 && sidx < 2 * V) redout[sidx] = acc;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < V; ++k) {
    s0[k] = redout[k];
    s1[k] = redout[V + k];
  }
}

__device__ __forceinline__ bool wave_any(bool b) { return __builtin_amdgcn_ballot_w64(b) != 0; }

// Per-wave LDS scratch of the point solver.
template <int NS>
struct WaveLds {
  double mst[NS][kLanes];     // owned moment of the old state (D* or I*)
  double hist[4][NS][kLanes];  // Anderson history: Q_prev, F_prev, dQ_old, dF_old
  double red[2 * NS * kLanes];  // reduction staging
  double redout[16];
};

template <int NS, int NQ>
struct PointSolver {
  static_assert(NQ == 32, "lane layout is for 32 energy nodes");

  // Energy-coupling contraction: a1[t] = sum_j M1[j] X_t[j], a2[t] = sum_j M2[j] X_t[j]
  // where X_t = W D_t on number lanes and W (1 - D_t) on flux lanes.
  __device__ __forceinline__ static void contract(const double (&M1)[NQ], const double (&M2)[NQ],
                                                  const double (&XR)[NS][2], double (&a1)[NS], double (&a2)[NS]) {
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      a1[t] = 0.0;
      a2[t] = 0.0;
    }
    static_for<0, 2>([&](auto c) {
      static_for<0, 16>([&](auto i) {
        constexpr int C = decltype(c)::value, I = decltype(i)::value, j = 16 * C + I;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const double b = row_bcast<I>(XR[t][C]);
          a1[t] = __builtin_fma(M1[j], b, a1[t]);
          a2[t] = __builtin_fma(M2[j], b, a2[t]);
        }
      });
    });
  }

  // Kernel rows at temperature T (Eqs. nesRatesNodal, pairRatesNodal with the
  // kernels of Eqs. inOutInvarianceNES ... detailedBalancePair).  With
  // a = exp(-|e_q - e_j| / (2T)) and G_x = exp(-2 e_x / T):
  //   Phi_in  = A e_q e_j (a^3 if e_q > e_j else a),  Phi_out = A e_q e_j (a if e_q > e_j else a^3),
  //   Phi_ann = A' e_q e_j a^2,                       Phi_pro = A' e_q e_j G_max(q,j).
  // Every factor is <= 1, so nothing overflows at low temperature.
  __device__ __forceinline__ static void build_rows(int h, double epsq, double invT, double An, double Ap,
                                                    double (&M1)[NQ], double (&M2)[NQ]) {
    double ER[2], GR[2];
    swap16(epsq, ER[0], ER[1]);
    const double Gq = exp(-2.0 * epsq * invT);
    swap16(Gq, GR[0], GR[1]);
    const double hinv = 0.5 * invT;
    static_for<0, 2>([&](auto c) {
      static_for<0, 16>([&](auto i) {
        constexpr int C = decltype(c)::value, I = decltype(i)::value, j = 16 * C + I;
        const double ej = row_bcast<I>(ER[C]);
        const double Gj = row_bcast<I>(GR[C]);
        const double dl = epsq - ej;
        const double av = exp(-fabs(dl) * hinv);
        const double a2 = av * av;
        const double a3 = a2 * av;
        const double ee = epsq * ej;
        const bool above = dl > 0.0;
        M1[j] = An * ee * ((above != (h != 0)) ? a3 : av);
        M2[j] = Ap * ee * (h ? (above ? Gq : Gj) : a2);
      });
    });
  }

  __device__ static void solve(const FwdArgs& a, int64_t p, WaveLds<NS>& S) {
    const DevModel* __restrict__ md = a.mdl;
    const SolverParams& prm = a.prm;
    const int lane = threadIdx.x;
    const int h = lane >> 5;  // 0: number lanes, 1: flux lanes
    const int q = lane & 31;
    const double epsq = md->eps[q], w2q = md->w2[q], w3q = md->w3[q], shq = md->shape[q];
    const double dtau = a.dtau;
    const unsigned flags = md->flags;
    double* red = S.red;
    double* redout = S.redout;

    const double rho = a.rho11[p];
    const double ye_st = a.ye0[p], e_st = a.e0[p];
    const int64_t base = p * (int64_t)(NS * NQ);
    const double r3 = cbrt(rho);
    const bool fixedT = prm.fixed_matter && a.T_fixed;

    // the moment a lane owns: D* on number lanes, I* on flux lanes; D* on
    // every lane (flux lanes form W (1 - D) from it)
    double M[NS], Dcur[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      Dcur[t] = a.D0[base + t * NQ + q];
      M[t] = h ? a.I0[base + t * NQ + q] : Dcur[t];
    }

    if (rho < md->rho11_min) {
      // coupling disabled at low density (Sec. 7.2): pass the state through
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        if (h == 0) a.D[base + t * NQ + q] = M[t];
        else a.I[base + t * NQ + q] = M[t];
      }
      if (lane == 0) {
        a.ye[p] = ye_st;
        a.e[p] = e_st;
        a.T[p] = fixedT ? a.T_fixed[p]
                        : (e_st - md->eos_b * pow(ye_st, 4.0 / 3.0) * r3) / (md->eos_a * (1.0 + ye_st));
        a.n_outer[p] = 0;
        a.n_inner[p] = 0;
        a.status[p] = NMC_STATUS_OK;
      }
      return;
    }
#pragma unroll
    for (int t = 0; t < NS; ++t) S.mst[t][lane] = M[t];

    const double chi0 = a.chi0 ? a.chi0[p] : md->chi_ref * rho;
    const double An = (flags & NMC_NES) ? a.theta[NQ] * rho : 0.0;
    const double Ap = (flags & NMC_PAIR) ? a.theta[NQ + 1] * rho : 0.0;
    const bool coupled = (flags & (NMC_NES | NMC_PAIR)) != 0;

    // point-constant opacities: chi^EmAb = theta_q chi0 shape_q (electron
    // flavours), sigma^Iso = sigma_ratio chi0 shape_q
    const double shape = chi0 * shq;
    const double sig = (flags & NMC_ISO) ? md->sigma_ratio * shape : 0.0;
    const double emab_q = (flags & NMC_EMAB) ? a.theta[q] * shape : 0.0;

    // ||D_s||_W^2 of the initial moments (reference of the first inner loop)
    double nD[NS];
    {
      double v[NS], s0[NS], s1[NS];
#pragma unroll
      for (int t = 0; t < NS; ++t) v[t] = h ? 0.0 : w2q * Dcur[t] * Dcur[t];
      half_sums<NS>(v, s0, s1, red, redout);
#pragma unroll
      for (int t = 0; t < NS; ++t) nD[t] = s0[t];
    }

    double y0 = ye_st, y1 = e_st;  // matter iterate (Ye, e)
    // outer Anderson history: previous (q, f) and the older difference column
    double oq0 = 0, oq1 = 0, of0 = 0, of1 = 0, odq0 = 0, odq1 = 0, odf0 = 0, odf1 = 0;
    int status = NMC_STATUS_OK;
    bool fatal = false, inner_failed = false, outer_conv = false;
    int k, total_inner = 0;
    double T_last = fixedT ? a.T_fixed[p] : (e_st - md->eos_b * pow(ye_st, 4.0 / 3.0) * r3) / (md->eos_a * (1.0 + ye_st));

    double M1[NQ], M2[NQ];
    for (k = 1; k <= prm.max_outer; ++k) {
      // ---- ComputeOpacities(y^[k]) --------------------------------------
      const double T = fixedT ? a.T_fixed[p] : (y1 - md->eos_b * pow(y0, 4.0 / 3.0) * r3) / (md->eos_a * (1.0 + y0));
      const double mu = (prm.fixed_matter && a.mu_fixed) ? a.mu_fixed[p]
                                                         : md->mu_a * (y0 - md->mu_ye0) * r3 + md->mu_b * log(T / md->mu_t0);
      if (!(T > 0.0) || !(y0 >= 0.0) || !isfinite(T) || !isfinite(mu)) {
        status = NMC_STATUS_EOS_DOMAIN;
        fatal = true;
        break;
      }
      T_last = T;
      const double invT = 1.0 / T;

      // Eq. emissivityEmAbNodal with the nodal Fermi-Dirac equilibrium: the
      // number lanes need chi^EmAb D_eq and chi^EmAb, the flux lanes
      // chi^EmAb + sigma^Iso (transport opacity, Eq. transportOpacityNodal).
      double c1[NS], c2[NS];
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const double chia = md->emab[t] * emab_q;
        const double x = (epsq - md->musign[t] * mu) * invT;
        const double ex = exp(-fabs(x));
        const double deq = x > 0.0 ? ex / (1.0 + ex) : 1.0 / (1.0 + ex);
        c1[t] = h ? 0.0 : chia * deq;
        c2[t] = h ? chia + sig : chia;
      }

      // kernel rows in registers: number lanes Phi_in[q][:], Phi_ann[q][:];
      // flux lanes Phi_out[q][:], Phi_pro[q][:]
      if (coupled) build_rows(h, epsq, invT, An, Ap, M1, M2);

      // ---- inner loop over moments at fixed matter (M^[k,1] = M^[k-1,*]) --
      double dref0[NS];
#pragma unroll
      for (int t = 0; t < NS; ++t) dref0[t] = sqrt(nD[t]);
      double G11 = 0.0;
      bool conv = false;
      int l;
      for (l = 1; l <= prm.max_inner; ++l) {
        // ComputeRates(M^[k,l])
        double eta_c[NS], chi_c[NS];
        if (coupled) {
          double XR[NS][2];
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            const double x = h ? w2q * (1.0 - Dcur[t]) : w2q * Dcur[t];
            swap16(x, XR[t][0], XR[t][1]);
          }
          double a1[NS], a2[NS];
          contract(M1, M2, XR, a1, a2);
          // number lanes: a1 = eta^NES, a2 = Phi_ann W D (per partner);
          // flux lanes: a1 = Phi_out W (1 - D), a2 = eta^Pair (per partner)
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const int sb = md->partner[s];
            double pa = a2[0];
#pragma unroll
            for (int t = 1; t < NS; ++t) pa = (sb == t) ? a2[t] : pa;
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
          const double num = S.mst[t][lane] + dtau * (h ? 0.0 : c1[t] + eta_c[t]);
          const double den = 1.0 + dtau * (c2[t] + chi_c[t]);
          Q[t] = num / den;
          F[t] = Q[t] - M[t];
        }

        // Anderson step over the last min(l, M_inner) residuals
        double Mnew[NS];
        const int mem = l < prm.m_inner ? l : prm.m_inner;
        if (mem == 1) {
#pragma unroll
          for (int t = 0; t < NS; ++t) Mnew[t] = Q[t];
        } else {
          double dQ2[NS], dF2[NS];
          double v4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            dQ2[t] = Q[t] - S.hist[0][t][lane];
            dF2[t] = F[t] - S.hist[1][t][lane];
            const double dF1 = (mem == 3) ? S.hist[3][t][lane] : 0.0;
            v4[0] += dF1 * dF2[t];
            v4[1] += dF2[t] * dF2[t];
            v4[2] += dF1 * F[t];
            v4[3] += dF2[t] * F[t];
          }
          double s0[4], s1[4];
          half_sums<4>(v4, s0, s1, red, redout);
          const double G12 = s0[0] + s1[0], G22 = s0[1] + s1[1];
          const double b1 = s0[2] + s1[2], b2 = s0[3] + s1[3];
          double g1 = 0.0, g2 = 0.0;
          bool two = (mem == 3);
          if (two) {
            const double tr = G11 + G22;
            two = G11 > 1e-14 * tr;
            if (two) {
              const double L11 = sqrt(G11);
              const double L21 = G12 / L11;
              const double p2 = G22 - L21 * L21;
              two = p2 > 1e-14 * tr;
              if (two) {
                const double L22 = sqrt(p2);
                const double z1 = b1 / L11;
                const double z2 = (b2 - L21 * z1) / L22;
                g2 = z2 / L22;
                g1 = (z1 - L21 * g2) / L11;
              }
            }
          }
          if (!two) {
            // newest column only; Picard when it vanishes
            g1 = 0.0;
            if (G22 > 1e-14 * G22) {
              const double L = sqrt(G22);
              g2 = (b2 / L) / L;
            } else {
              g2 = 0.0;
            }
          }
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            double mn = Q[t] - g2 * dQ2[t];
            if (mem == 3) mn -= g1 * S.hist[2][t][lane];
            Mnew[t] = mn;
            S.hist[2][t][lane] = dQ2[t];
            S.hist[3][t][lane] = dF2[t];
          }
          G11 = G22;
        }
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          S.hist[0][t][lane] = Q[t];
          S.hist[1][t][lane] = F[t];
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
        // by the new norm)
        {
          double v[2 * NS], s0[2 * NS], s1[2 * NS];
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            const double d = Mnew[t] - M[t];
            v[t] = w2q * d * d;
            v[NS + t] = h ? 0.0 : w2q * Mnew[t] * Mnew[t];
          }
          half_sums<2 * NS>(v, s0, s1, red, redout);
          conv = true;
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            const double sd = s0[t], si = s1[t];
            const double dm = sqrt(sd > si ? sd : si);
            const double dn = sqrt(s0[NS + t]);
            const double dref = dref0[t] > dn ? dref0[t] : dn;
            if (!(dm <= prm.tol_inner * dref)) conv = false;
            nD[t] = s0[NS + t];
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
      total_inner += (l > prm.max_inner ? prm.max_inner : l);
      if (fatal) break;
      if (!conv) inner_failed = true;
      if (prm.fixed_matter) {
        outer_conv = true;
        break;
      }

      // ---- matter right-hand side (Eq. implicitFluidNodal at v = 0) -------
      double yq0, yq1;
      {
        double mv[2] = {0.0, 0.0}, s0[2], s1[2];
        if (h == 0) {
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            const double dd = M[t] - S.mst[t][lane];
            mv[0] += md->g[t] * w2q * dd;
            mv[1] += md->mult[t] * w3q * dd;
          }
        }
        half_sums<2>(mv, s0, s1, red, redout);
        const double K = md->kcoup / rho;
        yq0 = ye_st - K * s0[0];
        yq1 = e_st - K * s0[1];
      }
      const double f0 = yq0 - y0, f1 = yq1 - y1;

      // outer Anderson step on (Ye, e)
      const int omem = k < prm.m_outer ? k : prm.m_outer;
      double yn0, yn1;
      if (omem == 1) {
        yn0 = yq0;
        yn1 = yq1;
      } else {
        const double dq20 = yq0 - oq0, dq21 = yq1 - oq1;
        const double df20 = f0 - of0, df21 = f1 - of1;
        const double G22 = df20 * df20 + df21 * df21, b2 = df20 * f0 + df21 * f1;
        double g1 = 0.0, g2 = 0.0;
        bool two = (omem == 3);
        if (two) {
          const double G11o = odf0 * odf0 + odf1 * odf1;
          const double G12 = odf0 * df20 + odf1 * df21, b1 = odf0 * f0 + odf1 * f1;
          const double tr = G11o + G22;
          two = G11o > 1e-14 * tr;
          if (two) {
            const double L11 = sqrt(G11o);
            const double L21 = G12 / L11;
            const double p2 = G22 - L21 * L21;
            two = p2 > 1e-14 * tr;
            if (two) {
              const double L22 = sqrt(p2);
              const double z1 = b1 / L11;
              const double z2 = (b2 - L21 * z1) / L22;
              g2 = z2 / L22;
              g1 = (z1 - L21 * g2) / L11;
            }
          }
        }
        if (!two) {
          g1 = 0.0;
          if (G22 > 1e-14 * G22) {
            const double L = sqrt(G22);
            g2 = (b2 / L) / L;
          } else {
            g2 = 0.0;
          }
        }
        yn0 = yq0 - g2 * dq20;
        yn1 = yq1 - g2 * dq21;
        if (omem == 3) {
          yn0 -= g1 * odq0;
          yn1 -= g1 * odq1;
        }
        odq0 = dq20;
        odq1 = dq21;
        odf0 = df20;
        odf1 = df21;
      }
      oq0 = yq0;
      oq1 = yq1;
      of0 = f0;
      of1 = f1;
      if (!isfinite(yn0) || !isfinite(yn1)) {
        status = NMC_STATUS_NONFINITE;
        fatal = true;
        break;
      }
      // Algorithm outerConverged: componentwise against y*
      const bool oc = fabs(yn0 - y0) <= prm.tol_outer * fabs(ye_st) && fabs(yn1 - y1) <= prm.tol_outer * fabs(e_st);
      y0 = yn0;
      y1 = yn1;
      if (oc) {
        outer_conv = true;
        break;
      }
    }
    if (k > prm.max_outer) k = prm.max_outer;
    if (!fatal) {
      if (!outer_conv) status = NMC_STATUS_MAX_OUTER;
      else if (inner_failed) status = NMC_STATUS_MAX_INNER;
    }

    // ---- outputs --------------------------------------------------------
    double ye_out = ye_st, e_out = e_st, T_out = T_last;
    if (!prm.fixed_matter) {
      // final matter state from the final moments (exact lepton-number and
      // energy balance)
      double mv[2] = {0.0, 0.0}, s0[2], s1[2];
      if (h == 0) {
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const double dd = M[t] - S.mst[t][lane];
          mv[0] += md->g[t] * w2q * dd;
          mv[1] += md->mult[t] * w3q * dd;
        }
      }
      half_sums<2>(mv, s0, s1, red, redout);
      const double K = md->kcoup / rho;
      ye_out = ye_st - K * s0[0];
      e_out = e_st - K * s0[1];
      T_out = (e_out - md->eos_b * pow(ye_out, 4.0 / 3.0) * r3) / (md->eos_a * (1.0 + ye_out));
    }
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      if (h == 0) a.D[base + t * NQ + q] = M[t];
      else a.I[base + t * NQ + q] = M[t];
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

template <int NS, int NQ>
__global__ __launch_bounds__(kLanes, 2) void fwd_kernel(FwdArgs a) {
  __shared__ WaveLds<NS> S;
  if (a.queue) {
    // persistent grid: pop chunks of points from the work queue until drained
    for (;;) {
      int b = 0;
      if (threadIdx.x == 0) b = atomicAdd(a.queue, a.chunk);
      const int64_t b0 = __builtin_amdgcn_readfirstlane(b);
      if (b0 >= a.P) break;
      const int64_t end = b0 + a.chunk < a.P ? b0 + a.chunk : a.P;
      for (int64_t p = b0; p < end; ++p) PointSolver<NS, NQ>::solve(a, p, S);
    }
  } else {
    const int64_t b0 = (int64_t)blockIdx.x * a.chunk;
    const int64_t end = b0 + a.chunk < a.P ? b0 + a.chunk : a.P;
    for (int64_t p = b0; p < end; ++p) PointSolver<NS, NQ>::solve(a, p, S);
  }
}

__global__ void reset_counter_kernel(int* c) {
  if (threadIdx.x == 0) *c = 0;
}

template <int NS, int NQ>
hipError_t launch_fwd_t(const FwdArgs& a, const nmc_launch& L, int num_cu, hipStream_t s) {
  auto kern = fwd_kernel<NS, NQ>;
  int64_t grid;
  if (a.queue) {
    int bpc = L.blocks_per_cu;
    if (bpc <= 0) {
      // occupancy of this kernel variant, queried once per process
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

hipError_t launch_reset_counter(int* counter, hipStream_t s) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, counter);
  return hipGetLastError();
}

hipError_t launch_forward(const FwdArgs& a, int nq, int ns, const nmc_launch& L, int num_cu, hipStream_t s) {
  if (nq == 32) {
    switch (ns) {
      case 1: return launch_fwd_t<1, 32>(a, L, num_cu, s);
      case 2: return launch_fwd_t<2, 32>(a, L, num_cu, s);
      case 3: return launch_fwd_t<3, 32>(a, L, num_cu, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace nmc
