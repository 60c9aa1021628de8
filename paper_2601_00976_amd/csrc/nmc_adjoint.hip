// Adjoint (implicit-function-theorem) kernels of the coupling solve on CDNA4.
//
// At the converged state x = (D, Ye, e) of a point the reduced residual
//   R_D = D (1 + dtau chi) - D* - dtau eta          (Eq. implicitMomentsNodal, v = 0)
//   R_Y = Ye - Ye* + K sum_s g_s sum_q W_q (D - D*)  (Eq. implicitFluidNodal)
//   R_e = e  - e*  + K sum_s d_s sum_q W3_q (D - D*)
// vanishes (the flux moments drop out: nothing depends on I when v = 0).
// With J = dR/dx = [[A, B], [C, 1]] (A: moment block, B: the Ye / e columns
// through T(e, Ye) and mu(Ye, T), C: the conservation rows) the transposed
// system J^T lambda = dL/dx is solved by a Schur complement on the two matter
// unknowns:
//   Z = A^-T C^T,  (1 - B^T Z) lambda_m = (gY, -gE),  lambda_D = -Z lambda_m,
// and dL/dtheta_j = -lambda_D^T dR_D/dtheta_j for theta = (s_1..s_nq, a_nes,
// a_pair), L = gE (e* - e) + gY (Ye - Ye*).
//
// A is block diagonal over pair-coupled species: NES couples the nodes of one
// species, pair processes couple a species with its partner, so with species
// in id order the blocks are (nu_e, anti-nu_e) of size 64 and nu_x of size
// 32.  Each block is factorised in registers, one wavefront per point: lane r
// holds row r of A^T (column r of A) and the two right-hand sides.  Block
// Gaussian elimination with 2 x 2 pivot blocks runs without row exchanges
// (the W-scaled columns of A are strictly diagonally dominant), broadcasting
// the two pivot rows of each step through LDS; block back substitution
// follows.  Per-point terms go to a
// (P, nq + 2) array and are summed over points by a fixed-order two-stage
// reduction.
#include "nmc_wave.h"

namespace nmc {
namespace {

constexpr int NQ = 32;

template <int NS>
struct AdjLds {
  ModelLds m;
  SplitExp E;
  double tb[32 * kTileStride];  // pair factors b = exp(-|e_q - e_p| / (2T)) of the kernels
  double D[NS][NQ];
  // per-row results, row = (species, node)
  double chi[NS][NQ];         // total opacity chi of the row
  double b0[NS][NQ], b1[NS][NQ];  // dR_D / dYe, dR_D / de
  double da[NS][NQ], dp[NS][NQ], ds[NS][NQ];  // dR_D / d a_nes, / d a_pair, / d s_q
  double z0[NS][NQ], z1[NS][NQ];  // Z = A^-T C^T
  alignas(16) double prow[2 * (2 * NQ + 2)];  // pivot-row buffers of the block factorisation
};

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const uint32_t lo = __builtin_amdgcn_readlane((int)lo32(v), lane);
  const uint32_t hi = __builtin_amdgcn_readlane((int)hi32(v), lane);
  return mk64(lo, hi);
}

// ds_write2_b64 of (a, b) to LDS bytes base + 8 J and base + 8 (J + 1)
template <int J>
__device__ __forceinline__ void lds_write2_f64(uint32_t base, double a, double b) {
  static_assert(J + 1 <= 255, "ds_write2_b64 offsets are 8-bit");
  asm volatile("ds_write2_b64 %0, %1, %2 offset0:%3 offset1:%4" : : "v"(base), "v"(a), "v"(b), "i"(J), "i"(J + 1)
               : "memory");
}

// R[J + i] += bcast_{L + i}(u) b + bcast_{L + i}(w) a for i = 0..3, the
// column values u, w taken from lane L + i of the lane's 16-lane row
// (v_fmac_f64_dpp row_newbcast): the b term first, then the a term, each one
// rounding.  The leading s_nop covers a VALU write of u or w just before.
template <int L>
__device__ __forceinline__ void elim_cols4(double& r0, double& r1, double& r2, double& r3, double u, double w,
                                           double a, double b) {
  asm volatile(
      "s_nop 1\n"
      "v_fmac_f64_dpp %0, %5, %7 row_newbcast:%8 row_mask:0xf bank_mask:0xf\n"
      "v_fmac_f64_dpp %1, %5, %7 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n"
      "v_fmac_f64_dpp %2, %5, %7 row_newbcast:%10 row_mask:0xf bank_mask:0xf\n"
      "v_fmac_f64_dpp %3, %5, %7 row_newbcast:%11 row_mask:0xf bank_mask:0xf\n"
      "v_fmac_f64_dpp %0, %4, %6 row_newbcast:%8 row_mask:0xf bank_mask:0xf\n"
      "v_fmac_f64_dpp %1, %4, %6 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n"
      "v_fmac_f64_dpp %2, %4, %6 row_newbcast:%10 row_mask:0xf bank_mask:0xf\n"
      "v_fmac_f64_dpp %3, %4, %6 row_newbcast:%11 row_mask:0xf bank_mask:0xf\n"
      : "+v"(r0), "+v"(r1), "+v"(r2), "+v"(r3)
      : "v"(u), "v"(w), "v"(a), "v"(b), "i"(L), "i"(L + 1), "i"(L + 2), "i"(L + 3));
}

// Solves A^T z = c for one diagonal block of size N (lanes 0..N-1 active):
// lane r enters with R = row r of A^T and c = (c0, c1) its right-hand sides
// and leaves with (z0, z1) = entry r of the two solutions.  Returns false if
// a pivot block was singular or non-finite, detected as a non-finite
// solution entry (such a block turns the multipliers or the final quotients
// into inf or NaN, which propagate into z).
//
// Block Gauss-Jordan elimination with 2 x 2 pivot blocks and no row
// exchanges: with D in [0, 1] and non-negative kernels, diag(W) A is strictly
// diagonally dominant by columns (the off-diagonal column sums of the
// W-scaled NES and pair terms equal the kernel part of the diagonal opacity,
// leaving a margin W_p (1 + dtau chi^EmAb_p)), so A^T with its columns scaled
// by W is dominant by rows; elimination without pivoting, Gauss-Jordan
// included, is stable for such matrices, and their diagonal blocks and Schur
// complements stay dominant, so every 2 x 2 pivot block is nonsingular.
// Step k (even) removes columns k and k+1 from every row but k and k+1 (lanes
// k and k+1) with the multipliers [R[k], R[k+1]] B^-1 of the pivot block B.
// The two lanes write their rows (from column k on) and right-hand sides to
// two LDS row buffers; every lane then loads, per group of 16 columns, one
// entry of each pivot row (lane L of a 16-lane row loads column 16 g + L), and
// the update FMAs take column 16 g + L from lane L of the lane's row by DPP
// broadcast.  All lanes run the FMAs (a DPP source lane must be active); the
// pivot rows have zero multipliers, so their entries are unchanged.  The
// update starts at the 4-column block of column k + 2; the columns of that
// block left of k + 2 are updated too: they are eliminated columns or the
// row's own pivot block, which the row keeps in registers when it is
// eliminated, and are never read again.  Rows above the pivot are
// updated by the same instructions as the rows below, so the elimination
// costs no more than a one-sided one, and at the end every pivot pair holds
// only its own block: z = B^-1 c for each pair, from the partner's
// right-hand sides by DPP, with no back substitution.  A single wavefront
// runs the work-group, so its LDS accesses complete in program order and no
// barrier is needed.
template <int N>
__device__ __forceinline__ bool solve_block_transposed(double (&R)[N], double c0, double c1, double& z0,
                                                       double& z1, double* prow_generic) {
  static_assert(N % 16 == 0, "2 x 2 pivot blocks, 16-column groups");
  typedef double f64x2 __attribute__((ext_vector_type(2)));
  typedef __attribute__((address_space(3))) double lds_f64;
  typedef __attribute__((address_space(3))) f64x2 lds_f64x2;
  constexpr int RS = N + 2;  // doubles per row buffer: entries 0..N-1, right-hand sides at N, N+1
  const int lane = opaque((int)threadIdx.x);
  const int col = lane & 15;
  // the lane's pivot block, kept when its pair is eliminated: lane k (even)
  // solves z_k = (a11 c_k - a01 c_k+1) / det, lane k+1 z_k+1 = (a00 c_k+1 -
  // a10 c_k) / det, so each keeps its (x, y) = (a11, a01) or (a00, a10)
  double bx = 0.0, by = 0.0, brd = 0.0;
  static_for<0, N / 2>([&](auto kk) __attribute__((always_inline)) {
    constexpr int k = 2 * decltype(kk)::value;
    lds_f64* prow = (lds_f64*)prow_generic;
    lds_f64x2* prow2 = (lds_f64x2*)prow;
    // the pivot block B = [[a00, a01], [a10, a11]] (rows k, k+1, columns k, k+1)
    const double a00 = readlane_f64(R[k], k), a01 = readlane_f64(R[k + 1], k);
    const double a10 = readlane_f64(R[k], k + 1), a11 = readlane_f64(R[k + 1], k + 1);
    if (lane == k || lane == k + 1) {
      // rows k and k+1 (columns k..N-1) to their buffers: ds_write2_b64 from
      // one base register per lane with 8-byte-unit offsets
      const uint32_t base = (uint32_t)(uintptr_t)prow + (uint32_t)((lane - k) * RS * 8);
      static_for<0, (N - k) / 2>([&](auto ii) __attribute__((always_inline)) {
        constexpr int j = k + 2 * decltype(ii)::value;
        lds_write2_f64<j>(base, R[j], R[j + 1]);
      });
      lds_write2_f64<N>(base, c0, c1);
    }
    const double rdet = rcp_nr(a00 * a11 - a01 * a10);
    if (lane == k) {
      bx = a11;
      by = a01;
      brd = rdet;
    }
    if (lane == k + 1) {
      bx = a00;
      by = a10;
      brd = rdet;
    }
    const bool other = lane != k && lane != k + 1;
    const double nl0 = other ? -((R[k] * a11 - R[k + 1] * a10) * rdet) : 0.0;
    const double nl1 = other ? -((R[k + 1] * a00 - R[k] * a01) * rdet) : 0.0;
    static_for<(k + 2) / 16, N / 16>([&](auto gg) __attribute__((always_inline)) {
      constexpr int g = decltype(gg)::value;
      const double u = prow[16 * g + col], w = prow[RS + 16 * g + col];
      // in the group of column k + 2, the 4-column blocks left of it hold
      // only dead entries (eliminated columns, or the pivot blocks kept in
      // registers): skipped
      constexpr int q0 = g == (k + 2) / 16 ? ((k + 2) % 16) / 4 : 0;
      static_for<q0, 4>([&](auto qq) __attribute__((always_inline)) {
        constexpr int j = 16 * g + 4 * decltype(qq)::value;
        elim_cols4<j % 16>(R[j], R[j + 1], R[j + 2], R[j + 3], u, w, nl0, nl1);
      });
    });
    const f64x2 cu = prow2[N / 2], cv = prow2[(RS + N) / 2];
    c0 = __builtin_fma(nl0, cu.x, __builtin_fma(nl1, cv.x, c0));
    c1 = __builtin_fma(nl0, cu.y, __builtin_fma(nl1, cv.y, c1));
  });
  // each pivot pair (k, k+1) now solves its own block; the partner lane is
  // lane ^ 1 (quad_perm [1,0,3,2])
  const double o0 = dpp<0xB1>(c0), o1 = dpp<0xB1>(c1);
  z0 = (bx * c0 - by * o0) * brd;
  z1 = (bx * c1 - by * o1) * brd;
  // a singular or non-finite pivot block makes some entry of the solution
  // non-finite
  return __builtin_amdgcn_ballot_w64(lane < N && !(isfinite(z0) && isfinite(z1))) == 0;
}

template <int NS>
struct PointAdjoint {
  // Rows of A^T of one block of species [S0, S0 + NB): lane r = 32 si + p
  // holds column (S0 + si, p) of A.  Entries (Jacobian of R_D):
  //   same species (NES):  -dtau W_p [(1 - D_q) Phi_in[q][p] + D_q Phi_out[q][p]]
  //   partner species:     +dtau W_p [D_q Phi_ann[q][p] + (1 - D_q) Phi_pro[q][p]]
  //   diagonal:            1 + dtau chi_(s, p)
  // with the kernels at the point's amplitudes; Phi_out[q][p] = Phi_in[p][q].
  // The kernels are formed from the pair factors b: with c = rho e_q e_p,
  // Phi_in[q][p] = c (p > q ? b : b^3), Phi_out[q][p] = c (q > p ? b : b^3),
  // Phi_ann = c b^2, Phi_pro = c G_max(q, p).
  template <int S0, int NB>
  __device__ __forceinline__ static void block_rows(AdjLds<NS>& S, double dtau, double rho, double a_nes,
                                                    double a_pair, double (&R)[32 * NB]) {
    constexpr int ST = kTileStride;
    const int lane = opaque((int)threadIdx.x);  // laundered: lane-derived indices are not hoisted out of the point loop
    const int h = lane >> 5, p = lane & 31;
    const int si = NB == 2 ? h : 0;
    const int sp = S0 + si;  // species of this lane's column
    const double rwe = rho * S.m.w2[p] * S.m.eps[p];
    const double dwn = dtau * a_nes * rwe, dwp = dtau * a_pair * rwe;
    const double diag = 1.0 + dtau * S.chi[sp][p];
    const double Gp = S.E.G[p];
    // the moments are re-read here (an opaque zero offset keeps the compiler
    // from carrying the values loaded for the contractions through the
    // factorisation of the previous block in registers)
    int z = 0;
    asm volatile("" : "+s"(z));
    const double* __restrict__ Db = &S.D[S0][z];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double eq = S.m.eps[q], Gq = S.E.G[q];
      const double b = S.tb[q * ST + p], b2 = b * b, b3 = b2 * b;
      const double fin = p > q ? b : b3, fout = q > p ? b : b3;
      const double fpro = fmin(Gq, Gp);  // G of the higher node: G falls with energy
      const double nq = -dwn * eq, pq = dwp * eq;
      // row (s, q), column (sp, p): NES if s = sp, pair if s is sp's partner
      auto nes = [&](double d) { return nq * __builtin_fma(d, fout - fin, fin); };
      auto pair = [&](double d) { return pq * __builtin_fma(d, b2 - fpro, fpro); };
      const double dg = q == p ? diag : 0.0;
      if constexpr (NB == 2) {
        // d is the moment of the row's species: the lane's own species for
        // its NES row, the partner's for its pair row
        const double d0 = Db[q], d1 = Db[NQ + q];
        const double vn = nes(si == 0 ? d0 : d1) + dg, vp = pair(si == 0 ? d1 : d0);
        R[q] = si == 0 ? vn : vp;
        R[32 + q] = si == 0 ? vp : vn;
      } else {
        const double d = Db[q];
        R[q] = nes(d) + pair(d) + dg;
      }
      if ((q & 3) == 3) asm volatile("" ::: "memory");
    }
  }

  template <int S0, int NB>
  __device__ __forceinline__ static bool block_solve(AdjLds<NS>& S, const DevModel* md, double dtau, double rho,
                                                     double a_nes, double a_pair, double K) {
    double R[32 * NB];
    block_rows<S0, NB>(S, dtau, rho, a_nes, a_pair, R);
    const int lane = opaque((int)threadIdx.x);  // laundered: lane-derived indices are not hoisted out of the point loop
    const int h = lane >> 5, p = lane & 31;
    const int sp = S0 + (NB == 2 ? h : 0);
    // right-hand sides: column (sp, p) of the conservation rows C
    const double c0 = K * md->ig[sp] * S.m.w2[p];
    const double c1 = K * md->imult[sp] * S.m.w3[p];
    double z0, z1;
    const bool ok = solve_block_transposed<32 * NB>(R, c0, c1, z0, z1, S.prow);
    if (lane < 32 * NB) {
      S.z0[sp][p] = z0;
      S.z1[sp][p] = z1;
    }
    __syncthreads();
    return ok;
  }

  __device__ static void run(const AdjArgs& a, int64_t pt, AdjLds<NS>& S) {
    constexpr int ST = kTileStride;
    constexpr int NT = NQ + 2;
    const DevModel* __restrict__ md = a.mdl;
    const int lane = opaque((int)threadIdx.x);  // laundered: lane-derived indices are not hoisted out of the point loop
    const int h = lane >> 5, q = lane & 31;
    double* gout = a.grad_pp + pt * NT;
    if (a.status[pt] != NMC_STATUS_OK || a.n_outer[pt] == 0) {
      // skipped or failed points contribute nothing
      if (lane < NT) gout[lane] = 0.0;
      return;
    }
    const int64_t base = pt * (int64_t)(NS * NQ);
    if (lane < 32) {
#pragma unroll
      for (int t = 0; t < NS; ++t) S.D[t][lane] = a.D[base + md->ext[t] * NQ + lane];
    }
    const double rho = a.rho11[pt], ye = a.ye[pt], e = a.e[pt];
    const double chi0 = a.chi0 ? a.chi0[pt] : md->chi_ref * rho;
    const double dtau = a.dtau;
    // EOS and its derivatives
    const double r3 = cbrt(rho);
    const double ia = 1.0 / (md->eos_a * (1.0 + ye));
    const double T = (e - md->eos_b * ye43(ye) * r3) * ia;
    const double mu = md->mu_a * (ye - md->mu_ye0) * r3 + md->mu_b * log(T / md->mu_t0);
    const double invT = 1.0 / T;
    const double dT_de = ia;
    const double dT_dye = -(4.0 / 3.0) * md->eos_b * cbrt(ye) * r3 * ia - T / (1.0 + ye);
    const double dmu_dye = md->mu_a * r3 + md->mu_b * invT * dT_dye;
    const double dmu_de = md->mu_b * invT * dT_de;
    const double K = md->kcoup / rho;
    const unsigned flags = md->flags;
    const double a_nes = (flags & NMC_NES) ? S.m.theta[NQ] : 0.0;
    const double a_pair = (flags & NMC_PAIR) ? S.m.theta[NQ + 1] : 0.0;
    split_exp_prepare(S.m, invT, S.E);

    // ---- per-row contractions with unit-amplitude kernels (A = rho11) ----
    // group 0: species h (ns >= 2) or 0 (ns = 1, lanes < 32); group 1: nu_x (ns = 3, lanes < 32)
    constexpr int NG = NS == 3 ? 2 : 1;
    int sg[NG], sbg[NG];
    bool on[NG];
    sg[0] = NS >= 2 ? h : 0;
    on[0] = NS >= 2 || lane < 32;
    if constexpr (NG == 2) {
      sg[1] = 2;
      on[1] = lane < 32;
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) sbg[g] = NS == 3 ? (sg[g] < 2 ? 1 - sg[g] : 2) : (NS == 2 ? 1 - sg[g] : 0);
    const double eq = S.m.eps[q];
    // en, on (NES in / out), an, ep (pair ann / pro) and their temperature
    // derivatives times T^2
    double en[NG], onn[NG], an[NG], ep[NG], dn[NG], dout[NG], dan[NG], dpr[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) en[g] = onn[g] = an[g] = ep[g] = dn[g] = dout[g] = dan[g] = dpr[g] = 0.0;
    fill_tile<kTilePairFactor>(S.m, S.E, 1.0, h, q, S.tb);
    __syncthreads();
    // the kernels without their common factor rho e_q (applied to the sums)
    const double Gq = S.E.G[q];
#pragma unroll 2
    for (int p = 0; p < NQ; ++p) {
      const double epp = S.m.eps[p], we = S.m.w2[p] * epp, dl = eq - epp, adl = fabs(dl);
      const double b = S.tb[q * ST + p], b2 = b * b, b3 = b2 * b;
      const bool up = p > q;
      const double tin = we * (up ? b : b3), tout = we * (up ? b3 : b);
      const double tann = we * b2, tpro = we * fmin(S.E.G[p], Gq);
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const double d = S.D[sg[g]][p], db = S.D[sbg[g]][p];
        en[g] = __builtin_fma(tin, d, en[g]);
        dn[g] = __builtin_fma(tin * (adl + 0.5 * dl), d, dn[g]);
        onn[g] = __builtin_fma(tout, 1.0 - d, onn[g]);
        dout[g] = __builtin_fma(tout * (adl - 0.5 * dl), 1.0 - d, dout[g]);
        an[g] = __builtin_fma(tann, db, an[g]);
        dan[g] = __builtin_fma(tann * adl, db, dan[g]);
        ep[g] = __builtin_fma(tpro, 1.0 - db, ep[g]);
        dpr[g] = __builtin_fma(tpro * (adl + eq + epp), 1.0 - db, dpr[g]);
      }
    }
    {
      const double sc = rho * eq;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        en[g] *= sc;
        dn[g] *= sc;
        onn[g] *= sc;
        dout[g] *= sc;
        an[g] *= sc;
        dan[g] *= sc;
        ep[g] *= sc;
        dpr[g] *= sc;
      }
    }
    // ---- per-row Jacobian pieces ----------------------------------------
    {
      const double shape = chi0 * S.m.shape[q];
      const double iT2 = invT * invT;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        if (!on[g]) continue;
        const int s = sg[g];
        const double chia = (flags & NMC_EMAB) ? md->iemab[s] * S.m.theta[q] * shape : 0.0;
        const double x = (eq - md->imusign[s] * mu) * invT;
        const double ex = exp(-fabs(x));
        const double r = 1.0 / (1.0 + ex);
        const double f = x > 0.0 ? ex * r : r;   // Fermi-Dirac D_eq
        const double fc = x > 0.0 ? r : ex * r;  // 1 - D_eq
        const double ddeq_dT = f * fc * x * invT;
        const double ddeq_dmu = f * fc * md->imusign[s] * invT;
        const double Dq = S.D[s][q];
        const double chi = chia + a_nes * (en[g] + onn[g]) + a_pair * (ep[g] + an[g]);
        const double deta_dT = chia * ddeq_dT + (a_nes * dn[g] + a_pair * dpr[g]) * iT2;
        const double dchi_dT = (a_nes * (dn[g] + dout[g]) + a_pair * (dpr[g] + dan[g])) * iT2;
        const double dR_dT = dtau * (Dq * dchi_dT - deta_dT);
        const double dR_dmu = -dtau * chia * ddeq_dmu;
        S.chi[s][q] = chi;
        S.b0[s][q] = dR_dT * dT_dye + dR_dmu * dmu_dye;
        S.b1[s][q] = dR_dT * dT_de + dR_dmu * dmu_de;
        S.da[s][q] = (flags & NMC_NES) ? dtau * (Dq * (en[g] + onn[g]) - en[g]) : 0.0;
        S.dp[s][q] = (flags & NMC_PAIR) ? dtau * (Dq * (ep[g] + an[g]) - ep[g]) : 0.0;
        S.ds[s][q] = (flags & NMC_EMAB) ? dtau * shape * md->iemab[s] * (Dq - f) : 0.0;
      }
    }
    __syncthreads();

    // ---- Z = A^-T C^T, block by block ------------------------------------
    // (kernels at unit amplitude a = 1, i.e. A = rho11, scaled by a_nes, a_pair)
    bool ok;
    if constexpr (NS == 1) {
      ok = block_solve<0, 1>(S, md, dtau, rho, a_nes, a_pair, K);
    } else {
      ok = block_solve<0, 2>(S, md, dtau, rho, a_nes, a_pair, K);
      if constexpr (NS == 3) ok = block_solve<2, 1>(S, md, dtau, rho, a_nes, a_pair, K) && ok;
    }

    // ---- Schur complement on (Ye, e), multipliers and gradient ------------
    double v4[4] = {0.0, 0.0, 0.0, 0.0};
    if (lane < 32) {
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        v4[0] += S.b0[t][q] * S.z0[t][q];
        v4[1] += S.b0[t][q] * S.z1[t][q];
        v4[2] += S.b1[t][q] * S.z0[t][q];
        v4[3] += S.b1[t][q] * S.z1[t][q];
      }
    }
    double bz[4];
    wave_sums4(v4, bz);
    const double s00 = 1.0 - bz[0], s01 = -bz[1], s10 = -bz[2], s11 = 1.0 - bz[3];
    const double g_e = a.gbar[2 * pt], g_y = a.gbar[2 * pt + 1];
    const double r0 = g_y, r1 = -g_e;  // dL/dYe, dL/de
    const double idet = 1.0 / (s00 * s11 - s01 * s10);
    const double l0 = (s11 * r0 - s01 * r1) * idet;
    const double l1 = (s00 * r1 - s10 * r0) * idet;
    double gq = 0.0, v2[4] = {0.0, 0.0, 0.0, 0.0};
    if (lane < 32) {
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const double lam = -(S.z0[t][q] * l0 + S.z1[t][q] * l1);
        gq -= lam * S.ds[t][q];
        v2[0] -= lam * S.da[t][q];
        v2[1] -= lam * S.dp[t][q];
      }
    }
    double gs[4];
    wave_sums4(v2, gs);
    const double nan = __builtin_nan("");
    if (lane < 32) gout[lane] = ok ? gq : nan;
    if (lane == 32) gout[NQ] = ok ? gs[0] : nan;
    if (lane == 33) gout[NQ + 1] = ok ? gs[1] : nan;
    __syncthreads();
  }
};

template <int NS>
__global__ __launch_bounds__(kLanes) void adj_kernel(AdjArgs a) {
  __shared__ AdjLds<NS> S;
  load_model(a.mdl, a.theta, S.m);
  for (int64_t p = blockIdx.x; p < a.P; p += gridDim.x) PointAdjoint<NS>::run(a, p, S);
}

// Column sums of a (P, ncol) row-major array in a fixed order: block b sums
// its contiguous range of rows, then one block adds the block partials in
// order into out (accumulating).
__global__ void reduce_stage1(const double* __restrict__ x, int64_t P, int ncol, int64_t rows_per_block,
                              double* __restrict__ partial) {
  const int c = threadIdx.x;
  if (c >= ncol) return;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < P ? r0 + rows_per_block : P;
  double s = 0.0;
  for (int64_t r = r0; r < r1; ++r) s += x[r * ncol + c];
  partial[(int64_t)blockIdx.x * ncol + c] = s;
}

__global__ __launch_bounds__(256) void reduce_stage2(const double* __restrict__ partial, int nblk, int ncol,
                                                     double* __restrict__ out) {
  // per column: thread t sums partials t, t + 256, ... in order, then a
  // fixed-shape tree over the 256 threads
  __shared__ double red[256];
  const int t = threadIdx.x;
  for (int c = 0; c < ncol; ++c) {
    double s = 0.0;
    for (int b = t; b < nblk; b += 256) s += partial[(int64_t)b * ncol + c];
    red[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    if (t == 0) out[c] += red[0];
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_adjoint(const AdjArgs& a, int nq, int ns, int num_cu, hipStream_t s) {
  if (nq != NQ || ns < 1 || ns > 3) return hipErrorInvalidValue;
  if (a.P == 0) return hipSuccess;
  const int64_t want = (int64_t)num_cu * 16;
  const unsigned grid = (unsigned)(a.P < want ? a.P : want);
  switch (ns) {
    case 1: hipLaunchKernelGGL(adj_kernel<1>, dim3(grid), dim3(kLanes), 0, s, a); break;
    case 2: hipLaunchKernelGGL(adj_kernel<2>, dim3(grid), dim3(kLanes), 0, s, a); break;
    default: hipLaunchKernelGGL(adj_kernel<3>, dim3(grid), dim3(kLanes), 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_reduce_columns(const double* x, int64_t P, int ncol, double* partial, double* out,
                                 hipStream_t s) {
  if (P == 0) return hipSuccess;
  if (ncol > 256) return hipErrorInvalidValue;
  const int64_t nblk = P < kReduceBlocks ? P : kReduceBlocks;
  const int64_t rows = (P + nblk - 1) / nblk;
  const int64_t used = (P + rows - 1) / rows;
  hipLaunchKernelGGL(reduce_stage1, dim3((unsigned)used), dim3(256), 0, s, x, P, ncol, rows, partial);
  hipLaunchKernelGGL(reduce_stage2, dim3(1), dim3(256), 0, s, partial, (int)used, ncol, out);
  return hipGetLastError();
}

}  // namespace nmc
