// Building blocks of the two-points-per-wavefront solve kernels (CDNA4): the
// lane half of a wave solves one point and lane q of the half owns node q of
// every species.  Half-wave reductions, the pair-factor tile of a point, and
// the rate contraction over the point's 32 columns broadcast by DPP
// row_newbcast (Eqs. nesRatesNodal, pairRatesNodal).
#pragma once

#include "nmc_wave.h"

namespace nmc {
namespace pairk {

constexpr int NQP = 32;
// widest exponent range (powers of two of exp(-e / (2T)) over the grid) of
// the symmetric contraction: its scaled vectors and row factors then stay
// within 2^(+-(kSymBits / 2 + 1)), far from overflow
constexpr int kSymBits = 1800;
// widest exponent range of g for which a lane forms its row of the
// symmetric core directly from the squared scaled factors h = g^2 and 1 / h
// (within 2^(+-(kDirectBits + 4)), inside the normal range)
constexpr int kDirectBits = 1000;

// Row q of the symmetric core B2(q, j) = exp(-|e_q - e_j| / T), q this
// lane's node, from the scaled h = exp(-e / T) 2^2c of every node of the
// point and their reciprocals, held in registers: after swap16, H[g] and
// RH[g] carry nodes [16 g, 16 g + 16) in every 16-lane row, and column j is
// taken from lane j % 16 of the row by DPP broadcast.  Of the two
// orientations h_j / h_q and h_q / h_j the smaller is B2 (the other is its
// reciprocal, or overflows to +inf).  The diagonal comes out as h_q / h_q,
// one to within two roundings.
__device__ __forceinline__ void direct_row_regs(double hq, double rhq, double (&B)[32]) {
  double H[2], RH[2];
  swap16(hq, H[0], H[1]);
  swap16(rhq, RH[0], RH[1]);
  static_for<0, 32>([&](auto jj) __attribute__((always_inline)) {
    constexpr int j = decltype(jj)::value;
    B[j] = min_f64(row_bcast<j % 16>(H[j / 16]) * rhq, hq * row_bcast<j % 16>(RH[j / 16]));
  });
}

// Sums over the lane's half-wave of 2K values, in every lane of the half:
// rows (0, 2) carry slot k, rows (1, 3) slot K + k, then a row butterfly and
// a row swap.  The K chains advance stage by stage.  Fixed order.
template <int K>
__device__ __forceinline__ void half_own_sums(const double (&v)[2 * K], double (&s)[2 * K]) {
  double r[K];
#pragma unroll
  for (int k = 0; k < K; ++k) r[k] = halve16(v[k], v[K + k]);
#pragma unroll
  for (int k = 0; k < K; ++k) r[k] += dpp<0xB1>(r[k]);   // quad_perm [1,0,3,2]
#pragma unroll
  for (int k = 0; k < K; ++k) r[k] += dpp<0x4E>(r[k]);   // quad_perm [2,3,0,1]
#pragma unroll
  for (int k = 0; k < K; ++k) r[k] += dpp<0x141>(r[k]);  // row_half_mirror
#pragma unroll
  for (int k = 0; k < K; ++k) r[k] += dpp<0x140>(r[k]);  // row_mirror
#pragma unroll
  for (int k = 0; k < K; ++k) swap16(r[k], s[k], s[K + k]);
}


// The value of species class c (spread_class) from per-species values s[t]
// held in every lane; zero beyond NS.
template <int NS, int N>
__device__ __forceinline__ double class_pick(const double (&s)[N], int c) {
  static_assert(N >= NS, "one value per species");
  double r = 0.0;
#pragma unroll
  for (int t = 0; t < NS; ++t) r = c == t ? s[t] : r;
  return r;
}

// Species class of a lane for the spread sums below: c = 2 r + m with r the
// row of the lane within its half and m = 1 for lanes 8..15 of the row.
__device__ __forceinline__ int spread_class(int lane) { return ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1); }

// One value per species folded to its lane class (spread_class): the rows
// of a half split the species pairs (0, 1) and (2, 3), and row_mirror folds
// the pairs apart.  Species at or beyond NS count as zero.
template <int NS>
__device__ __forceinline__ double species_fold(const double (&v)[NS]) {
  double p[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) p[c] = c < NS ? v[c < NS ? c : 0] : 0.0;
  return fold_pair<0x140, 0x3>(halve16(p[0], p[2]), halve16(p[1], p[3]));
}

// Sums over the half-wave of the inner convergence test, spread over its
// lanes instead of copied into all of them: lane class c (spread_class)
// holds species c, or zeros where c >= NS.  Terms: dm[m] the squared change
// of owned moment m of each species (M of them, M even), xn the squared new
// D.  On return y[j] holds moment 2j's sum in lanes with bit 2 clear and
// moment 2j + 1's in the others (row_half_mirror folds each pair), and n the
// sum of xn; all over the half's 32 nodes.  Fixed order; every lane of a
// class and bank pair holds the same bits.
template <int NS, int M>
__device__ __forceinline__ void spread_conv_sums(const double (&dm)[M][NS], const double (&xn)[NS],
                                                 double (&y)[M / 2], double& n) {
  static_assert(M % 2 == 0, "moments are folded in pairs");
  double f[M];
#pragma unroll
  for (int m = 0; m < M; ++m) f[m] = species_fold<NS>(dm[m]);
  double x = species_fold<NS>(xn);
#pragma unroll
  for (int j = 0; j < M / 2; ++j) y[j] = fold_pair<0x141, 0x5>(f[2 * j], f[2 * j + 1]);  // lanes 0..3, 8..11 keep 2j
  x += dpp<0x141>(x);
#pragma unroll
  for (int j = 0; j < M / 2; ++j) y[j] += dpp<0xB1>(y[j]);  // quad_perm [1,0,3,2]
  x += dpp<0xB1>(x);
#pragma unroll
  for (int j = 0; j < M / 2; ++j) y[j] += dpp<0x4E>(y[j]);  // quad_perm [2,3,0,1]
  x += dpp<0x4E>(x);
  n = x;
}

// Four sums over the half-wave, in every lane of the half: folded pairwise
// by row_mirror and row_half_mirror (lanes 0..3 of a row carry v0, 4..7 v2,
// 8..11 v1, 12..15 v3), two quad stages, the half's two rows added, and each
// sum broadcast from its bank.  Fixed order.
__device__ __forceinline__ void half_sums4(const double (&v)[4], double (&s)[4]) {
  const double x01 = fold_pair<0x140, 0x3>(v[0], v[1]);
  const double x23 = fold_pair<0x140, 0x3>(v[2], v[3]);
  double z = fold_pair<0x141, 0x5>(x01, x23);
  z += dpp<0xB1>(z);
  z += dpp<0x4E>(z);
  z = halve16(z, z);
  s[0] = row_bcast<0>(z);
  s[1] = row_bcast<8>(z);
  s[2] = row_bcast<4>(z);
  s[3] = row_bcast<12>(z);
}

// max(a, -b) of two non-NaN values as one v_max_f64 with a negated operand
__device__ __forceinline__ double max_neg_f64(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, -%2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Pair factors of one point into its 32 x 32 tile T (row-major).  SYM: the
// symmetric core b^2 (diagonal written by the caller).  Otherwise signed:
// for every unordered node pair (lo, hi), T[hi][lo] = +b and T[lo][hi] = -b
// with b = exp(-|e_lo - e_hi| / (2T)) = P_lo R_hi 2^(n_lo - n_hi).  Lane q
// forms the pairs (q, q + d mod 32) for d = 1..15 and, if q < 16, d = 16,
// from its own split (Pq, Rq, nq) and its partner's in LDS.  Of the two
// orientations 2^(x_q - x_j) and 2^(x_j - x_q) the smaller is b (the other
// is its reciprocal, or overflows), so no compare picks the formula; the
// sign goes by whether q is the lower node.
template <bool SYM>
__device__ __forceinline__ void pair_tile_rows(double* __restrict__ T, const double* __restrict__ P2,
                                               const double* __restrict__ R2, const int* __restrict__ n2, int q,
                                               double Pq, double Rq, int nq) {
  constexpr int N = 32;
  double Pp[N / 2], Rp[N / 2];
  int np[N / 2];
#pragma unroll
  for (int d = 1; d <= N / 2; ++d) {  // every partner load first: one LDS round trip
    const int j = (q + d) & (N - 1);
    Pp[d - 1] = P2[j];
    Rp[d - 1] = R2[j];
    np[d - 1] = n2[j];
  }
#pragma unroll
  for (int d = 1; d <= N / 2; ++d) {
    const int j = (q + d) & (N - 1);
    const int e = nq - np[d - 1];
    const double b = min_f64(ldexp(Pq * Rp[d - 1], e), ldexp(Pp[d - 1] * Rq, -e));
    if (d < N / 2 || q < N / 2) {
      if constexpr (SYM) {
        const double b2 = b * b;
        T[j * N + q] = b2;
        T[q * N + j] = b2;
      } else {
        const double sb = q + d < N ? b : -b;  // + where j is the upper node
        T[j * N + q] = sb;
        T[q * N + j] = -sb;
      }
    }
  }
}

// any lane of this lane's half
__device__ __forceinline__ bool half_any(bool b) {
  const uint64_t m = __builtin_amdgcn_ballot_w64(b);
  return ((threadIdx.x >> 5) ? (m >> 32) : (m & 0xffffffffull)) != 0;
}

// One column of the rate contraction: the moment vectors' column L of each
// 16-lane row is broadcast into the FMAs (v_fmac_f64_dpp row_newbcast:L, the
// DPP operand being src0).  eN += Phi_in x_s, oN += Phi_out y_s,
// aP += Phi_ann x_sbar, eP += Phi_ann (h y)_sbar, the last being Phi_pro y_sbar
// by detailed balance once the row sum is scaled by h_q (h = exp(-e / T)).
// The leading s_nop covers the VALU-write to DPP-read distance for registers
// written just before.
template <int NS>
struct ColFmac;

template <>
struct ColFmac<3> {
  template <int L>
  __device__ __forceinline__ static void run(double (&eN)[3], double (&oN)[3], double (&aP)[3], double (&eP)[3],
                                             const double (&x)[3], const double (&y)[3], const double (&hy)[3],
                                             double fi, double fo, double fa) {
    asm volatile(
        "s_nop 1\n"
        "v_fmac_f64_dpp %0, %12, %21 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %13, %21 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %14, %21 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %15, %22 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %4, %16, %22 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %5, %17, %22 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %6, %13, %23 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %7, %12, %23 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %8, %14, %23 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %9, %19, %23 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %10, %18, %23 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %11, %20, %23 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n"
        : "+v"(eN[0]), "+v"(eN[1]), "+v"(eN[2]), "+v"(oN[0]), "+v"(oN[1]), "+v"(oN[2]), "+v"(aP[0]), "+v"(aP[1]),
          "+v"(aP[2]), "+v"(eP[0]), "+v"(eP[1]), "+v"(eP[2])
        : "v"(x[0]), "v"(x[1]), "v"(x[2]), "v"(y[0]), "v"(y[1]), "v"(y[2]), "v"(hy[0]), "v"(hy[1]), "v"(hy[2]),
          "v"(fi), "v"(fo), "v"(fa), "i"(L));
  }
};

template <>
struct ColFmac<2> {
  template <int L>
  __device__ __forceinline__ static void run(double (&eN)[2], double (&oN)[2], double (&aP)[2], double (&eP)[2],
                                             const double (&x)[2], const double (&y)[2], const double (&hy)[2],
                                             double fi, double fo, double fa) {
    asm volatile(
        "s_nop 1\n"
        "v_fmac_f64_dpp %0, %8, %14 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %9, %14 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %10, %15 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %11, %15 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %4, %9, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %5, %8, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %6, %13, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %7, %12, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        : "+v"(eN[0]), "+v"(eN[1]), "+v"(oN[0]), "+v"(oN[1]), "+v"(aP[0]), "+v"(aP[1]), "+v"(eP[0]), "+v"(eP[1])
        : "v"(x[0]), "v"(x[1]), "v"(y[0]), "v"(y[1]), "v"(hy[0]), "v"(hy[1]), "v"(fi), "v"(fo), "v"(fa), "i"(L));
  }
};

template <>
struct ColFmac<1> {
  template <int L>
  __device__ __forceinline__ static void run(double (&eN)[1], double (&oN)[1], double (&aP)[1], double (&eP)[1],
                                             const double (&x)[1], const double (&y)[1], const double (&hy)[1],
                                             double fi, double fo, double fa) {
    asm volatile(
        "s_nop 1\n"
        "v_fmac_f64_dpp %0, %4, %7 row_newbcast:%10 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %5, %8 row_newbcast:%10 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %4, %9 row_newbcast:%10 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %6, %9 row_newbcast:%10 row_mask:0xf bank_mask:0xf\n"
        : "+v"(eN[0]), "+v"(oN[0]), "+v"(aP[0]), "+v"(eP[0])
        : "v"(x[0]), "v"(y[0]), "v"(hy[0]), "v"(fi), "v"(fo), "v"(fa), "i"(L));
  }
};

// Four columns L0 .. L0 + 3 of the rate contraction on the symmetric core
// B2 = b^2 of the kernels (the per-node exponential factors ride on the
// vectors, see the solver): eN += B2 a_s, oN += B2 b_s, aP += B2 c_sbar,
// eP += B2 d_sbar, the vectors' column broadcast into the FMAs
// (row_newbcast) and B2 from VGPRs m0 .. m3.  12 FMAs per column for three
// species and nothing else; one leading s_nop per four columns covers the
// VALU-write to DPP-read distance of the vectors.
template <int NS>
struct ColSym;

template <>
struct ColSym<3> {
  template <int L0>
  __device__ __forceinline__ static void run(double (&eN)[3], double (&oN)[3], double (&aP)[3], double (&eP)[3],
                                             const double (&a)[3], const double (&b)[3], const double (&c)[3],
                                             const double (&d)[3], double m0, double m1, double m2, double m3) {
    asm volatile(
        "s_nop 1\n"
        "v_fmac_f64_dpp %0, %12, %24 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %13, %24 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %14, %24 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %15, %24 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %4, %16, %24 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %5, %17, %24 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %6, %19, %24 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %7, %18, %24 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %8, %20, %24 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %9, %22, %24 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %10, %21, %24 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %11, %23, %24 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %12, %25 row_newbcast:%29 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %13, %25 row_newbcast:%29 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %14, %25 row_newbcast:%29 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %15, %25 row_newbcast:%29 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %4, %16, %25 row_newbcast:%29 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %5, %17, %25 row_newbcast:%29 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %6, %19, %25 row_newbcast:%29 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %7, %18, %25 row_newbcast:%29 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %8, %20, %25 row_newbcast:%29 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %9, %22, %25 row_newbcast:%29 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %10, %21, %25 row_newbcast:%29 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %11, %23, %25 row_newbcast:%29 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %12, %26 row_newbcast:%30 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %13, %26 row_newbcast:%30 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %14, %26 row_newbcast:%30 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %15, %26 row_newbcast:%30 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %4, %16, %26 row_newbcast:%30 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %5, %17, %26 row_newbcast:%30 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %6, %19, %26 row_newbcast:%30 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %7, %18, %26 row_newbcast:%30 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %8, %20, %26 row_newbcast:%30 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %9, %22, %26 row_newbcast:%30 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %10, %21, %26 row_newbcast:%30 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %11, %23, %26 row_newbcast:%30 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %12, %27 row_newbcast:%31 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %13, %27 row_newbcast:%31 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %14, %27 row_newbcast:%31 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %15, %27 row_newbcast:%31 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %4, %16, %27 row_newbcast:%31 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %5, %17, %27 row_newbcast:%31 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %6, %19, %27 row_newbcast:%31 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %7, %18, %27 row_newbcast:%31 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %8, %20, %27 row_newbcast:%31 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %9, %22, %27 row_newbcast:%31 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %10, %21, %27 row_newbcast:%31 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %11, %23, %27 row_newbcast:%31 row_mask:0xf bank_mask:0xf\n"
        : "+v"(eN[0]), "+v"(eN[1]), "+v"(eN[2]), "+v"(oN[0]), "+v"(oN[1]), "+v"(oN[2]), "+v"(aP[0]), "+v"(aP[1]), "+v"(aP[2]), "+v"(eP[0]), "+v"(eP[1]), "+v"(eP[2])
        : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(b[0]), "v"(b[1]), "v"(b[2]), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(d[0]), "v"(d[1]), "v"(d[2]), "v"(m0), "v"(m1), "v"(m2), "v"(m3), "i"(L0 + 0), "i"(L0 + 1), "i"(L0 + 2), "i"(L0 + 3));
  }
};

template <>
struct ColSym<2> {
  template <int L0>
  __device__ __forceinline__ static void run(double (&eN)[2], double (&oN)[2], double (&aP)[2], double (&eP)[2],
                                             const double (&a)[2], const double (&b)[2], const double (&c)[2],
                                             const double (&d)[2], double m0, double m1, double m2, double m3) {
    asm volatile(
        "s_nop 1\n"
        "v_fmac_f64_dpp %0, %8, %16 row_newbcast:%20 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %9, %16 row_newbcast:%20 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %10, %16 row_newbcast:%20 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %11, %16 row_newbcast:%20 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %4, %13, %16 row_newbcast:%20 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %5, %12, %16 row_newbcast:%20 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %6, %15, %16 row_newbcast:%20 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %7, %14, %16 row_newbcast:%20 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %8, %17 row_newbcast:%21 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %9, %17 row_newbcast:%21 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %10, %17 row_newbcast:%21 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %11, %17 row_newbcast:%21 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %4, %13, %17 row_newbcast:%21 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %5, %12, %17 row_newbcast:%21 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %6, %15, %17 row_newbcast:%21 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %7, %14, %17 row_newbcast:%21 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %8, %18 row_newbcast:%22 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %9, %18 row_newbcast:%22 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %10, %18 row_newbcast:%22 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %11, %18 row_newbcast:%22 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %4, %13, %18 row_newbcast:%22 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %5, %12, %18 row_newbcast:%22 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %6, %15, %18 row_newbcast:%22 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %7, %14, %18 row_newbcast:%22 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %8, %19 row_newbcast:%23 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %9, %19 row_newbcast:%23 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %10, %19 row_newbcast:%23 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %11, %19 row_newbcast:%23 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %4, %13, %19 row_newbcast:%23 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %5, %12, %19 row_newbcast:%23 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %6, %15, %19 row_newbcast:%23 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %7, %14, %19 row_newbcast:%23 row_mask:0xf bank_mask:0xf\n"
        : "+v"(eN[0]), "+v"(eN[1]), "+v"(oN[0]), "+v"(oN[1]), "+v"(aP[0]), "+v"(aP[1]), "+v"(eP[0]), "+v"(eP[1])
        : "v"(a[0]), "v"(a[1]), "v"(b[0]), "v"(b[1]), "v"(c[0]), "v"(c[1]), "v"(d[0]), "v"(d[1]), "v"(m0), "v"(m1), "v"(m2), "v"(m3), "i"(L0 + 0), "i"(L0 + 1), "i"(L0 + 2), "i"(L0 + 3));
  }
};

template <>
struct ColSym<1> {
  template <int L0>
  __device__ __forceinline__ static void run(double (&eN)[1], double (&oN)[1], double (&aP)[1], double (&eP)[1],
                                             const double (&a)[1], const double (&b)[1], const double (&c)[1],
                                             const double (&d)[1], double m0, double m1, double m2, double m3) {
    asm volatile(
        "s_nop 1\n"
        "v_fmac_f64_dpp %0, %4, %8 row_newbcast:%12 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %5, %8 row_newbcast:%12 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %6, %8 row_newbcast:%12 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %7, %8 row_newbcast:%12 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %4, %9 row_newbcast:%13 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %5, %9 row_newbcast:%13 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %6, %9 row_newbcast:%13 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %7, %9 row_newbcast:%13 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %4, %10 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %5, %10 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %6, %10 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %7, %10 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %4, %11 row_newbcast:%15 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %5, %11 row_newbcast:%15 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %6, %11 row_newbcast:%15 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %7, %11 row_newbcast:%15 row_mask:0xf bank_mask:0xf\n"
        : "+v"(eN[0]), "+v"(oN[0]), "+v"(aP[0]), "+v"(eP[0])
        : "v"(a[0]), "v"(b[0]), "v"(c[0]), "v"(d[0]), "v"(m0), "v"(m1), "v"(m2), "v"(m3), "i"(L0 + 0), "i"(L0 + 1), "i"(L0 + 2), "i"(L0 + 3));
  }
};

}  // namespace pairk
}  // namespace nmc
