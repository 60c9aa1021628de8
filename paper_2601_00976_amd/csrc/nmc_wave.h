// Wave-level building blocks shared by the solve kernels (CDNA4, 64-lane
// wavefronts): lane permutations, register reductions, the DPP contraction
// blocks, and the LDS assembly of the energy-coupling kernel matrices.
#pragma once

#include <type_traits>
#include <utility>

#include "nmc_internal.h"

namespace nmc {

constexpr int kLanes = 64;

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// DPP lane permutation within 16-lane rows for controls that read a valid
// lane for every lane (quad_perm, row mirrors), so no "old" value is needed
template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  const long v = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(long, x), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, v);
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
// s1[k] = sum over lanes 32..63.  Four lanes share each of the 2V sums; lane
// r of a group adds the entries r, r + 4, ..., r + 28 of its half, starting
// at a group-dependent rotation so that the 16 lanes of every LDS access
// cycle hit 16 different banks.  Fixed summation order (deterministic).
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
    const double* b = red + k * kLanes + hh * 32;
    const int rot = sidx & 3;
    double part[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) part[i] = b[(r + 4 * ((i + rot) & 7)) & 31];
    acc = ((part[0] + part[1]) + (part[2] + part[3])) + ((part[4] + part[5]) + (part[6] + part[7]));
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

// Register-only reductions (no LDS round trip).  Within a 16-lane row the
// butterfly xor 1, xor 2 (quad_perm), half-row mirror and row mirror leaves
// the row total in every lane, bitwise identical across the row.
__device__ __forceinline__ double row_allsum(double v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  return v;
}

// a from lanes 0..31 and b from lanes 32..63 halved into one register:
// lanes 0..31 get a(l) + a(l + 32), lanes 32..63 get b(l - 32) + b(l)
__device__ __forceinline__ double halve32(double a, double b) {
  auto x = __builtin_amdgcn_permlane32_swap(lo32(a), lo32(b), false, false);
  auto y = __builtin_amdgcn_permlane32_swap(hi32(a), hi32(b), false, false);
  return mk64(x[0], y[0]) + mk64(x[1], y[1]);
}

// min(a, b) of two non-NaN values as one v_min_f64 (the library fmin first
// quiets signalling NaNs, which a value loaded from memory cannot rule out)
__device__ __forceinline__ double min_f64(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// rows (0, 2) keep a summed with the partner row, rows (1, 3) keep b
__device__ __forceinline__ double halve16(double a, double b) {
  auto x = __builtin_amdgcn_permlane16_swap(lo32(a), lo32(b), false, false);
  auto y = __builtin_amdgcn_permlane16_swap(hi32(a), hi32(b), false, false);
  return mk64(x[0], y[0]) + mk64(x[1], y[1]);
}

// Lanes whose DPP bank (4-lane group of a 16-lane row, bit b of BANKS for
// lanes 4b..4b+3) is enabled take src from their DPP source lane of CTRL; the
// others keep old.
template <int CTRL, int BANKS>
__device__ __forceinline__ double dpp_banks(double old, double src) {
  const long v = __builtin_amdgcn_update_dpp(__builtin_bit_cast(long, old), __builtin_bit_cast(long, src), CTRL,
                                             0xF, BANKS, false);
  return __builtin_bit_cast(double, v);
}

// A butterfly stage that folds the sums of two values into one register:
// CTRL pairs every lane of the banks in A with a lane outside them
// (row_mirror with A = banks 0, 1; row_half_mirror with A = banks 0, 2), and
// after it lanes in A hold a + a(partner), the others b + b(partner).  Two
// masked moves and one add, where two separate stages cost four moves and
// two adds; the next stages then carry one value instead of two.
template <int CTRL, int A>
__device__ __forceinline__ double fold_pair(double a, double b) {
  const double x = dpp_banks<CTRL, A>(b, a);
  const double y = dpp_banks<CTRL, 0xF ^ A>(a, b);
  return x + y;
}

// Sums over the whole wave of the inner convergence test of a one-point
// kernel (64 nodes, lane = node), spread over the lanes: the 16-lane row c
// (lane >> 4) holds species c (zeros where c >= NS).  d is the squared change
// of D_c in lanes with bit 3 clear and of I_c in the others; n is the squared
// norm of the new D_c.  The wave halves split the species pairs (0, 1) and
// (2, 3), the rows of a half split the pairs, row_mirror folds the D and I
// changes apart, and three more DPP stages finish.  Fixed order; every lane
// of a row and bank pair holds the same bits.
template <int NS>
__device__ __forceinline__ void spread_conv_sums64(const double (&dd)[NS], const double (&di)[NS],
                                                   const double (&xn)[NS], double& d, double& n) {
  double pd[4], pi[4], pn[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    pd[c] = c < NS ? dd[c < NS ? c : 0] : 0.0;
    pi[c] = c < NS ? di[c < NS ? c : 0] : 0.0;
    pn[c] = c < NS ? xn[c < NS ? c : 0] : 0.0;
  }
  // halve32: lanes 0..31 carry species (0, 1), lanes 32..63 (2, 3); halve16:
  // the even row of a half the first of its pair, the odd row the second
  const double fd = halve16(halve32(pd[0], pd[2]), halve32(pd[1], pd[3]));
  const double fi = halve16(halve32(pi[0], pi[2]), halve32(pi[1], pi[3]));
  double x = halve16(halve32(pn[0], pn[2]), halve32(pn[1], pn[3]));
  double y = fold_pair<0x140, 0x3>(fd, fi);  // row_mirror: lanes 0..7 keep D
  x += dpp<0x140>(x);
  y += dpp<0x141>(y);  // row_half_mirror
  x += dpp<0x141>(x);
  y += dpp<0xB1>(y);  // quad_perm [1,0,3,2]
  x += dpp<0xB1>(x);
  y += dpp<0x4E>(y);  // quad_perm [2,3,0,1]
  x += dpp<0x4E>(x);
  d = y;
  n = x;
}

// Sums of 4 values over all 64 lanes, returned in every lane.
__device__ __forceinline__ void wave_sums4(const double (&v)[4], double (&out)[4]) {
  // lanes 0..31: (v0, v1) over the wave halves; lanes 32..63: (v2, v3)
  const double h01 = halve32(v[0], v[2]);
  const double h23 = halve32(v[1], v[3]);
  // row r now carries slot r summed over 4 lanes per column
  const double r = row_allsum(halve16(h01, h23));
  // rows (0,0,2,2) and (1,1,3,3), then both halves
  double f, sc;
  swap16(r, f, sc);
  double f0, f1, s0, s1;
  swap32(f, f0, f1);
  swap32(sc, s0, s1);
  out[0] = f0;
  out[1] = s0;
  out[2] = f1;
  out[3] = s1;
}

// Per-half sums of 2 K values (K = 1..3): s0 over lanes 0..31, s1 over lanes
// 32..63, returned in every lane.  The K reduction chains are advanced stage
// by stage, so that their dependent permute / add steps interleave.
template <int K>
__device__ __forceinline__ void half_sums_reg(const double (&v)[2 * K], double (&s0)[2 * K], double (&s1)[2 * K]) {
  // rows (0, 2): slot k over the row pair; rows (1, 3): slot K + k
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
  for (int k = 0; k < K; ++k) {
    double f, sc;
    swap16(r[k], f, sc);  // f: slot k of this half, sc: slot K + k
    double a0, a1, b0, b1;
    swap32(f, a0, a1);
    swap32(sc, b0, b1);
    s0[k] = a0;
    s1[k] = a1;
    s0[K + k] = b0;
    s1[K + k] = b1;
  }
}

__device__ __forceinline__ bool wave_any(bool b) { return __builtin_amdgcn_ballot_w64(b) != 0; }

// a wave-uniform 64-bit integer held in scalar registers
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Opaque copies: values derived from these are recomputed where they are
// used instead of being hoisted out of the outer loop (hoisted invariants
// end up spilled, which costs far more than recomputing them).
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}
template <class T>
__device__ __forceinline__ const T* opaque_ptr(const T* p) {
  asm volatile("" : "+s"(p));
  return p;
}
// A uniform pointer to read-only global data viewed in the constant address
// space, so that loads through it are scalar loads (s_load, scalar cache);
// laundered like opaque_ptr.
template <class T>
using const_ptr = const __attribute__((address_space(4))) T*;
template <class T>
__device__ __forceinline__ const_ptr<T> scalar_ptr(const T* p) {
  const_ptr<T> c = (const_ptr<T>)p;
  asm volatile("" : "+s"(c));
  return c;
}

// Four columns of the contraction for every species and both matrices in one
// asm block: acc1[t] += bcast(x[t], L0 + jj) * m1[jj], acc2[t] += bcast(x[t], L0 + jj) * m2[jj].
// The leading s_nop 1 provides the two wait states a DPP source needs after
// a VALU write, whatever the compiler schedules before the block.
template <int NS>
struct Fmac4;

template <>
struct Fmac4<1> {
  template <int L0>
  __device__ __forceinline__ static void run(double (&a1)[1], double (&a2)[1], const double (&x)[1], double m10,
                                             double m11, double m12, double m13, double m20, double m21, double m22,
                                             double m23) {
    asm volatile(
        "s_nop 1\n"
        "v_fmac_f64_dpp %0, %2, %3 row_newbcast:%11 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %2, %7 row_newbcast:%11 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %2, %4 row_newbcast:%12 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %2, %8 row_newbcast:%12 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %2, %5 row_newbcast:%13 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %2, %9 row_newbcast:%13 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %2, %6 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %2, %10 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n"
        : "+v"(a1[0]), "+v"(a2[0])
        : "v"(x[0]), "v"(m10), "v"(m11), "v"(m12), "v"(m13), "v"(m20), "v"(m21), "v"(m22), "v"(m23), "i"(L0),
          "i"(L0 + 1), "i"(L0 + 2), "i"(L0 + 3));
  }
};

template <>
struct Fmac4<2> {
  template <int L0>
  __device__ __forceinline__ static void run(double (&a1)[2], double (&a2)[2], const double (&x)[2], double m10,
                                             double m11, double m12, double m13, double m20, double m21, double m22,
                                             double m23) {
    asm volatile(
        "s_nop 1\n"
        "v_fmac_f64_dpp %0, %4, %6 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %5, %6 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %4, %10 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %5, %10 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %4, %7 row_newbcast:%15 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %5, %7 row_newbcast:%15 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %4, %11 row_newbcast:%15 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %5, %11 row_newbcast:%15 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %4, %8 row_newbcast:%16 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %5, %8 row_newbcast:%16 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %4, %12 row_newbcast:%16 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %5, %12 row_newbcast:%16 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %4, %9 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %5, %9 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %4, %13 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %5, %13 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        : "+v"(a1[0]), "+v"(a1[1]), "+v"(a2[0]), "+v"(a2[1])
        : "v"(x[0]), "v"(x[1]), "v"(m10), "v"(m11), "v"(m12), "v"(m13), "v"(m20), "v"(m21), "v"(m22), "v"(m23),
          "i"(L0), "i"(L0 + 1), "i"(L0 + 2), "i"(L0 + 3));
  }
};

template <>
struct Fmac4<3> {
  template <int L0>
  __device__ __forceinline__ static void run(double (&a1)[3], double (&a2)[3], const double (&x)[3], double m10,
                                             double m11, double m12, double m13, double m20, double m21, double m22,
                                             double m23) {
    asm volatile(
        "s_nop 1\n"
        "v_fmac_f64_dpp %0, %6, %9 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %7, %9 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %8, %9 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %6, %13 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %4, %7, %13 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %5, %8, %13 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %6, %10 row_newbcast:%18 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %7, %10 row_newbcast:%18 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %8, %10 row_newbcast:%18 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %6, %14 row_newbcast:%18 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %4, %7, %14 row_newbcast:%18 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %5, %8, %14 row_newbcast:%18 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %6, %11 row_newbcast:%19 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %7, %11 row_newbcast:%19 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %8, %11 row_newbcast:%19 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %6, %15 row_newbcast:%19 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %4, %7, %15 row_newbcast:%19 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %5, %8, %15 row_newbcast:%19 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %0, %6, %12 row_newbcast:%20 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %1, %7, %12 row_newbcast:%20 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %2, %8, %12 row_newbcast:%20 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %3, %6, %16 row_newbcast:%20 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %4, %7, %16 row_newbcast:%20 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f64_dpp %5, %8, %16 row_newbcast:%20 row_mask:0xf bank_mask:0xf\n"
        : "+v"(a1[0]), "+v"(a1[1]), "+v"(a1[2]), "+v"(a2[0]), "+v"(a2[1]), "+v"(a2[2])
        : "v"(x[0]), "v"(x[1]), "v"(x[2]), "v"(m10), "v"(m11), "v"(m12), "v"(m13), "v"(m20), "v"(m21), "v"(m22),
          "v"(m23), "i"(L0), "i"(L0 + 1), "i"(L0 + 2), "i"(L0 + 3));
  }
};

// 1 / x from the hardware estimate refined by two Newton steps, for finite x
// of normal magnitude (|x| and 1 / |x| both above the denormal range)
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Natural logarithm of a positive finite double: x = m 2^e with m in
// [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s) = 2 (s + s^3 / 3 + ... + s^19 / 19)
// with s = (m - 1) / (m + 1), |s| <= 0.1716 (the remainder of the series is
// below 2^-53 of its sum), and e ln 2 split in a high part exact in the
// product and a low part (Cody and Waite).  Within 2 ulp of the correctly
// rounded value.  Not for x <= 0, inf or NaN.
__device__ __forceinline__ double log_pos(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  const bool lo = m < 0.70710678118654752440;
  m = lo ? m + m : m;
  e = lo ? e - 1 : e;
  const double num = m - 1.0, den = m + 1.0;  // m - 1 exact
  const double r = rcp_nr(den);
  double s = num * r;
  s = __builtin_fma(__builtin_fma(-s, den, num), r, s);
  const double z = s * s;
  double p = 1.0 / 19.0;
  p = __builtin_fma(p, z, 1.0 / 17.0);
  p = __builtin_fma(p, z, 1.0 / 15.0);
  p = __builtin_fma(p, z, 1.0 / 13.0);
  p = __builtin_fma(p, z, 1.0 / 11.0);
  p = __builtin_fma(p, z, 1.0 / 9.0);
  p = __builtin_fma(p, z, 1.0 / 7.0);
  p = __builtin_fma(p, z, 1.0 / 5.0);
  p = __builtin_fma(p, z, 1.0 / 3.0);
  const double s2 = s + s, ef = (double)e;
  constexpr double kLn2Hi = 6.93147180369123816490e-01, kLn2Lo = 1.90821492927058770002e-10;
  return __builtin_fma(ef, kLn2Hi, s2 + __builtin_fma(ef, kLn2Lo, (s2 * z) * p));
}

// Coefficients (g1, g2) of an Anderson step over two difference columns
// (1 the older, 2 the newer) from their normal equations, by LDL^T (the
// Cholesky pivots G11 and G22 - G12^2 / G11, without square roots).  A pivot
// <= 1e-14 trace drops the older column, and with no column left the step is
// Picard (g = 0).  two_cols says whether the older column exists; without
// it G12 and b1 are not used (any value, NaN included, gives the same g2 and
// g1 = 0), so callers need not zero the older column's products.
// Branch-free, with Newton-refined reciprocals of the positive pivots.
__device__ __forceinline__ void anderson2(bool two_cols, double G11, double G12, double G22, double b1, double b2,
                                          double& g1, double& g2) {
  const double tr = G11 + G22;
  const bool use2 = two_cols && G11 > 1e-14 * tr;
  const double r11 = rcp_nr(use2 ? G11 : 1.0);
  const double l21 = G12 * r11;
  const double p2 = G22 - G12 * l21;
  const bool two = use2 && p2 > 1e-14 * tr;
  const bool one = G22 > 1e-14 * G22;
  const double rp = rcp_nr(two ? p2 : (one ? G22 : 1.0));
  g2 = two ? (b2 - l21 * b1) * rp : (one ? b2 * rp : 0.0);
  g1 = two ? (b1 - G12 * g2) * r11 : 0.0;
}

// Per-node model tables copied into LDS once per work-group (lane-indexed
// reads of them are then LDS hits); the uniform scalars of the model stay in
// the global table, where the scalar cache serves them.
template <int NQ>
struct ModelLdsN {
  double eps[NQ], w2[NQ], w3[NQ], shape[NQ];
  double theta[NQ + 2];  // per-node EmAb scales, a_nes, a_pair
};
using ModelLds = ModelLdsN<32>;

template <int NQ>
__device__ __forceinline__ void load_model(const DevModel* __restrict__ md, const double* __restrict__ theta,
                                           ModelLdsN<NQ>& m) {
  const int l = threadIdx.x;
  if (l < NQ) {
    m.eps[l] = md->eps[l];
    m.w2[l] = md->w2[l];
    m.w3[l] = md->w3[l];
    m.shape[l] = md->shape[l];
  }
  for (int i = l; i < NQ + 2; i += kLanes) m.theta[i] = theta[i];
  __syncthreads();
}

// Work queue of the persistent kernels: up to kQueues counters, each on its
// own 256-byte line, one per class of work-group ids (id mod nq: one per XCD
// when work-groups are dealt round-robin to the 8 XCDs).  The chunk indices
// are cut into blocks of kQueueRun * nq; counter c hands out, in every block,
// the run of kQueueRun consecutive chunks at offset c * kQueueRun, so every
// queue sees the same mix of cheap and expensive points while the per-point
// scalar inputs and outputs of a run share cache lines within one XCD.  The
// chunks past the last whole block are dealt round-robin (c, c + nq, ...).
// Every work-group loops until its queue is exhausted, so the grid drains
// before the kernel ends.
constexpr int kQueues = 8;
constexpr int kQueueStride = 64;  // ints
constexpr int kQueueRun = 32;     // chunks

struct WorkQueue {
  int* ctr;
  int64_t nchunks, full;  // chunks; tickets per counter inside whole blocks
  int nq, c;
  int pend;  // lane 0: ticket returned by the grab in flight
  int cur;   // ticket of the next chunk (uniform)
  __device__ __forceinline__ WorkQueue(int* queue, int64_t P, int chunk) {
    nq = gridDim.x < kQueues ? (int)gridDim.x : kQueues;
    c = blockIdx.x % nq;
    ctr = queue + c * kQueueStride;
    nchunks = (P + chunk - 1) / chunk;
    full = nchunks / ((int64_t)kQueueRun * nq) * kQueueRun;
    pend = 0;
    if (threadIdx.x == 0) pend = atomicAdd(ctr, 1);
    cur = __builtin_amdgcn_readfirstlane(pend);
  }
  // next chunk index of this work-group (uniform), or -1 once drained; the
  // following grab is issued here and must be settled before the next call
  __device__ __forceinline__ int64_t next() {
    const int64_t t = cur;
    const int64_t g = t < full ? (t / kQueueRun) * kQueueRun * nq + (int64_t)c * kQueueRun + t % kQueueRun
                               : full * nq + (t - full) * nq + c;
    if (g >= nchunks) return -1;
    if (threadIdx.x == 0) pend = atomicAdd(ctr, 1);
    return g;
  }
  // takes the result of the grab in flight.  Called once the chunk's inputs
  // are loaded: the wait for the atomic then overlaps that of the loads
  // instead of the drain of the chunk's output stores (vector memory
  // counters complete in order).
  __device__ __forceinline__ void settle() { cur = __builtin_amdgcn_readfirstlane(pend); }
};

// Pair partner of internal species s (species sorted by id: nu_e, anti-nu_e
// are partners, nu_x is its own partner).  Models without pair processes
// have zero pair kernels, so the map is irrelevant for them.
template <int NS>
__device__ __forceinline__ constexpr int pair_partner(int s) {
  return NS == 3 ? (s < 2 ? 1 - s : 2) : (NS == 2 ? 1 - s : 0);
}


// Ye^(4/3) of the EOS
__device__ __forceinline__ double ye43(double ye) { return ye * cbrt(ye); }

// ---------------------------------------------------------------------------
// Kernel matrices at temperature T (Eqs. nesRatesNodal, pairRatesNodal with
// the kernels of Eqs. inOutInvarianceNES ... detailedBalancePair).  With
// b = exp(-(e_hi - e_lo) / (2T)) for e_hi >= e_lo and G_x = exp(-2 e_x / T):
//   Phi_in[hi][lo] = A e e' b^3,  Phi_in[lo][hi] = A e e' b,  Phi_out = Phi_in^T,
//   Phi_ann = A' e e' b^2,  Phi_pro = A' e e' G_hi  (both symmetric).
// b is assembled from per-node exponent splits x = e log2(e) / (2T) =
// n + f, P = 2^f, R = 2^-f:  b = ldexp(P_lo R_hi, n_lo - n_hi), so every
// factor stays <= 1 and nothing overflows at low temperature.
constexpr int kTileStride = 33;  // padded row stride of a 32 x 32 LDS tile

struct alignas(16) SplitExp {
  double P2[32], R2[32], G[32];
  int n2[32];
};

// Exponent split of y = v log2(e) / (2T): y = n + f with n = floor(y), and
// P = 2^f in [1, 2), R = 2^-f.  exp(-v / T) = 2^(-2n) R^2 without exp().
struct ExpSplit {
  double P, R;
  int n;
};
__device__ __forceinline__ ExpSplit exp_split(double v, double invT) {
  const double y = v * (0.5 * invT) * 1.4426950408889634;  // log2(e)
  const double n = floor(y);
  ExpSplit r;
  r.P = exp2(y - n);
  r.R = rcp_nr(r.P);
  r.n = (int)n;
  return r;
}

// lanes 0..31 fill the per-node factors of temperature 1 / invT
// (G = exp(-2 e / T) = 2^(-4n) R^4); ends with a barrier
__device__ __forceinline__ void split_exp_prepare(const ModelLds& m, double invT, SplitExp& E) {
  const int lane = threadIdx.x;
  if (lane < 32) {
    const ExpSplit x = exp_split(m.eps[lane], invT);
    E.P2[lane] = x.P;
    E.R2[lane] = x.R;
    E.n2[lane] = x.n;
    const double R2 = x.R * x.R;
    E.G[lane] = ldexp(R2 * R2, -4 * x.n);
  }
  __syncthreads();
}

enum TileKind { kTilePhiIn, kTilePhiAnn, kTilePhiPro, kTilePairFactor };

// Writes the full 32 x 32 matrix of the given kind with amplitude amp into
// the tile (row-major, stride kTileStride); kTilePairFactor is the symmetric
// b = exp(-|e_q - e_j| / (2T)) itself (amp unused, exactly 1 on the
// diagonal).  Pair slot i of lane (h, q)
// covers nodes (q, q + d mod 32), d = h + 2 i; the d = 16 pairs are taken by
// q < 16 only, so each of the 528 unordered pairs (diagonal included) is
// written exactly once.  h = lane / 32 and q = lane mod 32 are passed in
// (callers launder them so that the index arithmetic is not hoisted out of
// their loops).  No barrier: the caller synchronises.
template <TileKind K>
__device__ __forceinline__ void fill_tile(const ModelLds& m, const SplitExp& E, double amp, int h, int q,
                                          double* T0) {
  constexpr int ST = kTileStride;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int d = h + 2 * i;
    const int j = (q + d) & 31;
    const int lo = q < j ? q : j, hi = q < j ? j : q;
    if (d < 16 || (d == 16 && q < 16)) {
      const double ee = amp * (m.eps[lo] * m.eps[hi]);
      if constexpr (K == kTilePairFactor) {
        const double b = lo == hi ? 1.0 : ldexp(E.P2[lo] * E.R2[hi], E.n2[lo] - E.n2[hi]);
        T0[hi * ST + lo] = b;
        T0[lo * ST + hi] = b;
      } else if constexpr (K == kTilePhiPro) {
        const double v = ee * E.G[hi];
        T0[hi * ST + lo] = v;
        T0[lo * ST + hi] = v;
      } else {
        const double b = ldexp(E.P2[lo] * E.R2[hi], E.n2[lo] - E.n2[hi]);
        if constexpr (K == kTilePhiIn) {
          T0[hi * ST + lo] = ee * (b * b * b);
          T0[lo * ST + hi] = ee * b;
        } else {
          const double v = ee * (b * b);
          T0[hi * ST + lo] = v;
          T0[lo * ST + hi] = v;
        }
      }
    }
  }
}

}  // namespace nmc
