// Primitive-moment recovery (Sec. 3.4) and the stage combination of the
// PD-ARS IMEX step (Eq. butcherPDARS) of the coupling.
//
// Recovery: one thread per (point, species, node).  Given the conserved
// moments U = (N, G_j) and the fluid velocity v, the primitive moments
// M = (D, I_j) solve N = D + v^i I_i, G_j = I_j + v^i K_ij(M) (Eq.
// conservedToPrimitive); the thread iterates the fixed-point map of Eq.
// c2p_FP, M <- (1 - lam) M + lam (N - v.I, G_j - v^i K_ij(M)),
// lam = 1 / (1 + |v|), from M = U (Eq. c2p_sequence) with Anderson
// acceleration over its last `mem` residuals, its 4-vector state and history
// in registers, until ||M^[k+1] - M^[k]|| <= tol ||U|| (Euclidean).  The
// accesses of consecutive threads are consecutive nodes, so every load and
// store of a wavefront is one coalesced run per array.
#include "nmc_closure.h"

namespace nmc {
namespace {

// the fixed-point recovery of a node whose conserved moments are of order one
__device__ __forceinline__ int c2p_scaled(double N, const double (&G)[3], const double (&v)[3], double lam, double oml,
                                          int mem, double tol2, int max_it, double (&M)[4]) {
  const double U[4] = {N, G[0], G[1], G[2]};
  const double un2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
  double Qp[4], Fp[4], dQo[4] = {0.0, 0.0, 0.0, 0.0}, dFo[4] = {0.0, 0.0, 0.0, 0.0};
  double G11 = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) M[i] = U[i];
  for (int k = 1; k <= max_it; ++k) {
    double vI, vK[3];
    const double I3[3] = {M[1], M[2], M[3]};
    closure_terms_unit(M[0], I3, v, vI, vK);
    double g[4], F[4], Mn[4];
    g[0] = oml * M[0] + lam * (N - vI);
#pragma unroll
    for (int j = 0; j < 3; ++j) g[1 + j] = oml * M[1 + j] + lam * (G[j] - vK[j]);
#pragma unroll
    for (int i = 0; i < 4; ++i) F[i] = g[i] - M[i];
    const int m_k = k < mem ? k : mem;
    if (m_k == 1) {
#pragma unroll
      for (int i = 0; i < 4; ++i) Mn[i] = g[i];
    } else {
      double dQ2[4], dF2[4], G12 = 0.0, G22 = 0.0, b1 = 0.0, b2 = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        dQ2[i] = g[i] - Qp[i];
        dF2[i] = F[i] - Fp[i];
        G12 += dFo[i] * dF2[i];
        G22 += dF2[i] * dF2[i];
        b1 += dFo[i] * F[i];
        b2 += dF2[i] * F[i];
      }
      double g1, g2;
      anderson2(m_k == 3, G11, G12, G22, b1, b2, g1, g2);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        Mn[i] = g[i] - g2 * dQ2[i] - g1 * dQo[i];
        dQo[i] = dQ2[i];
        dFo[i] = dF2[i];
      }
      G11 = G22;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      Qp[i] = g[i];
      Fp[i] = F[i];
    }
    bool fin = true;
    double d2 = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      fin = fin && isfinite(Mn[i]);
      d2 += (Mn[i] - M[i]) * (Mn[i] - M[i]);
      M[i] = Mn[i];
    }
    if (!fin) return -2;
    if (d2 <= tol2 * un2) return k;
  }
  return -1;
}

// the fixed-point recovery of one node; returns the iterations taken, -1 at
// the cap, -2 on a non-finite iterate.  The map is homogeneous of degree one
// in U (the Eddington factor depends on |I| / D only), so the node is solved
// for U scaled by a power of two that brings its largest component near 1
// and the result scaled back: exact scalings that keep the Anderson Gram
// products of a faint node (a far tail's 1e-160) out of the denormal range,
// where the hardware reciprocal of its normal equations would overflow.
__device__ __forceinline__ int c2p_node(double N0, const double (&G0)[3], const double (&v)[3], int mem, double tol2,
                                        int max_it, double (&M)[4]) {
  const double lam = 1.0 / (1.0 + sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
  const double oml = 1.0 - lam;
  int ex = 0;
  {
    const double big = fmax(fmax(fabs(N0), fabs(G0[0])), fmax(fabs(G0[1]), fabs(G0[2])));
    if (big > 0.0 && isfinite(big)) frexp(big, &ex);
  }
  const double N = ldexp(N0, -ex);
  const double G[3] = {ldexp(G0[0], -ex), ldexp(G0[1], -ex), ldexp(G0[2], -ex)};
  const int it = c2p_scaled(N, G, v, lam, oml, mem, tol2, max_it, M);
#pragma unroll
  for (int i = 0; i < 4; ++i) M[i] = ldexp(M[i], ex);
  return it;
}

// conserved moments of primitive ones at velocity v (Eq. conservedToPrimitive)
__device__ __forceinline__ void p2c_node(double D, const double (&I)[3], const double (&v)[3], double& N,
                                         double (&G)[3]) {
  double vI, vK[3];
  closure_terms(D, I, v, vI, vK);
  N = D + vI;
#pragma unroll
  for (int j = 0; j < 3; ++j) G[j] = I[j] + vK[j];
}

__global__ __launch_bounds__(256) void c2p_kernel(int64_t P, int ns, int nq, const double* __restrict__ N,
                                                  const double* __restrict__ G, const double* __restrict__ v,
                                                  int mem, double tol2, int max_it, double* __restrict__ D,
                                                  double* __restrict__ I, int32_t* __restrict__ iters) {
  const int64_t n = P * ns * nq;
  // nq is a power of two (32 or 64) and ns is 1..3: the node, (point,
  // species) and point indices by shifts, a mask and a division by the
  // constant 3
  const int lq = 31 - __builtin_clz(nq);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ps = i >> lq;
    const int q = (int)(i & (nq - 1));
    const int64_t p = ns == 3 ? ps / 3 : ps >> (ns - 1);
    const double vv[3] = {v[3 * p], v[3 * p + 1], v[3 * p + 2]};
    const double Gq[3] = {G[(ps * 3 + 0) * nq + q], G[(ps * 3 + 1) * nq + q], G[(ps * 3 + 2) * nq + q]};
    double M[4];
    const int it = c2p_node(N[i], Gq, vv, mem, tol2, max_it, M);
    D[i] = M[0];
#pragma unroll
    for (int j = 0; j < 3; ++j) I[(ps * 3 + j) * nq + q] = M[1 + j];
    iters[i] = it;
  }
}

// PD-ARS stage 3 input: per (point, species, node), U^(3*) = U^n + w (U^(2) -
// U^n) in conserved variables at the stage velocities, recovered to primitive
// moments at v^(3*) = v^n + w (v^(2) - v^n); the matter state likewise (one
// thread per point).  Points below the coupling density pass through.
__global__ __launch_bounds__(256) void pdars_stage3_kernel(PdarsArgs a) {
  const int ns = a.ns, nq = a.nq;
  const int64_t n = a.P * ns * nq;
  const double w = a.w;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ps = i / nq;
    const int q = (int)(i - ps * nq);
    const int64_t p = ps / ns;
    const bool skip = a.rho11[p] < a.rho11_min;
    const double vn[3] = {a.v0[3 * p], a.v0[3 * p + 1], a.v0[3 * p + 2]};
    const double v2[3] = {a.v2[3 * p], a.v2[3 * p + 1], a.v2[3 * p + 2]};
    double v3[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) v3[j] = skip ? vn[j] : vn[j] + w * (v2[j] - vn[j]);
    double In[3], I2[3], Gn[3], G2[3], G3[3], Nn, N2;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      In[j] = a.I0[(ps * 3 + j) * nq + q];
      I2[j] = a.I2[(ps * 3 + j) * nq + q];
    }
    const double Dn = a.D0[i];
    double M[4] = {Dn, In[0], In[1], In[2]};
    int it = 0;
    if (!skip) {
      p2c_node(Dn, In, vn, Nn, Gn);
      p2c_node(a.D2[i], I2, v2, N2, G2);
      const double N3 = Nn + w * (N2 - Nn);
#pragma unroll
      for (int j = 0; j < 3; ++j) G3[j] = Gn[j] + w * (G2[j] - Gn[j]);
      it = c2p_node(N3, G3, v3, a.mem, a.tol2, a.max_it, M);
    }
    a.D3[i] = M[0];
#pragma unroll
    for (int j = 0; j < 3; ++j) a.I3[(ps * 3 + j) * nq + q] = M[1 + j];
    a.iters[i] = it;
    if (i - p * ns * nq == 0) {
      a.ye3[p] = skip ? a.ye0[p] : a.ye0[p] + w * (a.ye2[p] - a.ye0[p]);
      a.ef3[p] = skip ? a.ef0[p] : a.ef0[p] + w * (a.ef2[p] - a.ef0[p]);
#pragma unroll
      for (int j = 0; j < 3; ++j) a.v3[3 * p + j] = v3[j];
    }
  }
}

// the step's counts and status: iterations of both solves; the first non-OK
// status of stage 2, the recovery (MAX_INNER at its cap, NONFINITE), stage 3
__global__ __launch_bounds__(256) void pdars_merge_kernel(int64_t P, int nn, const int32_t* __restrict__ no2,
                                                          const int32_t* __restrict__ ni2,
                                                          const int32_t* __restrict__ st2,
                                                          const int32_t* __restrict__ iters, int32_t* n_outer,
                                                          int32_t* n_inner, int32_t* status) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    int c2p = NMC_STATUS_OK;
    for (int i = 0; i < nn; ++i) {
      const int it = iters[p * nn + i];
      if (it == -2) c2p = NMC_STATUS_NONFINITE;
      if (it == -1 && c2p == NMC_STATUS_OK) c2p = NMC_STATUS_MAX_INNER;
    }
    if (st2[p] != NMC_STATUS_OK) status[p] = st2[p];
    else if (c2p != NMC_STATUS_OK) status[p] = c2p;
    n_outer[p] += no2[p];
    n_inner[p] += ni2[p];
  }
}

int64_t grid_for(int64_t n, int num_cu) {
  int64_t g = (n + 255) / 256, cap = (int64_t)num_cu * 32;
  g = g < cap ? g : cap;
  return g < 1 ? 1 : g;
}

}  // namespace

hipError_t launch_c2p(int64_t P, int ns, int nq, const double* N, const double* G, const double* v, int mem,
                      double tol, int max_it, double* D, double* I, int32_t* iters, int num_cu, hipStream_t s) {
  // the kernel's index arithmetic takes nq a power of two and ns in 1..3
  if (nq <= 0 || (nq & (nq - 1)) != 0 || ns < 1 || ns > 3) return hipErrorInvalidValue;
  const int64_t n = P * ns * nq;
  hipLaunchKernelGGL(c2p_kernel, dim3((unsigned)grid_for(n, num_cu)), dim3(256), 0, s, P, ns, nq, N, G, v, mem,
                     tol * tol, max_it, D, I, iters);
  return hipGetLastError();
}

hipError_t launch_pdars_stage3(const PdarsArgs& a, int num_cu, hipStream_t s) {
  hipLaunchKernelGGL(pdars_stage3_kernel, dim3((unsigned)grid_for(a.P * a.ns * a.nq, num_cu)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pdars_merge(int64_t P, int nn, const int32_t* no2, const int32_t* ni2, const int32_t* st2,
                              const int32_t* iters, int32_t* n_outer, int32_t* n_inner, int32_t* status, int num_cu,
                              hipStream_t s) {
  hipLaunchKernelGGL(pdars_merge_kernel, dim3((unsigned)grid_for(P, num_cu)), dim3(256), 0, s, P, nn, no2, ni2, st2,
                     iters, n_outer, n_inner, status);
  return hipGetLastError();
}

}  // namespace nmc
