// Internal declarations of the nmc library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nmc.h"

namespace nmc {

constexpr int kMaxNq = 64;
constexpr int kMaxNs = 3;
constexpr int kReduceBlocks = 1024;  // first-stage blocks of the point reduction

// Model table resident in device memory.  The kernels copy the per-node
// tables into LDS once per work-group and read the uniform scalars through
// the scalar cache.
struct DevModel {
  int ns, nq;
  unsigned flags;
  int pad0;
  int species[kMaxNs];
  int partner[kMaxNs];  // index of the pair partner in the species list, or -1
  double g[kMaxNs];       // lepton number of the species
  double mult[kMaxNs];    // energy multiplicity (4 for the heavy-lepton stand-in)
  double musign[kMaxNs];  // chemical potential = musign * mu_nu_e
  double emab[kMaxNs];    // 1 if the species has emission/absorption
  // Internal species order used by the solve kernels: sorted by species id,
  // so that pair partners sit at compile-time positions (nu_e, anti-nu_e at
  // 0, 1 and nu_x last).  ext[t] is the caller's slot of internal species t;
  // the i* arrays are the per-species constants in internal order.
  int ext[kMaxNs];
  double ig[kMaxNs], imult[kMaxNs], imusign[kMaxNs], iemab[kMaxNs];
  double eps[kMaxNq];     // node energies [MeV]
  double w2[kMaxNq];      // w eps^2 dEps [MeV^3]
  double w3[kMaxNq];      // w2 eps [MeV^4]
  double shape[kMaxNq];   // (eps / eps_ref)^chi_power
  double chi_ref, sigma_ratio;
  double eos_a, eos_b, mu_a, mu_ye0, mu_b, mu_t0;
  double inv_mu_t0;       // 1 / mu_t0
  double kcoup;           // K * rho11 [MeV^-3]
  double rho11_min;
  double phi1_nes, phi1_pair;  // Phi_1 / Phi_0 of the NES and pair kernels
  // projected equilibrium (Eq. fermiDiracProjection) with its limiter bounds
  // D_min and 1 - D_max, and per-node tables of the node's element: edges,
  // l_1 eps^2 = pl[0] eps^3 + pl[1] eps^2 and l_2 likewise (pl[2], pl[3]),
  // the node's row of the inverse eps^2 mass matrix, 1 / int eps^2, and the
  // node's own basis function at the element's lower and upper edge
  int fd_projection;
  double deq_min, ceq_min;
  double pelo[kMaxNq], pehi[kMaxNq];
  double pl[kMaxNq][4];
  double pinv[kMaxNq][2];
  double prm0[kMaxNq];
  double pedge[kMaxNq][2];
};

struct SolverParams {
  double tol_inner, tol_outer;
  int m_inner, m_outer, max_inner, max_outer, fixed_matter;
};

struct FwdArgs {
  const DevModel* mdl;
  SolverParams prm;
  double tol_inner2;  // tol_inner^2 (the inner test is evaluated squared)
  int64_t P;
  double dtau;
  const double *D0, *I0, *rho11, *ye0, *e0, *chi0, *T_fixed, *mu_fixed, *theta;
  double *D, *I, *ye, *e, *T;
  int32_t *n_outer, *n_inner, *status;
  double* kstore;  // per-point kernel matrices (kernel_store = HBM) or nullptr
  int* queue;  // work-queue counter (persistent mode) or nullptr
  int chunk;   // points per grab
};

// O(v) forward solve (nonzero fluid velocity): moments D (P, ns, nq) and I
// (P, ns, 3, nq), matter (Ye, ef, v) with v (P, 3)
struct FwdVArgs {
  const DevModel* mdl;
  SolverParams prm;
  double tol_inner2;
  int64_t P;
  double dtau;
  const double *D0, *I0, *rho11, *ye0, *ef0, *v0, *chi0, *theta;
  double *D, *I, *ye, *ef, *v, *T;
  int32_t *n_outer, *n_inner, *status;
  int* queue;
  int chunk;
};

// the stage-3 input of a PD-ARS step (see nmc_primitive.hip)
struct PdarsArgs {
  int64_t P;
  int ns, nq;
  double w;          // a_32 / a_22: weight of stage 2 in U^(3*)
  double rho11_min;  // coupling density
  const double *rho11, *D0, *I0, *ye0, *ef0, *v0;  // the step's initial state
  const double *D2, *I2, *ye2, *ef2, *v2;          // stage-2 solution
  double *D3, *I3, *ye3, *ef3, *v3;                // stage-3 initial state
  int32_t* iters;    // recovery iterations per (point, species, node)
  int mem, max_it;   // recovery: Anderson memory and cap
  double tol2;       // recovery: squared relative tolerance
};

struct AdjArgs {
  const DevModel* mdl;
  int64_t P;
  double dtau;
  const double *rho11, *chi0, *theta;
  const double *D, *ye, *e;
  const int32_t *status, *n_outer;
  const double* gbar;
  double* grad_pp;     // (P, nq + 2) per-point terms, always written
};

// launchers (defined in the kernel translation units)
hipError_t launch_forward(const FwdArgs& a, int nq, int ns, bool coupled, bool proj, const nmc_launch& L,
                          int num_cu, hipStream_t s);
hipError_t launch_forward64(const FwdArgs& a, int ns, bool coupled, const nmc_launch& L, int num_cu,
                            hipStream_t s);
hipError_t launch_forward_pair(const FwdArgs& a, int ns, bool coupled, bool proj, const nmc_launch& L,
                               int num_cu, hipStream_t s);
hipError_t launch_forward_v(const FwdVArgs& a, int ns, bool coupled, bool phi1, const nmc_launch& L, int num_cu,
                            hipStream_t s);
hipError_t launch_forward_vpair(const FwdVArgs& a, int ns, bool coupled, bool phi1, const nmc_launch& L, int num_cu,
                                hipStream_t s);
hipError_t launch_reset_counter(int* counter, hipStream_t s);
hipError_t launch_c2p(int64_t P, int ns, int nq, const double* N, const double* G, const double* v, int mem,
                      double tol, int max_it, double* D, double* I, int32_t* iters, int num_cu, hipStream_t s);
hipError_t launch_pdars_stage3(const PdarsArgs& a, int num_cu, hipStream_t s);
hipError_t launch_pdars_merge(int64_t P, int nn, const int32_t* no2, const int32_t* ni2, const int32_t* st2,
                              const int32_t* iters, int32_t* n_outer, int32_t* n_inner, int32_t* status, int num_cu,
                              hipStream_t s);
// near-equilibrium initial state from raw draws
hipError_t launch_init_state(const DevModel* mdl, int ns, int nq, int64_t P, const double* T, const double* mu,
                             const double* rho11, const double* ye, const double* uD, const double* uI, double a,
                             double b, double c, double* D0, double* I0, double* e0, hipStream_t s);
hipError_t launch_adjoint(const AdjArgs& a, int nq, int ns, int num_cu, hipStream_t s);
hipError_t launch_reduce_columns(const double* grad_pp, int64_t P, int ncol, double* partial, double* grad_theta,
                                 hipStream_t s);

}  // namespace nmc
