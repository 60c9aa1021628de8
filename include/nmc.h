/*
 * nmc.h -- C ABI of the MI355X implicit neutrino-matter coupling solver.
 *
 * The library solves, independently at every spatial point of a batch, the
 * backward-Euler neutrino-matter coupling problem of the DG-IMEX two-moment
 * scheme of arXiv 2601.00976 (Sec. 3.5, "Neutrino-matter Coupling"):
 *
 *   [M, y] = SolveNeutrinoMatterCoupling(dtau, M*, y*)
 *
 * with neutrino number moments D and number fluxes I on an energy-node grid
 * for up to three species (nu_e, anti-nu_e, and nu_x standing for the four
 * heavy-lepton flavours), and matter state y = (Ye, e) at zero fluid velocity
 * (nmc_solve_batch) or y = (Ye, ef, v) with the O(v) terms (nmc_solve_batch_v).
 * The moment equations are Eqs. implicitNumberNodal / implicitNumberFluxNodal,
 * the rates Eqs. emissivityNodal ... pairRatesNodal, the matter update Eq.
 * implicitFluidNodal, and the iteration the nested fixed point with Anderson
 * acceleration of Algorithm neutrinoMatterCoupling with the convergence tests
 * of Algorithms innerConverged and outerConverged.
 *
 * Microphysics is a synthetic closed-form stand-in for the tabulated opacities
 * and equation of state:
 *   chi_EmAb(s,q) = theta_q * chi0 * (eps_q/eps_ref)^chi_power  (nu_e, anti-nu_e)
 *   sigma_Iso(s,q) = sigma_ratio * chi0 * (eps_q/eps_ref)^chi_power
 *   D_eq(s,q) = 1 / (exp((eps_q - mu_s)/T) + 1), mu_s = (+mu, -mu, 0)
 *   NES:  Phi_in = A eps eps' exp(-(|d| + d/2)/T), Phi_out = A eps eps' exp(-(|d| - d/2)/T),
 *         d = eps - eps', A = theta_{nq} * rho11
 *   pair: Phi_ann = A' eps eps' exp(-|d|/T), Phi_pro = Phi_ann exp(-(eps + eps')/T),
 *         A' = theta_{nq+1} * rho11
 *   EOS:  e = eos_a T (1 + Ye) + eos_b Ye^(4/3) rho11^(1/3)   [MeV / baryon]
 *         mu = mu_a (Ye - mu_ye0) rho11^(1/3) + mu_b ln(T / mu_t0)   [MeV]
 * These kernels satisfy the in-out invariance and detailed-balance relations
 * of Eqs. inOutInvarianceNES ... detailedBalancePair exactly.
 *
 * Units: energies in MeV, lengths in km (c = 1, so dtau is in km and
 * opacities in 1/km), density rho11 in 1e11 g/cm^3, matter energy e in
 * MeV per baryon.
 *
 * Conventions
 *  - Every function returns NMC_OK (0) or a negative NMC_E_* code.  Arguments
 *    are validated on the host before anything is enqueued; no C++ exception
 *    crosses the ABI.  nmc_last_error() gives a thread-local message.
 *  - Handles are opaque, owned by the library, immutable after creation and
 *    safe to share across streams and threads.  Creation allocates device
 *    memory; solve calls never allocate, free or synchronize, so they may be
 *    captured into a HIP graph.
 *  - Array arguments of solve calls are caller-owned DEVICE pointers that must
 *    stay valid until the stream reaches the enqueued work.  Layouts are
 *    structure-of-arrays: moments are (P, ns, nq) row-major with the energy
 *    node fastest; per-point scalars are (P).
 *  - Numerical failure of a point is never an error return; it is reported in
 *    status[p] (NMC_STATUS_*).
 *  - `stream` is a hipStream_t (NULL = the default stream).
 */
#ifndef NMC_H
#define NMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NMC_OK 0
#define NMC_E_INVALID_ARG (-1) /* null pointer, non-positive size, bad value */
#define NMC_E_UNSUPPORTED (-2) /* e.g. node count not 32/64, more than 3 species */
#define NMC_E_HIP (-3)         /* a HIP runtime call failed */
#define NMC_E_WORKSPACE (-4)   /* workspace too small */

/* per-point status */
#define NMC_STATUS_OK 0         /* converged (or skipped below rho11_min: n_outer = 0) */
#define NMC_STATUS_MAX_OUTER 1  /* outer (matter) iteration hit max_outer */
#define NMC_STATUS_MAX_INNER 2  /* some inner (moment) loop hit max_inner */
#define NMC_STATUS_NONFINITE 3  /* a non-finite iterate appeared; last finite state returned */
#define NMC_STATUS_EOS_DOMAIN 4 /* T <= 0 or Ye < 0 from the EOS; last valid moments returned */

/* species */
#define NMC_NU_E 0
#define NMC_NU_E_BAR 1
#define NMC_NU_X 2

/* physics flags */
#define NMC_EMAB 1u /* emission / absorption (nu_e, anti-nu_e only) */
#define NMC_ISO 2u  /* isoenergetic scattering (flux moments only) */
#define NMC_NES 4u  /* inelastic neutrino-electron scattering kernels */
#define NMC_PAIR 8u /* pair processes */
#define NMC_ALL_PHYSICS 15u

/* energy-grid spacing */
#define NMC_SPACING_LOG 0  /* geometric element edges eps_lo (eps_hi/eps_lo)^(e/n_elem) */
#define NMC_SPACING_ZOOM 1 /* dEps_{e+1} = zoom dEps_e on [0, eps_hi] (Table energyGrids) */

typedef struct nmc_grid nmc_grid;
typedef struct nmc_model nmc_model;

typedef struct {
  int n_elem;          /* energy elements; nq = 2 n_elem must be 32 or 64 */
  int nodes_per_elem;  /* Legendre-Gauss nodes per element: must be 2 (k = 1) */
  double eps_lo;       /* MeV (LOG spacing) */
  double eps_hi;       /* MeV */
  int spacing;         /* NMC_SPACING_LOG or NMC_SPACING_ZOOM */
  double zoom;         /* ZOOM spacing only */
} nmc_grid_desc;

typedef struct {
  int n_species;       /* 1..3 */
  int species[3];      /* NMC_NU_E / NMC_NU_E_BAR / NMC_NU_X, each at most once */
  unsigned flags;      /* NMC_EMAB | NMC_ISO | NMC_NES | NMC_PAIR */
  double chi_ref;      /* absorption scale per rho11 when no chi0 array is given [1/km] (10) */
  double eps_ref;      /* MeV (10) */
  double chi_power;    /* (2) */
  double sigma_ratio;  /* (0.5) */
  double eos_a, eos_b; /* (1.5, 3) */
  double mu_a, mu_ye0, mu_b, mu_t0; /* (20, 0.3, 5, 5) */
  double hc_mev_cm;    /* (1.239841984e-10) */
  double m_u_g;        /* (1.66053906660e-24) */
  double rho11_min;    /* points below this density are passed through unsolved (1e-4 = 1e7 g/cm^3) */
  /* linear-order (l = 1) NES and pair kernels as fractions of the isotropic
   * ones, Phi_1 = phi1 Phi_0 (0, 0); nonzero values add the Phi_1 terms of
   * Eqs. zerothMomentCollisionTerm_NES/_Pair and
   * firstMomentCollisionTerm_NES/_Pair to nmc_solve_batch_v (the zero-velocity
   * solve, with one flux component and no closure, ignores them); each in
   * [-1/3, 1/3], the range that keeps the linear angular kernel non-negative */
  double phi1_nes, phi1_pair;
  /* equilibrium D^Eq (Sec. 3.5.2).  0 (default): the Fermi-Dirac function at
   * the nodes.  1: the eps^2-weighted L2 projection of the Fermi-Dirac
   * distribution onto each energy element (Eq. fermiDiracProjection) with the
   * bound-enforcing limiter that keeps it in [deq_min, deq_max] at the nodes
   * and element edges without changing the element average; the NES and pair
   * kernels then take their detailed-balance factors from its odds D / (1 -
   * D), per species (Eqs. detailedBalanceNES, detailedBalancePair).  The
   * projection runs in nmc_solve_batch with 32 nodes and kernel_store
   * NMC_KERNELS_ON_CHIP or NMC_KERNELS_PAIRED; the O(v) solve, the PD-ARS
   * step and the adjoint return NMC_E_UNSUPPORTED for it. */
  int fd_projection;
  double deq_min;      /* D_min, in [1e-150, 1e-3] (1e-150) */
  double deq_max;      /* D_max, in [0.999, 1 - 1e-15] (1 - 1e-12) */
} nmc_model_desc;

typedef struct {
  double tol_inner;    /* Algorithm innerConverged tolerance (1e-10) */
  double tol_outer;    /* Algorithm outerConverged tolerance (1e-10) */
  int m_inner;         /* Anderson memory of the inner loop, 1 (Picard) .. 3 (3) */
  int m_outer;         /* Anderson memory of the outer loop, 1 .. 3 (3) */
  int max_inner;       /* cap per inner loop (100) */
  int max_outer;       /* cap on outer iterations (50) */
  int fixed_matter;    /* 1: opacities once at y*, no matter update (semi-implicit) */
} nmc_solver_params;

typedef struct {
  const double* D0;    /* (P, ns, nq) number moments D* */
  const double* I0;    /* (P, ns, nq) number-flux moments I* */
  const double* rho11; /* (P) */
  const double* ye0;   /* (P) Ye* */
  const double* e0;    /* (P) e* [MeV/baryon] */
  const double* chi0;  /* (P) absorption scale [1/km] or NULL for chi_ref * rho11 */
  const double* T_fixed;  /* (P) or NULL: with fixed_matter, temperature used instead of the EOS */
  const double* mu_fixed; /* (P) or NULL: with fixed_matter, nu_e chemical potential used instead */
  const double* theta; /* (nq + 2): per-node EmAb scales s_q, then a_nes, a_pair [1/(km MeV^5) per rho11] */
} nmc_batch_in;

typedef struct {
  double* D;           /* (P, ns, nq); may alias D0 */
  double* I;           /* (P, ns, nq); may alias I0 */
  double* ye;          /* (P); may alias ye0 */
  double* e;           /* (P); may alias e0 */
  double* T;           /* (P) temperature of the output state */
  int32_t* n_outer;    /* (P) outer iterations (0 for skipped points) */
  int32_t* n_inner;    /* (P) inner iterations summed over outer iterations */
  int32_t* status;     /* (P) NMC_STATUS_* */
} nmc_batch_out;

typedef struct {
  int blocks_per_cu;   /* resident work-groups per compute unit for the persistent grid (0 = auto) */
  int chunk;           /* points taken per work-queue grab (>= 1) */
  int persistent;      /* 1: persistent grid with an atomic work queue; 0: one work-group per chunk */
  int kernel_store;    /* NMC_KERNELS_ON_CHIP or NMC_KERNELS_HBM (see below) */
} nmc_launch;

/* Where the energy-coupling kernel matrices live during a solve, and how
 * the 32-node solve maps points to wavefronts.
 * ON_CHIP: the library's default.  32 nodes: as PAIRED; 64 nodes: as REGEN.
 * HBM: 64-node solve only, for the roofline study of precomputed kernels:
 *   Phi_in, Phi_out and Phi_ann of every point are written to the workspace
 *   once per outer iteration and re-read by every inner iteration; the
 *   workspace then needs nmc_kernel_store_bytes(m, P) more bytes after the
 *   nmc_workspace_bytes(m, P) ones. */
#define NMC_KERNELS_ON_CHIP 0
#define NMC_KERNELS_HBM 1
/* REGEN: kernel entries regenerated from per-node factors in every inner
 * iteration, nothing stored (the 64-node solve always works this way; for 32
 * nodes it is an alternative to the register-resident rows). */
#define NMC_KERNELS_REGEN 2
/* REGISTERS: 32 nodes only: the kernel rows are assembled once per outer
 * iteration (LDS tile) and held in VGPRs; the inner iterations contract them
 * with DPP row broadcasts. */
#define NMC_KERNELS_REGISTERS 3
/* PAIRED: 32 nodes only: two points per wavefront, one per half; each lane
 * owns one node of its point (both moments) and contracts all 32 columns of
 * its row, the columns broadcast from registers (DPP); the lane's pair
 * factors exp(-|e - e'| / (2T)) are computed once per outer iteration and
 * kept in VGPRs. */
#define NMC_KERNELS_PAIRED 4
/* WAVE: 32 nodes only: one point per wavefront, the two lane halves owning
 * the number and flux moments and splitting the 32 columns; the lane's 16
 * pair factors are computed once per outer iteration and kept in VGPRs. */
#define NMC_KERNELS_WAVE 5

/* Defaults of the descriptors above (values in parentheses). */
void nmc_model_desc_default(nmc_model_desc* desc);
void nmc_solver_params_default(nmc_solver_params* prm);

/* Energy grid (Sec. 3.1.2; Eq. energy_integration_weights): nodes eps_q and
 * weights w2_q = w_q eps_q^2 dEps_e [MeV^3], w3_q = w2_q eps_q, with the
 * 2-point Legendre-Gauss rule on (-1/2, 1/2).  The constant 4 pi / h^3 of
 * W^(2) is folded into the coupling constant and kernel amplitudes. */
int nmc_grid_create(const nmc_grid_desc* desc, nmc_grid** out);
/* Host copies of the grid; any output pointer may be NULL. */
int nmc_grid_query(const nmc_grid* g, int* nq, double* eps, double* w2, double* w3);
int nmc_grid_destroy(nmc_grid* g);

/* Model: species set, physics flags and constants on a grid.  The matter
 * coupling constant is K = (4 pi / (hc)^3) * m_u / (1e11 rho11) [MeV^-3].
 * NMC_PAIR requires every species' pair partner to be present. */
int nmc_model_create(const nmc_grid* g, const nmc_model_desc* desc, nmc_model** out);
int nmc_model_destroy(nmc_model* m);
/* Bytes of device workspace a solve call with P points needs. */
size_t nmc_workspace_bytes(const nmc_model* m, int64_t P);
/* Extra workspace bytes of a solve with kernel_store = NMC_KERNELS_HBM:
 * 3 nq^2 doubles per point (0 if the model cannot use that mode). */
size_t nmc_kernel_store_bytes(const nmc_model* m, int64_t P);

/* Batched forward solve: Algorithm neutrinoMatterCoupling at every point.
 * Outputs may alias inputs (in-place step).  The output matter state is the
 * matter right-hand side evaluated at the final moments, so lepton number and
 * energy balance hold to rounding.  `ws` is device workspace of at least
 * nmc_workspace_bytes(m, P) bytes, 256-byte aligned, not shared with a
 * concurrently running call.  `launch` may be NULL: persistent grid, one
 * point per grab, kernels on chip (the Python layer passes the autotuned
 * shape).  Returns NMC_E_UNSUPPORTED for grids other than 32 or 64 nodes. */
int nmc_solve_batch(const nmc_model* m, const nmc_solver_params* prm, int64_t P, double dtau,
                    const nmc_batch_in* in, const nmc_batch_out* out, void* ws, size_t ws_bytes,
                    const nmc_launch* launch, void* stream);

/* The batched forward solve of nmc_solve_batch for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  It takes no workspace: the work-queue
 * counters live in a static device array of 4 MiB (one copy per device,
 * held until the process ends) that the call clears with a kernel before
 * its solve.  Inputs, outputs, launch and stream are as for
 * nmc_solve_batch, with the same results; nothing is allocated or freed.
 * With launch->kernel_store = NMC_KERNELS_HBM the kernel store also lives
 * there, so P is limited to what fits (NMC_E_WORKSPACE beyond: 2 KiB of
 * counters plus nmc_kernel_store_bytes(m, P) must not exceed 4 MiB).
 * Every call on a device shares that device's array, so calls that overlap
 * on one device (concurrent streams, threads) race and must be serialised
 * by the caller; a call on a model whose device has no scratch address
 * returns NMC_E_HIP. */
int nmc_solve_batch_noalloc(const nmc_model* m, const nmc_solver_params* prm, int64_t P, double dtau,
                            const nmc_batch_in* in, const nmc_batch_out* out, const nmc_launch* launch,
                            void* stream);

/* Implicit-function-theorem adjoint of the forward solve at its converged
 * state (fwd holds the forward outputs for inputs `in`, solved with `prm`;
 * NULL means the defaults).  The adjoint differentiates the coupled system
 * (moments and matter), so a forward run with prm->fixed_matter set is
 * rejected with NMC_E_UNSUPPORTED.  With per-point loss
 * L_p = gbar[2p] (e*_p - e_p) + gbar[2p+1] (Ye_p - Ye*_p), it ADDS
 * dL/dtheta = sum_p -lambda_p^T dR_p/dtheta to grad_theta (nq + 2), where
 * R_x^T lambda_p = dL_p/dx at x = (D, Ye, e); grad_pp (P, nq + 2) receives the
 * per-point terms if not NULL.  Points with nonzero status or skipped points
 * contribute zero.  The summation over points is deterministic.
 * Reads in->rho11, in->theta, in->chi0 (may be NULL) and fwd->{D, ye, e,
 * status, n_outer}; gbar is (P, 2) on the device.  `ws` as for the forward
 * call (nmc_workspace_bytes(m, P), 256-byte aligned).  32-node grids only
 * (NMC_E_UNSUPPORTED otherwise).  A singular Jacobian (a zero or non-finite
 * pivot) makes that point's terms NaN. */
int nmc_solve_batch_adjoint(const nmc_model* m, const nmc_solver_params* prm, int64_t P, double dtau,
                            const nmc_batch_in* in, const nmc_batch_out* fwd, const double* gbar,
                            double* grad_theta, double* grad_pp, void* ws, size_t ws_bytes, void* stream);

/* O(v) solve: nonzero fluid velocity (the O(v/c) two-moment model of
 * Sec. 2, solved as in Sec. 3.5).  The moment equations keep every velocity
 * term of Eqs. implicitNumberNodal / implicitNumberFluxNodal and are
 * iterated in the fixed-point form of Eq. implicitMomentsNodal with
 * lambda = 1 / (1 + |v|); the flux equation is closed with the Minerbo
 * Eddington tensor (Eqs. eddingtonFactorMinerbo, eddingtonTensor; flux
 * factor |I| / D limited to [0, 1]).  The matter state y = (Ye, ef, v) holds
 * the specific fluid energy ef = e + m_u c^2 |v|^2 / 2 [MeV/baryon] (the EOS
 * sees e) and the velocity v in units of c; Eq. implicitFluidNodal moves
 * into it the changes of the Eulerian neutrino lepton number, energy and
 * momentum of Eqs. eulerianNumberLG, eulerianEnergyLG, eulerianMomentumLG
 * (momentum per baryon divided by m_u c^2 = 931.494 MeV).  The old state is
 * given in primitive moments; the old conserved moments N* = D* + v*.I* and
 * G*_j = I*_j + v*^i K*_ij are formed from it.  The outer test compares Ye
 * and ef against y* componentwise and each velocity component against the
 * speed max(|v*|, |v^[k+1]|).  The output matter state is the matter
 * right-hand side at the final moments and the matter iterate they were
 * solved at.  Same status codes, skip rule and in-place aliasing as
 * nmc_solve_batch. */
typedef struct {
  const double* D0;    /* (P, ns, nq) number moments D* */
  const double* I0;    /* (P, ns, 3, nq) number-flux moments: component j of species s at [p][s][j][:] */
  const double* rho11; /* (P) */
  const double* ye0;   /* (P) Ye* */
  const double* ef0;   /* (P) ef* [MeV/baryon], internal plus kinetic */
  const double* v0;    /* (P, 3) fluid velocity v* [c] */
  const double* chi0;  /* (P) absorption scale [1/km] or NULL for chi_ref * rho11 */
  const double* theta; /* (nq + 2) as in nmc_batch_in */
} nmc_batch_v_in;

typedef struct {
  double* D;           /* (P, ns, nq); may alias D0 */
  double* I;           /* (P, ns, 3, nq); may alias I0 */
  double* ye;          /* (P); may alias ye0 */
  double* ef;          /* (P); may alias ef0 */
  double* v;           /* (P, 3); may alias v0 */
  double* T;           /* (P) temperature of the output state */
  int32_t* n_outer;    /* (P) */
  int32_t* n_inner;    /* (P) */
  int32_t* status;     /* (P) NMC_STATUS_* */
} nmc_batch_v_out;

/* Batched O(v) forward solve.  32-node grids only (NMC_E_UNSUPPORTED
 * otherwise).  launch->kernel_store NMC_KERNELS_ON_CHIP (default) or
 * NMC_KERNELS_PAIRED: two points per wavefront, each lane owning the four
 * moments of its node; NMC_KERNELS_WAVE: one point per wavefront.  Both
 * carry the linear-order corrections when phi1_nes or phi1_pair is nonzero.
 * Other modes return NMC_E_UNSUPPORTED.  Workspace, launch, stream and error
 * rules as for nmc_solve_batch; dtau must be positive. */
int nmc_solve_batch_v(const nmc_model* m, const nmc_solver_params* prm, int64_t P, double dtau,
                      const nmc_batch_v_in* in, const nmc_batch_v_out* out, void* ws, size_t ws_bytes,
                      const nmc_launch* launch, void* stream);

/* Primitive-moment recovery (Sec. 3.4): for every point, species and node,
 * the primitive moments M = (D, I_j) of the conserved ones U = (N, G_j) at
 * fluid velocity v, i.e. N = D + v^i I_i, G_j = I_j + v^i K_ij(M) with the
 * Minerbo tensor (Eq. conservedToPrimitive), by the fixed-point sequence of
 * Eqs. c2p_FP / c2p_sequence (lambda = 1 / (1 + |v|), from M = U) with
 * Anderson acceleration, until ||M^[k+1] - M^[k]|| <= tol ||U||
 * (Euclidean over the four moments). */
typedef struct {
  int mem;       /* Anderson memory, 1 (Picard) .. 3 (3) */
  double tol;    /* relative tolerance (1e-8) */
  int max_it;    /* iteration cap (100) */
} nmc_c2p_params;
void nmc_c2p_params_default(nmc_c2p_params* cp);

/* N (P, ns, nq), G (P, ns, 3, nq), v (P, 3) -> D (P, ns, nq), I (P, ns, 3, nq);
 * iters (P, ns, nq) int32: iterations taken, -1 where the cap was reached
 * (the last iterate is returned), -2 on a non-finite iterate.  Device arrays;
 * D and I must not alias N and G.  Any node count and species set of the
 * model. */
int nmc_primitive_recovery(const nmc_model* m, const nmc_c2p_params* cp, int64_t P, const double* N,
                           const double* G, const double* v, double* D, double* I, int32_t* iters, void* stream);

/* One time step of the IMEX scheme with the PD-ARS tableau (Eq.
 * butcherPDARS) for the neutrino-matter coupling alone (the explicit
 * operator, phase-space advection, is outside this library and zero here):
 * stage 2 solves the modified backward-Euler problem of nmc_solve_batch_v
 * with step dt from the initial state; the stage-3 initial state is
 * U^n + (a_32 / a_22)(U^(2) - U^n) in conserved moments (and likewise the
 * matter state), recovered to primitive moments as nmc_primitive_recovery
 * does; stage 3 solves with step dt / 2 from it, and its solution is the
 * step's result (the scheme is globally stiffly accurate).  Points below
 * the coupling density pass through.  n_outer / n_inner count both solves;
 * status is the first non-OK of stage 2, the recovery (MAX_INNER where it hit
 * its cap, NONFINITE) and stage 3.  Inputs, outputs, aliasing and launch as
 * for nmc_solve_batch_v; ws: nmc_pdars_workspace_bytes(m, P) bytes,
 * 256-byte aligned. */
size_t nmc_pdars_workspace_bytes(const nmc_model* m, int64_t P);
int nmc_pdars_step_v(const nmc_model* m, const nmc_solver_params* prm, const nmc_c2p_params* cp, int64_t P,
                     double dt, const nmc_batch_v_in* in, const nmc_batch_v_out* out, void* ws, size_t ws_bytes,
                     const nmc_launch* launch, void* stream);

/* Initial neutrino state from raw draws: e0 = EOS(T, Ye, rho11),
 * D0 = clip(D_eq(T, mu) (a + b uD), 0, 1 - 1e-12), I0 = c D0 uI, with mu from
 * the EOS when mu is NULL.  All arrays are device pointers; e0 may be NULL. */
int nmc_init_state(const nmc_model* m, int64_t P, const double* T, const double* mu,
                   const double* rho11, const double* ye, const double* uD, const double* uI,
                   double a, double b, double c, double* D0, double* I0, double* e0, void* stream);

const char* nmc_error_string(int code);
const char* nmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NMC_H */
