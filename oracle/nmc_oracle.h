/*
 * Test infrastructure, not product code.
 *
 * Plain, slow, obviously-correct FP64 CPU oracle for the implicit (backward
 * Euler) neutrino-matter coupling solve of the two-moment DG-IMEX scheme
 * (paper Sec. 3.5, Eqs. implicitNumberNodal ... implicitFluidNodal and
 * Algorithms neutrinoMatterCoupling / innerConverged / outerConverged).
 *
 * It shares no code with the HIP library: only tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  Every routine cites the
 * passage it follows; readings of silent or garbled passages are listed in the
 * design notes of the repository.
 */
#ifndef NMC_ORACLE_H
#define NMC_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORA_MAX_NQ 64
#define ORA_MAX_NS 3

/* species identities */
#define ORA_NU_E 0
#define ORA_NU_E_BAR 1
#define ORA_NU_X 2

/* physics flags */
#define ORA_EMAB 1u
#define ORA_ISO 2u
#define ORA_NES 4u
#define ORA_PAIR 8u

/* per-point status */
#define ORA_OK 0
#define ORA_MAX_OUTER 1
#define ORA_MAX_INNER 2
#define ORA_NONFINITE 3
#define ORA_EOS_DOMAIN 4

typedef struct {
  int nq, ns;
  int species[ORA_MAX_NS];
  double eps[ORA_MAX_NQ]; /* node energies [MeV] */
  double w2[ORA_MAX_NQ];  /* w_q eps_q^2 dEps [MeV^3] (4 pi / h^3 factored out) */
  double w3[ORA_MAX_NQ];  /* w2 * eps [MeV^4] */
  unsigned flags;
  double chi_ref, eps_ref, chi_power, sigma_ratio;
  double eos_a, eos_b, mu_a, mu_ye0, mu_b, mu_t0;
  double kcoup; /* (4 pi/(hc)^3) * m_u / 1e11 [MeV^-3]; K = kcoup / rho11 */
  double rho11_min; /* coupling disabled below this density (Sec. 7.2) */
  /* linear-order (l = 1) Legendre coefficients of the NES and pair kernels as
   * fractions of the isotropic ones: Phi_1^{In/Out} = phi1_nes Phi_0^{In/Out},
   * Phi_1^{Pro/Ann} = phi1_pair Phi_0^{Pro/Ann} (0: isotropic kernels).  They
   * enter the O(v) solve through Eqs. zerothMomentCollisionTerm_NES/_Pair and
   * firstMomentCollisionTerm_NES/_Pair. */
  double phi1_nes, phi1_pair;
  /* 1: the equilibrium D_eq is the weighted L2 projection of the Fermi-Dirac
   * distribution onto each energy element with the bound-enforcing limiter
   * into [deq_min, deq_max] (Eq. fermiDiracProjection), and the NES and pair
   * kernels obey detailed balance with it (Eqs. detailedBalanceNES,
   * detailedBalancePair); 0: pointwise nodal values */
  int fd_projection;
  double deq_min, deq_max;
  double edges[ORA_MAX_NQ / 2 + 1]; /* element edges [MeV], nq / 2 + 1 of them */
} ora_model;

typedef struct {
  double tol_inner, tol_outer;
  int m_inner, m_outer, max_inner, max_outer, fixed_matter;
} ora_params;

/* grids */
int ora_grid_loguniform(int n_elem, double eps_lo, double eps_hi, double* edges, double* eps, double* w2,
                        double* w3);
int ora_grid_zoom(int n_elem, double zoom, double width, double* edges, double* eps, double* w2, double* w3);

/* model default constants */
void ora_model_defaults(ora_model* m);

/* thermodynamics */
double ora_fermi_dirac(double eps, double mu, double T);
double ora_fermi_dirac_complement(double eps, double mu, double T);
double ora_eos_energy(const ora_model* m, double T, double ye, double rho11);
double ora_eos_temperature(const ora_model* m, double e, double ye, double rho11);
double ora_eos_mu(const ora_model* m, double ye, double T, double rho11);

/* Gauss-Legendre rule with n points on (-1, 1) */
int ora_gauss_legendre(int n, double* x, double* w);
/* weighted L2 projection of the Fermi-Dirac distribution f(eps; mu, T) onto
 * the linear polynomials of every energy element (Eq. fermiDiracProjection):
 * dtil (nq) the projection's nodal values, dlim (nq) after the
 * bound-enforcing limiter, clim (nq) the limited complement 1 - D (any may be
 * NULL) */
void ora_fd_projection(const ora_model* m, double T, double mu, double* dtil, double* dlim, double* clim);
/* NES and pair kernels of species s with detailed balance for equilibrium
 * odds o_s = D_eq / (1 - D_eq) (Eqs. detailedBalanceNES, detailedBalancePair):
 * odds (ns, nq) -> phi_in, phi_out, phi_pro (ns, nq, nq), phi_ann (nq, nq) */
void ora_kernels_odds(const ora_model* m, const double* theta, double rho11, double T, const double* odds,
                      double* phi_in, double* phi_out, double* phi_pro, double* phi_ann);

/* opacities and kernels at (T, mu) for one point */
void ora_kernels(const ora_model* m, const double* theta, double rho11, double T,
                 double* phi_in, double* phi_out, double* phi_pro, double* phi_ann);
void ora_rates(const ora_model* m, const double* theta, double rho11, double chi0, double T, double mu,
               const double* D, double* eta, double* chi, double* kappa);

/* Anderson step on generic vectors (history oldest first) */
int ora_anderson(int n, int mem, const double* Qh, const double* Fh, double* out);

/* batched forward solve (Algorithm neutrinoMatterCoupling) */
int ora_solve_batch(const ora_model* m, const ora_params* prm, const double* theta, long P, double dtau,
                    const double* D0, const double* I0, const double* rho11, const double* ye0,
                    const double* e0, const double* chi0, const double* T_fixed, const double* mu_fixed,
                    double* D, double* I, double* ye, double* e, double* T,
                    int* n_outer, int* n_inner, int* status, int nthreads);

/* implicit-system residual (definition of the result) at one point */
void ora_residual(const ora_model* m, const double* theta, double dtau, double rho11, double chi0,
                  const double* Dstar, const double* Istar, double ye_star, double e_star,
                  const double* D, const double* I, double ye, double e, double* R);

/* analytic Jacobian of the (D, Ye, e) residual block at one point, n = ns*nq + 2, row-major */
int ora_jacobian(const ora_model* m, const double* theta, double dtau, double rho11, double chi0,
                 const double* D, double ye, double e, double* J);

/* dense Newton on the full residual (tiny problems) */
int ora_newton(const ora_model* m, const double* theta, double dtau, double rho11, double chi0,
               const double* Dstar, const double* Istar, double ye_star, double e_star,
               double* D, double* I, double* ye, double* e, double tol, int max_it);

/* implicit-function-theorem adjoint, dense LU, summed gradient */
int ora_adjoint_batch(const ora_model* m, const double* theta, long P, double dtau, const double* rho11,
                      const double* chi0, const double* D, const double* ye, const double* e,
                      const double* gbar, double* grad_theta, double* grad_pp, int nthreads);

/* ---- O(v) coupling: nonzero fluid velocity (Sec. 3.5.1 in full) ----------
 * Moments per point: D (ns, nq) and the three flux components I (ns, 3, nq);
 * matter y = (Ye, ef, v_1, v_2, v_3) with ef the specific fluid energy
 * (internal plus kinetic) in MeV per baryon and v in units of c. */
#define ORA_MU_C2 931.49410242 /* atomic mass unit rest energy [MeV] */

/* Minerbo Eddington factor psi(h) (Eq. eddingtonFactorMinerbo) */
double ora_minerbo_psi(double h);
/* flux factor h = |I| / D used by the closure, in [0, 1] */
double ora_flux_factor(double D, double Imag);
/* K_ij = k_ij D (Eq. eddingtonTensor with the Minerbo factor), 3x3 row-major */
void ora_eddington(double D, const double* I3, double* K9);

/* linear-order corrections of the NES and pair collision terms at one point
 * (Eqs. linearCorrectionsNES, linearCorrectionsPair and their use in Eqs.
 * zerothMomentCollisionTerm_NES/_Pair, firstMomentCollisionTerm_NES/_Pair):
 * C1D (ns, nq) adds to the number equation, C1I (ns, 3, nq) to the flux
 * equations, at moments D (ns, nq), I (ns, 3, nq) and temperature T */
void ora_phi1_terms(const ora_model* m, const double* theta, double rho11, double T, const double* D,
                    const double* I, double* C1D, double* C1I);

/* batched O(v) forward solve (Algorithm neutrinoMatterCoupling with
 * Eqs. implicitMomentsNodal at lambda = 1/(1+|v|), implicitFluidNodal,
 * eulerianMomentumLG, eulerianEnergyLG, eulerianNumberLG) */
int ora_solve_batch_v(const ora_model* m, const ora_params* prm, const double* theta, long P, double dtau,
                      const double* D0, const double* I0, const double* rho11, const double* ye0,
                      const double* ef0, const double* v0, const double* chi0,
                      double* D, double* I, double* ye, double* ef, double* v, double* T,
                      int* n_outer, int* n_inner, int* status, int nthreads);

/* primitive-moment recovery (Sec. 3.4, Eqs. c2p_FP, c2p_sequence): conserved
 * N (P, ns, nq), G (P, ns, 3, nq) at velocity v (P, 3) -> primitive D, I;
 * iters (P, ns, nq): iterations, -1 at the cap, -2 on a non-finite iterate */
int ora_primitive_batch(const ora_model* m, long P, const double* N, const double* G, const double* v, int mem,
                        double tol, int max_it, double* D, double* I, int* iters, int nthreads);

/* one IMEX step with the PD-ARS tableau (Eq. butcherPDARS) of the coupling
 * alone: two modified backward-Euler solves (steps dt, dt/2) with the stage
 * combination in conserved variables and primitive recovery between them */
int ora_pdars_step_v(const ora_model* m, const ora_params* prm, const double* theta, long P, double dt,
                     const double* D0, const double* I0, const double* rho11, const double* ye0,
                     const double* ef0, const double* v0, const double* chi0, int c2p_mem, double c2p_tol,
                     int c2p_max, double* D, double* I, double* ye, double* ef, double* v, double* T,
                     int* n_outer, int* n_inner, int* status, int nthreads);

/* initial state from raw draws */
int ora_init_state(const ora_model* m, long P, const double* T, const double* mu, const double* rho11,
                   const double* ye, const double* uD, const double* uI, double a, double b, double c,
                   double* D0, double* I0, double* e0);

#ifdef __cplusplus
}
#endif
#endif
