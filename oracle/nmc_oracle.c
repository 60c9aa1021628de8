/*
 * Test infrastructure, not product code: the plain FP64 CPU oracle of the
 * implicit neutrino-matter coupling solve.  Only tests, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code, header, table
 * or helper with the HIP library.
 *
 * Built with -O2 -ffp-contract=off so every multiply and add rounds as written.
 * Loops are plain; nothing is blocked, fused or reordered beyond what the
 * paper's definitions state.  Citations name sections, equations and
 * algorithms of the paper (arXiv 2601.00976).
 *
 * Parity pins (tests/test_oracle_*.py): grid and weights (Table energyGrids,
 * Eq. energy_integration_weights), Fermi-Dirac and EOS closed forms, kernel
 * in-out invariance and detailed balance (Eqs. inOutInvarianceNES ...
 * detailedBalancePair), number / lepton-number conservation of the collision
 * contractions, the emission-absorption closed form (Eqs. implicitNumberNodal,
 * implicitNumberFluxNodal, emissivityEmAbNodal), the equilibrium fixed point,
 * the large-dtau equilibrium limit, Newton on tiny problems, Anderson finite
 * termination on linear maps, and finite differences for the Jacobian and the
 * adjoint.  The O(v) solve is pinned by the Minerbo closure's limits, trace
 * and eigen-structure and its fit to the exact maximum-entropy closure, the
 * dtau = 0 identity, the moving-equilibrium fixed point, the reduction to the
 * static solve at v = 0 without flux, and dense Newton on the unrearranged
 * implicit equations.  Exact iteration counts and intermediate iterates are
 * parity unpinned.
 */
#include "nmc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXN (2 * ORA_MAX_NS * ORA_MAX_NQ)
#define MAXMEM 8

/* ------------------------------------------------------------------------ */
/* Energy grid: Sec. 3.1.2 (nodes eps_q = eps_e + dEps_e xi_q on the reference
 * interval (-1/2, 1/2), Legendre-Gauss points, weights summing to one) and
 * Eq. energy_integration_weights (W2 = 4 pi w eps^2 dEps / h^3; the constant
 * 4 pi / h^3 is carried by the coupling constants instead). */

static void lg2(double* xi, double* w) {
  /* 2-point Legendre-Gauss rule on (-1/2, 1/2): xi = -/+ 1/(2 sqrt 3), w = 1/2 */
  xi[0] = -0.5 / sqrt(3.0);
  xi[1] = 0.5 / sqrt(3.0);
  w[0] = 0.5;
  w[1] = 0.5;
}

static void fill_nodes(int n_elem, const double* edges, double* eps, double* w2, double* w3) {
  double xi[2], w[2];
  lg2(xi, w);
  for (int e = 0; e < n_elem; ++e) {
    double lo = edges[e], hi = edges[e + 1];
    double c = 0.5 * (lo + hi), d = hi - lo;
    for (int q = 0; q < 2; ++q) {
      int g = e * 2 + q; /* global energy index (Sec. 3.1.2) */
      eps[g] = c + d * xi[q];
      w2[g] = w[q] * eps[g] * eps[g] * d;
      w3[g] = w2[g] * eps[g];
    }
  }
}

int ora_grid_loguniform(int n_elem, double eps_lo, double eps_hi, double* edges, double* eps, double* w2,
                        double* w3) {
  /* geometric element edges eps_lo * (eps_hi/eps_lo)^(e/n_elem) */
  if (n_elem < 1 || 2 * n_elem > ORA_MAX_NQ || !(eps_lo > 0) || !(eps_hi > eps_lo)) return -1;
  for (int e = 0; e <= n_elem; ++e) edges[e] = eps_lo * pow(eps_hi / eps_lo, (double)e / n_elem);
  edges[n_elem] = eps_hi;
  fill_nodes(n_elem, edges, eps, w2, w3);
  return 0;
}

int ora_grid_zoom(int n_elem, double zoom, double width, double* edges, double* eps, double* w2, double* w3) {
  /* Table energyGrids: dEps_{e+1} = zoom * dEps_e on [0, width] */
  if (n_elem < 1 || 2 * n_elem > ORA_MAX_NQ || !(zoom > 0) || !(width > 0)) return -1;
  double d1;
  if (zoom == 1.0) d1 = width / n_elem;
  else d1 = width * (zoom - 1.0) / (pow(zoom, n_elem) - 1.0);
  edges[0] = 0.0;
  double d = d1;
  for (int e = 0; e < n_elem; ++e) {
    edges[e + 1] = edges[e] + d;
    d *= zoom;
  }
  fill_nodes(n_elem, edges, eps, w2, w3);
  return 0;
}

void ora_model_defaults(ora_model* m) {
  memset(m, 0, sizeof(*m));
  m->flags = ORA_EMAB | ORA_ISO | ORA_NES | ORA_PAIR;
  m->chi_ref = 10.0;   /* km^-1 per rho11 */
  m->eps_ref = 10.0;   /* MeV */
  m->chi_power = 2.0;
  m->sigma_ratio = 0.5;
  m->eos_a = 1.5;
  m->eos_b = 3.0;
  m->mu_a = 20.0;
  m->mu_ye0 = 0.3;
  m->mu_b = 5.0;
  m->mu_t0 = 5.0;
  {
    const double hc = 1.239841984e-10;    /* MeV cm */
    const double m_u = 1.66053906660e-24; /* g */
    const double pi = 3.14159265358979323846;
    m->kcoup = 4.0 * pi / (hc * hc * hc) * m_u / 1.0e11;
  }
  m->rho11_min = 1.0e-4; /* 1e7 g/cm^3 */
  m->fd_projection = 0;
  m->deq_min = 1.0e-150;
  m->deq_max = 1.0 - 1.0e-12;
}

/* ------------------------------------------------------------------------ */
/* Thermodynamics.  Fermi-Dirac equilibrium: App. B, Eq. FermiDiracDistribution,
 * evaluated at the node energy (pointwise nodal values). */

double ora_fermi_dirac(double eps, double mu, double T) {
  double x = (eps - mu) / T;
  if (x > 0.0) {
    double t = exp(-x);
    return t / (1.0 + t);
  }
  return 1.0 / (1.0 + exp(x));
}

double ora_fermi_dirac_complement(double eps, double mu, double T) {
  double x = (eps - mu) / T;
  if (x > 0.0) return 1.0 / (1.0 + exp(-x));
  double t = exp(x);
  return t / (1.0 + t);
}

/* synthetic closed-form EOS: e = a T (1 + Ye) + b Ye^(4/3) rho11^(1/3) [MeV/baryon] */
double ora_eos_energy(const ora_model* m, double T, double ye, double rho11) {
  return m->eos_a * T * (1.0 + ye) + m->eos_b * pow(ye, 4.0 / 3.0) * cbrt(rho11);
}

double ora_eos_temperature(const ora_model* m, double e, double ye, double rho11) {
  return (e - m->eos_b * pow(ye, 4.0 / 3.0) * cbrt(rho11)) / (m->eos_a * (1.0 + ye));
}

/* mu_nu_e = mu_a (Ye - ye0) rho11^(1/3) + mu_b ln(T / T0) [MeV] */
double ora_eos_mu(const ora_model* m, double ye, double T, double rho11) {
  return m->mu_a * (ye - m->mu_ye0) * cbrt(rho11) + m->mu_b * log(T / m->mu_t0);
}

/* ------------------------------------------------------------------------ */
/* Species bookkeeping: lepton numbers g = (+1, -1, 0) (Sec. 2.2), energy
 * multiplicity d = (1, 1, 4) for the heavy-lepton stand-in, chemical-potential
 * sign (+1, -1, 0), pair partner (nu_e <-> anti-nu_e, nu_x <-> nu_x) and
 * emission/absorption only for the electron flavours (Table opacities). */

static double sp_g(int id) { return id == ORA_NU_E ? 1.0 : (id == ORA_NU_E_BAR ? -1.0 : 0.0); }
static double sp_d(int id) { return id == ORA_NU_X ? 4.0 : 1.0; }
static double sp_musign(int id) { return id == ORA_NU_E ? 1.0 : (id == ORA_NU_E_BAR ? -1.0 : 0.0); }
static int sp_emab(int id) { return id != ORA_NU_X; }
static int sp_partner_id(int id) { return id == ORA_NU_E ? ORA_NU_E_BAR : (id == ORA_NU_E_BAR ? ORA_NU_E : ORA_NU_X); }

static int partner_index(const ora_model* m, int s) {
  int want = sp_partner_id(m->species[s]);
  for (int t = 0; t < m->ns; ++t)
    if (m->species[t] == want) return t;
  return -1;
}

/* ------------------------------------------------------------------------ */
/* Energy-coupling kernels (Eqs. nesRatesNodal, pairRatesNodal) built so that
 * in-out invariance (Eqs. inOutInvarianceNES, inOutInvariancePair) and detailed
 * balance (Eqs. detailedBalanceNES, detailedBalancePair) hold exactly with the
 * pointwise Fermi-Dirac equilibrium:
 *   S(e,e')   = A e e' exp(-|e-e'|/T)
 *   Phi_in    = S exp(-(e-e')/(2T)),  Phi_out = S exp(+(e-e')/(2T))
 *   Phi_ann   = A_p e e' exp(-|e-e'|/T),  Phi_pro = Phi_ann exp(-(e+e')/T)
 * Every exponent is written as exp(-(non-negative)/T). */

static void kernels_unit(const ora_model* m, double T, double a_nes, double a_pair, double* phi_in,
                         double* phi_out, double* phi_pro, double* phi_ann) {
  int nq = m->nq;
  for (int q = 0; q < nq; ++q) {
    for (int p = 0; p < nq; ++p) {
      double eq = m->eps[q], ep = m->eps[p];
      double dlt = eq - ep;
      double adl = fabs(dlt);
      double ee = eq * ep;
      phi_in[q * nq + p] = a_nes * ee * exp(-(adl + 0.5 * dlt) / T);
      phi_out[q * nq + p] = a_nes * ee * exp(-(adl - 0.5 * dlt) / T);
      phi_ann[q * nq + p] = a_pair * ee * exp(-adl / T);
      phi_pro[q * nq + p] = a_pair * ee * exp(-(adl + eq + ep) / T);
    }
  }
}

void ora_kernels(const ora_model* m, const double* theta, double rho11, double T, double* phi_in,
                 double* phi_out, double* phi_pro, double* phi_ann) {
  double a_nes = (m->flags & ORA_NES) ? theta[m->nq] * rho11 : 0.0;
  double a_pair = (m->flags & ORA_PAIR) ? theta[m->nq + 1] * rho11 : 0.0;
  kernels_unit(m, T, a_nes, a_pair, phi_in, phi_out, phi_pro, phi_ann);
}

/* ------------------------------------------------------------------------ */
/* Equilibrium by projection (Sec. 3.5.2, Eq. fermiDiracProjection): on every
 * energy element the linear polynomial D~ with
 *   int_K D~ l_a eps^2 deps = int_K f l_a eps^2 deps   (a = 1, 2),
 * l_a the Lagrange basis on the element's two Legendre-Gauss nodes, followed by
 * the bound-enforcing limiter (Zhang & Shu): D = Dbar + theta (D~ - Dbar) with
 * Dbar the eps^2-weighted element average and the largest theta in [0, 1]
 * that keeps D in [D_min, D_max] at the nodes and at both element edges.
 * The complement 1 - D is projected and limited alongside from 1 - f, so
 * that it keeps its relative accuracy where D is close to one. */

int ora_gauss_legendre(int n, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  if (n < 1 || n > 128) return -1;
  for (int i = 0; i < n; ++i) {
    /* Newton on P_n(z) from the usual cosine guess for its i-th largest root;
     * P_n and P_{n-1} by the three-term recurrence */
    double z = cos(pi * (i + 0.75) / (n + 0.5)), pn = 0.0, pm = 0.0;
    for (int it = 0; it < 100; ++it) {
      pm = 1.0;
      pn = z;
      for (int k = 2; k <= n; ++k) {
        double nx = ((2.0 * k - 1.0) * z * pn - (k - 1.0) * pm) / k;
        pm = pn;
        pn = nx;
      }
      double dz = pn / (n * (z * pn - pm) / (z * z - 1.0));
      z -= dz;
      if (fabs(dz) <= 1e-16) break;
    }
    pm = 1.0;
    pn = z;
    for (int k = 2; k <= n; ++k) {
      double nx = ((2.0 * k - 1.0) * z * pn - (k - 1.0) * pm) / k;
      pm = pn;
      pn = nx;
    }
    double dp = n * (z * pn - pm) / (z * z - 1.0);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  return 0;
}

/* int_a^b eps^2 l_k(eps) g(eps) deps for k = 1, 2, with g = f (comp = 0) or
 * g = 1 - f (comp = 1): composite 16-point Legendre-Gauss rule on pieces no
 * wider than 2T (the Fermi-Dirac function is analytic within pi T of the real
 * axis, so each piece converges to rounding) */
static void fd_moments(double a, double b, double e1, double e2, double mu, double T, int comp,
                       const double* gx, const double* gw, double* out) {
  out[0] = out[1] = 0.0;
  if (!(b > a)) return;
  int npc = (int)ceil((b - a) / (2.0 * T));
  if (npc < 1) npc = 1;
  double h = (b - a) / npc;
  for (int j = 0; j < npc; ++j) {
    double lo = a + j * h, hi = (j == npc - 1) ? b : a + (j + 1) * h;
    double c = 0.5 * (lo + hi), r = 0.5 * (hi - lo);
    for (int k = 0; k < 16; ++k) {
      double e = c + r * gx[k];
      double g = comp ? ora_fermi_dirac_complement(e, mu, T) : ora_fermi_dirac(e, mu, T);
      double wt = r * gw[k] * e * e * g;
      out[0] += wt * (e - e2) / (e1 - e2);
      out[1] += wt * (e - e1) / (e2 - e1);
    }
  }
}

static void fd_project(const ora_model* m, double T, double mu, double* dtil, double* ctil, double* dlim,
                       double* clim) {
  double gx[16], gw[16], x3[3], w3[3];
  ora_gauss_legendre(16, gx, gw);
  ora_gauss_legendre(3, x3, w3);
  const double dmin = m->deq_min, dmax = m->deq_max, cmin = 1.0 - m->deq_max;
  for (int el = 0; el < m->nq / 2; ++el) {
    double lo = m->edges[el], hi = m->edges[el + 1];
    double e1 = m->eps[2 * el], e2 = m->eps[2 * el + 1];
    /* mass matrix int_K l_a l_b eps^2 (degree 4: the 3-point rule is exact) */
    double M11 = 0.0, M12 = 0.0, M22 = 0.0;
    for (int k = 0; k < 3; ++k) {
      double e = 0.5 * (lo + hi) + 0.5 * (hi - lo) * x3[k], wt = 0.5 * (hi - lo) * w3[k] * e * e;
      double l1 = (e - e2) / (e1 - e2), l2 = (e - e1) / (e2 - e1);
      M11 += wt * l1 * l1;
      M12 += wt * l1 * l2;
      M22 += wt * l2 * l2;
    }
    /* right-hand sides; beyond 100 T past the chemical potential the
     * integrand is below exp(-100) of its value there and is dropped */
    double bf[2], bc[2];
    fd_moments(lo, fmin(hi, fmax(lo, mu) + 100.0 * T), e1, e2, mu, T, 0, gx, gw, bf);
    fd_moments(fmax(lo, fmin(hi, mu) - 100.0 * T), hi, e1, e2, mu, T, 1, gx, gw, bc);
    double det = M11 * M22 - M12 * M12;
    double d[2] = {(M22 * bf[0] - M12 * bf[1]) / det, (M11 * bf[1] - M12 * bf[0]) / det};
    double cc[2] = {(M22 * bc[0] - M12 * bc[1]) / det, (M11 * bc[1] - M12 * bc[0]) / det};
    double m0 = (hi * hi * hi - lo * lo * lo) / 3.0;
    double dbar = (bf[0] + bf[1]) / m0, cbar = (bc[0] + bc[1]) / m0;
    /* values at the nodes and at the element edges */
    double lo1 = (lo - e2) / (e1 - e2), lo2 = (lo - e1) / (e2 - e1);
    double hi1 = (hi - e2) / (e1 - e2), hi2 = (hi - e1) / (e2 - e1);
    double mD = fmin(fmin(d[0], d[1]), fmin(d[0] * lo1 + d[1] * lo2, d[0] * hi1 + d[1] * hi2));
    double mC = fmin(fmin(cc[0], cc[1]), fmin(cc[0] * lo1 + cc[1] * lo2, cc[0] * hi1 + cc[1] * hi2));
    for (int a = 0; a < 2; ++a) {
      if (dtil) dtil[2 * el + a] = d[a];
      if (ctil) ctil[2 * el + a] = cc[a];
    }
    double th = 1.0, Dn[2], Cn[2];
    if (dbar < dmin) {
      /* the element average itself lies below the bound: the element takes
       * the bound */
      Dn[0] = Dn[1] = dmin;
      Cn[0] = Cn[1] = 1.0 - dmin;
    } else if (cbar < cmin) {
      Dn[0] = Dn[1] = dmax;
      Cn[0] = Cn[1] = cmin;
    } else {
      if (mD < dmin) th = fmin(th, (dbar - dmin) / (dbar - mD));
      if (mC < cmin) th = fmin(th, (cbar - cmin) / (cbar - mC));
      for (int a = 0; a < 2; ++a) {
        Dn[a] = dbar + th * (d[a] - dbar);
        Cn[a] = cbar + th * (cc[a] - cbar);
      }
    }
    for (int a = 0; a < 2; ++a) {
      if (dlim) dlim[2 * el + a] = Dn[a];
      if (clim) clim[2 * el + a] = Cn[a];
    }
  }
}

void ora_fd_projection(const ora_model* m, double T, double mu, double* dtil, double* dlim, double* clim) {
  fd_project(m, T, mu, dtil, NULL, dlim, clim);
}

/* Kernels of one species with detailed balance for its equilibrium odds o and
 * its pair partner's ob (Eqs. detailedBalanceNES, detailedBalancePair) and
 * in-out invariance (Eqs. inOutInvarianceNES, inOutInvariancePair): the
 * symmetric S splits as Phi_in = S sqrt(o_q / o_p), Phi_out = S sqrt(o_p / o_q),
 * and Phi_pro = o_q ob_p Phi_ann.  With pointwise equilibrium, o = exp((mu -
 * eps)/T), these are the kernels above. */
static void kernels_odds_species(const ora_model* m, double T, double a_nes, double a_pair, const double* o,
                                 const double* ob, double* phi_in, double* phi_out, double* phi_pro,
                                 double* phi_ann) {
  int nq = m->nq;
  for (int q = 0; q < nq; ++q) {
    for (int p = 0; p < nq; ++p) {
      double eq = m->eps[q], ep = m->eps[p];
      double base = eq * ep * exp(-fabs(eq - ep) / T);
      double S = a_nes * base;
      phi_in[q * nq + p] = S * sqrt(o[q] / o[p]);
      phi_out[q * nq + p] = S * sqrt(o[p] / o[q]);
      phi_ann[q * nq + p] = a_pair * base;
      phi_pro[q * nq + p] = ob ? o[q] * ob[p] * (a_pair * base) : 0.0;
    }
  }
}

void ora_kernels_odds(const ora_model* m, const double* theta, double rho11, double T, const double* odds,
                      double* phi_in, double* phi_out, double* phi_pro, double* phi_ann) {
  int nq = m->nq;
  double a_nes = (m->flags & ORA_NES) ? theta[nq] * rho11 : 0.0;
  double a_pair = (m->flags & ORA_PAIR) ? theta[nq + 1] * rho11 : 0.0;
  for (int s = 0; s < m->ns; ++s) {
    int sb = partner_index(m, s);
    kernels_odds_species(m, T, a_nes, a_pair, odds + s * nq, sb >= 0 ? odds + sb * nq : NULL,
                         phi_in + s * nq * nq, phi_out + s * nq * nq, phi_pro + s * nq * nq, phi_ann);
  }
}

/* per-point opacity state, recomputed once per outer iteration
 * (ComputeOpacities in Algorithm neutrinoMatterCoupling) */
typedef struct {
  double T, mu;
  double deq[ORA_MAX_NS * ORA_MAX_NQ];
  double chia[ORA_MAX_NS * ORA_MAX_NQ];
  double sig[ORA_MAX_NS * ORA_MAX_NQ];
  /* per species (ns, nq, nq): with the projected equilibrium the detailed
   * balance factors differ between species */
  double phi_in[ORA_MAX_NS * ORA_MAX_NQ * ORA_MAX_NQ];
  double phi_out[ORA_MAX_NS * ORA_MAX_NQ * ORA_MAX_NQ];
  double phi_pro[ORA_MAX_NS * ORA_MAX_NQ * ORA_MAX_NQ];
  double phi_ann[ORA_MAX_NQ * ORA_MAX_NQ];
} opac;

static void compute_opacities(const ora_model* m, const double* theta, double rho11, double chi0, double T,
                              double mu, opac* o) {
  int nq = m->nq, ns = m->ns;
  o->T = T;
  o->mu = mu;
  double odds[ORA_MAX_NS * ORA_MAX_NQ];
  for (int s = 0; s < ns; ++s) {
    int id = m->species[s];
    double mus = sp_musign(id) * mu;
    if (m->fd_projection) {
      double comp[ORA_MAX_NQ];
      fd_project(m, T, mus, NULL, NULL, o->deq + s * nq, comp);
      for (int q = 0; q < nq; ++q) odds[s * nq + q] = o->deq[s * nq + q] / comp[q];
    }
    for (int q = 0; q < nq; ++q) {
      double shape = chi0 * pow(m->eps[q] / m->eps_ref, m->chi_power);
      /* Eq. emissivityEmAbNodal: eta^EmAb = chi^EmAb * D^Eq */
      if (!m->fd_projection) o->deq[s * nq + q] = ora_fermi_dirac(m->eps[q], mus, T);
      o->chia[s * nq + q] = ((m->flags & ORA_EMAB) && sp_emab(id)) ? theta[q] * shape : 0.0;
      o->sig[s * nq + q] = (m->flags & ORA_ISO) ? m->sigma_ratio * shape : 0.0;
    }
  }
  if (m->fd_projection) {
    ora_kernels_odds(m, theta, rho11, T, odds, o->phi_in, o->phi_out, o->phi_pro, o->phi_ann);
  } else {
    /* pointwise equilibrium: one set of kernels serves every species */
    ora_kernels(m, theta, rho11, T, o->phi_in, o->phi_out, o->phi_pro, o->phi_ann);
    for (int s = 1; s < ns; ++s) {
      memcpy(o->phi_in + s * nq * nq, o->phi_in, sizeof(double) * nq * nq);
      memcpy(o->phi_out + s * nq * nq, o->phi_out, sizeof(double) * nq * nq);
      memcpy(o->phi_pro + s * nq * nq, o->phi_pro, sizeof(double) * nq * nq);
    }
  }
}

/* Eqs. emissivityNodal, opacityNodal, transportOpacityNodal, nesRatesNodal,
 * pairRatesNodal: eta, chi, kappa at every (species, node) for moments D. */
static void rates(const ora_model* m, const opac* o, const double* D, double* eta, double* chi, double* kappa) {
  int nq = m->nq, ns = m->ns;
  for (int s = 0; s < ns; ++s) {
    int sb = partner_index(m, s);
    const double *pin = o->phi_in + s * nq * nq, *pout = o->phi_out + s * nq * nq;
    const double* ppro = o->phi_pro + s * nq * nq;
    for (int q = 0; q < nq; ++q) {
      double eta_nes = 0.0, out_nes = 0.0, eta_pair = 0.0, ann_pair = 0.0;
      if (m->flags & ORA_NES) {
        for (int p = 0; p < nq; ++p) {
          eta_nes += m->w2[p] * pin[q * nq + p] * D[s * nq + p];
          out_nes += m->w2[p] * pout[q * nq + p] * (1.0 - D[s * nq + p]);
        }
      }
      if ((m->flags & ORA_PAIR) && sb >= 0) {
        for (int p = 0; p < nq; ++p) {
          eta_pair += m->w2[p] * ppro[q * nq + p] * (1.0 - D[sb * nq + p]);
          ann_pair += m->w2[p] * o->phi_ann[q * nq + p] * D[sb * nq + p];
        }
      }
      double chi_nes = eta_nes + out_nes;
      double chi_pair = eta_pair + ann_pair;
      int i = s * nq + q;
      eta[i] = o->chia[i] * o->deq[i] + eta_nes + eta_pair;
      chi[i] = o->chia[i] + chi_nes + chi_pair;
      kappa[i] = chi[i] + o->sig[i];
    }
  }
}

void ora_rates(const ora_model* m, const double* theta, double rho11, double chi0, double T, double mu,
               const double* D, double* eta, double* chi, double* kappa) {
  opac* o = (opac*)malloc(sizeof(opac));
  compute_opacities(m, theta, rho11, chi0, T, mu, o);
  rates(m, o, D, eta, chi, kappa);
  free(o);
}

/* ------------------------------------------------------------------------ */
/* Anderson acceleration step (Algorithm neutrinoMatterCoupling, the least
 * squares problems for alpha / beta with sum-to-one constraint).  The
 * constrained problem over the last `mem` residuals is solved in its
 * equivalent difference form: with dF_i = F_{i+1} - F_i, dQ_i likewise,
 *   gamma = argmin || F_last - sum_i gamma_i dF_i ||_2,
 *   x_new = Q_last - sum_i gamma_i dQ_i.
 * Normal equations by Cholesky; a pivot <= 1e-14 * trace drops the oldest
 * column and retries; with no column left the step is Picard.  Returns the
 * number of difference columns used. */
int ora_anderson(int n, int mem, const double* Qh, const double* Fh, double* out) {
  const double* Qlast = Qh + (size_t)(mem - 1) * n;
  const double* Flast = Fh + (size_t)(mem - 1) * n;
  int first = 0; /* oldest difference column in use */
  int ncol = mem - 1;
  double gamma[MAXMEM];
  while (ncol > 0) {
    double G[MAXMEM][MAXMEM], b[MAXMEM], L[MAXMEM][MAXMEM];
    for (int i = 0; i < ncol; ++i) {
      int ci = first + i;
      for (int j = 0; j <= i; ++j) {
        int cj = first + j;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) {
          double di = Fh[(size_t)(ci + 1) * n + k] - Fh[(size_t)ci * n + k];
          double dj = Fh[(size_t)(cj + 1) * n + k] - Fh[(size_t)cj * n + k];
          acc += di * dj;
        }
        G[i][j] = acc;
        G[j][i] = acc;
      }
      double acc = 0.0;
      for (int k = 0; k < n; ++k) {
        double di = Fh[(size_t)(ci + 1) * n + k] - Fh[(size_t)ci * n + k];
        acc += di * Flast[k];
      }
      b[i] = acc;
    }
    double tr = 0.0;
    for (int i = 0; i < ncol; ++i) tr += G[i][i];
    int ok = 1;
    for (int i = 0; i < ncol && ok; ++i) {
      for (int j = 0; j <= i; ++j) {
        double s = G[i][j];
        for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
        if (i == j) {
          if (!(s > 1e-14 * tr)) {
            ok = 0;
            break;
          }
          L[i][i] = sqrt(s);
        } else {
          L[i][j] = s / L[j][j];
        }
      }
    }
    if (!ok) {
      first += 1;
      ncol -= 1;
      continue;
    }
    double y[MAXMEM];
    for (int i = 0; i < ncol; ++i) {
      double s = b[i];
      for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
      y[i] = s / L[i][i];
    }
    for (int i = ncol - 1; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < ncol; ++k) s -= L[k][i] * gamma[k];
      gamma[i] = s / L[i][i];
    }
    break;
  }
  for (int k = 0; k < n; ++k) {
    double v = Qlast[k];
    for (int i = 0; i < ncol; ++i) {
      int ci = first + i;
      double dq = Qh[(size_t)(ci + 1) * n + k] - Qh[(size_t)ci * n + k];
      v -= gamma[i] * dq;
    }
    out[k] = v;
  }
  return ncol;
}

/* push (Q, F) into a history of at most `cap` entries (oldest first) */
static void hist_push(double* Qh, double* Fh, int* count, int cap, int n, const double* Q, const double* F) {
  if (*count == cap) {
    memmove(Qh, Qh + n, sizeof(double) * (size_t)n * (cap - 1));
    memmove(Fh, Fh + n, sizeof(double) * (size_t)n * (cap - 1));
    *count = cap - 1;
  }
  memcpy(Qh + (size_t)(*count) * n, Q, sizeof(double) * n);
  memcpy(Fh + (size_t)(*count) * n, F, sizeof(double) * n);
  *count += 1;
}

/* matter right-hand side (Eqs. implicitFluidNodal, eulerianEnergyLG,
 * eulerianNumberLG at v = 0; the energy per baryon and the lepton fraction
 * change by the neutrino energy and lepton number absorbed, divided by the
 * baryon density, K = kcoup / rho11) */
static void matter_rhs(const ora_model* m, double rho11, const double* D, const double* Dstar, double ye_star,
                       double e_star, double* yq) {
  int nq = m->nq, ns = m->ns;
  double K = m->kcoup / rho11;
  double dn = 0.0, de = 0.0;
  for (int s = 0; s < ns; ++s) {
    int id = m->species[s];
    for (int q = 0; q < nq; ++q) {
      double dd = D[s * nq + q] - Dstar[s * nq + q];
      dn += sp_g(id) * m->w2[q] * dd;
      de += sp_d(id) * m->w3[q] * dd;
    }
  }
  yq[0] = ye_star - K * dn;
  yq[1] = e_star - K * de;
}

static int all_finite(const double* x, int n) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(x[i])) return 0;
  return 1;
}

/* weighted norm ||D_s||_W2 of one species (Algorithm innerConverged) */
static double wnorm(const ora_model* m, const double* v) {
  double acc = 0.0;
  for (int q = 0; q < m->nq; ++q) acc += m->w2[q] * v[q] * v[q];
  return sqrt(acc);
}

typedef struct {
  double M[MAXN], Mnew[MAXN], Q[MAXN], F[MAXN];
  double Qh[MAXMEM * MAXN], Fh[MAXMEM * MAXN];
  double eta[ORA_MAX_NS * ORA_MAX_NQ], chi[ORA_MAX_NS * ORA_MAX_NQ], kap[ORA_MAX_NS * ORA_MAX_NQ];
  opac o;
} work;

/* Algorithm neutrinoMatterCoupling for one spatial point (Sec. 3.5.3). */
static int solve_point(const ora_model* m, const ora_params* prm, const double* theta, double dtau,
                       const double* Dst, const double* Ist, double rho11, double ye_st, double e_st, double chi0,
                       int have_T, double T_in, int have_mu, double mu_in, double* D, double* I, double* ye_out,
                       double* e_out, double* T_out, int* n_outer, int* n_inner, work* w) {
  int nq = m->nq, ns = m->ns, nn = ns * nq, n = 2 * nn;
  double ystar[2] = {ye_st, e_st};
  double y[2] = {ye_st, e_st};
  double qh[MAXMEM * 2], fh[MAXMEM * 2];
  int ocount = 0;
  int status = ORA_OK, inner_failed = 0, outer_conv = 0, fatal = 0;
  int total_inner = 0, k;
  double T_last = (prm->fixed_matter && have_T) ? T_in : ora_eos_temperature(m, e_st, ye_st, rho11);

  /* initial guesses: y^[1] = y*, M^[1,1] = M* */
  for (int i = 0; i < nn; ++i) {
    w->M[i] = Dst[i];
    w->M[nn + i] = Ist[i];
  }

  for (k = 1; k <= prm->max_outer; ++k) {
    /* ComputeOpacities(y^[k]) */
    double T, mu;
    /* with matter held fixed the caller may prescribe T and mu directly */
    T = (prm->fixed_matter && have_T) ? T_in : ora_eos_temperature(m, y[1], y[0], rho11);
    mu = (prm->fixed_matter && have_mu) ? mu_in : ora_eos_mu(m, y[0], T, rho11);
    if (!(T > 0.0) || !(y[0] >= 0.0) || !isfinite(T) || !isfinite(mu)) {
      status = ORA_EOS_DOMAIN;
      fatal = 1;
      break;
    }
    T_last = T;
    compute_opacities(m, theta, rho11, chi0, T, mu, &w->o);

    /* inner loop over moments with matter held fixed; M^[k,1] = M^[k-1,*] */
    double dref0[ORA_MAX_NS];
    for (int s = 0; s < ns; ++s) dref0[s] = wnorm(m, w->M + s * nq);
    int icount = 0, conv = 0, l;
    for (l = 1; l <= prm->max_inner; ++l) {
      /* ComputeRates and moment right-hand side, Eq. implicitMomentsNodal at
       * v = 0 (lambda = 1): Q_D = (D* + dtau eta) / (1 + dtau chi),
       * Q_I = I* / (1 + dtau kappa) */
      rates(m, &w->o, w->M, w->eta, w->chi, w->kap);
      for (int i = 0; i < nn; ++i) {
        w->Q[i] = (Dst[i] + dtau * w->eta[i]) / (1.0 + dtau * w->chi[i]);
        w->Q[nn + i] = Ist[i] / (1.0 + dtau * w->kap[i]);
      }
      for (int i = 0; i < n; ++i) w->F[i] = w->Q[i] - w->M[i];
      hist_push(w->Qh, w->Fh, &icount, prm->m_inner, n, w->Q, w->F);
      ora_anderson(n, icount, w->Qh, w->Fh, w->Mnew);
      if (!all_finite(w->Mnew, n)) {
        status = ORA_NONFINITE;
        fatal = 1;
        break;
      }
      /* Algorithm innerConverged: per species, sqrt(max over moments of
       * sum_q W2 dM^2) <= tol * ||D_s||, reference guarded by the new norm */
      conv = 1;
      for (int s = 0; s < ns; ++s) {
        double sd = 0.0, si = 0.0;
        for (int q = 0; q < nq; ++q) {
          int i = s * nq + q;
          double dd = w->Mnew[i] - w->M[i];
          double di = w->Mnew[nn + i] - w->M[nn + i];
          sd += m->w2[q] * dd * dd;
          si += m->w2[q] * di * di;
        }
        double dm = sqrt(sd > si ? sd : si);
        double dnew = wnorm(m, w->Mnew + s * nq);
        double dref = dref0[s] > dnew ? dref0[s] : dnew;
        if (!(dm <= prm->tol_inner * dref)) conv = 0;
      }
      memcpy(w->M, w->Mnew, sizeof(double) * n);
      if (conv) break;
    }
    if (fatal) {
      total_inner += (l > prm->max_inner ? prm->max_inner : l);
      break;
    }
    total_inner += (l > prm->max_inner ? prm->max_inner : l);
    if (!conv) inner_failed = 1;

    if (prm->fixed_matter) {
      outer_conv = 1;
      break;
    }

    /* matter right-hand side and residual; outer Anderson step */
    double yq[2], f[2], ynew[2];
    matter_rhs(m, rho11, w->M, Dst, ye_st, e_st, yq);
    f[0] = yq[0] - y[0];
    f[1] = yq[1] - y[1];
    hist_push(qh, fh, &ocount, prm->m_outer, 2, yq, f);
    ora_anderson(2, ocount, qh, fh, ynew);
    if (!isfinite(ynew[0]) || !isfinite(ynew[1])) {
      status = ORA_NONFINITE;
      fatal = 1;
      break;
    }
    /* Algorithm outerConverged: componentwise against y* */
    int oc = fabs(ynew[0] - y[0]) <= prm->tol_outer * fabs(ystar[0]) &&
             fabs(ynew[1] - y[1]) <= prm->tol_outer * fabs(ystar[1]);
    y[0] = ynew[0];
    y[1] = ynew[1];
    if (oc) {
      outer_conv = 1;
      break;
    }
  }
  if (k > prm->max_outer) k = prm->max_outer;
  if (!fatal) {
    if (!outer_conv) status = ORA_MAX_OUTER;
    else if (inner_failed) status = ORA_MAX_INNER;
  }

  for (int i = 0; i < nn; ++i) {
    D[i] = w->M[i];
    I[i] = w->M[nn + i];
  }
  if (prm->fixed_matter) {
    *ye_out = ye_st;
    *e_out = e_st;
    *T_out = T_last;
  } else {
    /* output matter state recomputed from the final moments so that lepton
     * number and energy balance hold to rounding */
    double yq[2];
    matter_rhs(m, rho11, w->M, Dst, ye_st, e_st, yq);
    *ye_out = yq[0];
    *e_out = yq[1];
    *T_out = ora_eos_temperature(m, yq[1], yq[0], rho11);
  }
  *n_outer = k;
  *n_inner = total_inner;
  return status;
}

int ora_solve_batch(const ora_model* m, const ora_params* prm, const double* theta, long P, double dtau,
                    const double* D0, const double* I0, const double* rho11, const double* ye0,
                    const double* e0, const double* chi0, const double* T_fixed, const double* mu_fixed,
                    double* D, double* I, double* ye, double* e, double* T,
                    int* n_outer, int* n_inner, int* status, int nthreads) {
  if (m->nq < 1 || m->nq > ORA_MAX_NQ || m->ns < 1 || m->ns > ORA_MAX_NS) return -1;
  if (prm->m_inner < 1 || prm->m_inner > MAXMEM || prm->m_outer < 1 || prm->m_outer > MAXMEM) return -1;
  if (prm->max_inner < 1 || prm->max_outer < 1) return -1;
  if ((m->flags & ORA_PAIR))
    for (int s = 0; s < m->ns; ++s)
      if (partner_index(m, s) < 0) return -1;
  int nn = m->ns * m->nq;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    work* w = (work*)malloc(sizeof(work));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
    for (long p = 0; p < P; ++p) {
      double c0 = chi0 ? chi0[p] : m->chi_ref * rho11[p];
      if (rho11[p] < m->rho11_min) {
        /* neutrino-matter coupling is disabled at low density (Sec. 7.2):
         * the state passes through unchanged */
        for (int i = 0; i < nn; ++i) {
          D[p * nn + i] = D0[p * nn + i];
          I[p * nn + i] = I0[p * nn + i];
        }
        ye[p] = ye0[p];
        e[p] = e0[p];
        T[p] = (prm->fixed_matter && T_fixed) ? T_fixed[p] : ora_eos_temperature(m, e0[p], ye0[p], rho11[p]);
        n_outer[p] = 0;
        n_inner[p] = 0;
        status[p] = ORA_OK;
        continue;
      }
      status[p] = solve_point(m, prm, theta, dtau, D0 + p * nn, I0 + p * nn, rho11[p], ye0[p], e0[p], c0,
                              T_fixed != NULL, T_fixed ? T_fixed[p] : 0.0, mu_fixed != NULL,
                              mu_fixed ? mu_fixed[p] : 0.0, D + p * nn, I + p * nn, ye + p, e + p, T + p,
                              n_outer + p, n_inner + p, w);
    }
    free(w);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Residual of the implicit system (definition of the result): Eqs.
 * implicitNumberNodal, implicitNumberFluxNodal at v = 0 and Eq.
 * implicitFluidNodal.  Layout: [R_D (ns*nq), R_I (ns*nq), R_Ye, R_e]. */
void ora_residual(const ora_model* m, const double* theta, double dtau, double rho11, double chi0,
                  const double* Dstar, const double* Istar, double ye_star, double e_star,
                  const double* D, const double* I, double ye, double e, double* R) {
  int nn = m->ns * m->nq;
  double T = ora_eos_temperature(m, e, ye, rho11);
  double mu = ora_eos_mu(m, ye, T, rho11);
  double* eta = (double*)malloc(sizeof(double) * 3 * nn);
  double *chi = eta + nn, *kap = eta + 2 * nn;
  ora_rates(m, theta, rho11, chi0, T, mu, D, eta, chi, kap);
  for (int i = 0; i < nn; ++i) {
    R[i] = D[i] - Dstar[i] - dtau * (eta[i] - chi[i] * D[i]);
    R[nn + i] = I[i] - Istar[i] + dtau * kap[i] * I[i];
  }
  double yq[2];
  matter_rhs(m, rho11, D, Dstar, ye_star, e_star, yq);
  R[2 * nn] = ye - yq[0];
  R[2 * nn + 1] = e - yq[1];
  free(eta);
}

/* ------------------------------------------------------------------------ */
/* Analytic Jacobian of the reduced residual x = (D, Ye, e):
 *   R_D = D (1 + dtau chi) - D* - dtau eta,
 *   R_Y = Ye - Ye* + K sum g W2 (D - D*),  R_e = e - e* + K sum d W3 (D - D*),
 * with T = T(e, Ye) and mu = mu(Ye, T).  The flux block drops out because no
 * output of the reduced system depends on I when v = 0. */

typedef struct {
  double dPin[ORA_MAX_NQ * ORA_MAX_NQ], dPout[ORA_MAX_NQ * ORA_MAX_NQ];
  double dPpro[ORA_MAX_NQ * ORA_MAX_NQ], dPann[ORA_MAX_NQ * ORA_MAX_NQ];
  opac o;
} jwork;

static void jacobian_core(const ora_model* m, const double* theta, double dtau, double rho11, double chi0,
                          const double* D, double ye, double e, double* J, jwork* w) {
  int nq = m->nq, ns = m->ns, nn = ns * nq, n = nn + 2;
  double T = ora_eos_temperature(m, e, ye, rho11);
  double mu = ora_eos_mu(m, ye, T, rho11);
  opac* o = &w->o;
  compute_opacities(m, theta, rho11, chi0, T, mu, o);
  /* d Phi / dT = Phi * c / T^2 with c the non-negative exponent numerator */
  for (int q = 0; q < nq; ++q)
    for (int p = 0; p < nq; ++p) {
      double dlt = m->eps[q] - m->eps[p], adl = fabs(dlt);
      int i = q * nq + p;
      w->dPin[i] = o->phi_in[i] * (adl + 0.5 * dlt) / (T * T);
      w->dPout[i] = o->phi_out[i] * (adl - 0.5 * dlt) / (T * T);
      w->dPann[i] = o->phi_ann[i] * adl / (T * T);
      w->dPpro[i] = o->phi_pro[i] * (adl + m->eps[q] + m->eps[p]) / (T * T);
    }
  double eta[ORA_MAX_NS * ORA_MAX_NQ], chi[ORA_MAX_NS * ORA_MAX_NQ], kap[ORA_MAX_NS * ORA_MAX_NQ];
  rates(m, o, D, eta, chi, kap);
  memset(J, 0, sizeof(double) * n * n);
  double r3 = cbrt(rho11);
  double dT_de = 1.0 / (m->eos_a * (1.0 + ye));
  double dT_dye = -(4.0 / 3.0) * m->eos_b * cbrt(ye) * r3 / (m->eos_a * (1.0 + ye)) - T / (1.0 + ye);
  double dmu_dye = m->mu_a * r3 + m->mu_b / T * dT_dye;
  double dmu_de = m->mu_b / T * dT_de;
  int nes = (m->flags & ORA_NES) != 0, pair = (m->flags & ORA_PAIR) != 0;
  for (int s = 0; s < ns; ++s) {
    int id = m->species[s];
    int sb = partner_index(m, s);
    double sgn = sp_musign(id);
    for (int q = 0; q < nq; ++q) {
      int i = s * nq + q;
      double Dq = D[i];
      J[i * n + i] += 1.0 + dtau * chi[i];
      if (nes)
        for (int p = 0; p < nq; ++p) {
          double a_in = m->w2[p] * o->phi_in[q * nq + p];
          double a_out = m->w2[p] * o->phi_out[q * nq + p];
          /* d eta_nes / dD_s' = W Phi_in ; d chi_nes / dD_s' = W (Phi_in - Phi_out) */
          J[i * n + s * nq + p] += dtau * (Dq * (a_in - a_out) - a_in);
        }
      if (pair && sb >= 0)
        for (int p = 0; p < nq; ++p) {
          double a_pro = m->w2[p] * o->phi_pro[q * nq + p];
          double a_ann = m->w2[p] * o->phi_ann[q * nq + p];
          /* d eta_pair / dDbar' = -W Phi_pro ; d chi_pair / dDbar' = W (Phi_ann - Phi_pro) */
          J[i * n + sb * nq + p] += dtau * (Dq * (a_ann - a_pro) + a_pro);
        }
      /* temperature and chemical-potential derivatives */
      double f = o->deq[i];
      double fc = ora_fermi_dirac_complement(m->eps[q], sgn * mu, T);
      double ddeq_dT = f * fc * (m->eps[q] - sgn * mu) / (T * T);
      double ddeq_dmu = f * fc / T * sgn;
      double deta_dT = o->chia[i] * ddeq_dT, dchi_dT = 0.0;
      if (nes)
        for (int p = 0; p < nq; ++p) {
          double t_in = m->w2[p] * w->dPin[q * nq + p] * D[s * nq + p];
          double t_out = m->w2[p] * w->dPout[q * nq + p] * (1.0 - D[s * nq + p]);
          deta_dT += t_in;
          dchi_dT += t_in + t_out;
        }
      if (pair && sb >= 0)
        for (int p = 0; p < nq; ++p) {
          double t_pro = m->w2[p] * w->dPpro[q * nq + p] * (1.0 - D[sb * nq + p]);
          double t_ann = m->w2[p] * w->dPann[q * nq + p] * D[sb * nq + p];
          deta_dT += t_pro;
          dchi_dT += t_pro + t_ann;
        }
      double dR_dT = dtau * (Dq * dchi_dT - deta_dT);
      double dR_dmu = -dtau * o->chia[i] * ddeq_dmu;
      J[i * n + nn] += dR_dT * dT_dye + dR_dmu * dmu_dye;
      J[i * n + nn + 1] += dR_dT * dT_de + dR_dmu * dmu_de;
    }
  }
  double K = m->kcoup / rho11;
  for (int s = 0; s < ns; ++s) {
    int id = m->species[s];
    for (int q = 0; q < nq; ++q) {
      J[nn * n + s * nq + q] = K * sp_g(id) * m->w2[q];
      J[(nn + 1) * n + s * nq + q] = K * sp_d(id) * m->w3[q];
    }
  }
  J[nn * n + nn] = 1.0;
  J[(nn + 1) * n + nn + 1] = 1.0;
}

int ora_jacobian(const ora_model* m, const double* theta, double dtau, double rho11, double chi0,
                 const double* D, double ye, double e, double* J) {
  if (m->fd_projection) return -2; /* derivatives of the projection: not written out */
  jwork* w = (jwork*)malloc(sizeof(jwork));
  jacobian_core(m, theta, dtau, rho11, chi0, D, ye, e, J, w);
  free(w);
  return 0;
}

/* dense LU with partial pivoting, in place; solves A x = b (trans = 0) or
 * A^T x = b (trans = 1) */
static int lu_factor(double* A, int n, int* piv) {
  for (int k = 0; k < n; ++k) {
    int pr = k;
    double best = fabs(A[k * n + k]);
    for (int i = k + 1; i < n; ++i)
      if (fabs(A[i * n + k]) > best) {
        best = fabs(A[i * n + k]);
        pr = i;
      }
    piv[k] = pr;
    if (best == 0.0) return -1;
    if (pr != k)
      for (int j = 0; j < n; ++j) {
        double t = A[k * n + j];
        A[k * n + j] = A[pr * n + j];
        A[pr * n + j] = t;
      }
    for (int i = k + 1; i < n; ++i) {
      A[i * n + k] /= A[k * n + k];
      double l = A[i * n + k];
      for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
    }
  }
  return 0;
}

static void lu_solve(const double* A, int n, const int* piv, double* x, int trans) {
  if (!trans) {
    for (int k = 0; k < n; ++k) {
      double t = x[k];
      x[k] = x[piv[k]];
      x[piv[k]] = t;
    }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) x[i] -= A[i * n + j] * x[j];
    for (int i = n - 1; i >= 0; --i) {
      for (int j = i + 1; j < n; ++j) x[i] -= A[i * n + j] * x[j];
      x[i] /= A[i * n + i];
    }
  } else {
    /* (P^T L U)^T y = b  ->  U^T z = b, L^T w = z, y = P^T w */
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < i; ++j) x[i] -= A[j * n + i] * x[j];
      x[i] /= A[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i)
      for (int j = i + 1; j < n; ++j) x[i] -= A[j * n + i] * x[j];
    for (int k = n - 1; k >= 0; --k) {
      double t = x[k];
      x[k] = x[piv[k]];
      x[piv[k]] = t;
    }
  }
}

/* Dense Newton on the reduced (D, Ye, e) system, then I from its closed form
 * I = I* / (1 + dtau kappa).  Used only to pin the fixed-point solution on
 * tiny problems. */
int ora_newton(const ora_model* m, const double* theta, double dtau, double rho11, double chi0,
               const double* Dstar, const double* Istar, double ye_star, double e_star,
               double* D, double* I, double* ye, double* e, double tol, int max_it) {
  if (m->fd_projection) return -2; /* its Jacobian is written for the pointwise equilibrium */
  int nn = m->ns * m->nq, n = nn + 2;
  double* J = (double*)malloc(sizeof(double) * n * n);
  double* R = (double*)malloc(sizeof(double) * (2 * nn + 2));
  double* dx = (double*)malloc(sizeof(double) * n);
  int* piv = (int*)malloc(sizeof(int) * n);
  jwork* w = (jwork*)malloc(sizeof(jwork));
  int it, rc = -1;
  for (it = 0; it < max_it; ++it) {
    ora_residual(m, theta, dtau, rho11, chi0, Dstar, Istar, ye_star, e_star, D, I, *ye, *e, R);
    for (int i = 0; i < nn; ++i) dx[i] = -R[i];
    dx[nn] = -R[2 * nn];
    dx[nn + 1] = -R[2 * nn + 1];
    jacobian_core(m, theta, dtau, rho11, chi0, D, *ye, *e, J, w);
    if (lu_factor(J, n, piv) != 0) break;
    lu_solve(J, n, piv, dx, 0);
    double step = 0.0, scale = 0.0;
    for (int i = 0; i < nn; ++i) {
      D[i] += dx[i];
      step += m->w2[i % m->nq] * dx[i] * dx[i];
      scale += m->w2[i % m->nq] * D[i] * D[i];
    }
    *ye += dx[nn];
    *e += dx[nn + 1];
    if (sqrt(step) <= tol * sqrt(scale) && fabs(dx[nn]) <= tol * fabs(*ye) && fabs(dx[nn + 1]) <= tol * fabs(*e)) {
      rc = it + 1;
      break;
    }
  }
  /* flux moments from their closed form at the converged D and T */
  {
    double T = ora_eos_temperature(m, *e, *ye, rho11);
    double mu = ora_eos_mu(m, *ye, T, rho11);
    double* eta = (double*)malloc(sizeof(double) * 3 * nn);
    ora_rates(m, theta, rho11, chi0, T, mu, D, eta, eta + nn, eta + 2 * nn);
    for (int i = 0; i < nn; ++i) I[i] = Istar[i] / (1.0 + dtau * eta[2 * nn + i]);
    free(eta);
  }
  free(J);
  free(R);
  free(dx);
  free(piv);
  free(w);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Implicit-function-theorem adjoint.  At the converged x (R(x, theta) = 0):
 *   R_x^T lambda = L_x^T,  dL/dtheta = -lambda^T R_theta,
 * with L = gE (e* - e) + gY (Ye - Ye*) per point, theta = (s_1..s_nq, a_nes,
 * a_pair).  s_q scales chi^EmAb only; a_nes and a_pair scale the NES and pair
 * kernels linearly (A = a * rho11). */
int ora_adjoint_batch(const ora_model* m, const double* theta, long P, double dtau, const double* rho11,
                      const double* chi0, const double* D, const double* ye, const double* e,
                      const double* gbar, double* grad_theta, double* grad_pp, int nthreads) {
  if (m->fd_projection) return -2; /* as ora_jacobian */
  int nq = m->nq, ns = m->ns, nn = ns * nq, n = nn + 2, nt = nq + 2;
  double* gsum = (double*)calloc((size_t)nt, sizeof(double));
  int bad = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    double* J = (double*)malloc(sizeof(double) * n * n);
    double* lam = (double*)malloc(sizeof(double) * n);
    int* piv = (int*)malloc(sizeof(int) * n);
    jwork* w = (jwork*)malloc(sizeof(jwork));
    double* gl = (double*)calloc((size_t)nt, sizeof(double));
    opac* ou = (opac*)malloc(sizeof(opac));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
    for (long p = 0; p < P; ++p) {
      if (rho11[p] < m->rho11_min) {
        /* coupling switched off (Sec. 7.2): the step passes the state
         * through, so nothing depends on theta */
        if (grad_pp)
          for (int j = 0; j < nt; ++j) grad_pp[p * nt + j] = 0.0;
        continue;
      }
      double c0 = chi0 ? chi0[p] : m->chi_ref * rho11[p];
      const double* Dp = D + p * nn;
      jacobian_core(m, theta, dtau, rho11[p], c0, Dp, ye[p], e[p], J, w);
      if (lu_factor(J, n, piv) != 0) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
        bad = 1;
        continue;
      }
      for (int i = 0; i < n; ++i) lam[i] = 0.0;
      lam[nn] = gbar[2 * p + 1];   /* dL/dYe */
      lam[nn + 1] = -gbar[2 * p];  /* dL/de (L_E = e* - e) */
      lu_solve(J, n, piv, lam, 1);
      double T = w->o.T, mu = w->o.mu;
      /* unit-amplitude kernels for the a_nes / a_pair derivatives */
      kernels_unit(m, T, rho11[p], rho11[p], ou->phi_in, ou->phi_out, ou->phi_pro, ou->phi_ann);
      double gp[ORA_MAX_NQ + 2];
      for (int j = 0; j < nt; ++j) gp[j] = 0.0;
      for (int s = 0; s < ns; ++s) {
        int id = m->species[s];
        int sb = partner_index(m, s);
        for (int q = 0; q < nq; ++q) {
          int i = s * nq + q;
          double Dq = Dp[i];
          if ((m->flags & ORA_EMAB) && sp_emab(id)) {
            double shape = c0 * pow(m->eps[q] / m->eps_ref, m->chi_power);
            gp[q] -= lam[i] * dtau * shape * (Dq - w->o.deq[i]);
          }
          if (m->flags & ORA_NES) {
            double en = 0.0, on = 0.0;
            for (int r = 0; r < nq; ++r) {
              en += m->w2[r] * ou->phi_in[q * nq + r] * Dp[s * nq + r];
              on += m->w2[r] * ou->phi_out[q * nq + r] * (1.0 - Dp[s * nq + r]);
            }
            gp[nq] -= lam[i] * dtau * (Dq * (en + on) - en);
          }
          if ((m->flags & ORA_PAIR) && sb >= 0) {
            double ep = 0.0, an = 0.0;
            for (int r = 0; r < nq; ++r) {
              ep += m->w2[r] * ou->phi_pro[q * nq + r] * (1.0 - Dp[sb * nq + r]);
              an += m->w2[r] * ou->phi_ann[q * nq + r] * Dp[sb * nq + r];
            }
            gp[nq + 1] -= lam[i] * dtau * (Dq * (ep + an) - ep);
          }
        }
      }
      (void)mu;
      if (grad_pp)
        for (int j = 0; j < nt; ++j) grad_pp[p * nt + j] = gp[j];
      for (int j = 0; j < nt; ++j) gl[j] += gp[j];
    }
#ifdef _OPENMP
#pragma omp critical
#endif
    for (int j = 0; j < nt; ++j) gsum[j] += gl[j];
    free(J);
    free(lam);
    free(piv);
    free(w);
    free(gl);
    free(ou);
  }
  for (int j = 0; j < nt; ++j) grad_theta[j] += gsum[j];
  free(gsum);
  return bad ? -2 : 0;
}

/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* O(v) coupling: the moment equations and matter update of Sec. 3.5.1 with a
 * nonzero fluid velocity.  Unknowns D (ns, nq) and I (ns, 3, nq); matter
 * y = (Ye, ef, v_1, v_2, v_3) with ef the specific fluid energy (internal
 * plus kinetic, MeV per baryon) and v in units of c. */

/* Minerbo closure: Eddington factor as a polynomial in the flux factor
 * (Eq. eddingtonFactorMinerbo). */
double ora_minerbo_psi(double h) { return 1.0 / 3.0 + (2.0 / 15.0) * (3.0 - h + 3.0 * h * h) * h * h; }

/* flux factor h = |I| / D, taken as 0 without flux and limited to the
 * realizable range [0, 1] (1 also when D <= 0 carries a flux) */
double ora_flux_factor(double D, double Imag) {
  if (!(Imag > 0.0)) return 0.0;
  if (!(D > 0.0)) return 1.0;
  double h = Imag / D;
  return h < 1.0 ? h : 1.0;
}

/* K_ij = k_ij D with k_ij = ((1 - psi) delta_ij + (3 psi - 1) n_i n_j) / 2,
 * n = I / |I| (Eq. eddingtonTensor, flat metric) */
void ora_eddington(double D, const double* I3, double* K9) {
  double Imag = sqrt(I3[0] * I3[0] + I3[1] * I3[1] + I3[2] * I3[2]);
  double psi = ora_minerbo_psi(ora_flux_factor(D, Imag));
  double a = 0.5 * (1.0 - psi), b = 0.5 * (3.0 * psi - 1.0);
  double n[3] = {0.0, 0.0, 0.0};
  if (Imag > 0.0)
    for (int i = 0; i < 3; ++i) n[i] = I3[i] / Imag;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) K9[3 * i + j] = D * ((i == j ? a : 0.0) + b * n[i] * n[j]);
}

/* the three flux components of species s at node q */
static void flux3(const ora_model* m, const double* I, int s, int q, double* I3) {
  for (int j = 0; j < 3; ++j) I3[j] = I[(s * 3 + j) * m->nq + q];
}

/* Eulerian neutrino lepton number, energy and momentum with the LG
 * quadrature (Eqs. eulerianNumberLG, eulerianEnergyLG, eulerianMomentumLG;
 * the common factor 4 pi / h^3 is folded into the coupling constant):
 * X = (N, E, F_1, F_2, F_3) */
static void eulerian_v(const ora_model* m, const double* D, const double* I, const double* v, double* X) {
  int nq = m->nq, ns = m->ns;
  for (int i = 0; i < 5; ++i) X[i] = 0.0;
  for (int s = 0; s < ns; ++s) {
    int id = m->species[s];
    for (int q = 0; q < nq; ++q) {
      double Dq = D[s * nq + q], I3[3], K9[9];
      flux3(m, I, s, q, I3);
      ora_eddington(Dq, I3, K9);
      double vI = v[0] * I3[0] + v[1] * I3[1] + v[2] * I3[2];
      X[0] += sp_g(id) * m->w2[q] * (Dq + vI);
      X[1] += sp_d(id) * m->w3[q] * (Dq + 2.0 * vI);
      for (int j = 0; j < 3; ++j) {
        double vK = v[0] * K9[3 * j] + v[1] * K9[3 * j + 1] + v[2] * K9[3 * j + 2];
        X[2 + j] += sp_d(id) * m->w3[q] * (I3[j] + v[j] * Dq + vK);
      }
    }
  }
}

/* matter right-hand side q(M, y) (Eq. implicitFluidNodal): the changes of
 * the Eulerian neutrino lepton number, energy and momentum per baryon are
 * removed from the matter; the momentum change per baryon divided by the
 * baryon rest energy m_u c^2 is the velocity change. */
static void matter_rhs_v(const ora_model* m, double rho11, const double* D, const double* I, const double* y,
                         const double* X0, const double* ystar, double* yq) {
  double X[5], K = m->kcoup / rho11;
  eulerian_v(m, D, I, y + 2, X);
  yq[0] = ystar[0] - K * (X[0] - X0[0]);
  yq[1] = ystar[1] - K * (X[1] - X0[1]);
  for (int j = 0; j < 3; ++j) yq[2 + j] = ystar[2 + j] - (K / ORA_MU_C2) * (X[2 + j] - X0[2 + j]);
}

static double norm3(const double* v) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

/* temperature from the EOS at the internal energy ef - m_u c^2 |v|^2 / 2 */
static double eos_temperature_v(const ora_model* m, const double* y, double rho11) {
  double vm = norm3(y + 2);
  return ora_eos_temperature(m, y[1] - 0.5 * ORA_MU_C2 * vm * vm, y[0], rho11);
}

/* Linear-order corrections (Sec. 2.4): with the angular kernels expanded to
 * linear order in the scattering angle, the number and flux equations of
 * species s gain, at node q,
 *   NES:  L_in^i  = sum_p W_p Phi_1^In[q][p] I_s^i(p),   L_out^i likewise
 *         (Eq. linearCorrectionsNES);
 *   pair: L_pro^i = sum_p W_p Phi_1^Pro[q][p] Ibar_s^i(p), L_ann^i likewise,
 *         Ibar the flux of the pair partner (Eq. linearCorrectionsPair);
 *   number equation: -(L_in^i - L_out^i) I_i + (L_pro^i - L_ann^i) I_i
 *         (Eqs. zerothMomentCollisionTerm_NES, zerothMomentCollisionTerm_Pair);
 *   flux equation j: (1/3)(delta_ij - 3 K_ij) L_in^i + K_ij L_out^i
 *         - (1/3)(delta_ij - 3 K_ij) L_pro^i - K_ij L_ann^i
 *         (Eqs. firstMomentCollisionTerm_NES, firstMomentCollisionTerm_Pair),
 * K_ij the Eddington tensor of species s at node q (flat metric).  The
 * synthetic Phi_1 are fixed fractions of the isotropic kernels (model fields
 * phi1_nes, phi1_pair), which keeps their in-out invariance and detailed
 * balance. */
static void phi1_terms(const ora_model* m, const opac* o, const double* D, const double* I, double* C1D,
                       double* C1I) {
  int nq = m->nq, ns = m->ns;
  for (int s = 0; s < ns; ++s) {
    int sb = partner_index(m, s);
    const double *pin = o->phi_in + s * nq * nq, *pout = o->phi_out + s * nq * nq;
    const double* ppro = o->phi_pro + s * nq * nq;
    for (int q = 0; q < nq; ++q) {
      double Lin[3] = {0.0, 0.0, 0.0}, Lout[3] = {0.0, 0.0, 0.0};
      double Lpro[3] = {0.0, 0.0, 0.0}, Lann[3] = {0.0, 0.0, 0.0};
      for (int i = 0; i < 3; ++i)
        for (int p = 0; p < nq; ++p) {
          if (m->flags & ORA_NES) {
            double Ii = I[(s * 3 + i) * nq + p];
            Lin[i] += m->w2[p] * (m->phi1_nes * pin[q * nq + p]) * Ii;
            Lout[i] += m->w2[p] * (m->phi1_nes * pout[q * nq + p]) * Ii;
          }
          if ((m->flags & ORA_PAIR) && sb >= 0) {
            double Ib = I[(sb * 3 + i) * nq + p];
            Lpro[i] += m->w2[p] * (m->phi1_pair * ppro[q * nq + p]) * Ib;
            Lann[i] += m->w2[p] * (m->phi1_pair * o->phi_ann[q * nq + p]) * Ib;
          }
        }
      double I3[3], K9[9];
      flux3(m, I, s, q, I3);
      ora_eddington(D[s * nq + q], I3, K9);
      double c0 = 0.0;
      for (int i = 0; i < 3; ++i) c0 += -(Lin[i] - Lout[i]) * I3[i] + (Lpro[i] - Lann[i]) * I3[i];
      C1D[s * nq + q] = c0;
      for (int j = 0; j < 3; ++j) {
        double cj = 0.0;
        for (int i = 0; i < 3; ++i) {
          double g3 = ((i == j ? 1.0 : 0.0) - 3.0 * K9[3 * i + j]) / 3.0;
          cj += g3 * Lin[i] + K9[3 * i + j] * Lout[i] - g3 * Lpro[i] - K9[3 * i + j] * Lann[i];
        }
        C1I[(s * 3 + j) * nq + q] = cj;
      }
    }
  }
}

void ora_phi1_terms(const ora_model* m, const double* theta, double rho11, double T, const double* D,
                    const double* I, double* C1D, double* C1I) {
  opac* o = (opac*)malloc(sizeof(opac));
  compute_opacities(m, theta, rho11, m->chi_ref * rho11, T, 0.0, o);
  phi1_terms(m, o, D, I, C1D, C1I);
  free(o);
}

#define MAXNV (4 * ORA_MAX_NS * ORA_MAX_NQ)
typedef struct {
  double M[MAXNV], Mnew[MAXNV], Q[MAXNV], F[MAXNV];
  double Qh[MAXMEM * MAXNV], Fh[MAXMEM * MAXNV];
  double Nst[ORA_MAX_NS * ORA_MAX_NQ], Gst[3 * ORA_MAX_NS * ORA_MAX_NQ];
  double eta[ORA_MAX_NS * ORA_MAX_NQ], chi[ORA_MAX_NS * ORA_MAX_NQ], kap[ORA_MAX_NS * ORA_MAX_NQ];
  double c1d[ORA_MAX_NS * ORA_MAX_NQ], c1i[3 * ORA_MAX_NS * ORA_MAX_NQ];
  opac o;
} work_v;

/* Algorithm neutrinoMatterCoupling for one spatial point with v != 0. */
static int solve_point_v(const ora_model* m, const ora_params* prm, const double* theta, double dtau,
                         const double* Dst, const double* Ist, double rho11, const double* ystar, double chi0,
                         double* D, double* I, double* yout, double* T_out, int* n_outer, int* n_inner,
                         work_v* w) {
  int nq = m->nq, ns = m->ns, nn = ns * nq, n = 4 * nn;
  double y[5], yused[5], X0[5];
  double qh[MAXMEM * 5], fh[MAXMEM * 5];
  int ocount = 0;
  int status = ORA_OK, inner_failed = 0, outer_conv = 0, fatal = 0;
  int total_inner = 0, k;
  for (int i = 0; i < 5; ++i) y[i] = yused[i] = ystar[i];
  double T_last = eos_temperature_v(m, ystar, rho11);

  /* number and number-flux densities of the old state, N* = D* + v*.I* and
   * G*_j = I*_j + v*^i K*_ij (Eq. numberDensityEulerian and the left-hand
   * sides of Eqs. implicitNumberNodal, implicitNumberFluxNodal at M*, v*), and
   * the old Eulerian lepton number, energy and momentum */
  for (int s = 0; s < ns; ++s)
    for (int q = 0; q < nq; ++q) {
      double Dq = Dst[s * nq + q], I3[3], K9[9];
      const double* vs = ystar + 2;
      flux3(m, Ist, s, q, I3);
      ora_eddington(Dq, I3, K9);
      w->Nst[s * nq + q] = Dq + (vs[0] * I3[0] + vs[1] * I3[1] + vs[2] * I3[2]);
      for (int j = 0; j < 3; ++j)
        w->Gst[(s * 3 + j) * nq + q] = I3[j] + (vs[0] * K9[3 * j] + vs[1] * K9[3 * j + 1] + vs[2] * K9[3 * j + 2]);
    }
  eulerian_v(m, Dst, Ist, ystar + 2, X0);

  /* initial guesses: y^[1] = y*, M^[1,1] = M* */
  for (int i = 0; i < nn; ++i) w->M[i] = Dst[i];
  for (int i = 0; i < 3 * nn; ++i) w->M[nn + i] = Ist[i];

  for (k = 1; k <= prm->max_outer; ++k) {
    const double* v = y + 2;
    double vmag = norm3(v);
    /* step-size parameter lambda = 1 / (1 + |v|) (remark on the choice of lambda) */
    double lam = 1.0 / (1.0 + vmag);
    double T = eos_temperature_v(m, prm->fixed_matter ? ystar : y, rho11);
    double mu = ora_eos_mu(m, y[0], T, rho11);
    if (!(T > 0.0) || !(y[0] >= 0.0) || !isfinite(T) || !isfinite(mu)) {
      status = ORA_EOS_DOMAIN;
      fatal = 1;
      break;
    }
    T_last = T;
    for (int i = 0; i < 5; ++i) yused[i] = y[i];
    compute_opacities(m, theta, rho11, chi0, T, mu, &w->o);

    double dref0[ORA_MAX_NS];
    for (int s = 0; s < ns; ++s) dref0[s] = wnorm(m, w->M + s * nq);
    int icount = 0, conv = 0, l;
    for (l = 1; l <= prm->max_inner; ++l) {
      /* ComputeRates and the moment right-hand side Q (Eq. implicitMomentsNodal):
       * Q_D = ((1 - lam) D + lam (N* - v.I + dtau eta)) / (1 + lam dtau chi),
       * Q_Ij = ((1 - lam) I_j + lam (G*_j - v^i K_ij)) / (1 + lam dtau kappa) */
      rates(m, &w->o, w->M, w->eta, w->chi, w->kap);
      /* the linear-order corrections are evaluated at the current iterate,
       * as the emissivity is, and join the right-hand sides */
      int lin = m->phi1_nes != 0.0 || m->phi1_pair != 0.0;
      if (lin) phi1_terms(m, &w->o, w->M, w->M + nn, w->c1d, w->c1i);
      for (int s = 0; s < ns; ++s)
        for (int q = 0; q < nq; ++q) {
          int i = s * nq + q;
          double Dq = w->M[i], I3[3], K9[9];
          flux3(m, w->M + nn, s, q, I3);
          ora_eddington(Dq, I3, K9);
          double vI = v[0] * I3[0] + v[1] * I3[1] + v[2] * I3[2];
          double srcD = lin ? w->eta[i] + w->c1d[i] : w->eta[i];
          w->Q[i] = ((1.0 - lam) * Dq + lam * (w->Nst[i] - vI + dtau * srcD)) / (1.0 + lam * dtau * w->chi[i]);
          for (int j = 0; j < 3; ++j) {
            int ij = (s * 3 + j) * nq + q;
            double vK = v[0] * K9[3 * j] + v[1] * K9[3 * j + 1] + v[2] * K9[3 * j + 2];
            double num = (1.0 - lam) * I3[j] + lam * (w->Gst[ij] - vK);
            if (lin) num = (1.0 - lam) * I3[j] + lam * (w->Gst[ij] - vK + dtau * w->c1i[ij]);
            w->Q[nn + ij] = num / (1.0 + lam * dtau * w->kap[i]);
          }
        }
      for (int i = 0; i < n; ++i) w->F[i] = w->Q[i] - w->M[i];
      hist_push(w->Qh, w->Fh, &icount, prm->m_inner, n, w->Q, w->F);
      ora_anderson(n, icount, w->Qh, w->Fh, w->Mnew);
      if (!all_finite(w->Mnew, n)) {
        status = ORA_NONFINITE;
        fatal = 1;
        break;
      }
      /* Algorithm innerConverged over the four moments D, I_1, I_2, I_3 */
      conv = 1;
      for (int s = 0; s < ns; ++s) {
        double sm[4] = {0.0, 0.0, 0.0, 0.0};
        for (int q = 0; q < nq; ++q) {
          double dd = w->Mnew[s * nq + q] - w->M[s * nq + q];
          sm[0] += m->w2[q] * dd * dd;
          for (int j = 0; j < 3; ++j) {
            int ij = nn + (s * 3 + j) * nq + q;
            double di = w->Mnew[ij] - w->M[ij];
            sm[1 + j] += m->w2[q] * di * di;
          }
        }
        double mx = sm[0];
        for (int j = 1; j < 4; ++j)
          if (sm[j] > mx) mx = sm[j];
        double dnew = wnorm(m, w->Mnew + s * nq);
        double dref = dref0[s] > dnew ? dref0[s] : dnew;
        if (!(sqrt(mx) <= prm->tol_inner * dref)) conv = 0;
      }
      memcpy(w->M, w->Mnew, sizeof(double) * n);
      if (conv) break;
    }
    total_inner += (l > prm->max_inner ? prm->max_inner : l);
    if (fatal) break;
    if (!conv) inner_failed = 1;

    if (prm->fixed_matter) {
      outer_conv = 1;
      break;
    }

    /* matter right-hand side, residual and outer Anderson step on y */
    double yq[5], f[5], ynew[5];
    matter_rhs_v(m, rho11, w->M, w->M + nn, y, X0, ystar, yq);
    for (int i = 0; i < 5; ++i) f[i] = yq[i] - y[i];
    hist_push(qh, fh, &ocount, prm->m_outer, 5, yq, f);
    ora_anderson(5, ocount, qh, fh, ynew);
    if (!all_finite(ynew, 5)) {
      status = ORA_NONFINITE;
      fatal = 1;
      break;
    }
    /* Algorithm outerConverged: Ye and ef componentwise against y*; each
     * velocity component against the speed max(|v*|, |v^[k+1]|) */
    double vref = norm3(ystar + 2), vn = norm3(ynew + 2);
    if (vn > vref) vref = vn;
    int oc = fabs(ynew[0] - y[0]) <= prm->tol_outer * fabs(ystar[0]) &&
             fabs(ynew[1] - y[1]) <= prm->tol_outer * fabs(ystar[1]);
    for (int j = 0; j < 3; ++j) oc = oc && fabs(ynew[2 + j] - y[2 + j]) <= prm->tol_outer * vref;
    for (int i = 0; i < 5; ++i) y[i] = ynew[i];
    if (oc) {
      outer_conv = 1;
      break;
    }
  }
  if (k > prm->max_outer) k = prm->max_outer;
  if (!fatal) {
    if (!outer_conv) status = ORA_MAX_OUTER;
    else if (inner_failed) status = ORA_MAX_INNER;
  }

  for (int i = 0; i < nn; ++i) D[i] = w->M[i];
  for (int i = 0; i < 3 * nn; ++i) I[i] = w->M[nn + i];
  if (prm->fixed_matter) {
    for (int i = 0; i < 5; ++i) yout[i] = ystar[i];
    *T_out = T_last;
  } else {
    /* output matter state: the matter right-hand side at the final moments
     * and the matter iterate they were solved at */
    matter_rhs_v(m, rho11, w->M, w->M + nn, yused, X0, ystar, yout);
    *T_out = eos_temperature_v(m, yout, rho11);
  }
  *n_outer = k;
  *n_inner = total_inner;
  return status;
}

int ora_solve_batch_v(const ora_model* m, const ora_params* prm, const double* theta, long P, double dtau,
                      const double* D0, const double* I0, const double* rho11, const double* ye0,
                      const double* ef0, const double* v0, const double* chi0,
                      double* D, double* I, double* ye, double* ef, double* v, double* T,
                      int* n_outer, int* n_inner, int* status, int nthreads) {
  if (m->nq < 1 || m->nq > ORA_MAX_NQ || m->ns < 1 || m->ns > ORA_MAX_NS) return -1;
  if (prm->m_inner < 1 || prm->m_inner > MAXMEM || prm->m_outer < 1 || prm->m_outer > MAXMEM) return -1;
  if (prm->max_inner < 1 || prm->max_outer < 1) return -1;
  if ((m->flags & ORA_PAIR))
    for (int s = 0; s < m->ns; ++s)
      if (partner_index(m, s) < 0) return -1;
  int nn = m->ns * m->nq;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    work_v* w = (work_v*)malloc(sizeof(work_v));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
    for (long p = 0; p < P; ++p) {
      double c0 = chi0 ? chi0[p] : m->chi_ref * rho11[p];
      double ystar[5] = {ye0[p], ef0[p], v0[3 * p], v0[3 * p + 1], v0[3 * p + 2]}, yo[5];
      if (rho11[p] < m->rho11_min) {
        /* coupling disabled at low density (Sec. 7.2): pass through */
        for (int i = 0; i < nn; ++i) D[p * nn + i] = D0[p * nn + i];
        for (int i = 0; i < 3 * nn; ++i) I[p * 3 * nn + i] = I0[p * 3 * nn + i];
        for (int i = 0; i < 5; ++i) yo[i] = ystar[i];
        T[p] = eos_temperature_v(m, ystar, rho11[p]);
        n_outer[p] = 0;
        n_inner[p] = 0;
        status[p] = ORA_OK;
      } else {
        status[p] = solve_point_v(m, prm, theta, dtau, D0 + p * nn, I0 + p * 3 * nn, rho11[p], ystar, c0,
                                  D + p * nn, I + p * 3 * nn, yo, T + p, n_outer + p, n_inner + p, w);
      }
      ye[p] = yo[0];
      ef[p] = yo[1];
      for (int j = 0; j < 3; ++j) v[3 * p + j] = yo[2 + j];
    }
    free(w);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Primitive-moment recovery (Sec. 3.4): for one species at one node, given
 * the conserved moments U = (N, G_j) and the velocity v, find M = (D, I_j)
 * with N = D + v^i I_i and G_j = I_j + v^i K_ij(M) (Eq.
 * conservedToPrimitive) by the fixed-point sequence of Eqs. c2p_FP,
 * c2p_sequence,
 *   M^[k+1] = (1 - lam) M^[k] + lam (N - v.I^[k], G_j - v^i K_ij(M^[k])),
 * lam = 1 / (1 + |v|), from M^[0] = U, with Anderson acceleration over the
 * last `mem` residuals, until ||M^[k+1] - M^[k]|| <= tol ||U|| (Euclidean).
 * Returns the iterations taken, or -1 when max_it is reached, -2 on a
 * non-finite iterate.  The map is homogeneous of degree one in U (K_ij = D
 * k_ij(|I| / D)), and so is the stopping test: the node is solved for U / s,
 * s = max_i |U_i|, and the result multiplied by s, so that the squared norms
 * and Anderson's Gram products of a faint node (a cold tail's 1e-200) do not
 * underflow; s is the power of two at max_i |U_i|, so the scaling is exact. */
static int c2p_scaled(double N, const double* G, const double* v, int mem, double tol, int max_it, double* M);

static int c2p_node(double N, const double* G, const double* v, int mem, double tol, int max_it, double* M) {
  double s = fabs(N);
  for (int j = 0; j < 3; ++j)
    if (fabs(G[j]) > s) s = fabs(G[j]);
  int e = 0;
  if (s > 0.0 && isfinite(s)) frexp(s, &e);
  s = ldexp(1.0, e);
  double Gs[3] = {G[0] / s, G[1] / s, G[2] / s};
  int it = c2p_scaled(N / s, Gs, v, mem, tol, max_it, M);
  for (int i = 0; i < 4; ++i) M[i] *= s;
  return it;
}

static int c2p_scaled(double N, const double* G, const double* v, int mem, double tol, int max_it, double* M) {
  double lam = 1.0 / (1.0 + norm3(v));
  double U[4] = {N, G[0], G[1], G[2]};
  double unorm = sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2] + U[3] * U[3]);
  double Qh[MAXMEM * 4], Fh[MAXMEM * 4], Mn[4];
  int count = 0;
  for (int i = 0; i < 4; ++i) M[i] = U[i];
  for (int k = 1; k <= max_it; ++k) {
    double K9[9], g[4], f[4];
    ora_eddington(M[0], M + 1, K9);
    g[0] = (1.0 - lam) * M[0] + lam * (N - (v[0] * M[1] + v[1] * M[2] + v[2] * M[3]));
    for (int j = 0; j < 3; ++j)
      g[1 + j] = (1.0 - lam) * M[1 + j] + lam * (G[j] - (v[0] * K9[3 * j] + v[1] * K9[3 * j + 1] + v[2] * K9[3 * j + 2]));
    for (int i = 0; i < 4; ++i) f[i] = g[i] - M[i];
    hist_push(Qh, Fh, &count, mem, 4, g, f);
    ora_anderson(4, count, Qh, Fh, Mn);
    if (!all_finite(Mn, 4)) return -2;
    double d2 = 0.0;
    for (int i = 0; i < 4; ++i) d2 += (Mn[i] - M[i]) * (Mn[i] - M[i]);
    for (int i = 0; i < 4; ++i) M[i] = Mn[i];
    if (sqrt(d2) <= tol * unorm) return k;
  }
  return -1;
}

int ora_primitive_batch(const ora_model* m, long P, const double* N, const double* G, const double* v, int mem,
                        double tol, int max_it, double* D, double* I, int* iters, int nthreads) {
  if (m->nq < 1 || m->nq > ORA_MAX_NQ || m->ns < 1 || m->ns > ORA_MAX_NS) return -1;
  if (mem < 1 || mem > MAXMEM || max_it < 1 || !(tol > 0.0)) return -1;
  int nq = m->nq, ns = m->ns;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
  for (long p = 0; p < P; ++p)
    for (int s = 0; s < ns; ++s)
      for (int q = 0; q < nq; ++q) {
        long i = (p * ns + s) * nq + q;
        double Gq[3], M[4];
        for (int j = 0; j < 3; ++j) Gq[j] = G[((p * ns + s) * 3 + j) * nq + q];
        iters[i] = c2p_node(N[i], Gq, v + 3 * p, mem, tol, max_it, M);
        D[i] = M[0];
        for (int j = 0; j < 3; ++j) I[((p * ns + s) * 3 + j) * nq + q] = M[1 + j];
      }
  return 0;
}

/* conserved moments of primitive ones at velocity v: N = D + v.I,
 * G_j = I_j + v^i K_ij (Eq. conservedToPrimitive), for one point */
static void p2c_point(const ora_model* m, const double* D, const double* I, const double* v, double* N, double* G) {
  int nq = m->nq, ns = m->ns;
  for (int s = 0; s < ns; ++s)
    for (int q = 0; q < nq; ++q) {
      double I3[3], K9[9];
      flux3(m, I, s, q, I3);
      ora_eddington(D[s * nq + q], I3, K9);
      N[s * nq + q] = D[s * nq + q] + v[0] * I3[0] + v[1] * I3[1] + v[2] * I3[2];
      for (int j = 0; j < 3; ++j)
        G[(s * 3 + j) * nq + q] = I3[j] + v[0] * K9[3 * j] + v[1] * K9[3 * j + 1] + v[2] * K9[3 * j + 2];
    }
}

/* One time step of the IMEX scheme with the PD-ARS tableau (Eq.
 * butcherPDARS) for the neutrino-matter coupling alone (the explicit
 * operator, phase-space advection, is zero here).  Stage i takes the
 * intermediate state U^(i*) = U^n + dt sum_{j<i} a_ij C^(j) (conserved
 * moments; the matter state likewise) and solves the modified backward-Euler
 * problem with step a_ii dt (Algorithm neutrinoMatterCoupling through
 * ora_solve_batch_v); C^(j) = (U^(j) - U^(j*)) / (a_jj dt) is the collision
 * term the stage-j solve applied.  Stage 1 has a_11 = 0 (U^(1) = U^n) and
 * enters no later stage (a_21 = a_31 = 0).  The stage-3 intermediate state is
 * recovered to primitive moments (primitive recovery, c2p parameters) before
 * its solve.  The scheme is globally stiffly accurate, so the step's result
 * is U^(3).  n_outer / n_inner sum over the two solves; status: the first
 * non-OK of stage 2, the primitive recovery (ORA_MAX_INNER when it does not
 * converge, ORA_NONFINITE), stage 3. */
int ora_pdars_step_v(const ora_model* m, const ora_params* prm, const double* theta, long P, double dt,
                     const double* D0, const double* I0, const double* rho11, const double* ye0,
                     const double* ef0, const double* v0, const double* chi0, int c2p_mem, double c2p_tol,
                     int c2p_max, double* D, double* I, double* ye, double* ef, double* v, double* T,
                     int* n_outer, int* n_inner, int* status, int nthreads) {
  static const double a[3][3] = {{0.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.5, 0.5}};
  int nq = m->nq, ns = m->ns, nn = ns * nq;
  if (!(dt > 0.0)) return -1;
  size_t szD = (size_t)P * nn, szI = (size_t)P * 3 * nn;
  double *D2 = malloc(szD * 8), *I2 = malloc(szI * 8), *y2e = malloc(P * 8), *y2f = malloc(P * 8);
  double *v2 = malloc(P * 3 * 8), *T2 = malloc(P * 8);
  double *D3 = malloc(szD * 8), *I3 = malloc(szI * 8), *y3e = malloc(P * 8), *y3f = malloc(P * 8),
         *v3 = malloc(P * 3 * 8);
  double *Nn = malloc(szD * 8), *Gn = malloc(szI * 8), *N2 = malloc(szD * 8), *G2 = malloc(szI * 8);
  double *N3 = malloc(szD * 8), *G3 = malloc(szI * 8);
  int *no2 = malloc(P * 4), *ni2 = malloc(P * 4), *st2 = malloc(P * 4), *it = malloc(szD * 4);
  int rc = 0;
  /* stage 2: U^(2*) = U^n; backward Euler with a_22 dt */
  rc = ora_solve_batch_v(m, prm, theta, P, a[1][1] * dt, D0, I0, rho11, ye0, ef0, v0, chi0, D2, I2, y2e, y2f, v2,
                         T2, no2, ni2, st2, nthreads);
  if (rc == 0) {
    /* stage 3: U^(3*) = U^n + dt a_32 C^(2), C^(2) = (U^(2) - U^(2*)) / (a_22 dt);
     * likewise the matter state */
    double w = a[2][1] / a[1][1];
    for (long p = 0; p < P; ++p) {
      p2c_point(m, D0 + p * nn, I0 + p * 3 * nn, v0 + 3 * p, Nn + p * nn, Gn + p * 3 * nn);
      p2c_point(m, D2 + p * nn, I2 + p * 3 * nn, v2 + 3 * p, N2 + p * nn, G2 + p * 3 * nn);
      for (int i = 0; i < nn; ++i) N3[p * nn + i] = Nn[p * nn + i] + w * (N2[p * nn + i] - Nn[p * nn + i]);
      for (int i = 0; i < 3 * nn; ++i)
        G3[p * 3 * nn + i] = Gn[p * 3 * nn + i] + w * (G2[p * 3 * nn + i] - Gn[p * 3 * nn + i]);
      y3e[p] = ye0[p] + w * (y2e[p] - ye0[p]);
      y3f[p] = ef0[p] + w * (y2f[p] - ef0[p]);
      for (int j = 0; j < 3; ++j) v3[3 * p + j] = v0[3 * p + j] + w * (v2[3 * p + j] - v0[3 * p + j]);
    }
    rc = ora_primitive_batch(m, P, N3, G3, v3, c2p_mem, c2p_tol, c2p_max, D3, I3, it, nthreads);
    /* points below the coupling density pass through the whole step */
    for (long p = 0; p < P && rc == 0; ++p)
      if (rho11[p] < m->rho11_min) {
        for (int i = 0; i < nn; ++i) {
          D3[p * nn + i] = D0[p * nn + i];
          it[p * nn + i] = 0;
        }
        for (int i = 0; i < 3 * nn; ++i) I3[p * 3 * nn + i] = I0[p * 3 * nn + i];
        y3e[p] = ye0[p];
        y3f[p] = ef0[p];
        for (int j = 0; j < 3; ++j) v3[3 * p + j] = v0[3 * p + j];
      }
  }
  if (rc == 0)
    rc = ora_solve_batch_v(m, prm, theta, P, a[2][2] * dt, D3, I3, rho11, y3e, y3f, v3, chi0, D, I, ye, ef, v, T,
                           n_outer, n_inner, status, nthreads);
  if (rc == 0)
    for (long p = 0; p < P; ++p) {
      int c2p = ORA_OK;
      for (int i = 0; i < nn; ++i) {
        if (it[p * nn + i] == -2) c2p = ORA_NONFINITE;
        if (it[p * nn + i] == -1 && c2p == ORA_OK) c2p = ORA_MAX_INNER;
      }
      if (st2[p] != ORA_OK) status[p] = st2[p];
      else if (c2p != ORA_OK) status[p] = c2p;
      n_outer[p] += no2[p];
      n_inner[p] += ni2[p];
    }
  free(D2); free(I2); free(y2e); free(y2f); free(v2); free(T2);
  free(D3); free(I3); free(y3e); free(y3f); free(v3);
  free(Nn); free(Gn); free(N2); free(G2); free(N3); free(G3);
  free(no2); free(ni2); free(st2); free(it);
  return rc;
}

/* Initial state from raw draws: e* from the EOS, D* = clip(D_eq (a + b uD),
 * 0, 1 - 1e-12), I* = c D* uI.  If mu is NULL it follows from the EOS. */
int ora_init_state(const ora_model* m, long P, const double* T, const double* mu, const double* rho11,
                   const double* ye, const double* uD, const double* uI, double a, double b, double c,
                   double* D0, double* I0, double* e0) {
  int nq = m->nq, ns = m->ns, nn = ns * nq;
  for (long p = 0; p < P; ++p) {
    double mup = mu ? mu[p] : ora_eos_mu(m, ye[p], T[p], rho11[p]);
    if (e0) e0[p] = ora_eos_energy(m, T[p], ye[p], rho11[p]);
    for (int s = 0; s < ns; ++s) {
      double mus = sp_musign(m->species[s]) * mup;
      for (int q = 0; q < nq; ++q) {
        long i = p * nn + s * nq + q;
        double d = ora_fermi_dirac(m->eps[q], mus, T[p]) * (a + b * uD[i]);
        if (d < 0.0) d = 0.0;
        if (d > 1.0 - 1e-12) d = 1.0 - 1e-12;
        D0[i] = d;
        I0[i] = c * d * uI[i];
      }
    }
  }
  return 0;
}
