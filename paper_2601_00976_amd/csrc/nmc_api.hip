// Host side of the nmc C ABI: handles, argument validation and launches.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>

#include "nmc_internal.h"

struct nmc_grid {
  int n_elem;
  int nq;
  double edges[nmc::kMaxNq / 2 + 1];
  double eps[nmc::kMaxNq];
  double w2[nmc::kMaxNq];
  double w3[nmc::kMaxNq];
};

struct nmc_model {
  nmc::DevModel host;
  nmc::DevModel* dev;
  int device;
  int num_cu;
  void* scratch;  // device address of the static scratch on `device`
  hipError_t scratch_err;  // result of its lookup
};

// Static scratch of nmc_solve_batch_noalloc: the work-queue counters (and,
// for kernels stored in HBM, the kernel store) of solves that may not
// allocate.  Each device holds its own copy for the life of the process.  In
// host code `scratch` is a host-side stand-in, never a device address: the
// device address comes from hipGetSymbolAddress, once per device.
static constexpr size_t kScratchBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(NMC_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

constexpr size_t kCounterBytes = 2048;  // work-queue counters: 8 lines of 256 bytes

// per-device addresses of the static scratch
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// device address of `scratch` on device `dev` (current), looked up once
hipError_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

int partner_id(int id) { return id == NMC_NU_E ? NMC_NU_E_BAR : (id == NMC_NU_E_BAR ? NMC_NU_E : NMC_NU_X); }

}  // namespace

extern "C" {

const char* nmc_error_string(int code) {
  switch (code) {
    case NMC_OK: return "ok";
    case NMC_E_INVALID_ARG: return "invalid argument";
    case NMC_E_UNSUPPORTED: return "unsupported configuration";
    case NMC_E_HIP: return "HIP runtime error";
    case NMC_E_WORKSPACE: return "workspace too small or misaligned";
    default: return "unknown error";
  }
}

const char* nmc_last_error(void) { return g_last_error.c_str(); }

void nmc_model_desc_default(nmc_model_desc* d) {
  if (!d) return;
  memset(d, 0, sizeof(*d));
  d->n_species = 3;
  d->species[0] = NMC_NU_E;
  d->species[1] = NMC_NU_E_BAR;
  d->species[2] = NMC_NU_X;
  d->flags = NMC_ALL_PHYSICS;
  d->chi_ref = 10.0;
  d->eps_ref = 10.0;
  d->chi_power = 2.0;
  d->sigma_ratio = 0.5;
  d->eos_a = 1.5;
  d->eos_b = 3.0;
  d->mu_a = 20.0;
  d->mu_ye0 = 0.3;
  d->mu_b = 5.0;
  d->mu_t0 = 5.0;
  d->hc_mev_cm = 1.239841984e-10;
  d->m_u_g = 1.66053906660e-24;
  d->rho11_min = 1.0e-4;
  d->fd_projection = 0;
  d->deq_min = 1.0e-150;
  d->deq_max = 1.0 - 1.0e-12;
}

void nmc_solver_params_default(nmc_solver_params* p) {
  if (!p) return;
  p->tol_inner = 1e-10;
  p->tol_outer = 1e-10;
  p->m_inner = 3;
  p->m_outer = 3;
  p->max_inner = 100;
  p->max_outer = 50;
  p->fixed_matter = 0;
}

// Energy grid: element edges, then 2 Legendre-Gauss nodes per element on the
// reference interval (-1/2, 1/2) with weights 1/2 (Sec. 3.1.2) and the
// integration weights of Eq. energy_integration_weights without 4 pi / h^3.
int nmc_grid_create(const nmc_grid_desc* desc, nmc_grid** out) {
  if (!desc || !out) return fail(NMC_E_INVALID_ARG, "grid_create: null argument");
  *out = nullptr;
  if (desc->nodes_per_elem != 2)
    return fail(NMC_E_UNSUPPORTED, "grid_create: nodes_per_elem must be 2 (got %d)", desc->nodes_per_elem);
  if (desc->n_elem < 1 || 2 * desc->n_elem > nmc::kMaxNq)
    return fail(NMC_E_INVALID_ARG, "grid_create: n_elem must be in [1, %d] (got %d)", nmc::kMaxNq / 2, desc->n_elem);
  if (!(desc->eps_hi > 0.0) || !isfinite(desc->eps_hi)) return fail(NMC_E_INVALID_ARG, "grid_create: bad eps_hi");
  nmc_grid* g = new (std::nothrow) nmc_grid();
  if (!g) return fail(NMC_E_INVALID_ARG, "grid_create: out of host memory");
  const int ne = desc->n_elem;
  g->n_elem = ne;
  g->nq = 2 * ne;
  if (desc->spacing == NMC_SPACING_LOG) {
    if (!(desc->eps_lo > 0.0) || !(desc->eps_hi > desc->eps_lo)) {
      delete g;
      return fail(NMC_E_INVALID_ARG, "grid_create: LOG spacing needs 0 < eps_lo < eps_hi");
    }
    for (int e = 0; e <= ne; ++e) g->edges[e] = desc->eps_lo * pow(desc->eps_hi / desc->eps_lo, (double)e / ne);
    g->edges[ne] = desc->eps_hi;
  } else if (desc->spacing == NMC_SPACING_ZOOM) {
    if (!(desc->zoom > 0.0) || !isfinite(desc->zoom)) {
      delete g;
      return fail(NMC_E_INVALID_ARG, "grid_create: ZOOM spacing needs zoom > 0");
    }
    const double z = desc->zoom;
    const double d1 = (z == 1.0) ? desc->eps_hi / ne : desc->eps_hi * (z - 1.0) / (pow(z, ne) - 1.0);
    g->edges[0] = 0.0;
    double d = d1;
    for (int e = 0; e < ne; ++e) {
      g->edges[e + 1] = g->edges[e] + d;
      d *= z;
    }
  } else {
    delete g;
    return fail(NMC_E_INVALID_ARG, "grid_create: unknown spacing %d", desc->spacing);
  }
  const double xi = 0.5 / sqrt(3.0);
  for (int e = 0; e < ne; ++e) {
    const double c = 0.5 * (g->edges[e] + g->edges[e + 1]);
    const double w = g->edges[e + 1] - g->edges[e];
    for (int k = 0; k < 2; ++k) {
      const int i = 2 * e + k;
      g->eps[i] = c + w * (k == 0 ? -xi : xi);
      g->w2[i] = 0.5 * g->eps[i] * g->eps[i] * w;
      g->w3[i] = g->w2[i] * g->eps[i];
    }
  }
  *out = g;
  return NMC_OK;
}

int nmc_grid_query(const nmc_grid* g, int* nq, double* eps, double* w2, double* w3) {
  if (!g) return fail(NMC_E_INVALID_ARG, "grid_query: null grid");
  if (nq) *nq = g->nq;
  if (eps) memcpy(eps, g->eps, sizeof(double) * g->nq);
  if (w2) memcpy(w2, g->w2, sizeof(double) * g->nq);
  if (w3) memcpy(w3, g->w3, sizeof(double) * g->nq);
  return NMC_OK;
}

int nmc_grid_destroy(nmc_grid* g) {
  delete g;
  return NMC_OK;
}

int nmc_model_create(const nmc_grid* g, const nmc_model_desc* d, nmc_model** out) {
  if (!g || !d || !out) return fail(NMC_E_INVALID_ARG, "model_create: null argument");
  *out = nullptr;
  if (g->nq != 32 && g->nq != 64)
    return fail(NMC_E_UNSUPPORTED, "model_create: the solver supports 32 or 64 energy nodes (grid has %d)", g->nq);
  if (d->n_species < 1 || d->n_species > nmc::kMaxNs)
    return fail(NMC_E_UNSUPPORTED, "model_create: n_species must be 1..3 (got %d)", d->n_species);
  if (d->flags & ~NMC_ALL_PHYSICS) return fail(NMC_E_INVALID_ARG, "model_create: unknown physics flags");
  nmc::DevModel m;
  memset(&m, 0, sizeof(m));
  m.ns = d->n_species;
  m.nq = g->nq;
  m.flags = d->flags;
  for (int s = 0; s < m.ns; ++s) {
    const int id = d->species[s];
    if (id < NMC_NU_E || id > NMC_NU_X) return fail(NMC_E_INVALID_ARG, "model_create: bad species id %d", id);
    for (int t = 0; t < s; ++t)
      if (d->species[t] == id) return fail(NMC_E_INVALID_ARG, "model_create: species %d listed twice", id);
    m.species[s] = id;
    m.g[s] = id == NMC_NU_E ? 1.0 : (id == NMC_NU_E_BAR ? -1.0 : 0.0);
    m.mult[s] = id == NMC_NU_X ? 4.0 : 1.0;
    m.musign[s] = id == NMC_NU_E ? 1.0 : (id == NMC_NU_E_BAR ? -1.0 : 0.0);
    m.emab[s] = id == NMC_NU_X ? 0.0 : 1.0;
  }
  for (int s = 0; s < m.ns; ++s) {
    m.partner[s] = -1;
    for (int t = 0; t < m.ns; ++t)
      if (m.species[t] == partner_id(m.species[s])) m.partner[s] = t;
    if ((m.flags & NMC_PAIR) && m.partner[s] < 0)
      return fail(NMC_E_UNSUPPORTED, "model_create: pair processes need the partner of species %d", m.species[s]);
  }
  for (int t = 0, k = 0; t < m.ns; ++t) {
    // t-th smallest species id
    int best = -1;
    for (int s = 0; s < m.ns; ++s) {
      bool taken = false;
      for (int u = 0; u < k; ++u) taken = taken || m.ext[u] == s;
      if (!taken && (best < 0 || m.species[s] < m.species[best])) best = s;
    }
    m.ext[k] = best;
    m.ig[k] = m.g[best];
    m.imult[k] = m.mult[best];
    m.imusign[k] = m.musign[best];
    m.iemab[k] = m.emab[best];
    ++k;
  }
  const double vals[] = {d->chi_ref, d->eps_ref, d->chi_power, d->sigma_ratio, d->eos_a, d->eos_b, d->mu_a,
                         d->mu_ye0, d->mu_b, d->mu_t0, d->hc_mev_cm, d->m_u_g, d->rho11_min, d->phi1_nes,
                         d->phi1_pair};
  for (double v : vals)
    if (!isfinite(v)) return fail(NMC_E_INVALID_ARG, "model_create: non-finite constant");
  if (!(d->eps_ref > 0) || !(d->eos_a > 0) || !(d->mu_t0 > 0) || !(d->hc_mev_cm > 0) || !(d->m_u_g > 0))
    return fail(NMC_E_INVALID_ARG, "model_create: eps_ref, eos_a, mu_t0, hc, m_u must be positive");
  for (int q = 0; q < m.nq; ++q) {
    m.eps[q] = g->eps[q];
    m.w2[q] = g->w2[q];
    m.w3[q] = g->w3[q];
    m.shape[q] = pow(g->eps[q] / d->eps_ref, d->chi_power);
  }
  m.chi_ref = d->chi_ref;
  m.sigma_ratio = d->sigma_ratio;
  m.eos_a = d->eos_a;
  m.eos_b = d->eos_b;
  m.mu_a = d->mu_a;
  m.mu_ye0 = d->mu_ye0;
  m.mu_b = d->mu_b;
  m.mu_t0 = d->mu_t0;
  m.inv_mu_t0 = 1.0 / d->mu_t0;
  const double pi = 3.14159265358979323846;
  const double hc = d->hc_mev_cm;
  m.kcoup = 4.0 * pi / (hc * hc * hc) * d->m_u_g / 1.0e11;
  m.rho11_min = d->rho11_min;
  if (!(fabs(d->phi1_nes) <= 1.0 / 3.0) || !(fabs(d->phi1_pair) <= 1.0 / 3.0))
    return fail(NMC_E_INVALID_ARG, "model_create: phi1_nes and phi1_pair must lie in [-1/3, 1/3]");
  m.phi1_nes = d->phi1_nes;
  m.phi1_pair = d->phi1_pair;
  if (d->fd_projection != 0 && d->fd_projection != 1)
    return fail(NMC_E_INVALID_ARG, "model_create: fd_projection must be 0 or 1");
  // bounds that keep the odds D / (1 - D), their square roots and the pair
  // products o o' normal doubles
  if (!(d->deq_min >= 1e-150) || !(d->deq_min <= 1e-3) || !(d->deq_max >= 0.999) || !(d->deq_max <= 1.0 - 1e-15))
    return fail(NMC_E_INVALID_ARG, "model_create: need 1e-150 <= deq_min <= 1e-3 and 0.999 <= deq_max <= 1 - 1e-15");
  m.fd_projection = d->fd_projection;
  m.deq_min = d->deq_min;
  m.ceq_min = 1.0 - d->deq_max;
  // per-node tables of the projection: eps^2 mass matrix of the element's
  // Lagrange basis by the 3-point Gauss rule (exact for its degree-4
  // integrands), inverted in closed form
  for (int e = 0; 2 * e < m.nq; ++e) {
    const double lo = g->edges[e], hi = g->edges[e + 1];
    const double e1 = g->eps[2 * e], e2 = g->eps[2 * e + 1];
    const double c = 0.5 * (lo + hi), r = 0.5 * (hi - lo), x3 = sqrt(0.6);
    const double gx[3] = {c - r * x3, c, c + r * x3}, gw[3] = {r * 5.0 / 9.0, r * 8.0 / 9.0, r * 5.0 / 9.0};
    double M11 = 0.0, M12 = 0.0, M22 = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double x = gx[k], w = gw[k] * x * x;
      const double l1 = (x - e2) / (e1 - e2), l2 = (x - e1) / (e2 - e1);
      M11 += w * l1 * l1;
      M12 += w * l1 * l2;
      M22 += w * l2 * l2;
    }
    const double det = M11 * M22 - M12 * M12;
    for (int side = 0; side < 2; ++side) {
      const int q = 2 * e + side;
      m.pelo[q] = lo;
      m.pehi[q] = hi;
      m.pl[q][0] = 1.0 / (e1 - e2);
      m.pl[q][1] = -e2 / (e1 - e2);
      m.pl[q][2] = 1.0 / (e2 - e1);
      m.pl[q][3] = -e1 / (e2 - e1);
      m.pinv[q][0] = (side == 0 ? M22 : -M12) / det;
      m.pinv[q][1] = (side == 0 ? -M12 : M11) / det;
      m.prm0[q] = 3.0 / (hi * hi * hi - lo * lo * lo);
      const double eo = side == 0 ? e2 : e1, es = side == 0 ? e1 : e2;
      m.pedge[q][0] = (lo - eo) / (es - eo);
      m.pedge[q][1] = (hi - eo) / (es - eo);
    }
  }

  nmc_model* mm = new (std::nothrow) nmc_model();
  if (!mm) return fail(NMC_E_INVALID_ARG, "model_create: out of host memory");
  mm->host = m;
  hipError_t e = hipGetDevice(&mm->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&mm->num_cu, hipDeviceAttributeMultiprocessorCount, mm->device);
  if (e == hipSuccess) e = hipMalloc((void**)&mm->dev, sizeof(nmc::DevModel));
  if (e == hipSuccess) e = hipMemcpy(mm->dev, &m, sizeof(m), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (mm->dev) (void)hipFree(mm->dev);
    delete mm;
    return hip_fail(e, "model_create");
  }
  // the static scratch of the no-allocation solve, looked up with the
  // model's device current; a failed lookup disables only that entry point
  mm->scratch_err = scratch_address(mm->device, &mm->scratch);
  if (mm->scratch_err != hipSuccess) mm->scratch = nullptr;
  *out = mm;
  return NMC_OK;
}

int nmc_model_destroy(nmc_model* m) {
  if (!m) return NMC_OK;
  hipError_t e = m->dev ? hipFree(m->dev) : hipSuccess;
  delete m;
  return e == hipSuccess ? NMC_OK : hip_fail(e, "model_destroy");
}

size_t nmc_workspace_bytes(const nmc_model* m, int64_t P) {
  if (!m || P < 0) return 0;
  // queue counters + per-point adjoint terms and a column-partial buffer
  const size_t nt = (size_t)m->host.nq + 2;
  const size_t pp = ((size_t)P * nt * sizeof(double) + 255) & ~(size_t)255;
  const size_t part = ((size_t)nmc::kReduceBlocks * nt * sizeof(double) + 255) & ~(size_t)255;
  return kCounterBytes + pp + part;
}

size_t nmc_kernel_store_bytes(const nmc_model* m, int64_t P) {
  if (!m || P < 0 || m->host.nq != 64) return 0;
  const size_t nq = (size_t)m->host.nq;
  return ((size_t)P * 3 * nq * nq * sizeof(double) + 255) & ~(size_t)255;
}

static int check_params(const nmc_solver_params* p) {
  if (!p) return fail(NMC_E_INVALID_ARG, "null solver params");
  if (!(p->tol_inner > 0.0) || !(p->tol_outer > 0.0) || !isfinite(p->tol_inner) || !isfinite(p->tol_outer))
    return fail(NMC_E_INVALID_ARG, "tolerances must be positive and finite");
  if (p->m_inner < 1 || p->m_inner > 3 || p->m_outer < 1 || p->m_outer > 3)
    return fail(NMC_E_UNSUPPORTED, "Anderson memories must be in 1..3 (got %d, %d)", p->m_inner, p->m_outer);
  if (p->max_inner < 1 || p->max_outer < 1 || p->max_inner > 100000 || p->max_outer > 100000)
    return fail(NMC_E_INVALID_ARG, "iteration caps must be in 1..100000");
  return NMC_OK;
}

// The batched forward solve behind nmc_solve_batch and
// nmc_solve_batch_noalloc: validation, then the launch with the work-queue
// counters at `ws` and, for kernels stored in HBM, the kernel store at
// `ws + kstore_off`.  `who` names the entry point in error messages.
static int solve_batch_impl(const char* who, const nmc_model* m, const nmc_solver_params* prm, int64_t P,
                            double dtau, const nmc_batch_in* in, const nmc_batch_out* out, void* ws,
                            size_t ws_bytes, size_t kstore_off, const nmc_launch* launch, void* stream) {
  if (!m || !in || !out) return fail(NMC_E_INVALID_ARG, "%s: null handle or descriptor", who);
  int rc = check_params(prm);
  if (rc) return rc;
  if (P < 0 || P > (int64_t(1) << 30)) return fail(NMC_E_INVALID_ARG, "%s: P out of range (%lld)", who, (long long)P);
  if (!(dtau > 0.0) || !isfinite(dtau)) return fail(NMC_E_INVALID_ARG, "%s: dtau must be positive", who);
  if (P == 0) return NMC_OK;
  if (!in->D0 || !in->I0 || !in->rho11 || !in->ye0 || !in->e0 || !in->theta)
    return fail(NMC_E_INVALID_ARG, "%s: null input array", who);
  if (!out->D || !out->I || !out->ye || !out->e || !out->T || !out->n_outer || !out->n_inner || !out->status)
    return fail(NMC_E_INVALID_ARG, "%s: null output array", who);
  if ((in->T_fixed || in->mu_fixed) && !prm->fixed_matter)
    return fail(NMC_E_INVALID_ARG, "%s: T_fixed / mu_fixed need fixed_matter", who);
  nmc_launch L = {0, 1, 1, NMC_KERNELS_ON_CHIP};
  if (launch) L = *launch;
  if (L.chunk < 1 || L.chunk > 4096 || L.blocks_per_cu < 0 || L.blocks_per_cu > 64)
    return fail(NMC_E_INVALID_ARG, "%s: bad launch configuration", who);
  if (L.kernel_store < NMC_KERNELS_ON_CHIP || L.kernel_store > NMC_KERNELS_WAVE)
    return fail(NMC_E_INVALID_ARG, "%s: bad kernel_store %d", who, L.kernel_store);
  double* kstore = nullptr;
  if (L.kernel_store == NMC_KERNELS_REGISTERS && m->host.nq != 32)
    return fail(NMC_E_UNSUPPORTED, "%s: register-resident kernel rows need 32 nodes", who);
  if ((L.kernel_store == NMC_KERNELS_PAIRED || L.kernel_store == NMC_KERNELS_WAVE) && m->host.nq != 32)
    return fail(NMC_E_UNSUPPORTED, "%s: kernel_store %d needs 32 nodes", who, L.kernel_store);
  if (m->host.fd_projection &&
      (m->host.nq != 32 || (L.kernel_store != NMC_KERNELS_ON_CHIP && L.kernel_store != NMC_KERNELS_PAIRED)))
    return fail(NMC_E_UNSUPPORTED, "%s: the projected equilibrium runs in the two-points-per-wave kernel (32 nodes, "
                "kernel_store ON_CHIP or PAIRED)", who);
  if (L.kernel_store == NMC_KERNELS_HBM) {
    if (m->host.nq != 64 || !(m->host.flags & (NMC_NES | NMC_PAIR)))
      return fail(NMC_E_UNSUPPORTED, "%s: kernels in HBM need 64 nodes and NES or pair physics", who);
    const size_t need = kstore_off + nmc_kernel_store_bytes(m, P);
    if (!ws || !aligned256(ws) || ws_bytes < need)
      return fail(NMC_E_WORKSPACE, "%s: kernels in HBM need %zu workspace bytes (%zu available)", who, need,
                  ws_bytes);
    kstore = (double*)((char*)ws + kstore_off);
  }
  if (L.persistent) {
    if (!ws || !aligned256(ws) || ws_bytes < kCounterBytes)
      return fail(NMC_E_WORKSPACE, "%s: persistent launch needs a 256-byte aligned workspace", who);
  }
  nmc::FwdArgs a;
  memset(&a, 0, sizeof(a));
  a.mdl = m->dev;
  a.prm.tol_inner = prm->tol_inner;
  a.prm.tol_outer = prm->tol_outer;
  a.prm.m_inner = prm->m_inner;
  a.prm.m_outer = prm->m_outer;
  a.prm.max_inner = prm->max_inner;
  a.prm.max_outer = prm->max_outer;
  a.prm.fixed_matter = prm->fixed_matter ? 1 : 0;
  a.tol_inner2 = prm->tol_inner * prm->tol_inner;
  a.P = P;
  a.dtau = dtau;
  a.D0 = in->D0;
  a.I0 = in->I0;
  a.rho11 = in->rho11;
  a.ye0 = in->ye0;
  a.e0 = in->e0;
  a.chi0 = in->chi0;
  a.T_fixed = in->T_fixed;
  a.mu_fixed = in->mu_fixed;
  a.theta = in->theta;
  a.D = out->D;
  a.I = out->I;
  a.ye = out->ye;
  a.e = out->e;
  a.T = out->T;
  a.n_outer = out->n_outer;
  a.n_inner = out->n_inner;
  a.status = out->status;
  a.chunk = L.chunk;
  a.kstore = kstore;
  hipStream_t s = (hipStream_t)stream;
  if (L.persistent) {
    a.queue = (int*)ws;
    hipError_t e = nmc::launch_reset_counter(a.queue, s);
    if (e != hipSuccess) return hip_fail(e, "counter reset");
  }
  const bool coupled = (m->host.flags & (NMC_NES | NMC_PAIR)) != 0;
  hipError_t e = nmc::launch_forward(a, m->host.nq, m->host.ns, coupled, m->host.fd_projection != 0, L, m->num_cu, s);
  if (e == hipErrorInvalidValue)
    return fail(NMC_E_UNSUPPORTED, "%s: no kernel for nq=%d ns=%d", who, m->host.nq, m->host.ns);
  if (e != hipSuccess) return hip_fail(e, "forward launch");
  return NMC_OK;
}

int nmc_solve_batch(const nmc_model* m, const nmc_solver_params* prm, int64_t P, double dtau,
                    const nmc_batch_in* in, const nmc_batch_out* out, void* ws, size_t ws_bytes,
                    const nmc_launch* launch, void* stream) {
  return solve_batch_impl("solve_batch", m, prm, P, dtau, in, out, ws, ws_bytes, m ? nmc_workspace_bytes(m, P) : 0,
                          launch, stream);
}

int nmc_solve_batch_noalloc(const nmc_model* m, const nmc_solver_params* prm, int64_t P, double dtau,
                            const nmc_batch_in* in, const nmc_batch_out* out, const nmc_launch* launch,
                            void* stream) {
  if (!m) return fail(NMC_E_INVALID_ARG, "solve_batch_noalloc: null model");
  if (!m->scratch)
    return fail(NMC_E_HIP, "solve_batch_noalloc: no static scratch address on device %d: %s", m->device,
                hipGetErrorString(m->scratch_err));
  if (launch && launch->kernel_store == NMC_KERNELS_HBM && P > 0) {
    const size_t need = kCounterBytes + nmc_kernel_store_bytes(m, P);
    if (need > kScratchBytes)
      return fail(NMC_E_WORKSPACE,
                  "solve_batch_noalloc: %lld points with kernels in HBM need %zu bytes of scratch; the static "
                  "scratch holds %zu",
                  (long long)P, need, kScratchBytes);
  }
  return solve_batch_impl("solve_batch_noalloc", m, prm, P, dtau, in, out, m->scratch, kScratchBytes,
                          kCounterBytes, launch, stream);
}

int nmc_solve_batch_v(const nmc_model* m, const nmc_solver_params* prm, int64_t P, double dtau,
                      const nmc_batch_v_in* in, const nmc_batch_v_out* out, void* ws, size_t ws_bytes,
                      const nmc_launch* launch, void* stream) {
  if (!m || !in || !out) return fail(NMC_E_INVALID_ARG, "solve_batch_v: null handle or descriptor");
  int rc = check_params(prm);
  if (rc) return rc;
  if (P < 0 || P > (int64_t(1) << 30)) return fail(NMC_E_INVALID_ARG, "solve_batch_v: P out of range (%lld)", (long long)P);
  if (!(dtau > 0.0) || !isfinite(dtau)) return fail(NMC_E_INVALID_ARG, "solve_batch_v: dtau must be positive");
  if (m->host.nq != 32)
    return fail(NMC_E_UNSUPPORTED, "solve_batch_v: implemented for 32 energy nodes (model has %d)", m->host.nq);
  if (m->host.fd_projection)
    return fail(NMC_E_UNSUPPORTED, "solve_batch_v: the projected equilibrium is implemented in nmc_solve_batch only");
  if (P == 0) return NMC_OK;
  if (!in->D0 || !in->I0 || !in->rho11 || !in->ye0 || !in->ef0 || !in->v0 || !in->theta)
    return fail(NMC_E_INVALID_ARG, "solve_batch_v: null input array");
  if (!out->D || !out->I || !out->ye || !out->ef || !out->v || !out->T || !out->n_outer || !out->n_inner ||
      !out->status)
    return fail(NMC_E_INVALID_ARG, "solve_batch_v: null output array");
  nmc_launch L = {0, 1, 1, NMC_KERNELS_ON_CHIP};
  if (launch) L = *launch;
  if (L.chunk < 1 || L.chunk > 4096 || L.blocks_per_cu < 0 || L.blocks_per_cu > 64)
    return fail(NMC_E_INVALID_ARG, "solve_batch_v: bad launch configuration");
  if (L.kernel_store != NMC_KERNELS_ON_CHIP && L.kernel_store != NMC_KERNELS_PAIRED &&
      L.kernel_store != NMC_KERNELS_WAVE)
    return fail(NMC_E_UNSUPPORTED, "solve_batch_v: kernel_store must be NMC_KERNELS_ON_CHIP or NMC_KERNELS_PAIRED (two "
                "points per wavefront) or NMC_KERNELS_WAVE (one point per wavefront)");
  if (L.persistent && (!ws || !aligned256(ws) || ws_bytes < kCounterBytes))
    return fail(NMC_E_WORKSPACE, "solve_batch_v: persistent launch needs a 256-byte aligned workspace");
  nmc::FwdVArgs a;
  memset(&a, 0, sizeof(a));
  a.mdl = m->dev;
  a.prm.tol_inner = prm->tol_inner;
  a.prm.tol_outer = prm->tol_outer;
  a.prm.m_inner = prm->m_inner;
  a.prm.m_outer = prm->m_outer;
  a.prm.max_inner = prm->max_inner;
  a.prm.max_outer = prm->max_outer;
  a.prm.fixed_matter = prm->fixed_matter ? 1 : 0;
  a.tol_inner2 = prm->tol_inner * prm->tol_inner;
  a.P = P;
  a.dtau = dtau;
  a.D0 = in->D0;
  a.I0 = in->I0;
  a.rho11 = in->rho11;
  a.ye0 = in->ye0;
  a.ef0 = in->ef0;
  a.v0 = in->v0;
  a.chi0 = in->chi0;
  a.theta = in->theta;
  a.D = out->D;
  a.I = out->I;
  a.ye = out->ye;
  a.ef = out->ef;
  a.v = out->v;
  a.T = out->T;
  a.n_outer = out->n_outer;
  a.n_inner = out->n_inner;
  a.status = out->status;
  a.chunk = L.chunk;
  hipStream_t s = (hipStream_t)stream;
  if (L.persistent) {
    a.queue = (int*)ws;
    hipError_t e = nmc::launch_reset_counter(a.queue, s);
    if (e != hipSuccess) return hip_fail(e, "solve_batch_v: counter reset");
  }
  const bool coupled = (m->host.flags & (NMC_NES | NMC_PAIR)) != 0;
  const bool phi1 = coupled && (m->host.phi1_nes != 0.0 || m->host.phi1_pair != 0.0);
  // two points per wavefront unless the one-point kernel is asked for; both
  // carry the linear-order corrections
  const bool one_point = L.kernel_store == NMC_KERNELS_WAVE;
  hipError_t e = one_point ? nmc::launch_forward_v(a, m->host.ns, coupled, phi1, L, m->num_cu, s)
                           : nmc::launch_forward_vpair(a, m->host.ns, coupled, phi1, L, m->num_cu, s);
  if (e == hipErrorInvalidValue) return fail(NMC_E_UNSUPPORTED, "solve_batch_v: no kernel for ns=%d", m->host.ns);
  if (e != hipSuccess) return hip_fail(e, "solve_batch_v: launch");
  return NMC_OK;
}

void nmc_c2p_params_default(nmc_c2p_params* cp) {
  if (!cp) return;
  cp->mem = 3;
  cp->tol = 1e-8;
  cp->max_it = 100;
}

static int check_c2p(const nmc_c2p_params* cp, const char* who) {
  if (!cp) return fail(NMC_E_INVALID_ARG, "%s: null recovery parameters", who);
  if (cp->mem < 1 || cp->mem > 3) return fail(NMC_E_UNSUPPORTED, "%s: recovery memory must be 1..3", who);
  if (!(cp->tol > 0.0) || !isfinite(cp->tol) || cp->max_it < 1 || cp->max_it > 100000)
    return fail(NMC_E_INVALID_ARG, "%s: recovery tolerance must be positive, cap in 1..100000", who);
  return NMC_OK;
}

int nmc_primitive_recovery(const nmc_model* m, const nmc_c2p_params* cp, int64_t P, const double* N, const double* G,
                           const double* v, double* D, double* I, int32_t* iters, void* stream) {
  if (!m) return fail(NMC_E_INVALID_ARG, "primitive_recovery: null model");
  int rc = check_c2p(cp, "primitive_recovery");
  if (rc) return rc;
  if (P < 0 || P > (int64_t(1) << 30)) return fail(NMC_E_INVALID_ARG, "primitive_recovery: P out of range");
  if (P == 0) return NMC_OK;
  if (!N || !G || !v || !D || !I || !iters) return fail(NMC_E_INVALID_ARG, "primitive_recovery: null array");
  hipError_t e = nmc::launch_c2p(P, m->host.ns, m->host.nq, N, G, v, cp->mem, cp->tol, cp->max_it, D, I, iters,
                                 m->num_cu, (hipStream_t)stream);
  return e == hipSuccess ? NMC_OK : hip_fail(e, "primitive_recovery: launch");
}

namespace {
// PD-ARS tableau of the implicit part (Eq. butcherPDARS): a_22 = 1, a_32 = a_33 = 1/2
constexpr double kA22 = 1.0, kA32 = 0.5, kA33 = 0.5;

// workspace of a PD-ARS step: the solve's own, then the stage-2 solution and
// the stage-3 initial state
struct PdarsWs {
  char* solve;
  double *D2, *I2, *ye2, *ef2, *T2, *v2;
  int32_t *no2, *ni2, *st2;
  double *D3, *I3, *ye3, *ef3, *v3;
  int32_t* iters;
  size_t total;
};

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

PdarsWs pdars_layout(const nmc_model* m, int64_t P, char* base) {
  PdarsWs w;
  const size_t nn = (size_t)m->host.ns * m->host.nq, pp = (size_t)P;
  size_t off = al256(nmc_workspace_bytes(m, P));
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += al256(bytes);
    return p;
  };
  w.solve = base;
  w.D2 = (double*)take(pp * nn * 8);
  w.I2 = (double*)take(pp * 3 * nn * 8);
  w.ye2 = (double*)take(pp * 8);
  w.ef2 = (double*)take(pp * 8);
  w.T2 = (double*)take(pp * 8);
  w.v2 = (double*)take(pp * 3 * 8);
  w.no2 = (int32_t*)take(pp * 4);
  w.ni2 = (int32_t*)take(pp * 4);
  w.st2 = (int32_t*)take(pp * 4);
  w.D3 = (double*)take(pp * nn * 8);
  w.I3 = (double*)take(pp * 3 * nn * 8);
  w.ye3 = (double*)take(pp * 8);
  w.ef3 = (double*)take(pp * 8);
  w.v3 = (double*)take(pp * 3 * 8);
  w.iters = (int32_t*)take(pp * nn * 4);
  w.total = off;
  return w;
}
}  // namespace

size_t nmc_pdars_workspace_bytes(const nmc_model* m, int64_t P) {
  if (!m || P < 0) return 0;
  return pdars_layout(m, P, nullptr).total;
}

int nmc_pdars_step_v(const nmc_model* m, const nmc_solver_params* prm, const nmc_c2p_params* cp, int64_t P,
                     double dt, const nmc_batch_v_in* in, const nmc_batch_v_out* out, void* ws, size_t ws_bytes,
                     const nmc_launch* launch, void* stream) {
  if (!m || !in || !out) return fail(NMC_E_INVALID_ARG, "pdars_step_v: null handle or descriptor");
  if (m->host.fd_projection)
    return fail(NMC_E_UNSUPPORTED, "pdars_step_v: the projected equilibrium is implemented in nmc_solve_batch only");
  int rc = check_c2p(cp, "pdars_step_v");
  if (rc) return rc;
  if (!(dt > 0.0) || !isfinite(dt)) return fail(NMC_E_INVALID_ARG, "pdars_step_v: dt must be positive");
  if (P < 0 || P > (int64_t(1) << 30)) return fail(NMC_E_INVALID_ARG, "pdars_step_v: P out of range");
  if (P == 0) return NMC_OK;
  if (!ws || !aligned256(ws) || ws_bytes < nmc_pdars_workspace_bytes(m, P))
    return fail(NMC_E_WORKSPACE, "pdars_step_v: workspace must be 256-byte aligned and at least "
                                 "nmc_pdars_workspace_bytes");
  if (!in->D0 || !in->I0 || !in->rho11 || !in->ye0 || !in->ef0 || !in->v0 || !in->theta)
    return fail(NMC_E_INVALID_ARG, "pdars_step_v: null input array");
  const PdarsWs w = pdars_layout(m, P, (char*)ws);
  hipStream_t s = (hipStream_t)stream;
  // stage 2: U^(2*) = U^n (a_21 = 0, no explicit operator), step a_22 dt
  nmc_batch_v_out o2 = {w.D2, w.I2, w.ye2, w.ef2, w.v2, w.T2, w.no2, w.ni2, w.st2};
  rc = nmc_solve_batch_v(m, prm, P, kA22 * dt, in, &o2, w.solve, nmc_workspace_bytes(m, P), launch, stream);
  if (rc) return rc;
  // stage 3: U^(3*) = U^n + dt a_32 C^(2) = U^n + (a_32 / a_22)(U^(2) - U^n), recovered to primitive moments
  nmc::PdarsArgs a;
  memset(&a, 0, sizeof(a));
  a.P = P;
  a.ns = m->host.ns;
  a.nq = m->host.nq;
  a.w = kA32 / kA22;
  a.rho11_min = m->host.rho11_min;
  a.rho11 = in->rho11;
  a.D0 = in->D0;
  a.I0 = in->I0;
  a.ye0 = in->ye0;
  a.ef0 = in->ef0;
  a.v0 = in->v0;
  a.D2 = w.D2;
  a.I2 = w.I2;
  a.ye2 = w.ye2;
  a.ef2 = w.ef2;
  a.v2 = w.v2;
  a.D3 = w.D3;
  a.I3 = w.I3;
  a.ye3 = w.ye3;
  a.ef3 = w.ef3;
  a.v3 = w.v3;
  a.iters = w.iters;
  a.mem = cp->mem;
  a.max_it = cp->max_it;
  a.tol2 = cp->tol * cp->tol;
  hipError_t e = nmc::launch_pdars_stage3(a, m->num_cu, s);
  if (e != hipSuccess) return hip_fail(e, "pdars_step_v: stage-3 input");
  nmc_batch_v_in i3 = {w.D3, w.I3, in->rho11, w.ye3, w.ef3, w.v3, in->chi0, in->theta};
  rc = nmc_solve_batch_v(m, prm, P, kA33 * dt, &i3, out, w.solve, nmc_workspace_bytes(m, P), launch, stream);
  if (rc) return rc;
  // globally stiffly accurate: the step's result is the stage-3 solution
  e = nmc::launch_pdars_merge(P, m->host.ns * m->host.nq, w.no2, w.ni2, w.st2, w.iters, out->n_outer, out->n_inner,
                              out->status, m->num_cu, s);
  return e == hipSuccess ? NMC_OK : hip_fail(e, "pdars_step_v: merge");
}

int nmc_solve_batch_adjoint(const nmc_model* m, const nmc_solver_params* prm, int64_t P, double dtau,
                            const nmc_batch_in* in, const nmc_batch_out* fwd, const double* gbar,
                            double* grad_theta, double* grad_pp, void* ws, size_t ws_bytes, void* stream) {
  if (!m || !in || !fwd) return fail(NMC_E_INVALID_ARG, "adjoint: null model, inputs or forward outputs");
  if (prm && prm->fixed_matter)
    return fail(NMC_E_UNSUPPORTED, "adjoint: the forward solve held the matter fixed; the adjoint differentiates "
                                   "the coupled system");
  if (P < 0 || P > (int64_t(1) << 30)) return fail(NMC_E_INVALID_ARG, "adjoint: P out of range");
  if (!(dtau > 0.0) || !isfinite(dtau)) return fail(NMC_E_INVALID_ARG, "adjoint: dtau must be positive and finite");
  if (!grad_theta) return fail(NMC_E_INVALID_ARG, "adjoint: null grad_theta");
  if (m->host.nq != 32) return fail(NMC_E_UNSUPPORTED, "adjoint: implemented for 32 energy nodes (model has %d)", m->host.nq);
  if (m->host.fd_projection)
    return fail(NMC_E_UNSUPPORTED, "adjoint: its Jacobian is written for the pointwise equilibrium");
  if (P == 0) return NMC_OK;
  if (!in->rho11 || !in->theta || !fwd->D || !fwd->ye || !fwd->e || !fwd->status || !fwd->n_outer || !gbar)
    return fail(NMC_E_INVALID_ARG, "adjoint: null array");
  if (!ws || !aligned256(ws) || ws_bytes < nmc_workspace_bytes(m, P))
    return fail(NMC_E_WORKSPACE, "adjoint: workspace must be 256-byte aligned and at least nmc_workspace_bytes");
  const int nt = m->host.nq + 2;
  const size_t pp = ((size_t)P * nt * sizeof(double) + 255) & ~(size_t)255;
  char* w = (char*)ws + kCounterBytes;
  nmc::AdjArgs a;
  memset(&a, 0, sizeof(a));
  a.mdl = m->dev;
  a.P = P;
  a.dtau = dtau;
  a.rho11 = in->rho11;
  a.chi0 = in->chi0;
  a.theta = in->theta;
  a.D = fwd->D;
  a.ye = fwd->ye;
  a.e = fwd->e;
  a.status = fwd->status;
  a.n_outer = fwd->n_outer;
  a.gbar = gbar;
  a.grad_pp = grad_pp ? grad_pp : (double*)w;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = nmc::launch_adjoint(a, m->host.nq, m->host.ns, m->num_cu, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint: launch");
  e = nmc::launch_reduce_columns(a.grad_pp, P, nt, (double*)(w + pp), grad_theta, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint: reduction");
  return NMC_OK;
}

int nmc_init_state(const nmc_model* m, int64_t P, const double* T, const double* mu, const double* rho11,
                   const double* ye, const double* uD, const double* uI, double a, double b, double c, double* D0,
                   double* I0, double* e0, void* stream) {
  if (!m) return fail(NMC_E_INVALID_ARG, "init_state: null model");
  if (P < 0 || P > (int64_t(1) << 30)) return fail(NMC_E_INVALID_ARG, "init_state: P out of range");
  if (P == 0) return NMC_OK;
  if (!T || !rho11 || !ye || !uD || !uI || !D0 || !I0) return fail(NMC_E_INVALID_ARG, "init_state: null array");
  if (!isfinite(a) || !isfinite(b) || !isfinite(c)) return fail(NMC_E_INVALID_ARG, "init_state: non-finite coefficient");
  hipError_t e = nmc::launch_init_state(m->dev, m->host.ns, m->host.nq, P, T, mu, rho11, ye, uD, uI, a, b, c, D0, I0,
                                        e0, (hipStream_t)stream);
  return e == hipSuccess ? NMC_OK : hip_fail(e, "init_state: launch");
}

}  // extern "C"

// ---------------------------------------------------------------------------
namespace nmc {
namespace {

// one thread per (point, species, node)
__global__ void init_state_kernel(const DevModel* __restrict__ md, int ns, int nq, int64_t P,
                                  const double* __restrict__ T, const double* __restrict__ mu,
                                  const double* __restrict__ rho11, const double* __restrict__ ye,
                                  const double* __restrict__ uD, const double* __restrict__ uI, double a, double b,
                                  double c, double* __restrict__ D0, double* __restrict__ I0, double* __restrict__ e0) {
  const int64_t n = P * ns * nq;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = i / (ns * nq);
    const int s = (int)((i / nq) % ns);
    const int q = (int)(i % nq);
    const double r3 = cbrt(rho11[p]);
    const double Tp = T[p];
    const double mup = mu ? mu[p] : md->mu_a * (ye[p] - md->mu_ye0) * r3 + md->mu_b * log(Tp / md->mu_t0);
    const double x = (md->eps[q] - md->musign[s] * mup) / Tp;
    const double ex = exp(-fabs(x));
    const double f = x > 0.0 ? ex / (1.0 + ex) : 1.0 / (1.0 + ex);
    double d = f * (a + b * uD[i]);
    d = d < 0.0 ? 0.0 : d;
    d = d > 1.0 - 1e-12 ? 1.0 - 1e-12 : d;
    D0[i] = d;
    I0[i] = c * d * uI[i];
    if (e0 && s == 0 && q == 0) e0[p] = md->eos_a * Tp * (1.0 + ye[p]) + md->eos_b * pow(ye[p], 4.0 / 3.0) * r3;
  }
}

}  // namespace

hipError_t launch_init_state(const DevModel* mdl, int ns, int nq, int64_t P, const double* T, const double* mu,
                             const double* rho11, const double* ye, const double* uD, const double* uI, double a,
                             double b, double c, double* D0, double* I0, double* e0, hipStream_t s) {
  const int64_t n = P * ns * nq;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(init_state_kernel, dim3((unsigned)blocks), dim3(256), 0, s, mdl, ns, nq, P, T, mu, rho11, ye,
                     uD, uI, a, b, c, D0, I0, e0);
  return hipGetLastError();
}

}  // namespace nmc
