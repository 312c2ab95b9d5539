// Host side of the C ABI declared in include/pic.h: validation, layout of the
// caller's device workspace, FP64 constants of the method, and the order of
// kernel launches of one step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pic.h"
#include "device.hpp"

namespace picmcc {
hipError_t launch_push(const Sim &S, int s, int64_t step, int grid, int block, hipStream_t st);
hipError_t launch_field(const Sim &S, int64_t step, int mode, hipStream_t st);
hipError_t launch_fixup(const Sim &S, hipStream_t st);
hipError_t launch_ionprep(const Sim &S, hipStream_t st);
hipError_t launch_pair(const Sim &S, int64_t step, int stage, int sp, int grid, hipStream_t st);
hipError_t launch_eiprep(const Sim &S, hipStream_t st);
hipError_t launch_meta_init(const Sim &S, int tab, hipStream_t st);
hipError_t launch_meta_solve(const Sim &S, double weight, double tau, double D, double nu_q, double h, hipStream_t st);
hipError_t launch_eion(const Sim &S, int64_t step, int grid, hipStream_t st);
hipError_t launch_sort(const Sim &S, int s, const Particles &dst, int grid, hipStream_t st);
hipError_t launch_reduce_field(const Sim &S, int push_grid, int64_t next_step, hipStream_t st);
hipError_t launch_diag(const Sim &S, int s, int grid, hipStream_t st);
hipError_t launch_load(const Sim &S, int s, int64_t count, float vth, int grid, hipStream_t st);
hipError_t launch_shift(const Sim &S, int s, int grid, hipStream_t st);
hipError_t launch_load_profile(const Sim &S, int s, int64_t count, const long long *cum, const float *vth, int grid,
                               hipStream_t st);
hipError_t launch_deposit(const Sim &S, int s, int grid, hipStream_t st);
hipError_t set_lds_limits(const Sim &S, int block);
hipError_t launch_reduce(const Sim &S, int s, int push_grid, hipStream_t st);
hipError_t launch_compact(const Sim &S, int s, const Particles &dst, int grid, hipStream_t st);
int max_push_grid();
size_t max_push_lds(const Sim &S, int block);
size_t push_lds_bytes(const Sim &S, int s, int bs);
size_t diag_lds_bytes(const Sim &S);
hipError_t batch_push_occupancy(int block, int s, size_t lds, int *per_cu);
hipError_t launch_field_b(const BatchLaunch &B, int rel, hipStream_t st);
hipError_t launch_push_b(const BatchLaunch &B, int s, uint64_t mask, int rel, hipStream_t st);
hipError_t launch_reduce_b(const BatchLaunch &B, int s, uint64_t mask, hipStream_t st);
hipError_t launch_ionprep_b(const BatchLaunch &B, uint64_t mask, hipStream_t st);
hipError_t launch_pair_b(const BatchLaunch &B, uint64_t mask, int rel, int stage, int sp, hipStream_t st);
hipError_t launch_eiprep_b(const BatchLaunch &B, uint64_t mask, hipStream_t st);
hipError_t launch_eion_b(const BatchLaunch &B, uint64_t mask, int rel, hipStream_t st);
hipError_t launch_diag_b(const BatchLaunch &B, uint64_t mask, hipStream_t st);
hipError_t launch_compact_b(const BatchLaunch &B, uint64_t mask, hipStream_t st);
hipError_t launch_advance_b(const BatchLaunch &B, int64_t add, hipStream_t st);
}  // namespace picmcc

using namespace picmcc;

namespace {

// SI constants (CODATA 2018; e and k_B exact)
constexpr double QE = 1.602176634e-19;
constexpr double KB = 1.380649e-23;
constexpr double EPS0 = 8.8541878128e-12;
constexpr int MAX_NG = 8192;

struct Layout {
  size_t total = 0;
  size_t part[NSP][2][6];   // two buffers x (w, off, vx, vy, vz, id)
  size_t pkey[NSP], pbkt[NSP], ptmp[NSP], bcnt;
  size_t Q, E, phi, sumQ, sumphi, esum, ecnt, edf, iedf, nacc, kleft, pcell, phist, sortcnt, sortbase, sortoff, sc, sigma,
      hbound, events, partials, ttot, blkcnt, prof, jsum, jcnt, jpow, kleft_neg, dens_ei, meta_src, na, na_f,
      meta_tmp, bal;
  size_t take(size_t bytes) {
    const size_t o = total;
    total += (bytes + 255) & ~(size_t)255;
    return o;
  }
};

Layout make_layout(const pic_config &c, const pic_species *sp, int nproc) {
  Layout L;
  for (int s = 0; s < NSP; ++s) {
    const size_t slots = ((size_t)sp[s].capacity + 255) & ~(size_t)255;   // whole 8-particle groups
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 6; ++a) L.part[s][b][a] = L.take(4 * slots);
    L.pkey[s] = L.take(8 * (size_t)c.max_products);
    L.pbkt[s] = L.take(4 * (size_t)c.max_products);
    L.ptmp[s] = L.take(8 * (size_t)c.max_products);
  }
  L.bcnt = L.take(4 * (size_t)NSP * NBKT);
  const size_t nn = c.ng + 1;
  L.Q = L.take(8 * NSP * nn);
  L.E = L.take(4 * nn);
  L.phi = L.take(8 * nn);
  L.sumQ = L.take(8 * NSP * nn);
  L.sumphi = L.take(8 * nn);
  L.esum = L.take(8 * NSP * (size_t)c.ng);
  L.ecnt = L.take(8 * NSP * (size_t)c.ng);
  L.edf = L.take(8 * NSP * NBIN);
  L.iedf = L.take(8 * NSP * 2 * NBIN);
  L.nacc = L.take(16);
  L.kleft = L.take(4 * (size_t)c.ng);
  L.pcell = L.take(sizeof(PairCell) * (size_t)c.ng);
  L.phist = L.take(4 * (size_t)256 * c.ng);
  L.sortcnt = L.take(4 * (size_t)c.ng);
  L.sortbase = L.take(4 * (size_t)c.ng);
  L.sortoff = L.take(4 * (size_t)SORT_GRID * c.ng);
  L.sc = L.take(sizeof(Scalars));
  L.sigma = L.take(4 * (size_t)nproc * c.table_n);
  L.hbound = L.take(8 * (size_t)nproc * (c.table_n - 1));
  L.events = L.take(32 * (size_t)c.event_capacity);
  L.partials = L.take(8 * nn * (size_t)(c.grid > 0 ? c.grid : max_push_grid()));
  L.bal = L.take(sizeof(PushBal));
  L.ttot = L.take(4 * (size_t)c.table_n);
  L.blkcnt = L.take(8 * 4096);
  L.prof = L.take((8 + 4) * NSP * (size_t)c.ng);   // warm-start loading: per-cell cumulative counts, speeds
  L.jsum = L.take(8 * (size_t)c.steps_per_cycle);   // current density per rf phase
  L.jcnt = L.take(8 * (size_t)c.steps_per_cycle);
  L.jpow = L.take(16);
  L.kleft_neg = L.take(4 * (size_t)c.ng);          // O- partners of electron-impact detachment
  L.dens_ei = L.take(4 * 2 * nn);                   // ion node densities for the electron-ion test
  L.meta_src = L.take(8 * nn);                      // O2(a) field: production tally, density, solver work
  L.na = L.take(8 * nn);
  L.na_f = L.take(4 * nn);
  L.meta_tmp = L.take(8 * nn);
  return L;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

std::string g_query_error;

int validate(const pic_config *c, const pic_species *sp, const pic_process *pr, int nproc, std::string &msg) {
  if (!c || !sp || (nproc > 0 && !pr)) { msg = "null argument"; return PIC_EINVAL; }
  if (!finite_pos(c->L)) { msg = "L must be > 0"; return PIC_EINVAL; }
  if (c->ng < 2 || c->ng > MAX_NG) { msg = "ng must be in [2, 8192]"; return PIC_EINVAL; }
  if (!std::isfinite(c->U) || !finite_pos(c->f)) { msg = "U finite and f > 0 required"; return PIC_EINVAL; }
  if (!(std::isfinite(c->p) && c->p >= 0.0) || !finite_pos(c->t_gas)) { msg = "p >= 0 and t_gas > 0 required"; return PIC_EINVAL; }
  if (c->steps_per_cycle < 1 || c->ksub < 1) { msg = "steps_per_cycle and ksub must be >= 1"; return PIC_EINVAL; }
  if (!(std::isfinite(c->c_meta) && c->c_meta >= 0.0)) { msg = "c_meta must be >= 0"; return PIC_EINVAL; }
  if (!finite_pos(c->weight)) { msg = "weight must be > 0"; return PIC_EINVAL; }
  if (c->diag_every < 0 || c->sort_every < 0) { msg = "diag_every and sort_every must be >= 0"; return PIC_EINVAL; }
  if (c->sort_kind != PIC_SORT_CELL && c->sort_kind != PIC_SORT_COMPACT) { msg = "sort_kind must be PIC_SORT_CELL or PIC_SORT_COMPACT"; return PIC_EINVAL; }
  if (!finite_pos(c->table_emin) || !(c->table_emax > c->table_emin) || !std::isfinite(c->table_emax)) {
    msg = "table range must satisfy 0 < emin < emax"; return PIC_EINVAL;
  }
  if (c->table_n < 2 || c->table_n > 4096) { msg = "table_n must be in [2, 4096]"; return PIC_EINVAL; }
  if (c->max_products < 1 || c->max_products > MAXPROD) { msg = "max_products must be in [1, 2^24]"; return PIC_EINVAL; }
  if (c->event_capacity < 0) { msg = "event_capacity must be >= 0"; return PIC_EINVAL; }
  if (!(c->block == 0 || c->block == 256 || c->block == 512 || c->block == 1024)) {
    msg = "block must be 0, 256, 512 or 1024"; return PIC_EINVAL;
  }
  if (c->grid < 0 || c->grid > max_push_grid()) { msg = "grid must be in [0, 2048]"; return PIC_EINVAL; }
  if (!std::isfinite(c->e_ext0) || !std::isfinite(c->e_ext1)) { msg = "external field must be finite"; return PIC_EINVAL; }
  const double want_q[NSP] = {-1.0, 1.0, -1.0};
  for (int s = 0; s < NSP; ++s) {
    if (sp[s].charge != want_q[s]) { msg = "species charges must be -1 (e), +1 (O2+), -1 (O-)"; return PIC_EINVAL; }
    if (!finite_pos(sp[s].mass) || !(std::isfinite(sp[s].t0_ev) && sp[s].t0_ev >= 0.0)) {
      msg = "species mass > 0 and t0_ev >= 0 required"; return PIC_EINVAL;
    }
    if (sp[s].count < 0 || sp[s].capacity < 1 || sp[s].count > sp[s].capacity || sp[s].capacity > 0x7FFFFFFFLL) {
      msg = "species need 0 <= count <= capacity < 2^31"; return PIC_EINVAL;
    }
  }
  if (nproc < 0 || nproc > MAXPROC) { msg = "at most 16 processes"; return PIC_EINVAL; }
  int per[NSP] = {0, 0, 0};
  for (int p = 0; p < nproc; ++p) {
    const pic_process &P = pr[p];
    if (P.species < 0 || P.species >= NSP) { msg = "process species out of range"; return PIC_EINVAL; }
    const bool ok = (P.species == 0 && ((P.kind >= PIC_ELASTIC && P.kind <= PIC_ATTACH) ||
                                        P.kind == PIC_RECOMB || P.kind == PIC_EDETACH)) ||
                    (P.species == 1 && (P.kind == PIC_CX || P.kind == PIC_ION_ELASTIC)) ||
                    (P.species == 2 && (P.kind == PIC_NEUTRALIZE || P.kind == PIC_DETACH || P.kind == PIC_ION_ELASTIC));
    if (!ok) { msg = "process kind not valid for its species"; return PIC_EINVAL; }
    const bool gridpos = P.kind == PIC_NEUTRALIZE || P.kind == PIC_RECOMB, gridneg = P.kind == PIC_EDETACH;
    if (P.target < PIC_T_O2 || P.target > PIC_T_GRIDNEG || ((P.target == PIC_T_GRIDPOS) != gridpos) ||
        ((P.target == PIC_T_GRIDNEG) != gridneg)) {
      msg = "process target invalid (grid densities: O2+ for neutralisation and recombination, O- for "
            "electron-impact detachment, and only there)";
      return PIC_EINVAL;
    }
    if (!(std::isfinite(P.e_th) && P.e_th >= 0.0) || !finite_pos(P.target_mass) || !P.sigma) {
      msg = "process needs e_th >= 0, target_mass > 0 and a table"; return PIC_EINVAL;
    }
    for (int k = 0; k < c->table_n; ++k)
      if (!(std::isfinite(P.sigma[k]) && P.sigma[k] >= 0.0)) { msg = "cross sections must be finite and >= 0"; return PIC_EINVAL; }
    if (++per[P.species] > MAXPROC_SP) { msg = "at most 12 processes per species"; return PIC_EINVAL; }
  }
  return PIC_OK;
}

}  // namespace

struct pic_handle {
  pic_config cfg;
  pic_species sp[NSP];
  std::vector<pic_process> pr;
  std::vector<std::vector<double>> sig;
  Layout L;
  unsigned char *ws = nullptr;
  hipStream_t stream = nullptr;
  Sim S;
  Particles buf[NSP][2];
  int cur[NSP] = {0, 0, 0};
  int64_t step = 0;
  double numax[NSP] = {0, 0, 0};
  int block = 512, grid[NSP] = {1, 1, 1}, hgrid = 1, pgrid = 1;
  int ncu = 1;
  bool batch_busy = false;         // stepped by a batch that has not been synchronised
  bool field_ready = false;        // the field of `step` was solved by the previous step's reduction
  std::string err;
  // spatially resolved O2(a): configuration and the step its tally window began
  bool meta_on = false;
  pic_metastable meta{};
  double meta_h = 0.0;
  int64_t meta_step0 = 0;
};

namespace {

int fail(pic_handle *h, int code, const std::string &m) {
  if (h) h->err = m;
  return code;
}

int hipfail(pic_handle *h, hipError_t e, const char *where) {
  return fail(h, PIC_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(h, expr)                                        \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) return hipfail((h), e_, #expr);      \
  } while (0)

Particles carve(unsigned char *ws, const size_t *o) {
  Particles P;
  P.w = (int32_t *)(ws + o[0]);
  P.off = (float *)(ws + o[1]);
  P.vx = (float *)(ws + o[2]);
  P.vy = (float *)(ws + o[3]);
  P.vz = (float *)(ws + o[4]);
  P.id = (uint32_t *)(ws + o[5]);
  return P;
}

double reduced_mass(const pic_handle *h, const pic_process &P) {
  const double m = h->sp[P.species].mass;
  if (P.species == 0) return m;                 // electrons: lab energy, target at rest
  return m * P.target_mass / (m + P.target_mass);
}

double target_n(const pic_handle *h, const pic_process &P, double n_o2) {
  return P.target == PIC_T_O2 ? n_o2 : (P.target == PIC_T_O2A ? h->cfg.c_meta * n_o2 : 0.0);
}

// max over table intervals of sum_p n_p max(sigma_k, sigma_k+1) g(E_k+1)
double nu_bound(const pic_handle *h, int s, double n_o2) {
  const pic_config &c = h->cfg;
  double best = 0.0;
  for (int k = 0; k + 1 < c.table_n; ++k) {
    const double ek1 = c.table_emin * std::pow(c.table_emax / c.table_emin, (double)(k + 1) / (double)(c.table_n - 1));
    double sum = 0.0;
    for (size_t p = 0; p < h->pr.size(); ++p) {
      const pic_process &P = h->pr[p];
      if (P.species != s) continue;
      const double sm = std::fmax(h->sig[p][k], h->sig[p][k + 1]);
      sum += target_n(h, P, n_o2) * sm * std::sqrt(2.0 * ek1 * QE / reduced_mass(h, P));
    }
    if (sum > best) best = sum;
  }
  return best;
}

Scalars read_scalars(pic_handle *h, hipError_t *e) {
  Scalars sc;
  *e = hipMemcpyAsync(&sc, h->ws + h->L.sc, sizeof(Scalars), hipMemcpyDeviceToHost, h->stream);
  if (*e == hipSuccess) *e = hipStreamSynchronize(h->stream);
  return sc;
}

int device_errors(pic_handle *h, const Scalars &sc) {
  if (sc.err & E_CAPACITY) return fail(h, PIC_ECAPACITY, "particle storage or per-step product buffer full");
  if (sc.err & E_IDOVERFLOW) return fail(h, PIC_EIDOVERFLOW, "32-bit particle ids exhausted");
  if (sc.err & E_NAN) return fail(h, PIC_ENAN, "non-finite particle position");
  return PIC_OK;
}

int set_scalar(pic_handle *h, size_t field_off, const void *v, size_t n) {
  HIPCHK(h, hipMemcpyAsync(h->ws + h->L.sc + field_off, v, n, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PIC_OK;
}

}  // namespace

extern "C" {

int32_t pic_version(void) { return 10000; }

const char *pic_strerror(int code) {
  switch (code) {
    case PIC_OK: return "ok";
    case PIC_EINVAL: return "invalid argument";
    case PIC_ECAPACITY: return "capacity exceeded";
    case PIC_EIDOVERFLOW: return "particle id overflow";
    case PIC_ENAN: return "non-finite particle state";
    case PIC_EHIP: return "HIP runtime error";
    case PIC_ENODEVICE: return "no gfx950 device";
    case PIC_EBUSY: return "handle busy in a batch";
    default: return "unknown error";
  }
}

const char *pic_last_error(const pic_handle *h) { return h ? h->err.c_str() : g_query_error.c_str(); }

int pic_query(const pic_config *cfg, const pic_species *sp, const pic_process *pr, int32_t nproc,
              uint64_t *workspace_bytes) {
  std::string msg;
  const int r = validate(cfg, sp, pr, nproc, msg);
  if (r != PIC_OK) { g_query_error = msg; return r; }
  if (!workspace_bytes) { g_query_error = "null workspace_bytes"; return PIC_EINVAL; }
  *workspace_bytes = make_layout(*cfg, sp, nproc).total;
  return PIC_OK;
}

int pic_create(const pic_config *cfg, const pic_species *sp, const pic_process *pr, int32_t nproc, void *workspace,
               uint64_t workspace_bytes, void *stream, pic_handle **out) {
  std::string msg;
  int r = validate(cfg, sp, pr, nproc, msg);
  if (r != PIC_OK) { g_query_error = msg; return r; }
  if (!out || !workspace) { g_query_error = "null workspace or handle pointer"; return PIC_EINVAL; }
  const Layout L = make_layout(*cfg, sp, nproc);
  if (workspace_bytes < L.total) { g_query_error = "workspace smaller than pic_query reported"; return PIC_EINVAL; }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    g_query_error = "no HIP device";
    return PIC_ENODEVICE;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    g_query_error = std::string("device is ") + prop.gcnArchName + ", the kernels are built for gfx950";
    return PIC_ENODEVICE;
  }
  pic_handle *h = new pic_handle();
  h->cfg = *cfg;
  std::memcpy(h->sp, sp, sizeof(h->sp));
  h->pr.assign(pr, pr + nproc);
  h->sig.resize(nproc);
  for (int p = 0; p < nproc; ++p) {
    h->sig[p].assign(pr[p].sigma, pr[p].sigma + cfg->table_n);
    h->pr[p].sigma = h->sig[p].data();
  }
  h->L = L;
  h->ws = (unsigned char *)workspace;
  h->stream = (hipStream_t)stream;
  h->ncu = prop.multiProcessorCount;
  h->block = cfg->block ? cfg->block : 512;

  const pic_config &c = h->cfg;
  Sim &S = h->S;
  std::memset(&S, 0, sizeof(S));
  const double dx = c.L / c.ng, dt = 1.0 / (c.f * c.steps_per_cycle), dti = dt * c.ksub;
  const double n_o2 = c.p / (KB * c.t_gas);        // section 2: O2 reservoir n = p / kT
  S.ng = c.ng; S.dx = dx; S.dt = dt; S.L = c.L; S.U = c.U; S.f = c.f;
  S.eps0 = EPS0; S.qcharge = QE * c.weight / 4294967296.0;
  S.e_ext0 = c.e_ext0; S.e_ext1 = c.e_ext1; S.flags = c.flags; S.ksub = c.ksub; S.seed = c.seed;
  S.max_products = c.max_products; S.n_o2 = n_o2; S.c_meta = c.c_meta; S.dti = dti;
  S.wd = c.weight / 4294967296.0 / dx;
  S.nplus_c = (float)S.wd;
  S.event_cap = c.event_capacity;
  S.ntab = c.table_n;
  S.lnemin = (float)std::log(c.table_emin);
  S.invdlt = (float)((double)(c.table_n - 1) / (std::log(c.table_emax) - std::log(c.table_emin)));
  {
    const double inv2 = (double)(c.table_n - 1) / (std::log2(c.table_emax) - std::log2(c.table_emin));
    S.invdlt2 = (float)inv2;
    S.l2emin_s = (float)(std::log2(c.table_emin) * inv2);
  }
  S.emin = (float)c.table_emin;
  S.emax = (float)c.table_emax;
  for (int s = 0; s < NSP; ++s) {
    const double dts = s == 0 ? dt : dti;
    const double m = sp[s].mass;
    S.cap[s] = sp[s].capacity;
    S.charge[s] = (int)sp[s].charge;
    S.qmdt[s] = (float)(sp[s].charge * QE / m * dts);
    S.dtdx[s] = (float)(dts / dx);
    S.half_m_e[s] = (float)(0.5 * m / QE);
    S.two_e_m[s] = (float)(2.0 * QE / m);
    S.mass[s] = m;
    S.vt_gas[s] = (float)std::sqrt(KB * c.t_gas / m);
    for (int b = 0; b < 2; ++b) h->buf[s][b] = carve(h->ws, L.part[s][b]);
    S.p[s] = h->buf[s][0];
    S.alt[s] = h->buf[s][1];
    S.pkey[s] = (uint64_t *)(h->ws + L.pkey[s]);
    S.pbkt[s] = (int32_t *)(h->ws + L.pbkt[s]);
    S.ptmp[s] = (uint64_t *)(h->ws + L.ptmp[s]);
  }
  // collision-frequency bounds of the null-collision method
  h->numax[0] = nu_bound(h, 0, n_o2);
  h->numax[1] = nu_bound(h, 1, n_o2);
  S.nd_e = h->numax[0] * dt;
  S.inv_nd_ef = S.nd_e > 0.0 ? (float)(1.0 / S.nd_e) : 0.0f;
  S.pnull_pos = 1.0 - std::exp(-h->numax[1] * dti);
  // electrons: the channels with neutral targets first (free flights, push), then
  // the electron-ion channels (the ion-step test)
  int order[MAXPROC], no = 0;
  for (int pass = 0; pass < 2; ++pass)
    for (int p = 0; p < nproc; ++p)
      if ((h->pr[p].kind == PIC_RECOMB || h->pr[p].kind == PIC_EDETACH) == (pass == 1)) order[no++] = p;
  for (int q = 0; q < nproc; ++q) {
    const int p = order[q];
    const pic_process &P = h->pr[p];
    const int s = P.species;
    const bool eion = P.kind == PIC_RECOMB || P.kind == PIC_EDETACH;
    ProcDev &d = eion ? S.proc[0][S.nproc_sp[0] + S.nei++] : S.proc[s][S.nproc_sp[s]++];
    const double mu = reduced_mass(h, P);
    d.kind = P.kind; d.target = P.target; d.tab = p;
    d.e_th = (float)P.e_th;
    const double n = target_n(h, P, n_o2);
    d.scale = s == 2 ? (float)n : (h->numax[s] > 0.0 ? (float)(n / h->numax[s]) : 0.0f);
    d.inv_mu2 = (float)(2.0 * QE / mu);
    d.half_mu_e = (float)(0.5 * mu / QE);
    d.vt = (float)std::sqrt(KB * c.t_gas / P.target_mass);
    d.tm_ratio = (float)(2.0 * sp[0].mass / P.target_mass);
    d.cmf = (float)(P.target_mass / (sp[s].mass + P.target_mass));
  }
  unsigned char *ws = h->ws;
  S.Q = (unsigned long long *)(ws + L.Q);
  S.E = (float *)(ws + L.E);
  S.phi = (double *)(ws + L.phi);
  S.sumQ = (double *)(ws + L.sumQ);
  S.sumphi = (double *)(ws + L.sumphi);
  S.esum = (unsigned long long *)(ws + L.esum);
  S.ecnt = (unsigned long long *)(ws + L.ecnt);
  S.edf = (unsigned long long *)(ws + L.edf);
  S.iedf = (unsigned long long *)(ws + L.iedf);
  S.nacc = (unsigned long long *)(ws + L.nacc);
  S.kleft = (int32_t *)(ws + L.kleft);
  S.kleft_neg = (int32_t *)(ws + L.kleft_neg);
  S.dens_ei = (float *)(ws + L.dens_ei);
  S.meta_src = (unsigned long long *)(ws + L.meta_src);
  S.na = (double *)(ws + L.na);
  S.na_f = (float *)(ws + L.na_f);
  S.meta_tmp = (double *)(ws + L.meta_tmp);
  S.pcell = (PairCell *)(ws + L.pcell);
  S.phist = (int32_t *)(ws + L.phist);
  S.sortcnt = (int32_t *)(ws + L.sortcnt);
  S.bcnt = (int32_t *)(ws + L.bcnt);
  S.sortbase = (int32_t *)(ws + L.sortbase);
  S.sortoff = (int32_t *)(ws + L.sortoff);
  S.sc = (Scalars *)(ws + L.sc);
  S.sigma = (const float *)(ws + L.sigma);
  S.hbound = (const double *)(ws + L.hbound);
  S.events = (long long *)(ws + L.events);
  S.part = (unsigned long long *)(ws + L.partials);
  S.bal = (PushBal *)(ws + L.bal);
  S.ttot_e = (const float *)(ws + L.ttot);
  S.blkcnt = (long long *)(ws + L.blkcnt);
  S.spc = c.steps_per_cycle;
  S.jsum = (double *)(ws + L.jsum);
  S.jcnt = (unsigned long long *)(ws + L.jcnt);
  S.jpow = (double *)(ws + L.jpow);

  // launch shapes.  The electron push keeps the state of its first candidates of
  // each pass in LDS; give it what the resident blocks (at most 1024 threads per
  // CU at the push kernels' 128 registers) leave free, beside at most 4 KB of static LDS.
  const size_t lds_cu = prop.maxSharedMemoryPerMultiProcessor ? prop.maxSharedMemoryPerMultiProcessor : prop.sharedMemPerBlock;
  {
    S.rq_cap = 0;
    const size_t base = push_lds_bytes(S, 0, h->block) + 4096;
    const size_t per_cu = std::max<size_t>(1, std::min<size_t>(lds_cu / base, 1024 / h->block));
    const size_t budget = std::min<size_t>(lds_cu / per_cu, prop.sharedMemPerBlock);
    S.rq_cap = budget > base ? (int)(std::min<size_t>(1024, (budget - base) / 26) & ~(size_t)3) : 0;
  }
  const size_t lds_need = max_push_lds(S, h->block);
  if (lds_need > prop.sharedMemPerBlock) {
    g_query_error = "grid too large for the LDS of one block (" + std::to_string(lds_need) + " bytes)";
    delete h;
    return PIC_EINVAL;
  }
  for (int s = 0; s < NSP; ++s) {
    const size_t lds = push_lds_bytes(S, s, h->block);
    int per_cu = (int)std::min<size_t>(2048 / h->block, std::max<size_t>(1, lds_cu / lds));
    const int gmax = std::max(1, per_cu * h->ncu);
    int64_t g = (sp[s].capacity + 8 * h->block - 1) / (8 * h->block);
    h->grid[s] = cfg->grid ? cfg->grid
                           : (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(g, gmax), max_push_grid()));
  }
  int64_t capmax = std::max(sp[0].capacity, std::max(sp[1].capacity, sp[2].capacity));
  h->hgrid = (int)std::max<int64_t>(1, std::min<int64_t>((capmax + 255) / 256, 4 * h->ncu));
  h->pgrid = (int)std::max<int64_t>(1, std::min<int64_t>((sp[1].capacity + 255) / 256, 4 * h->ncu));

  // tables: FP32 sigma for the kernels, FP64 interval bounds for the O- bound
  std::vector<float> sig32((size_t)nproc * c.table_n);
  std::vector<double> hb((size_t)nproc * (c.table_n - 1));
  for (int p = 0; p < nproc; ++p) {
    const double mu = reduced_mass(h, h->pr[p]);
    for (int k = 0; k < c.table_n; ++k) sig32[(size_t)p * c.table_n + k] = (float)h->sig[p][k];
    for (int k = 0; k + 1 < c.table_n; ++k) {
      const double ek1 = c.table_emin * std::pow(c.table_emax / c.table_emin, (double)(k + 1) / (double)(c.table_n - 1));
      hb[(size_t)p * (c.table_n - 1) + k] = std::fmax(h->sig[p][k], h->sig[p][k + 1]) * std::sqrt(2.0 * ek1 * QE / mu);
    }
  }
  // early null test of the electron MCC: sum over electron processes of (n_p / nu_max) sigma_p
  std::vector<float> ttot(c.table_n, 0.0f);
  for (int k = 0; k < c.table_n; ++k) {
    double t = 0.0;
    for (int p = 0; p < nproc; ++p)
      if (h->pr[p].species == 0 && h->numax[0] > 0.0) t += target_n(h, h->pr[p], n_o2) / h->numax[0] * h->sig[p][k];
    ttot[k] = (float)t;
  }
  hipError_t e = hipMemsetAsync(h->ws, 0, L.total, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->ws + L.ttot, ttot.data(), ttot.size() * 4, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess && nproc)
    e = hipMemcpyAsync(h->ws + L.sigma, sig32.data(), sig32.size() * 4, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess && nproc)
    e = hipMemcpyAsync(h->ws + L.hbound, hb.data(), hb.size() * 8, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = set_lds_limits(S, h->block);
  if (e != hipSuccess) {
    g_query_error = std::string("pic_create: ") + hipGetErrorString(e);
    delete h;
    return PIC_EHIP;
  }
  *out = h;
  return PIC_OK;
}

int pic_destroy(pic_handle *h) {
  if (!h) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  if (h->stream || true) (void)hipStreamSynchronize(h->stream);
  delete h;
  return PIC_OK;
}

int pic_prepare(pic_handle *h, int32_t shift) {
  if (!h) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  Sim &S = h->S;
  const size_t nn = h->cfg.ng + 1;
  {
    const int32_t z = 0;                          // the next field solve starts the current series
    const int r = set_scalar(h, offsetof(Scalars, jvalid), &z, 4);
    if (r != PIC_OK) return r;
  }
  HIPCHK(h, hipMemsetAsync(S.Q, 0, 8 * NSP * nn, h->stream));
  for (int s = 0; s < NSP; ++s) HIPCHK(h, launch_deposit(S, s, h->hgrid, h->stream));
  if (shift) {
    HIPCHK(h, launch_field(S, h->step, 1, h->stream));
    for (int s = 0; s < NSP; ++s) HIPCHK(h, launch_shift(S, s, h->hgrid, h->stream));
  }
  return PIC_OK;
}

int pic_load_uniform(pic_handle *h) {
  if (!h) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  HIPCHK(h, launch_fixup(h->S, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int s = 0; s < NSP; ++s) {
    const float vth = (float)std::sqrt(h->sp[s].t0_ev * QE / h->sp[s].mass);
    h->cur[s] = 0;
    h->S.p[s] = h->buf[s][0];
    h->S.alt[s] = h->buf[s][1];
    if (h->sp[s].count > 0) HIPCHK(h, launch_load(h->S, s, h->sp[s].count, vth, h->hgrid, h->stream));
    unsigned long long n = (unsigned long long)h->sp[s].count, z = 0;
    uint32_t nid = (uint32_t)h->sp[s].count;
    int r = set_scalar(h, offsetof(Scalars, n) + 8 * s, &n, 8);
    if (r == PIC_OK) r = set_scalar(h, offsetof(Scalars, nnew) + 8 * s, &z, 8);
    if (r == PIC_OK) r = set_scalar(h, offsetof(Scalars, next_id) + 4 * s, &nid, 4);
    if (r != PIC_OK) return r;
  }
  h->step = 0;
  return pic_prepare(h, 1);
}

}  // extern "C"

namespace {

// piecewise-linear profile at x (x / L), constant beyond the end points
#pragma clang fp contract(off)
double profile_at(int32_t n, const double *xs, const double *v, double x) {
  if (x <= xs[0]) return v[0];
  if (x >= xs[n - 1]) return v[n - 1];
  int32_t k = 0;
  while (xs[k + 1] <= x) ++k;
  return v[k] + (v[k + 1] - v[k]) * (x - xs[k]) / (xs[k + 1] - xs[k]);
}

bool valid_profile(int32_t n, const double *xs, const double *dens, const double *mean_ev) {
  if (n < 2 || !xs || !dens || !mean_ev) return false;
  for (int32_t k = 0; k < n; ++k) {
    if (!(xs[k] >= 0.0 && xs[k] <= 1.0) || (k > 0 && !(xs[k] > xs[k - 1]))) return false;
    for (int s = 0; s < NSP; ++s) {
      const double d = dens[s * n + k], e = mean_ev[s * n + k];
      if (!(std::isfinite(d) && d >= 0.0) || !(std::isfinite(e) && e > 0.0)) return false;
    }
  }
  return true;
}

// cumulative counts round(sum_{i <= j} n(x_i) dx / w) and thermal speeds per cell
#pragma clang fp contract(off)
void profile_counts(const pic_handle *h, int s, int32_t n, const double *xs, const double *dens,
                    const double *mean_ev, std::vector<long long> &cum, std::vector<float> &vth) {
  const int32_t ng = h->cfg.ng;
  const double dx = h->cfg.L / ng;
  cum.resize(ng);
  vth.resize(ng);
  double c = 0.0;
  for (int32_t j = 0; j < ng; ++j) {
    const double xc = ((double)j + 0.5) / (double)ng;
    const double nd = profile_at(n, xs, dens + s * n, xc);
    const double t_ev = (2.0 / 3.0) * profile_at(n, xs, mean_ev + s * n, xc);
    c += (nd * dx) / h->cfg.weight;
    cum[j] = (long long)std::floor(c + 0.5);
    vth[j] = (float)std::sqrt(t_ev * QE / h->sp[s].mass);
  }
}

}  // namespace

extern "C" {

int pic_load_profiles(pic_handle *h, int32_t n_pts, const double *x_over_L, const double *dens,
                      const double *mean_ev) {
  if (!h) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  if (!valid_profile(n_pts, x_over_L, dens, mean_ev)) {
    const int r = pic_load_uniform(h);
    if (r != PIC_OK) return r;
    h->err = "invalid profile: loaded uniformly instead";
    return PIC_WFALLBACK;
  }
  std::vector<long long> cum[NSP];
  std::vector<float> vth[NSP];
  for (int s = 0; s < NSP; ++s) {
    profile_counts(h, s, n_pts, x_over_L, dens, mean_ev, cum[s], vth[s]);
    if (cum[s].back() > h->sp[s].capacity) return fail(h, PIC_ECAPACITY, "profile needs more particles than the capacity");
  }
  HIPCHK(h, launch_fixup(h->S, h->stream));        // settle products still waiting for ids
  HIPCHK(h, hipStreamSynchronize(h->stream));
  const size_t ng = h->cfg.ng;
  long long *dcum = (long long *)(h->ws + h->L.prof);
  float *dvth = (float *)(h->ws + h->L.prof + 8 * NSP * ng);
  for (int s = 0; s < NSP; ++s) {
    HIPCHK(h, hipMemcpy(dcum + s * ng, cum[s].data(), 8 * ng, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(dvth + s * ng, vth[s].data(), 4 * ng, hipMemcpyHostToDevice));
  }
  for (int s = 0; s < NSP; ++s) {
    h->cur[s] = 0;
    h->S.p[s] = h->buf[s][0];
    h->S.alt[s] = h->buf[s][1];
    const long long count = cum[s].back();
    if (count > 0) HIPCHK(h, launch_load_profile(h->S, s, count, dcum + s * ng, dvth + s * ng, h->hgrid, h->stream));
    unsigned long long nn = (unsigned long long)count, z = 0;
    uint32_t nid = (uint32_t)count;
    int r = set_scalar(h, offsetof(Scalars, n) + 8 * s, &nn, 8);
    if (r == PIC_OK) r = set_scalar(h, offsetof(Scalars, nnew) + 8 * s, &z, 8);
    if (r == PIC_OK) r = set_scalar(h, offsetof(Scalars, next_id) + 4 * s, &nid, 4);
    if (r != PIC_OK) return r;
  }
  h->step = 0;
  return pic_prepare(h, 1);
}

int pic_set_particles(pic_handle *h, int32_t s, int64_t n, const int32_t *cell, const float *off, const float *vx,
                      const float *vy, const float *vz, const uint32_t *id, const int32_t *cd, uint32_t next_id) {
  if (!h || s < 0 || s >= NSP || n < 0) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  if (n > h->sp[s].capacity) return fail(h, PIC_ECAPACITY, "more particles than the species capacity");
  if (n > 0 && (!cell || !off || !vx || !vy || !vz || !id)) return fail(h, PIC_EINVAL, "null particle array");
  std::vector<int32_t> w((size_t)n);
  for (int64_t k = 0; k < n; ++k) {
    if (cell[k] < 0 || cell[k] >= h->cfg.ng || !(off[k] >= 0.0f && off[k] < 1.0f))
      return fail(h, PIC_EINVAL, "particle outside [0, L) or offset outside [0, 1)");
    int32_t word = cell[k];
    if (s == 0) {
      const int32_t c = cd ? cd[k] : 1;
      const int32_t steps = c & 0x7FFF;
      if (steps < 1) return fail(h, PIC_EINVAL, "electron countdown must be >= 1");
      word |= (steps << W_CD_SHIFT) | (c & 0x8000);
    }
    w[(size_t)k] = word;
  }
  HIPCHK(h, launch_fixup(h->S, h->stream));        // settle products still waiting for ids
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->cur[s] = 0;
  h->S.p[s] = h->buf[s][0];
  h->S.alt[s] = h->buf[s][1];
  const Particles &P = h->S.p[s];
  if (n > 0) {
    HIPCHK(h, hipMemcpy(P.w, w.data(), 4 * n, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(P.off, off, 4 * n, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(P.vx, vx, 4 * n, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(P.vy, vy, 4 * n, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(P.vz, vz, 4 * n, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(P.id, id, 4 * n, hipMemcpyHostToDevice));
  }
  unsigned long long nn = (unsigned long long)n, z = 0;
  const int32_t zi = 0;
  int r = set_scalar(h, offsetof(Scalars, jvalid), &zi, 4);
  if (r == PIC_OK) r = set_scalar(h, offsetof(Scalars, n) + 8 * s, &nn, 8);
  if (r == PIC_OK) r = set_scalar(h, offsetof(Scalars, nnew) + 8 * s, &z, 8);
  if (r == PIC_OK) r = set_scalar(h, offsetof(Scalars, next_id) + 4 * s, &next_id, 4);
  return r;
}

int pic_sync(pic_handle *h) {
  if (!h) return PIC_EINVAL;
  hipError_t e;
  const Scalars sc = read_scalars(h, &e);
  if (e != hipSuccess) return hipfail(h, e, "pic_sync");
  return device_errors(h, sc);
}

int pic_count(pic_handle *h, int32_t s, int64_t *n) {
  if (!h || s < 0 || s >= NSP || !n) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  HIPCHK(h, launch_fixup(h->S, h->stream));
  hipError_t e;
  const Scalars sc = read_scalars(h, &e);
  if (e != hipSuccess) return hipfail(h, e, "pic_count");
  std::vector<int32_t> w(sc.n[s]);
  if (sc.n[s]) HIPCHK(h, hipMemcpy(w.data(), h->S.p[s].w, 4 * sc.n[s], hipMemcpyDeviceToHost));
  int64_t c = 0;
  for (int32_t x : w) c += x >= 0;
  *n = c;
  return device_errors(h, sc);
}

int pic_get_particles(pic_handle *h, int32_t s, int64_t *n, int32_t *cell, float *off, float *vx, float *vy,
                      float *vz, uint32_t *id, int32_t *cd, uint32_t *next_id) {
  if (!h || s < 0 || s >= NSP || !n) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  HIPCHK(h, launch_fixup(h->S, h->stream));
  hipError_t e;
  const Scalars sc = read_scalars(h, &e);
  if (e != hipSuccess) return hipfail(h, e, "pic_get_particles");
  const size_t m = sc.n[s];
  std::vector<int32_t> w(m), ids(m);
  std::vector<float> o(m), x(m), y(m), z(m);
  const Particles &P = h->S.p[s];
  if (m) {
    HIPCHK(h, hipMemcpy(w.data(), P.w, 4 * m, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(o.data(), P.off, 4 * m, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(x.data(), P.vx, 4 * m, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(y.data(), P.vy, 4 * m, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(z.data(), P.vz, 4 * m, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(ids.data(), P.id, 4 * m, hipMemcpyDeviceToHost));
  }
  int64_t k = 0;
  for (size_t i = 0; i < m; ++i) {
    if (w[i] < 0) continue;
    if (k < *n) {
      if (cell) cell[k] = w[i] & (int32_t)W_CELL;
      if (off) off[k] = o[i];
      if (vx) vx[k] = x[i];
      if (vy) vy[k] = y[i];
      if (vz) vz[k] = z[i];
      if (id) id[k] = (uint32_t)ids[i];
      if (cd) cd[k] = s == 0 ? (((w[i] >> W_CD_SHIFT) & 0x7FFF) | (w[i] & (int32_t)W_CAP)) : 0;
    }
    ++k;
  }
  const bool fits = k <= *n;
  *n = k;
  if (next_id) *next_id = sc.next_id[s];
  if (!fits) return fail(h, PIC_ECAPACITY, "host arrays smaller than the live count");
  return device_errors(h, sc);
}

int pic_set_step(pic_handle *h, int64_t step) {
  if (!h || step < 0) return PIC_EINVAL;
  {
    const int32_t z = 0;
    if (!h->batch_busy) {
      const int r = set_scalar(h, offsetof(Scalars, jvalid), &z, 4);
      if (r != PIC_OK) return r;
    }
  }
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  h->step = step;
  return PIC_OK;
}

int pic_get_step(pic_handle *h, int64_t *step) {
  if (!h || !step) return PIC_EINVAL;
  *step = h->step;
  return PIC_OK;
}

// One step.  `more`: the caller enqueues the next step right after this one;
// then, when neither this step nor the next moves ions, the electron reduction
// also solves the next step's field (h->field_ready), so that state read
// between pic_step calls is never ahead of the step index.
static int enqueue_step(pic_handle *h, hipEvent_t ev0, hipEvent_t ev1, bool more) {
  Sim &S = h->S;
  const pic_config &c = h->cfg;
  const int64_t n = h->step;
  // electron-ion channels: the ion densities of this step's field, before it clears them
  const bool eion = S.nei > 0 && !(S.flags & F_NO_COLL) && n % c.ksub == 0;
  if (eion) HIPCHK(h, launch_eiprep(S, h->stream));
  if (!h->field_ready) HIPCHK(h, launch_field(S, n, 0, h->stream));
  h->field_ready = false;
  if (c.diag_every > 0 && n % c.diag_every == 0)
    for (int s = 0; s < NSP; ++s) HIPCHK(h, launch_diag(S, s, h->hgrid, h->stream));
  if (c.sort_every > 0 && n % c.sort_every == 0) {
    for (int s = 0; s < NSP; ++s) {
      const int other = 1 - h->cur[s];
      if (c.sort_kind == PIC_SORT_CELL) HIPCHK(h, launch_sort(S, s, h->buf[s][other], h->hgrid, h->stream));
      else HIPCHK(h, launch_compact(S, s, h->buf[s][other], h->hgrid, h->stream));
      h->cur[s] = other;
      S.p[s] = h->buf[s][other];
      S.alt[s] = h->buf[s][1 - other];
    }
  }
  if (ev0) HIPCHK(h, hipEventRecord(ev0, h->stream));
  HIPCHK(h, launch_push(S, 0, n, h->grid[0], h->block, h->stream));
  if (ev1) HIPCHK(h, hipEventRecord(ev1, h->stream));
  const bool fuse = more && n % c.ksub != 0 && (n + 1) % c.ksub != 0;
  if (fuse) HIPCHK(h, launch_reduce_field(S, h->grid[0], n + 1, h->stream));
  else HIPCHK(h, launch_reduce(S, 0, h->grid[0], h->stream));
  if (eion) HIPCHK(h, launch_eion(S, n, h->hgrid, h->stream));
  if (n % c.ksub == 0) {
    HIPCHK(h, launch_push(S, 1, n, h->grid[1], h->block, h->stream));
    HIPCHK(h, launch_reduce(S, 1, h->grid[1], h->stream));
    HIPCHK(h, launch_ionprep(S, h->stream));
    HIPCHK(h, launch_push(S, 2, n, h->grid[2], h->block, h->stream));
    HIPCHK(h, launch_reduce(S, 2, h->grid[2], h->stream));
    // partners: O2+ of neutralisation and recombination, then O- of electron-impact detachment
    for (int stage = 0; stage < 4; ++stage) HIPCHK(h, launch_pair(S, n, stage, 1, h->pgrid, h->stream));
    if (eion)
      for (int stage = 0; stage < 4; ++stage) HIPCHK(h, launch_pair(S, n, stage, 2, h->pgrid, h->stream));
  }
  h->step = n + 1;
  h->field_ready = fuse;
  return PIC_OK;
}

int pic_step(pic_handle *h, int64_t n_steps) {
  if (!h || n_steps < 0) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  for (int64_t k = 0; k < n_steps; ++k) {
    const int r = enqueue_step(h, nullptr, nullptr, k + 1 < n_steps);
    if (r != PIC_OK) return r;
  }
  return PIC_OK;
}

int pic_step_timed(pic_handle *h, int64_t n_steps, double *ms_push_e, double *ms_total, int64_t *launches) {
  if (!h || n_steps < 0) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  const int CH = 256;
  std::vector<hipEvent_t> ev(2 * CH);
  hipEvent_t t0, t1;
  for (auto &e : ev) HIPCHK(h, hipEventCreate(&e));
  HIPCHK(h, hipEventCreate(&t0));
  HIPCHK(h, hipEventCreate(&t1));
  double push = 0.0;
  int rc = PIC_OK;
  HIPCHK(h, hipEventRecord(t0, h->stream));
  for (int64_t k = 0; k < n_steps && rc == PIC_OK;) {
    const int m = (int)std::min<int64_t>(CH, n_steps - k);
    for (int j = 0; j < m && rc == PIC_OK; ++j) rc = enqueue_step(h, ev[2 * j], ev[2 * j + 1], k + j + 1 < n_steps);
    if (rc != PIC_OK) break;
    HIPCHK(h, hipEventSynchronize(ev[2 * m - 1]));
    for (int j = 0; j < m; ++j) {
      float ms = 0.0f;
      HIPCHK(h, hipEventElapsedTime(&ms, ev[2 * j], ev[2 * j + 1]));
      push += ms;
    }
    k += m;
  }
  HIPCHK(h, hipEventRecord(t1, h->stream));
  HIPCHK(h, hipEventSynchronize(t1));
  float tot = 0.0f;
  HIPCHK(h, hipEventElapsedTime(&tot, t0, t1));
  for (auto &e : ev) (void)hipEventDestroy(e);
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (ms_push_e) *ms_push_e = push;
  if (ms_total) *ms_total = tot;
  if (launches) *launches = n_steps;
  if (rc != PIC_OK) return rc;
  return pic_sync(h);
}

int pic_moments(pic_handle *h, pic_moments_out *out, int32_t reset) {
  if (!h || !out) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  const Layout &L = h->L;
  const size_t ng = h->cfg.ng, nn = ng + 1;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  unsigned long long na[2];
  HIPCHK(h, hipMemcpy(na, h->ws + L.nacc, 16, hipMemcpyDeviceToHost));
  out->nacc = (int64_t)na[0];
  out->ndiag = (int64_t)na[1];
  if (out->sum_q) HIPCHK(h, hipMemcpy(out->sum_q, h->ws + L.sumQ, 8 * NSP * nn, hipMemcpyDeviceToHost));
  if (out->sum_phi) HIPCHK(h, hipMemcpy(out->sum_phi, h->ws + L.sumphi, 8 * nn, hipMemcpyDeviceToHost));
  if (out->esum) HIPCHK(h, hipMemcpy(out->esum, h->ws + L.esum, 8 * NSP * ng, hipMemcpyDeviceToHost));
  if (out->ecnt) HIPCHK(h, hipMemcpy(out->ecnt, h->ws + L.ecnt, 8 * NSP * ng, hipMemcpyDeviceToHost));
  if (out->edf) HIPCHK(h, hipMemcpy(out->edf, h->ws + L.edf, 8 * NSP * NBIN, hipMemcpyDeviceToHost));
  if (out->iedf) HIPCHK(h, hipMemcpy(out->iedf, h->ws + L.iedf, 8 * NSP * 2 * NBIN, hipMemcpyDeviceToHost));
  const size_t spc = h->cfg.steps_per_cycle;
  if (out->current) HIPCHK(h, hipMemcpy(out->current, h->ws + L.jsum, 8 * spc, hipMemcpyDeviceToHost));
  if (out->current_n) HIPCHK(h, hipMemcpy(out->current_n, h->ws + L.jcnt, 8 * spc, hipMemcpyDeviceToHost));
  double jp[2];
  HIPCHK(h, hipMemcpy(jp, h->ws + L.jpow, 16, hipMemcpyDeviceToHost));
  out->power_sum = jp[0];
  out->power_n = (int64_t)jp[1];
  if (reset) {
    HIPCHK(h, hipMemsetAsync(h->ws + L.sumQ, 0, 8 * NSP * nn, h->stream));
    HIPCHK(h, hipMemsetAsync(h->ws + L.sumphi, 0, 8 * nn, h->stream));
    HIPCHK(h, hipMemsetAsync(h->ws + L.esum, 0, 8 * NSP * ng, h->stream));
    HIPCHK(h, hipMemsetAsync(h->ws + L.ecnt, 0, 8 * NSP * ng, h->stream));
    HIPCHK(h, hipMemsetAsync(h->ws + L.edf, 0, 8 * NSP * NBIN, h->stream));
    HIPCHK(h, hipMemsetAsync(h->ws + L.iedf, 0, 8 * NSP * 2 * NBIN, h->stream));
    HIPCHK(h, hipMemsetAsync(h->ws + L.nacc, 0, 16, h->stream));
    HIPCHK(h, hipMemsetAsync(h->ws + L.jsum, 0, 8 * spc, h->stream));
    HIPCHK(h, hipMemsetAsync(h->ws + L.jcnt, 0, 8 * spc, h->stream));
    HIPCHK(h, hipMemsetAsync(h->ws + L.jpow, 0, 16, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
  }
  return pic_sync(h);
}

int pic_get_hist(pic_handle *h, int64_t *q) {
  if (!h || !q) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  HIPCHK(h, launch_fixup(h->S, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HIPCHK(h, hipMemcpy(q, h->S.Q, 8 * NSP * (size_t)(h->cfg.ng + 1), hipMemcpyDeviceToHost));
  return pic_sync(h);
}

int pic_get_field(pic_handle *h, double *phi, float *e) {
  if (!h) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (phi) HIPCHK(h, hipMemcpy(phi, h->S.phi, 8 * (size_t)(h->cfg.ng + 1), hipMemcpyDeviceToHost));
  if (e) HIPCHK(h, hipMemcpy(e, h->S.E, 4 * (size_t)(h->cfg.ng + 1), hipMemcpyDeviceToHost));
  return pic_sync(h);
}

int pic_get_counters(pic_handle *h, int64_t *out) {
  if (!h || !out) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  hipError_t e;
  const Scalars sc = read_scalars(h, &e);
  if (e != hipSuccess) return hipfail(h, e, "pic_get_counters");
  for (int k = 0; k < NCOUNT; ++k) out[k] = (int64_t)sc.cnt[k];
  return device_errors(h, sc);
}

int pic_get_events(pic_handle *h, int64_t max, int64_t *rec, int64_t *n, int32_t clear) {
  if (!h || !n || max < 0) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  hipError_t e;
  const Scalars sc = read_scalars(h, &e);
  if (e != hipSuccess) return hipfail(h, e, "pic_get_events");
  *n = (int64_t)sc.nev;
  const int64_t m = std::min<int64_t>(std::min<int64_t>(max, *n), h->cfg.event_capacity);
  if (m > 0 && rec) HIPCHK(h, hipMemcpy(rec, h->S.events, 32 * m, hipMemcpyDeviceToHost));
  if (clear) {
    unsigned long long z = 0;
    const int r = set_scalar(h, offsetof(Scalars, nev), &z, 8);
    if (r != PIC_OK) return r;
  }
  return device_errors(h, sc);
}

int pic_metastable_config(pic_handle *h, const pic_metastable *m) {
  if (!h || !m) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  const int p = m->source_process;
  if (p < 0 || p >= (int)h->pr.size() || h->pr[p].species != 0 || h->pr[p].kind != PIC_EXCITE)
    return fail(h, PIC_EINVAL, "source_process must index an electron excitation channel");
  if (!(std::isfinite(m->diffusion) && m->diffusion > 0.0) || !(std::isfinite(m->quench_rate) && m->quench_rate >= 0.0) ||
      !(m->surface_loss >= 0.0 && m->surface_loss <= 1.0) || (m->surface_loss == 0.0 && m->quench_rate == 0.0))
    return fail(h, PIC_EINVAL, "need diffusion > 0, quench_rate >= 0, surface_loss in [0, 1], and some loss");
  const double vbar = std::sqrt(8.0 * KB * h->cfg.t_gas / (3.14159265358979323846 * h->pr[p].target_mass));
  h->meta = *m;
  h->meta_h = m->surface_loss * vbar / (2.0 * (2.0 - m->surface_loss));
  h->meta_on = true;
  h->meta_step0 = h->step;
  HIPCHK(h, launch_meta_init(h->S, p, h->stream));
  return PIC_OK;
}

int pic_metastable_update(pic_handle *h, double *n_out) {
  if (!h) return PIC_EINVAL;
  if (h->batch_busy) return fail(h, PIC_EBUSY, "member of a batch with unsynchronised work (call pic_batch_sync)");
  if (!h->meta_on) return fail(h, PIC_EINVAL, "pic_metastable_config has not been called");
  const double tau = (double)(h->step - h->meta_step0) * h->S.dt;
  if (!(tau > 0.0)) return fail(h, PIC_EINVAL, "no steps since the last update");
  HIPCHK(h, launch_meta_solve(h->S, h->cfg.weight, tau, h->meta.diffusion, h->meta.quench_rate, h->meta_h, h->stream));
  h->meta_step0 = h->step;
  if (n_out) {
    HIPCHK(h, hipMemcpyAsync(n_out, h->S.na, 8 * (size_t)(h->cfg.ng + 1), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
  }
  return PIC_OK;
}

int pic_nu_max(pic_handle *h, int32_t s, double *nu) {
  if (!h || !nu || s < 0 || s >= NSP) return PIC_EINVAL;
  if (s < 2) { *nu = h->numax[s]; return PIC_OK; }
  hipError_t e;
  const Scalars sc = read_scalars(h, &e);
  if (e != hipSuccess) return hipfail(h, e, "pic_nu_max");
  *nu = sc.numax_neg;
  return PIC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches
struct pic_batch {
  std::vector<pic_handle *> mem;
  hipStream_t stream = nullptr;
  unsigned char *ws = nullptr;
  Sim *d_sims = nullptr;
  BatchDev *d_bd = nullptr;
  pic_batch_config cfg{};
  int spc = 0;
  int rel = 0;                 // steps done in the running rf cycle
  bool on_device = false;      // the members' state lives in the device records
  BatchLaunch B{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int ncu = 1;
  size_t lds_max = 0;
  std::vector<Sim> host_sims;
  std::string err;
};

namespace {

std::string g_batch_error;

int bfail(pic_batch *b, int code, const std::string &m) {
  if (b) b->err = m;
  else g_batch_error = m;
  return code;
}

#define BHIP(b, expr)                                                                               \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) return bfail((b), PIC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t batch_bytes(int n) {
  return ((sizeof(Sim) * (size_t)n + 255) & ~(size_t)255) + ((sizeof(BatchDev) + 255) & ~(size_t)255);
}

uint64_t all_mask(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }

int batch_check_config(const pic_batch_config *c, int spc, std::string &msg) {
  if (!c) { msg = "null batch config"; return PIC_EINVAL; }
  if (!(c->block == 0 || c->block == 256 || c->block == 512 || c->block == 1024)) {
    msg = "batch block must be 0, 256, 512 or 1024"; return PIC_EINVAL;
  }
  if (c->sort_every < 0 || (c->sort_every > 0 && spc % c->sort_every != 0)) {
    msg = "batch sort_every must be 0 or divide steps_per_cycle"; return PIC_EINVAL;
  }
  if (c->grid < 0 || c->grid > max_push_grid()) { msg = "batch grid must be in [0, 2048]"; return PIC_EINVAL; }
  return PIC_OK;
}

void drop_graph(pic_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// launch shapes for the current configuration
int batch_shapes(pic_batch *b) {
  BatchLaunch &B = b->B;
  B.sims = b->d_sims;
  B.bd = b->d_bd;
  B.nmem = (int)b->mem.size();
  B.block = b->cfg.block ? b->cfg.block : 512;
  B.nn_max = 0;
  B.diag_lds = 0;
  for (pic_handle *h : b->mem) {
    B.nn_max = std::max(B.nn_max, h->cfg.ng + 1);
    B.diag_lds = std::max(B.diag_lds, diag_lds_bytes(h->S));
  }
  for (int s = 0; s < NSP; ++s) {
    size_t lds = 0;
    for (pic_handle *h : b->mem) lds = std::max(lds, push_lds_bytes(h->S, s, B.block));
    if (lds > b->lds_max) return bfail(b, PIC_EINVAL, "largest member grid does not fit the LDS of one block");
    int per_cu = 0;
    BHIP(b, batch_push_occupancy(B.block, s, lds, &per_cu));
    const int g = b->cfg.grid ? b->cfg.grid : std::max(1, per_cu) * b->ncu;
    B.push_grid[s] = std::min(g, max_push_grid());
    B.push_lds[s] = lds;
    if (s == 0) {
      // the balanced electron ranges need a cut table past the push's LDS; only
      // where it costs no occupancy
      B.bal_lds = 0;
      const size_t off = (lds + 15) & ~(size_t)15, tot = off + 8 * (size_t)(B.push_grid[0] + 1);
      int per_cu_bal = 0;
      if (tot <= b->lds_max) BHIP(b, batch_push_occupancy(B.block, 0, tot, &per_cu_bal));
      if (tot <= b->lds_max && per_cu_bal >= std::max(1, per_cu)) {
        B.push_lds[0] = tot;
        B.bal_lds = off;
      }
    }
  }
  B.cgrid = 64;
  B.pgrid = 16;
  B.dgrid = 32;
  return PIC_OK;
}

// the members' records go to the device; from here the batch owns their state
int batch_upload(pic_batch *b) {
  const int n = (int)b->mem.size();
  b->host_sims.resize(n);
  BatchDev bd;
  std::memset(&bd, 0, sizeof(bd));
  for (int m = 0; m < n; ++m) {
    pic_handle *h = b->mem[m];
    if (h->step % b->spc != 0)
      return bfail(b, PIC_EINVAL, "member " + std::to_string(m) + " is not at an rf-cycle boundary");
    Sim S = h->S;
    for (int s = 0; s < NSP; ++s) {
      S.p[s] = h->buf[s][h->cur[s]];
      S.alt[s] = h->buf[s][1 - h->cur[s]];
    }
    b->host_sims[m] = S;
    bd.base[m] = h->step;
  }
  BHIP(b, hipMemcpyAsync(b->d_sims, b->host_sims.data(), sizeof(Sim) * n, hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipMemcpyAsync(b->d_bd, &bd, sizeof(bd), hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  for (pic_handle *h : b->mem) h->batch_busy = true;
  b->on_device = true;
  b->rel = 0;
  return PIC_OK;
}

// the launches of step `r` of the rf cycle (device steps base[m] + r)
int launch_batch_step(pic_batch *b, int r) {
  const BatchLaunch &B = b->B;
  hipStream_t st = b->stream;
  const int n = B.nmem;
  const uint64_t all = all_mask(n);
  uint64_t dmask = 0ull, imask = 0ull, emask = 0ull;
  for (int m = 0; m < n; ++m) {
    const pic_config &c = b->mem[m]->cfg;
    if (c.diag_every > 0 && r % c.diag_every == 0) dmask |= 1ull << m;
    if (r % c.ksub == 0) {
      imask |= 1ull << m;
      // electron-ion channels (Table 1 (16), (22)) on this member's ion steps
      if (b->mem[m]->S.nei > 0 && !(c.flags & PIC_F_NO_COLL)) emask |= 1ull << m;
    }
  }
  if (emask) BHIP(b, launch_eiprep_b(B, emask, st));      // before the field kernel clears the ion histograms
  BHIP(b, launch_field_b(B, r, st));
  if (dmask) BHIP(b, launch_diag_b(B, dmask, st));
  if (b->cfg.sort_every > 0 && r % b->cfg.sort_every == 0) BHIP(b, launch_compact_b(B, all, st));
  BHIP(b, launch_push_b(B, 0, all, r, st));
  BHIP(b, launch_reduce_b(B, 0, all, st));
  if (emask) BHIP(b, launch_eion_b(B, emask, r, st));
  if (imask) {
    BHIP(b, launch_push_b(B, 1, imask, r, st));
    BHIP(b, launch_reduce_b(B, 1, imask, st));
    BHIP(b, launch_ionprep_b(B, imask, st));
    BHIP(b, launch_push_b(B, 2, imask, r, st));
    BHIP(b, launch_reduce_b(B, 2, imask, st));
    for (int stage = 0; stage < 4; ++stage) BHIP(b, launch_pair_b(B, imask, r, stage, 1, st));
    if (emask)
      for (int stage = 0; stage < 4; ++stage) BHIP(b, launch_pair_b(B, emask, r, stage, 2, st));
  }
  if (r == b->spc - 1) BHIP(b, launch_advance_b(B, b->spc, st));
  return PIC_OK;
}

void batch_advance_host(pic_batch *b, int64_t steps) {
  for (pic_handle *h : b->mem) h->step += steps;
  b->rel = (int)((b->rel + steps) % b->spc);
}

int batch_capture(pic_batch *b) {
  BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  int rc = PIC_OK;
  for (int r = 0; r < b->spc && rc == PIC_OK; ++r) rc = launch_batch_step(b, r);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (rc != PIC_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return bfail(b, PIC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  b->graph = g;
  BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return PIC_OK;
}

}  // namespace

extern "C" {

int pic_batch_query(int32_t n_members, uint64_t *workspace_bytes) {
  if (n_members < 1 || n_members > MAXBATCH || !workspace_bytes) {
    g_batch_error = "n_members must be in [1, 64] and workspace_bytes non-null";
    return PIC_EINVAL;
  }
  *workspace_bytes = batch_bytes(n_members);
  return PIC_OK;
}

int pic_batch_create(pic_handle *const *members, int32_t n, const pic_batch_config *cfg, void *workspace,
                     uint64_t workspace_bytes, void *stream, pic_batch **out) {
  if (!members || !out || !workspace || n < 1 || n > MAXBATCH)
    return bfail(nullptr, PIC_EINVAL, "need 1..64 members, a workspace and an output pointer");
  if (workspace_bytes < batch_bytes(n)) return bfail(nullptr, PIC_EINVAL, "workspace smaller than pic_batch_query reported");
  const int spc = members[0] ? members[0]->cfg.steps_per_cycle : 0;
  std::string msg;
  if (batch_check_config(cfg, spc, msg) != PIC_OK) return bfail(nullptr, PIC_EINVAL, msg);
  for (int m = 0; m < n; ++m) {
    const pic_handle *h = members[m];
    const std::string who = "member " + std::to_string(m) + ": ";
    if (!h) return bfail(nullptr, PIC_EINVAL, who + "null handle");
    for (int k = 0; k < m; ++k)
      if (members[k] == h) return bfail(nullptr, PIC_EINVAL, who + "listed twice");
    if (h->batch_busy) return bfail(nullptr, PIC_EBUSY, who + "busy in another batch");
    if (h->stream != (hipStream_t)stream) return bfail(nullptr, PIC_EINVAL, who + "created on another stream");
    const pic_config &c = h->cfg;
    if (c.steps_per_cycle != spc) return bfail(nullptr, PIC_EINVAL, who + "steps_per_cycle differs");
    if (spc % c.ksub != 0) return bfail(nullptr, PIC_EINVAL, who + "ksub must divide steps_per_cycle");
    if (c.diag_every > 0 && spc % c.diag_every != 0)
      return bfail(nullptr, PIC_EINVAL, who + "diag_every must divide steps_per_cycle");
    if (c.grid != 0) return bfail(nullptr, PIC_EINVAL, who + "grid must be 0 (full partial storage)");
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return bfail(nullptr, PIC_ENODEVICE, "no HIP device");
  pic_batch *b = new pic_batch();
  b->mem.assign(members, members + n);
  b->stream = (hipStream_t)stream;
  b->ws = (unsigned char *)workspace;
  b->d_sims = (Sim *)b->ws;
  b->d_bd = (BatchDev *)(b->ws + ((sizeof(Sim) * (size_t)n + 255) & ~(size_t)255));
  b->cfg = *cfg;
  b->spc = spc;
  b->ncu = prop.multiProcessorCount;
  b->lds_max = prop.sharedMemPerBlock;
  const int rc = batch_shapes(b);
  if (rc != PIC_OK) {
    g_batch_error = b->err;
    delete b;
    return rc;
  }
  *out = b;
  return PIC_OK;
}

int pic_batch_step_cycles(pic_batch *b, int64_t cycles) {
  if (!b || cycles < 0) return bfail(b, PIC_EINVAL, "null batch or negative cycle count");
  if (cycles == 0) return PIC_OK;
  if (!b->on_device) {
    const int rc = batch_upload(b);
    if (rc != PIC_OK) return rc;
  }
  if (b->rel != 0) return bfail(b, PIC_EINVAL, "batch not at an rf-cycle boundary");
  if (b->cfg.use_graph && b->stream) {
    if (!b->exec) {
      const int rc = batch_capture(b);
      if (rc != PIC_OK) return rc;
    }
    for (int64_t c = 0; c < cycles; ++c) {
      BHIP(b, hipGraphLaunch(b->exec, b->stream));
      batch_advance_host(b, b->spc);
    }
    return PIC_OK;
  }
  for (int64_t c = 0; c < cycles; ++c)
    for (int r = 0; r < b->spc; ++r) {
      const int rc = launch_batch_step(b, r);
      if (rc != PIC_OK) return rc;
      batch_advance_host(b, 1);
    }
  return PIC_OK;
}

int pic_batch_sync(pic_batch *b) {
  if (!b) return bfail(b, PIC_EINVAL, "null batch");
  BHIP(b, hipStreamSynchronize(b->stream));
  const int n = (int)b->mem.size();
  if (b->on_device) {
    BHIP(b, hipMemcpy(b->host_sims.data(), b->d_sims, sizeof(Sim) * n, hipMemcpyDeviceToHost));
    for (int m = 0; m < n; ++m) {
      pic_handle *h = b->mem[m];
      for (int s = 0; s < NSP; ++s) {
        h->cur[s] = b->host_sims[m].p[s].w == h->buf[s][0].w ? 0 : 1;
        h->S.p[s] = h->buf[s][h->cur[s]];
        h->S.alt[s] = h->buf[s][1 - h->cur[s]];
      }
      h->batch_busy = false;
    }
    b->on_device = false;
  }
  for (int m = 0; m < n; ++m) {
    const int rc = pic_sync(b->mem[m]);
    if (rc != PIC_OK) return bfail(b, rc, "member " + std::to_string(m) + ": " + b->mem[m]->err);
  }
  return PIC_OK;
}

int pic_batch_set_config(pic_batch *b, const pic_batch_config *cfg) {
  if (!b) return bfail(b, PIC_EINVAL, "null batch");
  std::string msg;
  if (batch_check_config(cfg, b->spc, msg) != PIC_OK) return bfail(b, PIC_EINVAL, msg);
  const pic_batch_config old = b->cfg;
  b->cfg = *cfg;
  drop_graph(b);
  const int rc = batch_shapes(b);
  if (rc != PIC_OK) {
    b->cfg = old;
    (void)batch_shapes(b);
  }
  return rc;
}

int pic_batch_get_config(const pic_batch *b, pic_batch_config *cfg) {
  if (!b || !cfg) return PIC_EINVAL;
  *cfg = b->cfg;
  if (!cfg->block) cfg->block = b->B.block;
  return PIC_OK;
}

int pic_batch_autotune(pic_batch *b, int32_t window, pic_batch_tuning *out) {
  if (!b || !out) return bfail(b, PIC_EINVAL, "null batch or output");
  if (window < 1 || b->spc % window != 0) return bfail(b, PIC_EINVAL, "window must divide steps_per_cycle");
  if (!b->on_device) {
    const int rc = batch_upload(b);
    if (rc != PIC_OK) return rc;
  }
  if (b->rel != 0) return bfail(b, PIC_EINVAL, "batch not at an rf-cycle boundary");
  const pic_batch_config keep = b->cfg;
  const int blocks[3] = {256, 512, 1024};
  const int sorts[7] = {10, 20, 50, 100, 200, 500, 1000};
  std::memset(out, 0, sizeof(*out));
  hipEvent_t e0, e1;
  BHIP(b, hipEventCreate(&e0));
  BHIP(b, hipEventCreate(&e1));
  int rc = PIC_OK;
  double best = 1e300;
  for (int bi = 0; bi < 3 && rc == PIC_OK; ++bi)
    for (int si = 0; si < 7 && rc == PIC_OK; ++si) {
      const int S = sorts[si];
      if (window % S != 0 || b->spc % S != 0 || out->n >= PIC_TUNE_MAX) continue;
      pic_batch_config c = keep;
      c.block = blocks[bi];
      c.sort_every = S;
      c.use_graph = 0;
      if (pic_batch_set_config(b, &c) != PIC_OK) { rc = PIC_OK; b->err.clear(); continue; }   // does not fit
      if (hipEventRecord(e0, b->stream) != hipSuccess) { rc = bfail(b, PIC_EHIP, "hipEventRecord"); break; }
      for (int k = 0; k < window && rc == PIC_OK; ++k) {
        rc = launch_batch_step(b, b->rel);
        if (rc == PIC_OK) batch_advance_host(b, 1);
      }
      if (rc != PIC_OK) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = bfail(b, PIC_EHIP, "trial timing");
        break;
      }
      const int k = out->n++;
      out->block[k] = c.block;
      out->sort_every[k] = S;
      out->ms_per_step[k] = (double)ms / window;
      if (out->ms_per_step[k] < best) { best = out->ms_per_step[k]; out->best = k; }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != PIC_OK) return rc;
  if (out->n == 0) return bfail(b, PIC_EINVAL, "no candidate fits (window must be a multiple of 10)");
  pic_batch_config c = keep;
  c.block = out->block[out->best];
  c.sort_every = out->sort_every[out->best];
  rc = pic_batch_set_config(b, &c);
  if (rc != PIC_OK) return rc;
  while (b->rel != 0) {                       // finish the rf cycle with the chosen launch shapes
    rc = launch_batch_step(b, b->rel);
    if (rc != PIC_OK) return rc;
    batch_advance_host(b, 1);
  }
  BHIP(b, hipStreamSynchronize(b->stream));
  return PIC_OK;
}

int pic_batch_destroy(pic_batch *b) {
  if (!b) return PIC_EINVAL;
  (void)hipStreamSynchronize(b->stream);
  if (b->on_device) (void)pic_batch_sync(b);
  drop_graph(b);
  for (pic_handle *h : b->mem) h->batch_busy = false;
  delete b;
  return PIC_OK;
}

const char *pic_batch_last_error(const pic_batch *b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

int pic_ksub_select(const pic_config *c, const pic_species *sp, double n_ion_max, double phi_max, int32_t *ksub) {
  if (!c || !sp || !ksub) { g_query_error = "null argument"; return PIC_EINVAL; }
  if (!finite_pos(c->L) || c->ng < 2 || !finite_pos(c->f) || c->steps_per_cycle < 1 ||
      !(std::isfinite(n_ion_max) && n_ion_max >= 0.0) || !(std::isfinite(phi_max) && phi_max >= 0.0)) {
    g_query_error = "need L > 0, ng >= 2, f > 0, steps_per_cycle >= 1, n_ion_max >= 0, phi_max >= 0";
    return PIC_EINVAL;
  }
  for (int s = 1; s < NSP; ++s)
    if (!finite_pos(sp[s].mass)) { g_query_error = "ion masses must be > 0"; return PIC_EINVAL; }
  const double dt = 1.0 / (c->f * c->steps_per_cycle), dx = c->L / c->ng;
  int best = 1;
  for (int k = 1; k <= c->steps_per_cycle; ++k) {
    if (c->steps_per_cycle % k != 0) continue;
    bool ok = true;
    for (int s = 1; s < NSP; ++s) {
      const double M = sp[s].mass;
      const double wpi = std::sqrt(n_ion_max * QE * QE / (EPS0 * M));
      const double vmax = std::sqrt(2.0 * QE * phi_max / M);
      if (wpi * k * dt > 0.2 || vmax * k * dt > dx) ok = false;
    }
    if (!ok) break;                  // both limits grow with k
    best = k;
  }
  *ksub = best;
  return PIC_OK;
}

}  // extern "C"
