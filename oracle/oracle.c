/*
 * FP64 CPU oracle for the 1D3V PIC-MCC oxygen discharge.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain, slow, obviously correct:
 * one particle at a time, one step at a time, in the order of the method.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* SI constants (CODATA 2018; e and k_B exact) */
static const double Q_E = 1.602176634e-19;
static const double K_B = 1.380649e-23;
static const double EPS0 = 8.8541878128e-12;
static const double TWO_PI = 6.283185307179586476925286766559;
static const double TWO32 = 4294967296.0;

#define MAXPROC 16

typedef struct {
  int64_t n, cap;
  double *xi, *vx, *vy, *vz;   /* xi: position in cell units, x = xi * dx */
  uint32_t *id;
  int32_t *cd;                 /* electrons: steps left in the free flight */
  uint8_t *capped, *alive;
  uint8_t *pband;              /* product whose own first draw fell in the band */
  uint64_t *pkey;              /* parent key of a product born this step */
  uint32_t next_id;
} orc_store;

struct orc_sim {
  orc_config c;
  orc_species sp[ORC_NSP];
  int32_t np;
  int32_t neion;               /* processes of Table 1 (16), (22) */
  orc_process pr[MAXPROC];
  double *sigma;               /* np * table_n */
  double dx, dt, n_o2;
  double numax[ORC_NSP];       /* collision-frequency bound per species */
  int64_t step;
  orc_store st[ORC_NSP];
  int64_t *Q;                  /* 3 * (ng+1) charge histograms, 2^-32 units */
  double *phi, *E;
  int64_t cnt[ORC_NCOUNT];
  /* moments */
  double *sumQ, *sumphi;
  int64_t nacc;
  int64_t *esum, *ecnt, *edf, *iedf, ndiag;
  /* pairing work: partners to remove per cell (O2+, O-) */
  int64_t *kcell, *kneg;
  /* event log */
  int32_t logon;
  int64_t nev, evcap, *ev;
  int64_t born_start[ORC_NSP];
  /* current density at the driven electrode, per phase of the rf cycle */
  double *jsum;                /* steps_per_cycle sums [A/m^2] */
  int64_t *jcnt;
  double psum;                 /* sum of U j over the samples [W/m^2] */
  int64_t pn;
  int32_t jvalid;              /* e0_prev, u_prev, abs0_prev hold the previous field solve */
  double e0_prev, u_prev;
  int64_t abs0_prev[ORC_NSP];
  /* spatially resolved O2(a1Delta_g) (section 4's proposed extension) */
  int32_t meta_on, meta_proc;
  double meta_D, meta_nuq, meta_h;
  int64_t *meta_src;           /* CIC tally of the source events, 2^-32 units per node */
  double *na;                  /* O2(a) density at the nodes [m^-3] */
  int64_t meta_step0;          /* step of the last update */
};

/* ------------------------------------------------------------------ */
/* Philox4x32-10 from its published definition: ten rounds of two 32x32->64
   multiplications with the Weyl key schedule. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream of one particle: counter (id, step, species|purpose|block, 0), key = seed. */
static void draw(const orc_sim *S, int s, uint32_t id, int64_t step, int purpose, int block, uint32_t out[4]) {
  uint32_t ctr[4] = {id, (uint32_t)step, ((uint32_t)s << 24) | ((uint32_t)purpose << 16) | (uint32_t)block, 0u};
  uint32_t key[2] = {(uint32_t)S->c.seed, (uint32_t)(S->c.seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

/* uniform in (0,1) from the top 23 bits: (k + 1/2) 2^-23 */
static double unif(uint32_t x) { return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0); }

/* Box-Muller pair */
static void normals(uint32_t a, uint32_t b, double *z0, double *z1) {
  double r = sqrt(-2.0 * log(unif(a)));
  double t = TWO_PI * unif(b);
  *z0 = r * cos(t);
  *z1 = r * sin(t);
}

/* isotropic unit vector: cos(theta) = 1 - 2u, phi = 2 pi u' */
static void iso_dir(uint32_t a, uint32_t b, double d[3]) {
  double ct = 1.0 - 2.0 * unif(a);
  double st = sqrt(fmax(0.0, 1.0 - ct * ct));
  double ph = TWO_PI * unif(b);
  d[0] = ct;
  d[1] = st * cos(ph);
  d[2] = st * sin(ph);
}

/* ------------------------------------------------------------------ */
/* cross-section table: linear in the log-energy index, clamped to the grid,
   zero below the threshold */
static double table_t(const orc_sim *S, double e) {
  double lo = log(S->c.table_emin), hi = log(S->c.table_emax);
  return (log(e) - lo) / ((hi - lo) / (double)(S->c.table_n - 1));
}

double orc_sigma(const orc_sim *S, int32_t p, double e) {
  const orc_process *P = &S->pr[p];
  if (e < P->e_th) return 0.0;
  double t = table_t(S, e);
  int nt = S->c.table_n;
  if (t < 0.0) t = 0.0;
  if (t > (double)(nt - 1)) t = (double)(nt - 1);
  int i = (int)floor(t);
  if (i > nt - 2) i = nt - 2;
  double w = t - (double)i;
  const double *tab = S->sigma + (size_t)p * nt;
  return (1.0 - w) * tab[i] + w * tab[i + 1];
}

static double clamp_e(orc_sim *S, double e) {
  if (e < S->c.table_emin) { S->cnt[ORC_C_CLAMP]++; return S->c.table_emin; }
  if (e > S->c.table_emax) { S->cnt[ORC_C_CLAMP]++; return S->c.table_emax; }
  return e;
}

static double reduced_mass(const orc_sim *S, int p) {
  int s = S->pr[p].species;
  double m = S->sp[s].mass, M = S->pr[p].target_mass;
  if (s == ORC_E) return m;                 /* electrons: target at rest, lab energy */
  return m * M / (m + M);
}

/* number density [m^-3] of ion species s at node j from its charge histogram
   (the end nodes own half a cell) */
static double node_density(const orc_sim *S, int s, int j) {
  double c = S->c.weight / TWO32 / S->dx;
  const int64_t *Qs = S->Q + (size_t)s * (S->c.ng + 1);
  return c * (double)Qs[j] * ((j == 0 || j == S->c.ng) ? 2.0 : 1.0);
}

/* density of the collision partner of process p at position xi; the ion
   partners are read from the grid with the linear weighting of the deposit */
static double target_density(const orc_sim *S, int p, double xi) {
  switch (S->pr[p].target) {
    case ORC_T_O2: return S->n_o2;
    case ORC_T_O2A: {
      if (!S->meta_on) return S->c.c_meta * S->n_o2;
      int j = (int)floor(xi);
      double w = xi - j;
      return (1.0 - w) * S->na[j] + w * S->na[j + 1];
    }
    default: {
      int s = S->pr[p].target == ORC_T_GRIDPOS ? ORC_POS : ORC_NEG;
      int j = (int)floor(xi);
      double w = xi - j;
      return (1.0 - w) * node_density(S, s, j) + w * node_density(S, s, j + 1);
    }
  }
}

/* Table 1 (16) and (22): electron collisions with the ions of the grid */
static int is_eion(const orc_process *P) {
  return P->species == ORC_E && (P->kind == ORC_RECOMB || P->kind == ORC_EDETACH);
}

/* max over the table intervals of sum_p n_p max(sigma_k, sigma_k+1) g(E_k+1),
   over the processes of species s with (eion = 1) or without (eion = 0) the
   electron-ion channels */
static double nu_bound(const orc_sim *S, int s, const double *np_override, int eion) {
  int nt = S->c.table_n;
  double best = 0.0;
  for (int k = 0; k + 1 < nt; ++k) {
    double ek1 = S->c.table_emin * pow(S->c.table_emax / S->c.table_emin, (double)(k + 1) / (double)(nt - 1));
    double sum = 0.0;
    for (int p = 0; p < S->np; ++p) {
      if (S->pr[p].species != s || is_eion(&S->pr[p]) != eion) continue;
      const double *tab = S->sigma + (size_t)p * nt;
      double sm = fmax(tab[k], tab[k + 1]);
      double n = np_override ? np_override[p] : target_density(S, p, 0.0);
      sum += n * sm * sqrt(2.0 * ek1 * Q_E / reduced_mass(S, p));
    }
    if (sum > best) best = sum;
  }
  return best;
}

double orc_nu_max(const orc_sim *S, int32_t s) { return S->numax[s]; }

void orc_info(const orc_sim *S, double *out) {
  out[0] = S->dx; out[1] = S->dt; out[2] = S->n_o2;
  out[3] = S->numax[0]; out[4] = S->numax[1]; out[5] = S->numax[2];
}

/* ------------------------------------------------------------------ */
static void store_reserve(orc_store *a, int64_t need) {
  if (need <= a->cap) return;
  int64_t cap = a->cap ? a->cap : 1024;
  while (cap < need) cap *= 2;
  a->xi = realloc(a->xi, cap * sizeof(double));
  a->vx = realloc(a->vx, cap * sizeof(double));
  a->vy = realloc(a->vy, cap * sizeof(double));
  a->vz = realloc(a->vz, cap * sizeof(double));
  a->id = realloc(a->id, cap * sizeof(uint32_t));
  a->cd = realloc(a->cd, cap * sizeof(int32_t));
  a->capped = realloc(a->capped, cap);
  a->alive = realloc(a->alive, cap);
  a->pband = realloc(a->pband, cap);
  a->pkey = realloc(a->pkey, cap * sizeof(uint64_t));
  a->cap = cap;
}

static int64_t store_push(orc_store *a) {
  store_reserve(a, a->n + 1);
  int64_t i = a->n++;
  a->alive[i] = 1; a->capped[i] = 0; a->cd[i] = 0; a->id[i] = 0; a->pkey[i] = 0; a->pband[i] = 0;
  return i;
}

static void log_event(orc_sim *S, int s, uint32_t id, int64_t code, int64_t band, int64_t aux) {
  if (!S->logon) return;
  if (S->nev == S->evcap) {
    S->evcap = S->evcap ? 2 * S->evcap : 4096;
    S->ev = realloc(S->ev, (size_t)S->evcap * 6 * sizeof(int64_t));
  }
  int64_t *r = S->ev + 6 * S->nev++;
  r[0] = S->step; r[1] = s; r[2] = id; r[3] = code; r[4] = band; r[5] = aux;
}

orc_sim *orc_create(const orc_config *cfg, const orc_species *sp, int32_t nproc, const orc_process *pr,
                    const double *sigma) {
  if (nproc > MAXPROC || cfg->ng < 2 || cfg->table_n < 2) return NULL;
  orc_sim *S = calloc(1, sizeof(orc_sim));
  S->c = *cfg;
  memcpy(S->sp, sp, sizeof(orc_species) * ORC_NSP);
  S->np = nproc;
  memcpy(S->pr, pr, sizeof(orc_process) * nproc);
  for (int p = 0; p < nproc; ++p) S->neion += is_eion(&pr[p]);
  S->sigma = malloc(sizeof(double) * nproc * cfg->table_n);
  memcpy(S->sigma, sigma, sizeof(double) * nproc * cfg->table_n);
  S->dx = cfg->L / cfg->ng;
  S->dt = 1.0 / (cfg->f * cfg->steps_per_cycle);
  S->n_o2 = cfg->p / (K_B * cfg->t_gas);           /* section 2: n = p / kT */
  int nn = cfg->ng + 1;
  S->Q = calloc((size_t)ORC_NSP * nn, sizeof(int64_t));
  S->phi = calloc(nn, sizeof(double));
  S->E = calloc(nn, sizeof(double));
  S->sumQ = calloc((size_t)ORC_NSP * nn, sizeof(double));
  S->sumphi = calloc(nn, sizeof(double));
  S->esum = calloc((size_t)ORC_NSP * cfg->ng, sizeof(int64_t));
  S->ecnt = calloc((size_t)ORC_NSP * cfg->ng, sizeof(int64_t));
  S->edf = calloc((size_t)ORC_NSP * ORC_NBIN, sizeof(int64_t));
  S->iedf = calloc((size_t)ORC_NSP * 2 * ORC_NBIN, sizeof(int64_t));
  S->kcell = calloc(cfg->ng, sizeof(int64_t));
  S->kneg = calloc(cfg->ng, sizeof(int64_t));
  S->meta_src = calloc(nn, sizeof(int64_t));
  S->na = calloc(nn, sizeof(double));
  S->jsum = calloc(cfg->steps_per_cycle, sizeof(double));
  S->jcnt = calloc(cfg->steps_per_cycle, sizeof(int64_t));
  S->numax[ORC_E] = nu_bound(S, ORC_E, NULL, 0);
  S->numax[ORC_POS] = nu_bound(S, ORC_POS, NULL, 0);
  S->numax[ORC_NEG] = 0.0;   /* set at each ion step from the O2+ density */
  return S;
}

void orc_destroy(orc_sim *S) {
  if (!S) return;
  for (int s = 0; s < ORC_NSP; ++s) {
    orc_store *a = &S->st[s];
    free(a->xi); free(a->vx); free(a->vy); free(a->vz); free(a->id); free(a->cd);
    free(a->capped); free(a->alive); free(a->pkey); free(a->pband);
  }
  free(S->sigma); free(S->Q); free(S->phi); free(S->E); free(S->sumQ); free(S->sumphi);
  free(S->esum); free(S->ecnt); free(S->edf); free(S->iedf); free(S->kcell); free(S->kneg); free(S->ev);
  free(S->jsum); free(S->jcnt); free(S->meta_src); free(S->na);
  free(S);
}

/* ------------------------------------------------------------------ */
/* free-flight length in steps: 1 + floor(tau / dt), tau exponential with rate
   nu_max; flights longer than ORC_CD_MAX steps are stored capped and redrawn
   (memoryless) when they expire */
static void new_flight(const orc_sim *S, uint32_t x, int32_t *cd, uint8_t *capped, int64_t *band) {
  double nd = S->numax[ORC_E] * S->dt;
  double tau = nd > 0.0 ? -log(unif(x)) / nd : INFINITY;
  /* decisions within 1e-6 (relative) of an integer step or of the cap lie in the band */
  if (band && isfinite(tau) && fabs(tau - (double)ORC_CD_MAX) < 1e-6 * tau) *band |= 2;
  if (tau >= (double)ORC_CD_MAX) { *cd = ORC_CD_MAX; *capped = 1; return; }
  double fl = floor(tau);
  if (band && (tau - fl < 1e-6 * fmax(1.0, tau) || fl + 1.0 - tau < 1e-6 * fmax(1.0, tau))) *band |= 2;
  *cd = 1 + (int32_t)fl;
  *capped = 0;
}

/* C.5-style uniform loading: positions on the 2^24-point lattice, Maxwellian
   velocities at the species' loading temperature */
void orc_load_uniform(orc_sim *S) {
  for (int s = 0; s < ORC_NSP; ++s) {
    orc_store *a = &S->st[s];
    a->n = 0;
    store_reserve(a, S->sp[s].count);
    double vth = sqrt(S->sp[s].t0_ev * Q_E / S->sp[s].mass);
    for (int64_t k = 0; k < S->sp[s].count; ++k) {
      int64_t i = store_push(a);
      uint32_t id = (uint32_t)k, r0[4], r1[4];
      draw(S, s, id, 0, ORC_P_LOAD, 0, r0);
      draw(S, s, id, 0, ORC_P_LOAD, 1, r1);
      uint64_t lat = (uint64_t)(r0[0] >> 8) * (uint64_t)S->c.ng;   /* lattice point * ng */
      a->xi[i] = (double)(lat >> 24) + (double)(lat & 0xFFFFFFu) / 16777216.0;
      double z0, z1, z2, z3;
      normals(r1[0], r1[1], &z0, &z1);
      normals(r1[2], r1[3], &z2, &z3);
      a->vx[i] = vth * z0; a->vy[i] = vth * z1; a->vz[i] = vth * z2;
      a->id[i] = id;
      if (s == ORC_E) new_flight(S, r0[1], &a->cd[i], &a->capped[i], NULL);
    }
    a->next_id = (uint32_t)S->sp[s].count;
  }
}

/* value of a piecewise-linear profile at x (x / L), constant beyond the end points */
static double profile_at(int32_t n, const double *xs, const double *v, double x) {
  if (x <= xs[0]) return v[0];
  if (x >= xs[n - 1]) return v[n - 1];
  int32_t k = 0;
  while (xs[k + 1] <= x) ++k;
  return v[k] + (v[k + 1] - v[k]) * (x - xs[k]) / (xs[k + 1] - xs[k]);
}

/* Warm-start loading.  Cell j (centre x_c = (j + 1/2) / ng) of species s is
   given round(sum_{i <= j} e_i) - round(sum_{i < j} e_i) particles, e_i =
   n_s(x_c) dx / w the expected number in cell i (rounding half up), with
   offsets on the 2^24-point lattice of the cell and a Maxwellian at
   T = (2/3) mean energy at x_c; particle k keeps the draws of uniform loading. */
int orc_load_profile(orc_sim *S, int32_t n_pts, const double *xs, const double *dens, const double *mean_ev) {
  if (n_pts < 2) return -1;
  for (int32_t k = 0; k < n_pts; ++k) {
    if (!(xs[k] >= 0.0 && xs[k] <= 1.0) || (k > 0 && !(xs[k] > xs[k - 1]))) return -1;
    for (int s = 0; s < ORC_NSP; ++s) {
      double d = dens[s * n_pts + k], e = mean_ev[s * n_pts + k];
      if (!(isfinite(d) && d >= 0.0) || !(isfinite(e) && e > 0.0)) return -1;
    }
  }
  int32_t ng = S->c.ng;
  for (int s = 0; s < ORC_NSP; ++s) {
    orc_store *a = &S->st[s];
    a->n = 0;
    double c = 0.0;
    int64_t prev = 0;
    for (int32_t j = 0; j < ng; ++j) {
      double xc = ((double)j + 0.5) / (double)ng;
      double n = profile_at(n_pts, xs, dens + s * n_pts, xc);
      double t_ev = (2.0 / 3.0) * profile_at(n_pts, xs, mean_ev + s * n_pts, xc);
      c += (n * S->dx) / S->c.weight;
      int64_t cum = (int64_t)floor(c + 0.5);
      double vth = sqrt(t_ev * Q_E / S->sp[s].mass);
      store_reserve(a, cum);
      for (int64_t k = prev; k < cum; ++k) {
        int64_t i = store_push(a);
        uint32_t id = (uint32_t)k, r0[4], r1[4];
        draw(S, s, id, 0, ORC_P_LOAD, 0, r0);
        draw(S, s, id, 0, ORC_P_LOAD, 1, r1);
        a->xi[i] = (double)j + (double)(r0[0] >> 8) / 16777216.0;
        double z0, z1, z2, z3;
        normals(r1[0], r1[1], &z0, &z1);
        normals(r1[2], r1[3], &z2, &z3);
        a->vx[i] = vth * z0; a->vy[i] = vth * z1; a->vz[i] = vth * z2;
        a->id[i] = id;
        if (s == ORC_E) new_flight(S, r0[1], &a->cd[i], &a->capped[i], NULL);
      }
      prev = cum;
    }
    a->next_id = (uint32_t)prev;
  }
  return 0;
}

int orc_set_particles(orc_sim *S, int32_t s, int64_t n, const int32_t *cell, const float *off,
                      const float *vx, const float *vy, const float *vz, const uint32_t *id,
                      const int32_t *cdw, uint32_t next_id) {
  S->jvalid = 0;
  orc_store *a = &S->st[s];
  a->n = 0;
  store_reserve(a, n);
  for (int64_t k = 0; k < n; ++k) {
    int64_t i = store_push(a);
    a->xi[i] = (double)cell[k] + (double)off[k];
    a->vx[i] = vx[k]; a->vy[i] = vy[k]; a->vz[i] = vz[k];
    a->id[i] = id[k];
    if (cdw) { a->cd[i] = cdw[k] & 0x7FFF; a->capped[i] = (cdw[k] & ORC_CD_CAP) ? 1 : 0; }
  }
  a->next_id = next_id;
  return 0;
}

int orc_set_particles64(orc_sim *S, int32_t s, int64_t n, const double *xi, const double *vx,
                        const double *vy, const double *vz, const uint32_t *id, const int32_t *cdw,
                        uint32_t next_id) {
  S->jvalid = 0;
  orc_store *a = &S->st[s];
  a->n = 0;
  store_reserve(a, n);
  for (int64_t k = 0; k < n; ++k) {
    int64_t i = store_push(a);
    a->xi[i] = xi[k]; a->vx[i] = vx[k]; a->vy[i] = vy[k]; a->vz[i] = vz[k];
    a->id[i] = id[k];
    if (cdw) { a->cd[i] = cdw[k] & 0x7FFF; a->capped[i] = (cdw[k] & ORC_CD_CAP) ? 1 : 0; }
  }
  a->next_id = next_id;
  return 0;
}

int64_t orc_count(const orc_sim *S, int32_t s) {
  int64_t c = 0;
  for (int64_t i = 0; i < S->st[s].n; ++i) c += S->st[s].alive[i];
  return c;
}
uint32_t orc_next_id(const orc_sim *S, int32_t s) { return S->st[s].next_id; }

void orc_get_particles(const orc_sim *S, int32_t s, double *xi, double *vx, double *vy, double *vz,
                       uint32_t *id, int32_t *cdw) {
  const orc_store *a = &S->st[s];
  int64_t k = 0;
  for (int64_t i = 0; i < a->n; ++i) {
    if (!a->alive[i]) continue;
    xi[k] = a->xi[i]; vx[k] = a->vx[i]; vy[k] = a->vy[i]; vz[k] = a->vz[i]; id[k] = a->id[i];
    if (cdw) cdw[k] = a->cd[i] | (a->capped[i] ? ORC_CD_CAP : 0);
    ++k;
  }
}

void orc_set_step(orc_sim *S, int64_t step) { S->step = step; S->jvalid = 0; }
int64_t orc_get_step(const orc_sim *S) { return S->step; }

/* ------------------------------------------------------------------ */
/* CIC charge assignment in fixed point: a particle at xi = j + s gives
   2^32 - a to node j and a to node j+1, a = rint(s 2^32) */
static void deposit_one(int64_t *Qs, double xi) {
  double fj = floor(xi);
  int64_t j = (int64_t)fj;
  int64_t a = llrint((xi - fj) * TWO32);
  Qs[j] += (int64_t)4294967296LL - a;
  Qs[j + 1] += a;
}

static void deposit_species(orc_sim *S, int s) {
  int64_t *Qs = S->Q + (size_t)s * (S->c.ng + 1);
  memset(Qs, 0, sizeof(int64_t) * (S->c.ng + 1));
  orc_store *a = &S->st[s];
  for (int64_t i = 0; i < a->n; ++i)
    if (a->alive[i]) deposit_one(Qs, a->xi[i]);
}

void orc_deposit_canonical(int32_t ng, int64_t n, const int32_t *cell, const float *off, int64_t *Q) {
  memset(Q, 0, sizeof(int64_t) * (ng + 1));
  for (int64_t k = 0; k < n; ++k) {
    int64_t a = llrint((double)off[k] * TWO32);
    Q[cell[k]] += (int64_t)4294967296LL - a;
    Q[cell[k] + 1] += a;
  }
}

/* Poisson: -eps0 (phi[j-1] - 2 phi[j] + phi[j+1]) / dx^2 = rho[j], j = 1..ng-1,
   phi[0] = phi0, phi[ng] = 0, by the Thomas algorithm.  Node fields: centred
   differences inside, Gauss's law over the half cells at the electrodes. */
void orc_poisson(int32_t ng, double dx, double phi0, const double *rho, double *phi, double *E) {
  int m = ng - 1;                      /* unknowns phi[1..ng-1] */
  double *cp = malloc(sizeof(double) * (m + 1)), *dp = malloc(sizeof(double) * (m + 1));
  /* row j: -phi[j-1] + 2 phi[j] - phi[j+1] = rho[j] dx^2 / eps0 */
  for (int r = 0; r < m; ++r) {
    int j = r + 1;
    double d = rho[j] * dx * dx / EPS0;
    if (j == 1) d += phi0;
    double a = (r == 0) ? 0.0 : -1.0, b = 2.0, c = (r == m - 1) ? 0.0 : -1.0;
    if (r == 0) { cp[r] = c / b; dp[r] = d / b; }
    else {
      double den = b - a * cp[r - 1];
      cp[r] = c / den;
      dp[r] = (d - a * dp[r - 1]) / den;
    }
  }
  phi[0] = phi0;
  phi[ng] = 0.0;
  for (int r = m - 1; r >= 0; --r) {
    double nxt = (r == m - 1) ? 0.0 : phi[r + 2];
    phi[r + 1] = dp[r] - cp[r] * nxt;
  }
  for (int j = 1; j < ng; ++j) E[j] = (phi[j - 1] - phi[j + 1]) / (2.0 * dx);
  E[0] = (phi[0] - phi[1]) / dx - rho[0] * dx / (2.0 * EPS0);
  E[ng] = (phi[ng - 1] - phi[ng]) / dx + rho[ng] * dx / (2.0 * EPS0);
  free(cp); free(dp);
}

static void field(orc_sim *S) {
  int ng = S->c.ng, nn = ng + 1;
  if (S->c.flags & ORC_F_EXT_FIELD) {
    for (int j = 0; j < nn; ++j) {
      S->E[j] = S->c.e_ext0 + S->c.e_ext1 * (j * S->dx - 0.5 * S->c.L);
      S->phi[j] = 0.0;
    }
    return;
  }
  double *rho = malloc(sizeof(double) * nn);
  double c = Q_E * S->c.weight / TWO32;
  for (int j = 0; j < nn; ++j) {
    double q = 0.0;
    for (int s = 0; s < ORC_NSP; ++s) q += S->sp[s].charge * (double)S->Q[(size_t)s * nn + j];
    double vol = (j == 0 || j == ng) ? 0.5 * S->dx : S->dx;
    rho[j] = c * q / vol;
  }
  double t = (double)S->step * S->dt;
  double phi0 = S->c.U * sin(TWO_PI * S->c.f * t);   /* driven electrode at x = 0 */
  orc_poisson(ng, S->dx, phi0, rho, S->phi, S->E);
  free(rho);
}

/* Section 3: current density through the discharge and power <U j> A.  Between two
   field solves (steps n-1 and n) the current density at x = 0 in +x is the
   displacement part eps0 (E_0^n - E_0^(n-1)) / dt plus the conduction part of the
   charge absorbed at x = 0 in between (moving in -x): -e w sum_s q_s dN_s / dt.
   It is summed at phase (n-1) mod steps_per_cycle; the power sums
   (U^(n-1) + U^n) / 2 times it. */
static void current_sample(orc_sim *S) {
  double e0 = S->E[0];
  double u = S->c.U * sin(TWO_PI * S->c.f * ((double)S->step * S->dt));
  if (S->jvalid) {
    double dq = 0.0;
    for (int s = 0; s < ORC_NSP; ++s) dq += S->sp[s].charge * (double)(S->cnt[ORC_C_ABS0 + s] - S->abs0_prev[s]);
    double j = EPS0 * (e0 - S->e0_prev) / S->dt - Q_E * S->c.weight * dq / S->dt;
    int64_t ph = (S->step - 1) % S->c.steps_per_cycle;
    S->jsum[ph] += j;
    S->jcnt[ph] += 1;
    S->psum += 0.5 * (S->u_prev + u) * j;
    S->pn += 1;
  }
  S->e0_prev = e0;
  S->u_prev = u;
  for (int s = 0; s < ORC_NSP; ++s) S->abs0_prev[s] = S->cnt[ORC_C_ABS0 + s];
  S->jvalid = 1;
}

void orc_prepare(orc_sim *S, int32_t shift) {
  S->jvalid = 0;
  for (int s = 0; s < ORC_NSP; ++s) deposit_species(S, s);
  if (!shift) return;
  field(S);
  for (int s = 0; s < ORC_NSP; ++s) {
    orc_store *a = &S->st[s];
    double dts = S->dt * (s == ORC_E ? 1 : S->c.ksub);
    double qm = S->sp[s].charge * Q_E / S->sp[s].mass;
    for (int64_t i = 0; i < a->n; ++i) {
      if (!a->alive[i]) continue;
      int j = (int)floor(a->xi[i]);
      double w = a->xi[i] - j;
      double Eg = (1.0 - w) * S->E[j] + w * S->E[j + 1];
      a->vx[i] -= qm * Eg * 0.5 * dts;
    }
  }
}

/* ------------------------------------------------------------------ */
static int ebin(double e) {
  if (!(e > 0.0)) return 0;
  int b = (int)floor((log10(e) + 3.0) * (ORC_NBIN / 6.0));
  if (b < 0) b = 0;
  if (b >= ORC_NBIN) b = ORC_NBIN - 1;
  return b;
}

static double kinetic_ev(const orc_sim *S, int s, double vx, double vy, double vz) {
  return 0.5 * S->sp[s].mass * (vx * vx + vy * vy + vz * vz) / Q_E;
}

/* new product of species s at position xi, parent key for id assignment */
static int64_t add_product(orc_sim *S, int s, double xi, double v[3], uint64_t pkey) {
  orc_store *a = &S->st[s];
  int64_t i = store_push(a);
  a->xi[i] = xi; a->vx[i] = v[0]; a->vy[i] = v[1]; a->vz[i] = v[2];
  a->pkey[i] = pkey;
  S->cnt[ORC_C_BORN + s]++;
  return i;
}

static void maxwellian(const orc_sim *S, double mass, const uint32_t r[4], double v[3]) {
  double vt = sqrt(K_B * S->c.t_gas / mass), z0, z1, z2, z3;
  normals(r[0], r[1], &z0, &z1);
  normals(r[2], r[3], &z2, &z3);
  v[0] = vt * z0; v[1] = vt * z1; v[2] = vt * z2;
}

/* electron candidate (free flight ended this step) */
static void collide_electron(orc_sim *S, int64_t i) {
  orc_store *a = &S->st[ORC_E];
  uint32_t id = a->id[i], c[4];
  int64_t band = 0;
  draw(S, ORC_E, id, S->step, ORC_P_CAND, 0, c);
  uint8_t was_capped = a->capped[i];
  new_flight(S, c[0], &a->cd[i], &a->capped[i], &band);
  if (was_capped) { S->cnt[ORC_C_REDRAW]++; log_event(S, ORC_E, id, -2, band, 0); return; }
  S->cnt[ORC_C_CAND + ORC_E]++;
  double me = S->sp[ORC_E].mass;
  double v2 = a->vx[i] * a->vx[i] + a->vy[i] * a->vy[i] + a->vz[i] * a->vz[i];
  double e = 0.5 * me * v2 / Q_E;
  double ec = clamp_e(S, e);
  double g = sqrt(2.0 * ec * Q_E / me);
  double target = unif(c[1]) * S->numax[ORC_E];
  double acc = 0.0;
  int chosen = -1;
  for (int p = 0; p < S->np; ++p) {
    if (S->pr[p].species != ORC_E || is_eion(&S->pr[p])) continue;
    acc += target_density(S, p, a->xi[i]) * orc_sigma(S, p, ec) * g;
    if (fabs(target - acc) < 1e-6 * S->numax[ORC_E]) band |= 1;
    if (chosen < 0 && target < acc) chosen = p;
  }
  log_event(S, ORC_E, id, chosen, band, 0);
  if (chosen < 0) { S->cnt[ORC_C_NULL + ORC_E]++; return; }
  S->cnt[ORC_C_EVENT + chosen]++;
  if (S->meta_on && chosen == S->meta_proc) deposit_one(S->meta_src, a->xi[i]);   /* O2(a) born here */
  const orc_process *P = &S->pr[chosen];
  double d[3], vmag = sqrt(v2);
  iso_dir(c[2], c[3], d);
  double enew;
  if (P->kind == ORC_ELASTIC) {
    double cchi = vmag > 0.0 ? (a->vx[i] * d[0] + a->vy[i] * d[1] + a->vz[i] * d[2]) / vmag : 0.0;
    enew = e * (1.0 - 2.0 * me / P->target_mass * (1.0 - cchi));
  } else if (P->kind == ORC_EXCITE) {
    enew = e - P->e_th;
  } else if (P->kind == ORC_IONIZE) {
    uint32_t p0[4], p1[4];
    draw(S, ORC_E, id, S->step, ORC_P_PROD, 0, p0);
    draw(S, ORC_E, id, S->step, ORC_P_PROD, 1, p1);
    double er = e - P->e_th, r = unif(p0[0]);
    enew = (1.0 - r) * er;
    /* secondary electron */
    double d2[3], v[3];
    iso_dir(p0[1], p0[2], d2);
    double v2m = sqrt(2.0 * r * er * Q_E / me);
    v[0] = v2m * d2[0]; v[1] = v2m * d2[1]; v[2] = v2m * d2[2];
    int64_t k = add_product(S, ORC_E, a->xi[i], v, ((uint64_t)ORC_E << 32) | id);
    int64_t pb = 0;
    new_flight(S, p0[3], &a->cd[k], &a->capped[k], &pb);
    a->pband[k] = pb != 0;
    /* new O2+ from the 300 K reservoir */
    maxwellian(S, S->sp[ORC_POS].mass, p1, v);
    add_product(S, ORC_POS, a->xi[i], v, ((uint64_t)ORC_E << 32) | id);
  } else { /* ORC_ATTACH: electron captured, O- appears */
    uint32_t p1[4];
    double v[3];
    draw(S, ORC_E, id, S->step, ORC_P_PROD, 1, p1);
    maxwellian(S, S->sp[ORC_NEG].mass, p1, v);
    add_product(S, ORC_NEG, a->xi[i], v, ((uint64_t)ORC_E << 32) | id);
    a->alive[i] = 0;
    return;
  }
  if (enew < 0.0) enew = 0.0;
  double vn = sqrt(2.0 * enew * Q_E / me);
  a->vx[i] = vn * d[0]; a->vy[i] = vn * d[1]; a->vz[i] = vn * d[2];
}

/* ion candidate test (per ion step, probability 1 - exp(-nu_max dt_i)) */
static void collide_ion(orc_sim *S, int s, int64_t i, double dts) {
  orc_store *a = &S->st[s];
  uint32_t id = a->id[i], c[4];
  int64_t band = 0;
  draw(S, s, id, S->step, ORC_P_CAND, 0, c);
  double pnull = 1.0 - exp(-S->numax[s] * dts);
  double u0 = unif(c[0]);
  if (fabs(u0 - pnull) < 1e-6) band |= 8;
  if (!(u0 < pnull)) { if (band) log_event(S, s, id, -4, band, 0); return; }
  S->cnt[ORC_C_CAND + s]++;
  uint32_t t[4];
  draw(S, s, id, S->step, ORC_P_TARGET, 0, t);
  double z0, z1, z2, z3;
  normals(t[0], t[1], &z0, &z1);
  normals(t[2], t[3], &z2, &z3);
  double m = S->sp[s].mass;
  double target = unif(c[1]) * S->numax[s];
  double acc = 0.0, erel_chosen = 0.0, vt_chosen[3] = {0, 0, 0};
  int chosen = -1;
  for (int p = 0; p < S->np; ++p) {
    if (S->pr[p].species != s) continue;
    double M = S->pr[p].target_mass, mu = m * M / (m + M);
    double vt = sqrt(K_B * S->c.t_gas / M);
    double vp[3] = {vt * z0, vt * z1, vt * z2};
    double gx = a->vx[i] - vp[0], gy = a->vy[i] - vp[1], gz = a->vz[i] - vp[2];
    double erel = 0.5 * mu * (gx * gx + gy * gy + gz * gz) / Q_E;   /* relative energy */
    double ec = clamp_e(S, erel);
    double g = sqrt(2.0 * ec * Q_E / mu);
    acc += target_density(S, p, a->xi[i]) * orc_sigma(S, p, ec) * g;
    if (fabs(target - acc) < 1e-6 * S->numax[s]) band |= 1;
    if (chosen < 0 && target < acc) {
      chosen = p; erel_chosen = erel;
      vt_chosen[0] = vp[0]; vt_chosen[1] = vp[1]; vt_chosen[2] = vp[2];
    }
  }
  log_event(S, s, id, chosen, band, 0);
  if (chosen < 0) { S->cnt[ORC_C_NULL + s]++; return; }
  S->cnt[ORC_C_EVENT + chosen]++;
  const orc_process *P = &S->pr[chosen];
  if (P->kind == ORC_CX) {
    /* charge transfer: the ion continues with the neutral partner's velocity */
    a->vx[i] = vt_chosen[0]; a->vy[i] = vt_chosen[1]; a->vz[i] = vt_chosen[2];
  } else if (P->kind == ORC_NEUTRALIZE) {
    a->alive[i] = 0;
    S->kcell[(int)floor(a->xi[i])]++;
  } else if (P->kind == ORC_ION_ELASTIC) {
    /* Table 1 (8): elastic scattering on the sampled neutral, isotropic in the
       centre-of-mass frame: v' = v_cm + M / (m + M) |g| n, n from the PROD draw */
    uint32_t p0[4];
    draw(S, s, id, S->step, ORC_P_PROD, 0, p0);
    double M = P->target_mass, d[3];
    double g[3] = {a->vx[i] - vt_chosen[0], a->vy[i] - vt_chosen[1], a->vz[i] - vt_chosen[2]};
    double gm = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    iso_dir(p0[0], p0[1], d);
    double f = M / (m + M);
    double vcm[3];
    for (int k = 0; k < 3; ++k) vcm[k] = (m * (k == 0 ? a->vx[i] : k == 1 ? a->vy[i] : a->vz[i]) + M * vt_chosen[k]) / (m + M);
    a->vx[i] = vcm[0] + f * gm * d[0];
    a->vy[i] = vcm[1] + f * gm * d[1];
    a->vz[i] = vcm[2] + f * gm * d[2];
  } else if (P->kind == ORC_DETACH) {
    /* Table 1 (19), (20): O- + O2 -> O + O2 + e and O- + O2(a) -> O3 + e; the
       electron carries the relative energy in excess of the threshold */
    uint32_t p0[4];
    draw(S, s, id, S->step, ORC_P_PROD, 0, p0);
    double d[3], v[3];
    iso_dir(p0[1], p0[2], d);
    double vm = sqrt(2.0 * fmax(erel_chosen - P->e_th, 0.0) * Q_E / S->sp[ORC_E].mass);
    v[0] = vm * d[0]; v[1] = vm * d[1]; v[2] = vm * d[2];
    int64_t k = add_product(S, ORC_E, a->xi[i], v, ((uint64_t)s << 32) | id);
    int64_t pb = 0;
    new_flight(S, p0[3], &S->st[ORC_E].cd[k], &S->st[ORC_E].capped[k], &pb);
    S->st[ORC_E].pband[k] = pb != 0;
    a->alive[i] = 0;
  }
}

static void push_species(orc_sim *S, int s, int64_t nstart) {
  orc_store *a = &S->st[s];
  double dts = S->dt * (s == ORC_E ? 1 : S->c.ksub);
  double qm = S->sp[s].charge * Q_E / S->sp[s].mass;
  double ng = (double)S->c.ng;
  for (int64_t i = 0; i < nstart; ++i) {
    if (!a->alive[i]) continue;
    S->cnt[ORC_C_PUSH + s]++;
    /* gather (linear weighting), leapfrog velocity then position */
    int j = (int)floor(a->xi[i]);
    double w = a->xi[i] - j;
    double Eg = (1.0 - w) * S->E[j] + w * S->E[j + 1];
    a->vx[i] += qm * Eg * dts;
    a->xi[i] += a->vx[i] * dts / S->dx;
    double xi = a->xi[i];
    if (xi < 0.0 || xi >= ng) {                   /* absorbing electrodes */
      int side = xi < 0.0 ? 0 : 1;
      int64_t band = (fabs(xi) < 1e-6 * ng || fabs(xi - ng) < 1e-6 * ng) ? 4 : 0;
      double e = kinetic_ev(S, s, a->vx[i], a->vy[i], a->vz[i]);
      S->cnt[(side ? ORC_C_ABSL : ORC_C_ABS0) + s]++;
      S->iedf[((size_t)s * 2 + side) * ORC_NBIN + ebin(e)]++;
      a->alive[i] = 0;
      log_event(S, s, a->id[i], -3, band, side);
      continue;
    }
    if (S->c.flags & ORC_F_NO_COLL) continue;
    if (s == ORC_E) {
      if (--a->cd[i] > 0) continue;
      collide_electron(S, i);
    } else {
      collide_ion(S, s, i, dts);
    }
  }
}

/* partners of the ion removals of this ion step: in every cell j with k[j]
   removals, the k[j] ions of species s with the smallest key (pairing draw, id)
   among those that were there before the step and are alive after its pushes;
   a cell holding fewer gives all it has and the rest is counted as a deficit.
   Each removal of Table 1 (16), (17) or (22) thus takes exactly one partner.
   O2+ partners of neutralisation (17) and recombination (16), O- partners of
   electron-impact detachment (22). */
typedef struct { int64_t cell; uint64_t key; int64_t i; } pair_cand;

static int cmp_pair(const void *x, const void *y) {
  const pair_cand *a = (const pair_cand *)x, *b = (const pair_cand *)y;
  if (a->cell != b->cell) return a->cell < b->cell ? -1 : 1;
  return a->key < b->key ? -1 : a->key > b->key;
}

static void pairing(orc_sim *S, int s, int64_t nstart_s, int64_t *k_cell, int c_paired, int c_deficit) {
  int ng = S->c.ng;
  orc_store *a = &S->st[s];
  int64_t want = 0;
  for (int j = 0; j < ng; ++j) want += k_cell[j];
  if (want == 0) return;
  /* every candidate partner of a cell with removals, sorted by (cell, key) */
  pair_cand *c = malloc(sizeof(pair_cand) * (size_t)(nstart_s > 0 ? nstart_s : 1));
  int64_t nc = 0;
  for (int64_t i = 0; i < nstart_s; ++i) {
    if (!a->alive[i]) continue;
    int j = (int)floor(a->xi[i]);
    if (k_cell[j] == 0) continue;
    uint32_t d[4];
    draw(S, s, a->id[i], S->step, ORC_P_PAIR, 0, d);
    c[nc].cell = j;
    c[nc].key = ((uint64_t)d[0] << 32) | a->id[i];
    c[nc].i = i;
    ++nc;
  }
  qsort(c, (size_t)nc, sizeof(pair_cand), cmp_pair);
  /* the first k[j] of each cell's run are removed */
  for (int64_t r = 0; r < nc;) {
    int64_t j = c[r].cell, e = r;
    while (e < nc && c[e].cell == j) ++e;
    int64_t take = k_cell[j] < e - r ? k_cell[j] : e - r;
    for (int64_t q = r; q < r + take; ++q) a->alive[c[q].i] = 0;
    S->cnt[c_paired] += take;
    k_cell[j] -= take;
    r = e;
  }
  for (int j = 0; j < ng; ++j) {
    S->cnt[c_deficit] += k_cell[j];
    k_cell[j] = 0;
  }
  free(c);
}

/* Table 1 (16) e + O2+ -> O + O and (22) e + O- -> O + 2e.  Once per ion step,
   after the electron push, every electron present at the start of the step is
   a candidate with probability 1 - exp(-nu_ei ksub dt): nu_ei bounds
   sum_p n_p(x) sigma_p(E) g over the gap with the largest node densities of the
   field solve, the ion taken at rest (g = electron speed, E its energy).  The
   channel follows from u nu_ei against the running sum at the electron's
   position.  (16): electron and an O2+ of its cell removed.  (22): E - E_th
   shared by the two electrons as (1 - r, r), both isotropic; an O- of the cell
   removed.  Partners go to the pairing. */
static void eion_pass(orc_sim *S, int64_t n_e) {
  int nn = S->c.ng + 1;
  double nmax[ORC_NSP] = {0.0, 0.0, 0.0};
  for (int s = ORC_POS; s <= ORC_NEG; ++s)
    for (int j = 0; j < nn; ++j) nmax[s] = fmax(nmax[s], node_density(S, s, j));
  double nover[MAXPROC];
  for (int p = 0; p < S->np; ++p)
    nover[p] = !is_eion(&S->pr[p]) ? 0.0 : nmax[S->pr[p].target == ORC_T_GRIDPOS ? ORC_POS : ORC_NEG];
  double nu = nu_bound(S, ORC_E, nover, 1);
  double pnull = 1.0 - exp(-nu * S->dt * S->c.ksub);
  double me = S->sp[ORC_E].mass;
  orc_store *a = &S->st[ORC_E];
  for (int64_t i = 0; i < n_e; ++i) {
    if (!a->alive[i]) continue;
    uint32_t id = a->id[i], c[4];
    int64_t band = 0;
    draw(S, ORC_E, id, S->step, ORC_P_EION, 0, c);
    double u0 = unif(c[0]);
    if (fabs(u0 - pnull) < 1e-6) band |= 8;
    if (!(u0 < pnull)) { if (band) log_event(S, ORC_EV_EION, id, -4, band, 0); continue; }
    S->cnt[ORC_C_EICAND]++;
    double v2 = a->vx[i] * a->vx[i] + a->vy[i] * a->vy[i] + a->vz[i] * a->vz[i];
    double e = 0.5 * me * v2 / Q_E;
    double ec = clamp_e(S, e);
    double g = sqrt(2.0 * ec * Q_E / me);
    double target = unif(c[1]) * nu, acc = 0.0;
    int chosen = -1;
    for (int p = 0; p < S->np; ++p) {
      if (!is_eion(&S->pr[p])) continue;
      acc += target_density(S, p, a->xi[i]) * orc_sigma(S, p, ec) * g;
      if (fabs(target - acc) < 1e-6 * nu) band |= 1;
      if (chosen < 0 && target < acc) chosen = p;
    }
    log_event(S, ORC_EV_EION, id, chosen, band, 0);
    if (chosen < 0) { S->cnt[ORC_C_EINULL]++; continue; }
    S->cnt[ORC_C_EVENT + chosen]++;
    int j = (int)floor(a->xi[i]);
    if (S->pr[chosen].kind == ORC_RECOMB) {
      a->alive[i] = 0;
      S->kcell[j]++;
    } else {
      uint32_t p0[4];
      draw(S, ORC_E, id, S->step, ORC_P_EION, 1, p0);
      double er = fmax(e - S->pr[chosen].e_th, 0.0), r = unif(p0[0]);
      double d[3], d2[3], v[3];
      iso_dir(c[2], c[3], d);
      double vn = sqrt(2.0 * (1.0 - r) * er * Q_E / me);
      a->vx[i] = vn * d[0]; a->vy[i] = vn * d[1]; a->vz[i] = vn * d[2];
      iso_dir(p0[1], p0[2], d2);
      double v2m = sqrt(2.0 * r * er * Q_E / me);
      v[0] = v2m * d2[0]; v[1] = v2m * d2[1]; v[2] = v2m * d2[2];
      int64_t k = add_product(S, ORC_E, a->xi[i], v, ((uint64_t)ORC_EV_EION << 32) | id);
      int64_t pb = 0;
      new_flight(S, p0[3], &a->cd[k], &a->capped[k], &pb);
      a->pband[k] = pb != 0;
      S->kneg[j]++;
    }
  }
}

/* ids of this step's products: per species, next_id + rank in (parent species, parent id) */
static int cmp_u64(const void *x, const void *y) {
  uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
  return a < b ? -1 : a > b;
}

static void assign_ids(orc_sim *S) {
  for (int s = 0; s < ORC_NSP; ++s) {
    orc_store *a = &S->st[s];
    int64_t b = S->born_start[s], nb = a->n - b;
    if (nb <= 0) continue;
    uint64_t *keys = malloc(sizeof(uint64_t) * nb);
    for (int64_t k = 0; k < nb; ++k) keys[k] = a->pkey[b + k];
    qsort(keys, nb, sizeof(uint64_t), cmp_u64);
    for (int64_t k = 0; k < nb; ++k) {
      /* rank of this product's key among the sorted keys (keys are unique) */
      uint64_t *hit = bsearch(&a->pkey[b + k], keys, nb, sizeof(uint64_t), cmp_u64);
      a->id[b + k] = a->next_id + (uint32_t)(hit - keys);
      if (a->pband[b + k]) log_event(S, s, a->id[b + k], -5, 2, 0);   /* product's own draw in the band */
    }
    a->next_id += (uint32_t)nb;
    free(keys);
  }
}

static void compact(orc_sim *S) {
  for (int s = 0; s < ORC_NSP; ++s) {
    orc_store *a = &S->st[s];
    int64_t k = 0;
    for (int64_t i = 0; i < a->n; ++i) {
      if (!a->alive[i]) continue;
      if (k != i) {
        a->xi[k] = a->xi[i]; a->vx[k] = a->vx[i]; a->vy[k] = a->vy[i]; a->vz[k] = a->vz[i];
        a->id[k] = a->id[i]; a->cd[k] = a->cd[i]; a->capped[k] = a->capped[i];
        a->alive[k] = 1; a->pkey[k] = a->pkey[i]; a->pband[k] = 0;
      }
      ++k;
    }
    a->n = k;
  }
}

static void diagnostics(orc_sim *S) {
  int ng = S->c.ng;
  for (int s = 0; s < ORC_NSP; ++s) {
    orc_store *a = &S->st[s];
    for (int64_t i = 0; i < a->n; ++i) {
      if (!a->alive[i]) continue;
      double e = kinetic_ev(S, s, a->vx[i], a->vy[i], a->vz[i]);
      int j = (int)floor(a->xi[i]);
      S->esum[(size_t)s * ng + j] += llrint(e * 1048576.0);   /* 2^-20 eV units */
      S->ecnt[(size_t)s * ng + j] += 1;
      S->edf[(size_t)s * ORC_NBIN + ebin(e)] += 1;
    }
  }
  S->ndiag++;
}

static void one_step(orc_sim *S) {
  int ng = S->c.ng, nn = ng + 1;
  /* 1. field from the charge left by the previous step; moments of that state */
  field(S);
  current_sample(S);
  for (int k = 0; k < ORC_NSP * nn; ++k) S->sumQ[k] += (double)S->Q[k];
  for (int j = 0; j < nn; ++j) S->sumphi[j] += S->phi[j];
  S->nacc++;
  if (S->c.diag_every > 0 && S->step % S->c.diag_every == 0) diagnostics(S);
  int64_t nstart[ORC_NSP];
  for (int s = 0; s < ORC_NSP; ++s) { nstart[s] = S->st[s].n; S->born_start[s] = S->st[s].n; }
  /* 2. electrons, every step */
  push_species(S, ORC_E, nstart[ORC_E]);
  int ion_step = (S->step % S->c.ksub) == 0;
  if (ion_step && S->neion > 0 && !(S->c.flags & ORC_F_NO_COLL)) eion_pass(S, nstart[ORC_E]);
  if (ion_step) {
    /* 3. O2+ then O- with dt_i = ksub dt and this step's field */
    push_species(S, ORC_POS, nstart[ORC_POS]);
    deposit_species(S, ORC_POS);
    /* bound for O-: the largest O2+ node density right now */
    double nmax = 0.0, c = S->c.weight / TWO32 / S->dx;
    const int64_t *Qp = S->Q + (size_t)ORC_POS * nn;
    for (int j = 0; j < nn; ++j) {
      double nj = c * (double)Qp[j] * ((j == 0 || j == ng) ? 2.0 : 1.0);
      if (nj > nmax) nmax = nj;
    }
    double nover[MAXPROC];
    double namax = 0.0;
    for (int j = 0; S->meta_on && j < nn; ++j) namax = fmax(namax, S->na[j]);
    for (int p = 0; p < S->np; ++p)
      nover[p] = S->pr[p].target == ORC_T_GRIDPOS ? nmax
               : (S->pr[p].target == ORC_T_O2A && S->meta_on) ? namax : target_density(S, p, 0.0);
    S->numax[ORC_NEG] = nu_bound(S, ORC_NEG, nover, 0);
    push_species(S, ORC_NEG, nstart[ORC_NEG]);
    pairing(S, ORC_POS, nstart[ORC_POS], S->kcell, ORC_C_PAIRED, ORC_C_DEFICIT);
    pairing(S, ORC_NEG, nstart[ORC_NEG], S->kneg, ORC_C_PAIRED_NEG, ORC_C_DEFICIT_NEG);
    deposit_species(S, ORC_POS);
    deposit_species(S, ORC_NEG);
  } else {
    /* ions stay put between ion steps; newborn ions add their charge */
    for (int s = ORC_POS; s <= ORC_NEG; ++s) {
      int64_t *Qs = S->Q + (size_t)s * nn;
      for (int64_t i = nstart[s]; i < S->st[s].n; ++i)
        if (S->st[s].alive[i]) deposit_one(Qs, S->st[s].xi[i]);
    }
  }
  deposit_species(S, ORC_E);
  assign_ids(S);
  compact(S);
  S->step++;
}

void orc_step(orc_sim *S, int64_t nsteps) {
  for (int64_t k = 0; k < nsteps; ++k) one_step(S);
}

/* ------------------------------------------------------------------ */
void orc_get_hist(const orc_sim *S, int64_t *Q) {
  memcpy(Q, S->Q, sizeof(int64_t) * ORC_NSP * (S->c.ng + 1));
}
/* test hook: histograms of a larger state, for pushing a sample of its particles */
void orc_set_hist(orc_sim *S, const int64_t *Q) {
  memcpy(S->Q, Q, sizeof(int64_t) * ORC_NSP * (S->c.ng + 1));
}

void orc_get_field(const orc_sim *S, double *phi, double *E) {
  if (phi) memcpy(phi, S->phi, sizeof(double) * (S->c.ng + 1));
  if (E) memcpy(E, S->E, sizeof(double) * (S->c.ng + 1));
}
void orc_get_counters(const orc_sim *S, int64_t *out) { memcpy(out, S->cnt, sizeof(S->cnt)); }

void orc_reset_moments(orc_sim *S) {
  int ng = S->c.ng, nn = ng + 1;
  memset(S->sumQ, 0, sizeof(double) * ORC_NSP * nn);
  memset(S->sumphi, 0, sizeof(double) * nn);
  memset(S->esum, 0, sizeof(int64_t) * ORC_NSP * ng);
  memset(S->ecnt, 0, sizeof(int64_t) * ORC_NSP * ng);
  memset(S->edf, 0, sizeof(int64_t) * ORC_NSP * ORC_NBIN);
  memset(S->iedf, 0, sizeof(int64_t) * ORC_NSP * 2 * ORC_NBIN);
  S->nacc = 0;
  S->ndiag = 0;
  memset(S->jsum, 0, sizeof(double) * S->c.steps_per_cycle);
  memset(S->jcnt, 0, sizeof(int64_t) * S->c.steps_per_cycle);
  S->psum = 0.0;
  S->pn = 0;
}

/* test hook: adds one sample of the energy moments of the current state (what
   a step with diag_every hitting records before it moves anything) */
void orc_sample_moments(orc_sim *S) { diagnostics(S); }

void orc_get_current(const orc_sim *S, double *jsum, int64_t *jcnt, double *psum, int64_t *pn) {
  if (jsum) memcpy(jsum, S->jsum, sizeof(double) * S->c.steps_per_cycle);
  if (jcnt) memcpy(jcnt, S->jcnt, sizeof(int64_t) * S->c.steps_per_cycle);
  if (psum) *psum = S->psum;
  if (pn) *pn = S->pn;
}

int64_t orc_get_moments(const orc_sim *S, double *sumQ, double *sumphi, int64_t *esum, int64_t *ecnt,
                        int64_t *edf, int64_t *iedf, int64_t *ndiag) {
  int ng = S->c.ng, nn = ng + 1;
  if (sumQ) memcpy(sumQ, S->sumQ, sizeof(double) * ORC_NSP * nn);
  if (sumphi) memcpy(sumphi, S->sumphi, sizeof(double) * nn);
  if (esum) memcpy(esum, S->esum, sizeof(int64_t) * ORC_NSP * ng);
  if (ecnt) memcpy(ecnt, S->ecnt, sizeof(int64_t) * ORC_NSP * ng);
  if (edf) memcpy(edf, S->edf, sizeof(int64_t) * ORC_NSP * ORC_NBIN);
  if (iedf) memcpy(iedf, S->iedf, sizeof(int64_t) * ORC_NSP * 2 * ORC_NBIN);
  if (ndiag) *ndiag = S->ndiag;
  return S->nacc;
}

/* ------------------------------------------------------------------ */
/* Spatially resolved O2(a1Delta_g), the extension section 4 proposes for the
   uniform n = C n(O2) of Eq. (1).  Steady state of
       D n'' - nu_q n + P(x) = 0,  0 < x < L,
   with the surface loss of the electrodes, flux gamma v / (2 (2 - gamma)) n
   (v the mean speed of the molecule), and P the production by the electron
   channel meta_proc (Table 1 (14)) tallied since the last update.  Finite
   volumes on the nodes (half volumes at the electrodes), FP64, tridiagonal. */
int orc_metastable_config(orc_sim *S, int32_t proc, double D, double nu_q, double gamma) {
  if (proc < 0 || proc >= S->np || S->pr[proc].species != ORC_E || S->pr[proc].kind != ORC_EXCITE) return -1;
  if (!(D > 0.0) || !(nu_q >= 0.0) || !(gamma >= 0.0 && gamma <= 1.0) || (gamma == 0.0 && nu_q == 0.0)) return -1;
  double M = S->pr[proc].target_mass;
  double vbar = sqrt(8.0 * K_B * S->c.t_gas / (0.5 * TWO_PI * M));   /* mean molecular speed */
  S->meta_on = 1;
  S->meta_proc = proc;
  S->meta_D = D;
  S->meta_nuq = nu_q;
  S->meta_h = gamma * vbar / (2.0 * (2.0 - gamma));
  int nn = S->c.ng + 1;
  for (int j = 0; j < nn; ++j) { S->na[j] = S->c.c_meta * S->n_o2; S->meta_src[j] = 0; }
  S->meta_step0 = S->step;
  return 0;
}

/* tridiagonal solve a_j x_{j-1} + b_j x_j + c_j x_{j+1} = r_j (Thomas) */
static void thomas(int n, const double *a, const double *b, const double *c, const double *r, double *x) {
  double *cp = malloc(sizeof(double) * n), *rp = malloc(sizeof(double) * n);
  cp[0] = c[0] / b[0];
  rp[0] = r[0] / b[0];
  for (int j = 1; j < n; ++j) {
    double m = b[j] - a[j] * cp[j - 1];
    cp[j] = c[j] / m;
    rp[j] = (r[j] - a[j] * rp[j - 1]) / m;
  }
  x[n - 1] = rp[n - 1];
  for (int j = n - 2; j >= 0; --j) x[j] = rp[j] - cp[j] * x[j + 1];
  free(cp); free(rp);
}

/* the steady profile for a production rate given per node [m^-3 s^-1] */
void orc_metastable_solve(int32_t ng, double dx, double D, double nu_q, double h, const double *prod, double *n) {
  int nn = ng + 1;
  double *a = calloc(nn, sizeof(double)), *b = calloc(nn, sizeof(double)), *c = calloc(nn, sizeof(double));
  double k = D / (dx * dx);
  for (int j = 1; j < ng; ++j) { a[j] = k; b[j] = -2.0 * k - nu_q; c[j] = k; }
  /* electrode nodes own half a cell: (D (n1 - n0) / dx - h n0) / (dx / 2) - nu_q n0 + P0 = 0 */
  b[0] = -2.0 * k - 2.0 * h / dx - nu_q; c[0] = 2.0 * k;
  a[ng] = 2.0 * k; b[ng] = -2.0 * k - 2.0 * h / dx - nu_q;
  double *r = malloc(sizeof(double) * nn);
  for (int j = 0; j < nn; ++j) r[j] = -prod[j];
  thomas(nn, a, b, c, r, n);
  free(a); free(b); free(c); free(r);
}

int orc_metastable_update(orc_sim *S, double *n_out) {
  if (!S->meta_on) return -1;
  int ng = S->c.ng, nn = ng + 1;
  double tau = (double)(S->step - S->meta_step0) * S->dt;
  if (!(tau > 0.0)) return -1;
  double *prod = malloc(sizeof(double) * nn);
  for (int j = 0; j < nn; ++j) {
    double vol = (j == 0 || j == ng) ? 0.5 * S->dx : S->dx;
    prod[j] = S->c.weight * ((double)S->meta_src[j] / TWO32) / (vol * tau);
    S->meta_src[j] = 0;
  }
  orc_metastable_solve(ng, S->dx, S->meta_D, S->meta_nuq, S->meta_h, prod, S->na);
  free(prod);
  S->meta_step0 = S->step;
  if (n_out) memcpy(n_out, S->na, sizeof(double) * nn);
  return 0;
}

/* test hook: a given O2(a) profile (after a config) */
int orc_metastable_set(orc_sim *S, const double *na) {
  if (!S->meta_on) return -1;
  memcpy(S->na, na, sizeof(double) * (S->c.ng + 1));
  return 0;
}

void orc_metastable_tally(const orc_sim *S, int64_t *src) {
  memcpy(src, S->meta_src, sizeof(int64_t) * (S->c.ng + 1));
}

void orc_log_events(orc_sim *S, int32_t on) { S->logon = on; S->nev = 0; }

int64_t orc_get_events(orc_sim *S, int64_t max, int64_t *rec) {
  int64_t n = S->nev < max ? S->nev : max;
  if (rec) memcpy(rec, S->ev, sizeof(int64_t) * 6 * n);
  return S->nev;
}
