/*
 * FP64 CPU oracle for the 1D3V PIC-MCC oxygen discharge.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the HIP path; both sides receive the same
 * input data (discharge parameters, species data, cross-section tables,
 * canonical particle states) and each implements the counter-based generator
 * Philox4x32-10 from its published definition (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11).
 *
 * Paper: Bronold, Matyash, Tskhakaya, Schneider, Fehske, "Particle-based
 * modeling of oxygen discharges" (ICPIG 2007).  Section 1: particle solution of
 * the Boltzmann-Poisson system, chemistry linked to the field through the
 * Poisson source term.  Section 2: 1D gap with three velocity components, one
 * electrode at U sin(2 pi f t), the other at 0, both absorbing, O2 reservoir at
 * n = p/kT with T = 300 K; free flights between collisions whose durations and
 * channel probabilities follow from the cross sections; species e, O-, O2+;
 * Table 1 channels; Eq. (1) for associative detachment with n(O2(a)) = C n(O2).
 *
 * Everything is FP64 except the canonical exchange format, which is the
 * single-precision particle record (cell, offset, vx, vy, vz, id, countdown).
 */
#ifndef PICMCC_ORACLE_H
#define PICMCC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_E = 0, ORC_POS = 1, ORC_NEG = 2, ORC_NSP = 3 };
enum { ORC_ELASTIC = 0, ORC_EXCITE = 1, ORC_IONIZE = 2, ORC_ATTACH = 3,
       ORC_CX = 4, ORC_NEUTRALIZE = 5, ORC_DETACH = 6, ORC_ION_ELASTIC = 7,
       ORC_RECOMB = 8,      /* e + O2+ -> O + O, Table 1 (16) */
       ORC_EDETACH = 9 };   /* e + O- -> O + 2e, Table 1 (22) */
enum { ORC_T_O2 = 0, ORC_T_O2A = 1, ORC_T_GRIDPOS = 2, ORC_T_GRIDNEG = 3 };
enum { ORC_P_LOAD = 1, ORC_P_CAND = 2, ORC_P_TARGET = 3, ORC_P_PROD = 4, ORC_P_PAIR = 5, ORC_P_EION = 6 };
/* species field of the event records of the electron-ion test */
enum { ORC_EV_EION = 3 };

/* flags */
#define ORC_F_EXT_FIELD  1   /* field = e_ext0 + e_ext1 (x - L/2) instead of Poisson */
#define ORC_F_NO_COLL    2   /* collisions off */

#define ORC_CD_MAX   32767   /* longest stored free flight, in steps */
#define ORC_CD_CAP   0x8000  /* canonical countdown word: bit 15 = capped flight */
#define ORC_NBIN     256     /* log energy bins, 1e-3 .. 1e3 eV */

/* counters (int64) */
enum {
  ORC_C_PUSH = 0,      /* +s: particles pushed */
  ORC_C_CAND = 3,      /* +s: collision candidates */
  ORC_C_NULL = 6,      /* +s: null collisions */
  ORC_C_ABS0 = 9,      /* +s: absorbed at x = 0 */
  ORC_C_ABSL = 12,     /* +s: absorbed at x = L */
  ORC_C_BORN = 15,     /* +s: products born */
  ORC_C_EVENT = 18,    /* +p (p < 16): real events per process */
  ORC_C_PAIRED = 34,   /* O2+ removed by pairing */
  ORC_C_DEFICIT = 35,  /* neutralisations without a partner */
  ORC_C_CLAMP = 36,    /* energies clamped to the table range */
  ORC_C_REDRAW = 37,   /* capped free flights redrawn */
  ORC_C_EICAND = 38,   /* electron-ion candidates */
  ORC_C_EINULL = 39,   /* electron-ion null collisions */
  ORC_C_PAIRED_NEG = 40,   /* O- removed as partners of electron-impact detachment */
  ORC_C_DEFICIT_NEG = 41,  /* electron-impact detachments without an O- partner */
  ORC_NCOUNT = 44
};

typedef struct {
  double L;               /* gap [m] */
  int32_t ng;             /* cells */
  double U;               /* voltage amplitude [V] */
  double f;               /* frequency [Hz] */
  double p;               /* pressure [Pa] */
  double t_gas;           /* gas temperature [K] */
  int32_t steps_per_cycle;
  int32_t ksub;           /* ion subcycling factor */
  double c_meta;          /* n(O2(a)) = c_meta * n(O2) */
  uint64_t seed;
  double weight;          /* physical particles per superparticle per m^2 */
  int32_t diag_every;     /* energy moments every D steps (0: never) */
  int32_t flags;
  double e_ext0, e_ext1;  /* external field hook [V/m], [V/m^2] */
  double table_emin, table_emax;
  int32_t table_n;
} orc_config;

typedef struct {
  double charge;          /* units of e */
  double mass;            /* kg */
  double t0_ev;           /* loading temperature [eV] */
  int64_t count;          /* superparticles loaded */
  int64_t capacity;       /* unused by the oracle (it grows), kept for symmetry */
} orc_species;

typedef struct {
  int32_t species, kind, target;
  double e_th;            /* eV */
  double target_mass;     /* kg */
} orc_process;

typedef struct orc_sim orc_sim;

orc_sim *orc_create(const orc_config *cfg, const orc_species *sp, int32_t nproc,
                    const orc_process *pr, const double *sigma);
void orc_destroy(orc_sim *S);

void orc_load_uniform(orc_sim *S);
/* Loading from profiles (warm start): n_pts points x[k] (x / L, strictly
   increasing in [0, 1]), densities dens[s][k] [m^-3] and mean energies
   mean_ev[s][k] [eV] per species.  Returns 0, or -1 for an invalid profile. */
int orc_load_profile(orc_sim *S, int32_t n_pts, const double *x, const double *dens, const double *mean_ev);
int orc_set_particles(orc_sim *S, int32_t s, int64_t n, const int32_t *cell, const float *off,
                      const float *vx, const float *vy, const float *vz, const uint32_t *id,
                      const int32_t *cdw, uint32_t next_id);
int orc_set_particles64(orc_sim *S, int32_t s, int64_t n, const double *xi, const double *vx,
                        const double *vy, const double *vz, const uint32_t *id, const int32_t *cdw,
                        uint32_t next_id);
int64_t orc_count(const orc_sim *S, int32_t s);
uint32_t orc_next_id(const orc_sim *S, int32_t s);
void orc_get_particles(const orc_sim *S, int32_t s, double *xi, double *vx, double *vy, double *vz,
                       uint32_t *id, int32_t *cdw);
void orc_set_step(orc_sim *S, int64_t step);
int64_t orc_get_step(const orc_sim *S);
void orc_prepare(orc_sim *S, int32_t shift);
void orc_step(orc_sim *S, int64_t nsteps);

void orc_get_hist(const orc_sim *S, int64_t *Q);
void orc_set_hist(orc_sim *S, const int64_t *Q);   /* test hook */
void orc_get_field(const orc_sim *S, double *phi, double *E);
void orc_get_counters(const orc_sim *S, int64_t *out);
double orc_nu_max(const orc_sim *S, int32_t s);
void orc_info(const orc_sim *S, double *out);   /* dx, dt, n_O2, nu_max[3] */
double orc_sigma(const orc_sim *S, int32_t p, double e_ev);

/* cycle accumulators */
void orc_reset_moments(orc_sim *S);
int64_t orc_get_moments(const orc_sim *S, double *sumQ, double *sumphi, int64_t *esum, int64_t *ecnt,
                        int64_t *edf, int64_t *iedf, int64_t *ndiag);
/* test hook: one sample of the energy moments (esum, ecnt, edf) of the state as it is */
void orc_sample_moments(orc_sim *S);

/* current density at the driven electrode (section 3): per phase of the rf cycle
   the sums of j [A/m^2] and their counts, and the sum of U j [W/m^2] over the
   samples; cleared with the other moments */
void orc_get_current(const orc_sim *S, double *jsum, int64_t *jcnt, double *psum, int64_t *pn);

/* spatially resolved O2(a1Delta_g) (section 4): production by the electron
   channel proc (an excitation, Table 1 (14)), diffusion D [m^2/s], volume loss
   nu_q [1/s], surface loss probability gamma at both electrodes.  Config starts
   from n = C n(O2) and clears the tally; update solves the steady profile from
   the events tallied since the last update and uses it for Eq. (1) detachment
   from then on.  Both return 0, or -1 for invalid arguments. */
int orc_metastable_config(orc_sim *S, int32_t proc, double D, double nu_q, double gamma);
int orc_metastable_update(orc_sim *S, double *n_out);
void orc_metastable_tally(const orc_sim *S, int64_t *src);
int orc_metastable_set(orc_sim *S, const double *na);   /* test hook */
void orc_metastable_solve(int32_t ng, double dx, double D, double nu_q, double h, const double *prod, double *n);

/* event log: records of 6 int64 {step, species, id, code, band, aux};
   code >= 0 process index, -1 null, -2 capped redraw, -3 absorbed, -4 candidate
   test in the band; species ORC_EV_EION for the electron-ion test of an electron */
void orc_log_events(orc_sim *S, int32_t on);
int64_t orc_get_events(orc_sim *S, int64_t max, int64_t *rec);

/* standalone definitions used by the pins */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_poisson(int32_t ng, double dx, double phi0, const double *rho, double *phi, double *E);
void orc_deposit_canonical(int32_t ng, int64_t n, const int32_t *cell, const float *off, int64_t *Q);

#ifdef __cplusplus
}
#endif
#endif
