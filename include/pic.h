/*
 * pic.h - C ABI of the MI355X (gfx950) PIC-MCC library for one-dimensional,
 * three-velocity (1D3V) capacitively coupled rf discharges in oxygen.
 *
 * Method: Bronold, Matyash, Tskhakaya, Schneider, Fehske, "Particle-based
 * modeling of oxygen discharges", ICPIG 2007.
 *   - Section 1: the discharge is the Boltzmann-Poisson system solved with
 *     pseudo-particles; collisions enter through cross sections and the
 *     chemistry reaches the field through the Poisson source term.
 *   - Section 2: gap 0 <= x <= L, velocities (vx, vy, vz); the electrode at
 *     x = 0 is driven at U sin(2 pi f t), the one at x = L is grounded; both
 *     absorb everything that reaches them (no secondary emission); the O2
 *     reservoir has density p / kT at T = 300 K; free flights alternate with
 *     collisions whose timing and channel follow from the cross sections;
 *     species e, O-, O2+; channels of Table 1; Eq. (1) for associative
 *     detachment with n(O2(a)) = C n(O2).
 *
 * Conventions shared by every call:
 *   - Species index 0 = electrons, 1 = O2+, 2 = O-.
 *   - Return value: 0 (PIC_OK) on success, a negative PIC_E* code on error.
 *     No call throws.  pic_last_error() gives a message for the last error.
 *   - Device memory: the library allocates none.  The caller allocates ONE
 *     device buffer of the size pic_query() reports, passes it to
 *     pic_create(), and keeps it alive until pic_destroy().  Host pointers
 *     passed to calls are read or written before the call returns.
 *   - Streams: all device work of a handle is enqueued on the hipStream_t
 *     given to pic_create().  pic_step() does not synchronise; calls that
 *     return data to the host synchronise that stream.  A handle is not
 *     thread-safe; different handles on different streams are independent.
 *   - Device-side errors (storage full, id overflow, NaN) are sticky flags
 *     reported by the next synchronising call.
 */
#ifndef PIC_H
#define PIC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_OK 0
#define PIC_EINVAL (-1)        /* invalid argument or configuration */
#define PIC_ECAPACITY (-2)     /* particle storage or per-step product buffer full */
#define PIC_EIDOVERFLOW (-3)   /* 32-bit particle ids exhausted */
#define PIC_ENAN (-5)          /* non-finite particle coordinate */
#define PIC_EHIP (-6)          /* HIP runtime error */
#define PIC_ENODEVICE (-7)     /* no usable gfx950 device */
#define PIC_WFALLBACK 1        /* warning: invalid warm-start profile, loaded uniformly instead */

/* process kinds (Table 1 channels handled by the library) */
#define PIC_ELASTIC 0      /* e + O2 elastic (7) */
#define PIC_EXCITE 1       /* e + O2 energy loss (10)-(15): E -> E - E_th */
#define PIC_IONIZE 2       /* e + O2 -> 2e + O2+ (21) */
#define PIC_ATTACH 3       /* e + O2 -> O + O- (18) */
#define PIC_CX 4           /* O2+ + O2 charge exchange (9) */
#define PIC_NEUTRALIZE 5   /* O- + O2+ -> O + O2 (17), partner density from the grid */
#define PIC_DETACH 6       /* O- + O2(a) -> O3 + e (20), O- + O2 -> O + O2 + e (19):
                              the electron takes the relative energy above e_th */
#define PIC_ION_ELASTIC 7  /* O- + O2 (8) or O2+ + O2 elastic: isotropic in the centre-of-mass frame */
/* electron collisions with the ions of the grid, tested once per ion step after
   the electron push (probability 1 - exp(-nu_ei ksub dt), nu_ei from the largest
   ion node densities of the field solve, the ion at rest); the struck ion is the
   pairing partner in the electron's cell.  Batches run them per member. */
#define PIC_RECOMB 8       /* e + O2+ -> O + O (16): electron and an O2+ removed; target PIC_T_GRIDPOS */
#define PIC_EDETACH 9      /* e + O- -> O + 2e (22): E - e_th shared (1 - r, r) by the two electrons,
                              isotropic; an O- removed; target PIC_T_GRIDNEG */

/* collision partners */
#define PIC_T_O2 0         /* O2 background, n = p / kT */
#define PIC_T_O2A 1        /* metastable O2(a), n = C p / kT */
#define PIC_T_GRIDPOS 2    /* O2+ density of the simulation grid */
#define PIC_T_GRIDNEG 3    /* O- density of the simulation grid */

/* configuration flags (test hooks) */
#define PIC_F_EXT_FIELD 1  /* E(x) = e_ext0 + e_ext1 (x - L/2) replaces the Poisson field */
#define PIC_F_NO_COLL 2    /* collisions off */

/* periodic re-ordering of the particle store (both drop absorbed and removed particles) */
#define PIC_SORT_CELL 0    /* counting sort by cell */
#define PIC_SORT_COMPACT 1 /* order-preserving compaction */

#define PIC_NBIN 256       /* log energy bins from 1e-3 to 1e3 eV */
#define PIC_NCOUNT 44      /* counters, layout below */

/* counter layout (int64): index + species or + process */
#define PIC_C_PUSH 0       /* +s particles pushed */
#define PIC_C_CAND 3       /* +s collision candidates */
#define PIC_C_NULL 6       /* +s null collisions */
#define PIC_C_ABS0 9       /* +s absorbed at x = 0 */
#define PIC_C_ABSL 12      /* +s absorbed at x = L */
#define PIC_C_BORN 15      /* +s products born */
#define PIC_C_EVENT 18     /* +p real collisions of process p (p < 16) */
#define PIC_C_PAIRED 34    /* O2+ removed as partners of neutralisation and recombination */
#define PIC_C_DEFICIT 35   /* neutralisations and recombinations that found no O2+ partner */
#define PIC_C_CLAMP 36     /* energies clamped into the table range */
#define PIC_C_REDRAW 37    /* capped free flights redrawn */
#define PIC_C_EICAND 38    /* electron-ion candidates */
#define PIC_C_EINULL 39    /* electron-ion null collisions */
#define PIC_C_PAIRED_NEG 40  /* O- removed as partners of electron-impact detachment */
#define PIC_C_DEFICIT_NEG 41 /* electron-impact detachments that found no O- partner */

typedef struct pic_config {
  double L;                /* gap [m], > 0 */
  int32_t ng;              /* cells, 2 .. 8192; nodes are ng + 1 */
  double U;                /* rf amplitude [V] at x = 0 */
  double f;                /* rf frequency [Hz] */
  double p;                /* O2 pressure [Pa] */
  double t_gas;            /* gas temperature [K] (300 in the paper) */
  int32_t steps_per_cycle; /* electron steps per rf period; dt = 1 / (f steps_per_cycle) */
  int32_t ksub;            /* ions move every ksub steps with dt_i = ksub dt */
  double c_meta;           /* C in n(O2(a)) = C n(O2), 0 <= C < 1 */
  uint64_t seed;           /* key of the counter-based random streams */
  double weight;           /* physical particles per superparticle per m^2 of electrode */
  int32_t diag_every;      /* energy moments sampled every diag_every steps (0 = never) */
  int32_t sort_every;      /* particles re-ordered by cell every sort_every steps (0 = never) */
  int32_t flags;           /* PIC_F_* */
  double e_ext0, e_ext1;   /* field of PIC_F_EXT_FIELD [V/m], [V/m^2] */
  double table_emin, table_emax; /* energy range of the tables [eV] */
  int32_t table_n;         /* points per table, log-spaced, 2 .. 4096 */
  int32_t max_products;    /* products per species per step, 1 .. 2^24 */
  int32_t event_capacity;  /* records of the collision event log (0 = off) */
  int32_t block;           /* threads per block of the particle kernels (0 = default) */
  int32_t grid;            /* blocks of the particle kernels (0 = default), <= 2048 */
  int32_t sort_kind;       /* PIC_SORT_CELL or PIC_SORT_COMPACT, applied every sort_every steps */
} pic_config;

typedef struct pic_species {
  double charge;           /* in units of e: -1 (e), +1 (O2+), -1 (O-) */
  double mass;             /* kg */
  double t0_ev;            /* Maxwellian loading temperature [eV] */
  int64_t count;           /* superparticles loaded by pic_load_uniform */
  int64_t capacity;        /* slots reserved in device memory (>= count) */
} pic_species;

typedef struct pic_process {
  int32_t species;         /* projectile species index */
  int32_t kind;            /* PIC_ELASTIC .. PIC_EDETACH; at most 12 processes per species */
  int32_t target;          /* PIC_T_* */
  double e_th;             /* threshold [eV]; sigma = 0 below it */
  double target_mass;      /* partner mass [kg] */
  const double *sigma;     /* host array of table_n cross sections [m^2] on the log grid
                              E_k = emin (emax/emin)^(k/(table_n-1)); copied by pic_create */
} pic_process;

/* Cycle accumulators returned by pic_moments (host arrays owned by the caller;
   any pointer may be NULL to skip that output). */
typedef struct pic_moments_out {
  double *sum_q;           /* [3][ng+1] sum over steps of the node charge (2^-32 superparticle units) */
  double *sum_phi;         /* [ng+1] sum over steps of the potential [V] */
  int64_t *esum;           /* [3][ng] sum of kinetic energies per cell, 2^-20 eV units */
  int64_t *ecnt;           /* [3][ng] particles counted per cell */
  int64_t *edf;            /* [3][PIC_NBIN] energy distribution counts */
  int64_t *iedf;           /* [3][2][PIC_NBIN] energies of particles absorbed at x=0 / x=L */
  int64_t nacc;            /* steps accumulated in sum_q / sum_phi */
  int64_t ndiag;           /* diagnostic samples in esum / ecnt / edf */
  /* Section 3, current density through the discharge and power <U j> A: between
     the field solves of steps n-1 and n the current density at x = 0 in +x is
     eps0 (E_0^n - E_0^(n-1)) / dt (displacement; E_0 the Gauss-law node field)
     plus -e w sum_s q_s dN_s / dt for the dN_s particles absorbed at x = 0 in
     between; it is summed at phase (n-1) mod steps_per_cycle.  Ions absorbed in
     an ion step appear in that step (the ions move every ksub steps). */
  double *current;         /* [steps_per_cycle] sums of j [A/m^2] per phase */
  int64_t *current_n;      /* [steps_per_cycle] samples per phase */
  double power_sum;        /* sum over the samples of (U^(n-1) + U^n) / 2 j [W/m^2] */
  int64_t power_n;         /* samples in power_sum; power per electrode area = power_sum / power_n */
} pic_moments_out;

typedef struct pic_handle pic_handle;

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t pic_version(void);

/* Validates the configuration and reports the device bytes pic_create needs.
   Pure host call. */
int pic_query(const pic_config *cfg, const pic_species *sp /* [3] */, const pic_process *pr,
              int32_t nproc, uint64_t *workspace_bytes);

/* Creates a discharge on the current HIP device.  `workspace` is caller-owned
   device memory of at least pic_query() bytes; `stream` is a hipStream_t (NULL =
   default stream).  Tables are copied; particles are empty until
   pic_load_uniform or pic_set_particles. */
int pic_create(const pic_config *cfg, const pic_species *sp, const pic_process *pr, int32_t nproc,
               void *workspace, uint64_t workspace_bytes, void *stream, pic_handle **out);

int pic_destroy(pic_handle *h);

/* Uniform loading (section 2 geometry): species s gets sp[s].count particles
   with ids 0..count-1 on the 2^24-point lattice of [0, L) and Maxwellian
   velocities at t0_ev, then pic_prepare(h, 1). */
int pic_load_uniform(pic_handle *h);

/* Warm start: loads every species from cycle-averaged profiles across the gap
   (the quantities the paper reports in section 3: densities and mean energies
   of e, O2+ and O-), e.g. predicted by the network of mlp.h.  n_pts points
   x_over_L (strictly increasing in [0, 1]); dens [3][n_pts] [m^-3] and
   mean_ev [3][n_pts] [eV] (> 0), host arrays, species order e, O2+, O-.
   Profiles are linear between points and constant beyond the end points.
   Cell j (centre x_c) of species s receives round(sum_{i<=j} e_i) -
   round(sum_{i<j} e_i) particles, e_i = n_s(x_c) dx / weight (rounding half
   up), ids 0..N_s-1 in cell order, offsets on the 2^24-point lattice of the
   cell, Maxwellian velocities at T = (2/3) mean energy at x_c; the particle
   draws are those of pic_load_uniform.  Then pic_prepare(h, 1), step 0.
   Returns PIC_WFALLBACK (> 0) after loading uniformly when the profile is
   invalid (too few points, x not increasing in [0, 1], a negative or
   non-finite density, a non-positive mean energy); PIC_ECAPACITY if a
   species needs more particles than its capacity. */
int pic_load_profiles(pic_handle *h, int32_t n_pts, const double *x_over_L, const double *dens,
                      const double *mean_ev);

/* Canonical particle record exchanged with the host (arrays of n):
   cell in [0, ng), off in [0, 1) (x = (cell + off) L / ng), vx, vy, vz [m/s],
   id, and for electrons the countdown word cd = steps left in the current free
   flight (1..32767) | 0x8000 when the flight was capped.  set replaces the
   species' particles; next_id is the id the next product receives. */
int pic_set_particles(pic_handle *h, int32_t s, int64_t n, const int32_t *cell, const float *off,
                      const float *vx, const float *vy, const float *vz, const uint32_t *id,
                      const int32_t *cd, uint32_t next_id);

/* Number of live particles of species s (synchronises). */
int pic_count(pic_handle *h, int32_t s, int64_t *n);

/* Copies the live particles of s into host arrays of at least *n entries;
   *n returns the count.  Order is unspecified (match by id). */
int pic_get_particles(pic_handle *h, int32_t s, int64_t *n, int32_t *cell, float *off, float *vx,
                      float *vy, float *vz, uint32_t *id, int32_t *cd, uint32_t *next_id);

/* Rebuilds the charge histograms from the particles; with shift != 0 also
   solves the field at the current step and moves every velocity back by half
   its step (leapfrog start). */
int pic_prepare(pic_handle *h, int32_t shift);

/* Sets / reads the index n of the next step (t_n = n dt). */
int pic_set_step(pic_handle *h, int64_t step);
int pic_get_step(pic_handle *h, int64_t *step);

/* Advances n_steps electron steps (ions every ksub-th): field solve, push,
   null-collision MCC, products, charge deposit, moments.  Asynchronous. */
int pic_step(pic_handle *h, int64_t n_steps);

/* Waits for the stream and reports sticky device errors. */
int pic_sync(pic_handle *h);

/* Copies the accumulators to the host (synchronises); reset != 0 clears them. */
int pic_moments(pic_handle *h, pic_moments_out *out, int32_t reset);

/* Charge histograms [3][ng+1] (2^-32 superparticle units), potential [ng+1]
   [V] and node field [ng+1] [V/m] of the last field solve, counters
   [PIC_NCOUNT].  All synchronise. */
int pic_get_hist(pic_handle *h, int64_t *q);
int pic_get_field(pic_handle *h, double *phi, float *e);
int pic_get_counters(pic_handle *h, int64_t *out);

/* Collision event log (config event_capacity > 0): records of 4 int64
   {step, species, id, code} (species 3: the electron-ion test of electron id);
   code >= 0 process index, -1 null collision,
   -2 capped flight redrawn, -3 absorbed (electrode in the id's record aux is
   not kept).  Returns the number of events since the last clear in *n; copies
   min(*n, max) records.  clear != 0 empties the log. */
int pic_get_events(pic_handle *h, int64_t max, int64_t *rec, int64_t *n, int32_t clear);

/* Spatially resolved O2(a1Delta_g), the extension section 4 proposes for the
   uniform n = C n(O2) of Eq. (1) (PIC_T_O2A partners).  The density on the nodes
   is the steady state of  D n'' - quench_rate n + P(x) = 0  between the
   electrodes, each losing gamma v / (2 (2 - gamma)) n per unit area (v the mean
   molecular speed at t_gas), with P the production by the excitation channel
   source_process (Table 1 (14)), tallied per node with the linear weighting of
   the charge deposit while the discharge steps; finite volumes on the nodes,
   FP64, solved on the device.
   pic_metastable_config: validates, starts from n = C n(O2) everywhere and
     clears the tally (asynchronous).  PIC_EINVAL: source_process not an
     electron excitation, diffusion <= 0, quench_rate < 0, surface_loss outside
     [0, 1], or no loss at all.
   pic_metastable_update: solves from the events since the config or the last
     update, P = w (events at the node) / (volume x elapsed time), and uses the
     new profile for Eq. (1) detachment and the O- collision bound from the next
     step on; copies the ng + 1 densities [m^-3] to n_out (host, may be NULL;
     then asynchronous).  PIC_EINVAL before a config or with no step since the
     last update. */
typedef struct pic_metastable {
  int32_t source_process;  /* index in the process list of the e + O2 -> e + O2(a) channel */
  double diffusion;        /* D of O2(a) in O2 at the run's pressure [m^2/s] */
  double quench_rate;      /* volume loss rate [1/s] */
  double surface_loss;     /* loss probability per wall collision, both electrodes */
} pic_metastable;
int pic_metastable_config(pic_handle *h, const pic_metastable *m);
int pic_metastable_update(pic_handle *h, double *n_out);

/* Collision-frequency bound used by the null-collision test of species s [1/s]
   (for O- the value of the last ion step). */
int pic_nu_max(pic_handle *h, int32_t s, double *nu);

/* Timing of the kernels of the next n_steps steps (synchronises): total device
   time of the electron push kernel and of everything else, measured with HIP
   events on the handle's stream, plus the launches of the push kernel. */
int pic_step_timed(pic_handle *h, int64_t n_steps, double *ms_push_e, double *ms_total,
                   int64_t *push_launches);

const char *pic_strerror(int code);
const char *pic_last_error(const pic_handle *h);

/* ------------------------------------------------------------------ batches
   Many discharges (different gaps, cells, voltages, pressures, particle counts,
   tables) advanced together.  Every kernel of a step is ONE launch over all
   members: the particle push is a persistent launch over a list of tiles cut
   from every member's store, the field solves and product-id assignments run
   as one block group per member.  One rf cycle of launches is captured once as
   a HIP graph and replayed; the step index each kernel uses is a per-member
   device counter advanced at the end of every cycle.

   The members are ordinary handles made by pic_create on the batch's stream;
   the batch does not own them and they must outlive it.  A member advanced in
   a batch reaches the same state as the same handle advanced alone by
   pic_step: the random streams are keyed by the member's own seed, and block
   size, grid and re-ordering interval change the storage order only.

   pic_batch_create checks: 1..64 distinct members created on `stream`, equal
   steps_per_cycle, every member's ksub and diag_every (if > 0) divide
   steps_per_cycle, member grid 0.  Between pic_batch_step_cycles /
   pic_batch_autotune and pic_batch_sync the members' own calls return
   PIC_EBUSY.  Member step indices must be multiples of steps_per_cycle when
   a batch call starts. */
#define PIC_EBUSY (-8)         /* member of a batch with unsynchronised work */

typedef struct pic_batch pic_batch;

typedef struct pic_batch_config {
  int32_t block;           /* threads per block of the batched push: 256, 512 or 1024 (0 = 512) */
  int32_t sort_every;      /* compaction of all members every sort_every steps (0 = never);
                              must divide steps_per_cycle */
  int32_t use_graph;       /* != 0: replay one captured rf cycle (needs a non-NULL stream) */
  int32_t grid;            /* blocks of the batched push (0 = all resident blocks), <= 2048 */
} pic_batch_config;

#define PIC_TUNE_MAX 32
typedef struct pic_batch_tuning {
  int32_t n;                        /* candidates timed */
  int32_t block[PIC_TUNE_MAX];
  int32_t sort_every[PIC_TUNE_MAX];
  double ms_per_step[PIC_TUNE_MAX]; /* device time per step of the trial window */
  int32_t best;                     /* index of the candidate now configured */
} pic_batch_tuning;

/* Device bytes of a batch of n_members (Sim records and counters). */
int pic_batch_query(int32_t n_members, uint64_t *workspace_bytes);

/* `workspace`: caller-owned device memory of at least pic_batch_query bytes. */
int pic_batch_create(pic_handle *const *members, int32_t n_members, const pic_batch_config *cfg,
                     void *workspace, uint64_t workspace_bytes, void *stream, pic_batch **out);

/* Advances every member by `cycles` rf cycles (steps_per_cycle steps each).
   Asynchronous: replays the cycle graph, or enqueues the launches directly. */
int pic_batch_step_cycles(pic_batch *b, int64_t cycles);

/* Waits for the stream, hands the members back (their particle buffers and
   step index) and reports the first member's sticky device error. */
int pic_batch_sync(pic_batch *b);

/* Changes block, grid, re-ordering interval or graph use (drops the graph). */
int pic_batch_set_config(pic_batch *b, const pic_batch_config *cfg);
int pic_batch_get_config(const pic_batch *b, pic_batch_config *cfg);

/* Autotuner: times every (block, sort_every) candidate over `window` steps of
   the running batch (block in {256, 512, 1024}; sort_every among 10, 20, 50,
   100, 200, 500, 1000 dividing both window and steps_per_cycle), configures the
   fastest, then completes the rf cycle so the members end on a cycle boundary.
   The trial steps are real steps of the members.  Synchronises. */
int pic_batch_autotune(pic_batch *b, int32_t window, pic_batch_tuning *out);

int pic_batch_destroy(pic_batch *b);
const char *pic_batch_last_error(const pic_batch *b);

/* Largest ion subcycling factor k dividing steps_per_cycle with
   (i) omega_pi k dt <= 0.2 for both ion species at ion density n_ion_max [m^-3]
   (leapfrog accuracy well inside its stability limit 2), and
   (ii) an ion that fell through the potential phi_max [V] moves at most one cell
   per ion step (CIC field of every crossed cell seen).  Pure host call; *ksub = 1
   when even k = 1 violates them. */
int pic_ksub_select(const pic_config *cfg, const pic_species *sp /* [3] */, double n_ion_max,
                    double phi_max, int32_t *ksub);

#ifdef __cplusplus
}
#endif
#endif
