// Internal layout shared by the host library (pic.cpp) and the gfx950 kernels
// (kernels.hip).  Not part of the public ABI.
#pragma once
#include <stdint.h>

namespace picmcc {

constexpr int NSP = 3;
constexpr int MAXPROC = 16;
constexpr int MAXPROC_SP = 12;     // processes per species
constexpr int NCOUNT = 44;
constexpr int NBIN = 256;
constexpr int CD_MAX = 32767;      // longest stored free flight [steps]
constexpr int MAXPROD = 1 << 24;   // products per species per step (24-bit local index)
constexpr int NBKT = 8192;         // parent-key buckets of the product id assignment

// packed cell word of a particle (int32):
//   bits 0..14 cell, bit 15 capped flight, bits 16..30 countdown, bit 31 dead
constexpr uint32_t W_CELL = 0x7FFFu;
constexpr uint32_t W_CAP = 0x8000u;
constexpr int W_CD_SHIFT = 16;
constexpr int32_t W_DEAD = -1;

enum { K_ELASTIC = 0, K_EXCITE = 1, K_IONIZE = 2, K_ATTACH = 3, K_CX = 4, K_NEUTRALIZE = 5, K_DETACH = 6,
       K_ION_ELASTIC = 7, K_RECOMB = 8, K_EDETACH = 9 };
enum { T_O2 = 0, T_O2A = 1, T_GRIDPOS = 2, T_GRIDNEG = 3 };
enum { P_LOAD = 1, P_CAND = 2, P_TARGET = 3, P_PROD = 4, P_PAIR = 5, P_EION = 6 };
enum { C_PUSH = 0, C_CAND = 3, C_NULL = 6, C_ABS0 = 9, C_ABSL = 12, C_BORN = 15, C_EVENT = 18,
       C_PAIRED = 34, C_DEFICIT = 35, C_CLAMP = 36, C_REDRAW = 37, C_EICAND = 38, C_EINULL = 39,
       C_PAIRED_NEG = 40, C_DEFICIT_NEG = 41 };
// parent-species code of the electron born in an electron-impact detachment (its
// parent key sorts after those of the three species) and the species field of
// the event records of the electron-ion test
constexpr int PS_EION = 3;
enum { E_CAPACITY = 1, E_IDOVERFLOW = 2, E_NAN = 4 };
enum { F_EXT_FIELD = 1, F_NO_COLL = 2 };

// device-resident scalars
struct Scalars {
  unsigned long long n[NSP];       // occupied slots (live + dead) per species
  unsigned long long nnew[NSP];    // products appended in the current step
  unsigned long long cnt[NCOUNT];
  unsigned long long nev;          // collision events logged
  uint32_t next_id[NSP];
  uint32_t err;
  double numax_neg;                // O- bound of the current ion step [1/s]
  double pnull_neg;                // 1 - exp(-numax_neg dt_i)
  float inv_numax_neg;
  int32_t pair_active;             // pending O2+ partners (neutralisation, recombination)
  uint32_t ticket;                 // last-block-done counter
  int32_t pair_active_neg;         // pending O- partners (electron-impact detachment)
  double numax_ei;                 // electron-ion bound of the current ion step [1/s]
  double pnull_ei;                 // 1 - exp(-numax_ei dt_i)
  float inv_numax_ei;
  int32_t meta_on;                 // spatially resolved O2(a): the field below replaces C n(O2)
  int32_t meta_tab;                // process whose events produce O2(a) (Table 1 (14))
  int32_t pair_nrec;               // keys listed by the pairing of the current ion step
  double na_max;                   // largest node density of the O2(a) field [m^-3]
  unsigned long long nsort[NSP];   // slots seen by the running sort
  // current density at the driven electrode: state of the previous field solve
  double e0_prev, u_prev;
  unsigned long long abs0_prev[NSP];
  int32_t jvalid;
  uint32_t field_ticket;            // reduction blocks done in k_reduce_field
};

constexpr int MAXGRID = 2048;      // largest push grid
constexpr int SORT_GRID = 256;     // most blocks of the cell sort (rows of sortoff)

// Load balance of the electron push: the slot range and the duration of every
// block in the last two launches (by step parity).  A launch cuts the store so
// that each block gets an equal share of the cost the previous launch measured.
struct PushBal {
  long long begin[2][MAXGRID + 1];
  long long dur[2][MAXGRID];
  int32_t grid[2];
};

// pairing record of one cell for the ion step being closed: every candidate key
// below bin bstar is taken, plus the `need` smallest of the `fill` keys of bin
// bstar listed from segoff on
struct PairCell { int32_t bstar, need, segoff, fill; };

struct Particles {
  int32_t *w;          // packed cell word
  float *off, *vx, *vy, *vz;
  uint32_t *id;
};

struct ProcDev {
  int32_t kind, target, tab;       // tab = row of the sigma table
  float e_th;
  float scale;                     // n_target / nu_max (constant targets)
  float inv_mu2;                   // 2 e / mu  (relative speed from energy)
  float half_mu_e;                 // mu / (2 e) (energy from relative speed)
  float vt;                        // sqrt(k T / M) of the partner
  float tm_ratio;                  // 2 m / M (electron elastic loss)
  float cmf;                       // M / (m + M): relative velocity share of the projectile in the CM frame
};

struct Sim {
  // geometry and drive
  int32_t ng;
  double dx, dt, L;
  double U, f;
  double eps0, qcharge;            // epsilon_0, e*w*2^-32 (charge per fixed-point unit per m^2)
  double e_ext0, e_ext1;
  int32_t flags, ksub;
  uint64_t seed;
  // species
  Particles p[NSP];
  Particles alt[NSP];              // the other buffer of each species (re-ordering target, pairing list)
  uint64_t *pkey[NSP];             // (parent species, parent id, local index) of this step's products
  int32_t *pbkt[NSP];              // bucket of each product's parent key
  uint64_t *ptmp[NSP];             // keys grouped by bucket during the id assignment
  int32_t *bcnt;                   // [3][NBKT] products per bucket this step
  int64_t cap[NSP];
  int32_t max_products;
  int32_t charge[NSP];
  float qmdt[NSP], dtdx[NSP];      // q/m dt_s, dt_s/dx
  float half_m_e[NSP];             // m / (2 e): energy [eV] from v^2
  float two_e_m[NSP];              // 2 e / m
  double mass[NSP];
  float vt_gas[NSP];               // sqrt(k T_gas / m_s): Maxwellian of newborn ions
  // processes
  int32_t nproc_sp[NSP];           // electrons: the channels with neutral targets only
  ProcDev proc[NSP][MAXPROC_SP];   // electrons: then nei electron-ion channels at [0][nproc_sp[0] + q]
  int32_t nei;
  const float *sigma;              // [nproc][ntab] FP32
  const double *hbound;            // [nproc][ntab-1] max(sigma_k, sigma_k+1) g(E_k+1), FP64
  int32_t ntab;
  float lnemin, invdlt, emin, emax;
  double n_o2, c_meta;
  double nd_e;                     // nu_max(e) dt
  float inv_nd_ef;                 // 1 / (nu_max(e) dt) in FP32, 0 if nu_max = 0
  float invdlt2, l2emin_s;         // table index t = log2(E) invdlt2 - l2emin_s
  const float *ttot_e;             // [ntab] sum over electron processes of scale_p sigma_p
  unsigned long long *part;        // [grid][ng+1] per-block charge partials
  PushBal *bal;                    // electron push ranges and durations
  long long *blkcnt;               // [grid] live counts / output offsets of the compaction
  double pnull_pos;                // 1 - exp(-nu_max(O2+) dt_i)
  double dti;
  double wd;                       // w 2^-32 / dx : node density per fixed-point unit (interior)
  float nplus_c;                   // the same in FP32
  // grid and accumulators
  unsigned long long *Q;           // [3][ng+1]
  float *E;                        // [ng+1]
  double *phi;                     // [ng+1]
  double *sumQ, *sumphi;           // [3][ng+1], [ng+1]
  unsigned long long *esum, *ecnt; // [3][ng]
  unsigned long long *edf, *iedf;  // [3][NBIN], [3][2][NBIN]
  unsigned long long *nacc;        // [2] nacc, ndiag
  int32_t *kleft;                  // [ng] O2+ partners still to remove per cell
  int32_t *kleft_neg;              // [ng] O- partners still to remove per cell
  float *dens_ei;                  // [2][ng+1] O2+, O- node densities of the field solve [m^-3]
  unsigned long long *meta_src;    // [ng+1] O2(a) production events, linear weighting in 2^-32 units
  double *na;                      // [ng+1] O2(a) density [m^-3]
  float *na_f;                     // [ng+1] the same in FP32 for the collision step
  double *meta_tmp;                // [ng+1] solver work
  PairCell *pcell;                 // [ng] pairing records
  int32_t *phist;                  // [ng][256] pairing key bins (zero between ion steps)
  int32_t *sortcnt, *sortbase;     // [ng], [ng]
  int32_t *sortoff;                // [SORT_GRID][ng]: each sort block's offset inside every cell
  Scalars *sc;
  long long *events;
  int64_t event_cap;
  int32_t rq_cap;                  // electron candidate records kept in LDS per pass
  int32_t spc;                     // steps per rf cycle
  double *jsum;                    // [spc] current density sums per phase [A/m^2]
  unsigned long long *jcnt;        // [spc] samples per phase
  double *jpow;                    // [2] sum of U j [W/m^2], number of samples (as a double)
};

// device state of a batch of discharges advanced together
constexpr int MAXBATCH = 64;
constexpr int CBLK = 1024;         // compaction blocks per species in a batch (blkcnt stride)
struct BatchDev {
  int64_t base[MAXBATCH];          // step of each member when the running cycle began
  int32_t rows[NSP][MAXBATCH];     // partial-histogram rows written by the last batched push
  PushBal bal;                     // electron push: tile ranges (in tiles) and durations per block
};

// launch shapes of a batch (host side)
struct BatchLaunch {
  Sim *sims;                       // device array [nmem]
  BatchDev *bd;
  int nmem;
  int block;                       // push block size
  int push_grid[NSP];              // persistent push grid per species
  size_t push_lds[NSP];            // largest member LDS per species (electrons: with the cut table)
  size_t bal_lds;                  // electrons: LDS offset of the balanced cut table, 0 = equal ranges
  int nn_max;                      // largest ng + 1
  size_t diag_lds;
  int cgrid, pgrid, dgrid;         // compaction / pairing / diagnostics blocks per member
};

}  // namespace picmcc
