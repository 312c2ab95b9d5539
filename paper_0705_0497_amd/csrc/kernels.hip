// gfx950 kernels of the 1D3V oxygen PIC-MCC step.
//
// Paper: Bronold et al., "Particle-based modeling of oxygen discharges"
// (ICPIG 2007), sections 1-2, Table 1, Eq. (1).  One step n:
//   k_field   charge -> potential -> node field (FP64), cycle sums, product ids
//   k_push<e> leapfrog push, absorbing walls, null-collision MCC with free
//             flights counted in steps, products, 64-bit fixed-point CIC deposit
//   on ion steps: k_push<O2+>, k_ionprep (O- bound), k_push<O->, k_pair (partners)
//   every S steps: counting sort by cell; every D steps: energy moments.
#include <hip/hip_runtime.h>
#include <math.h>

#include "device.hpp"

namespace picmcc {

// ---------------------------------------------------------------- random numbers
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplications with the Weyl key schedule.
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                     uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;   // one 32x32->64 product each
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
  }
  return {c0, c1, c2, c3};
}

// stream of one particle: counter (id, step, species|purpose|block, 0), key = seed
__device__ __forceinline__ U4 draw(const Sim &S, int s, uint32_t id, int64_t step, int purpose, int blk) {
  return philox(id, (uint32_t)step, ((uint32_t)s << 24) | ((uint32_t)purpose << 16) | (uint32_t)blk, 0u,
                (uint32_t)S.seed, (uint32_t)(S.seed >> 32));
}

// (k + 1/2) 2^-23 from the top 23 bits: exact in FP32 and FP64
__device__ __forceinline__ float unif(uint32_t x) { return fmaf((float)(x >> 9), 0x1p-23f, 0x1p-24f); }
__device__ __forceinline__ double unifd(uint32_t x) { return ((double)(x >> 9) + 0.5) * 0x1p-23; }

__device__ __forceinline__ void normals(uint32_t a, uint32_t b, float &z0, float &z1) {
  const float r = sqrtf(-2.0f * logf(unif(a)));
  float sn, cs;
  sincospif(2.0f * unif(b), &sn, &cs);
  z0 = r * cs;
  z1 = r * sn;
}

__device__ __forceinline__ void iso_dir(uint32_t a, uint32_t b, float &d0, float &d1, float &d2) {
  const float ct = 1.0f - 2.0f * unif(a);
  const float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
  float sn, cs;
  sincospif(2.0f * unif(b), &sn, &cs);
  d0 = ct;
  d1 = st * cs;
  d2 = st * sn;
}

// free flight in steps, 1 + floor(-ln u / (nu_max dt)), stored in the cell word;
// flights beyond CD_MAX steps are stored capped and redrawn when they expire
__device__ __forceinline__ uint32_t new_flight(double nd, uint32_t x) {
  const double tau = nd > 0.0 ? -log(unifd(x)) / nd : (double)CD_MAX;
  if (tau >= (double)CD_MAX) return ((uint32_t)CD_MAX << W_CD_SHIFT) | W_CAP;
  return (uint32_t)(1 + (int)floor(tau)) << W_CD_SHIFT;
}

// ---------------------------------------------------------------- small helpers
struct TabPos { int i; float w; };

__device__ __forceinline__ TabPos tab_pos(const Sim &S, float ec) {
  float t = fmaf(__log2f(ec), S.invdlt2, -S.l2emin_s);   // (log2 E - log2 Emin) / step in log2
  t = fminf(fmaxf(t, 0.0f), (float)(S.ntab - 1));
  const int i = min((int)t, S.ntab - 2);
  return {i, t - (float)i};
}

__device__ __forceinline__ float tab_sigma(const float *tab, TabPos tp) {
  const float a = tab[tp.i], b = tab[tp.i + 1];
  return fmaf(tp.w, b - a, a);
}

// CIC weight of node cell+1 in 2^-32 units: rint(off 2^32), exact scaling then RNE
__device__ __forceinline__ unsigned long long cic_a(float off) {
  return (unsigned long long)__float2uint_rn(off * 4294967296.0f);
}

__device__ __forceinline__ void dep_lds(unsigned long long *sQ, int cell, float off) {
  const unsigned long long a = cic_a(off);
  atomicAdd(&sQ[cell], 4294967296ull - a);
  atomicAdd(&sQ[cell + 1], a);
}

__device__ __forceinline__ void dep_global(unsigned long long *Q, int cell, float off) {
  const unsigned long long a = cic_a(off);
  atomicAdd(&Q[cell], 4294967296ull - a);
  atomicAdd(&Q[cell + 1], a);
}

__device__ __forceinline__ int ebin(float e) {
  if (!(e > 0.0f)) return 0;
  const int b = (int)floorf((log10f(e) + 3.0f) * ((float)NBIN / 6.0f));
  return min(max(b, 0), NBIN - 1);
}

__device__ __forceinline__ void log_event(const Sim &S, int64_t step, int s, uint32_t id, int code) {
  if (S.event_cap <= 0) return;
  const unsigned long long k = atomicAdd(&S.sc->nev, 1ull);
  if ((int64_t)k < S.event_cap) {
    long long *r = S.events + 4 * k;
    r[0] = step; r[1] = s; r[2] = id; r[3] = code;
  }
}

// reserve the slot of a product of species s born from parent (ps, pid).  Its
// parent key (ps, pid) goes to the id assignment, bucketed by its position in
// the ordered key space [0, next_id[0]) + [0, next_id[1]) + [0, next_id[2]) +
// [0, next_id[0]) (the last segment: ps = PS_EION, electrons of an
// electron-impact detachment, whose parent may also have ionised this step).
// What appends and collisions read of the step-start state: live counts, the
// parent-key space and the O2(a) switch.  None of it changes while particles
// move (only the product counters nnew do), so a push block reads it once.
struct StepCtx { int64_t n[NSP]; uint64_t off[NSP + 1]; uint64_t total; int meta_on, meta_tab; };

__device__ __forceinline__ StepCtx step_ctx(const Sim &S) {
  StepCtx r;
  uint64_t t = 0;
  for (int s = 0; s < NSP; ++s) { r.n[s] = (int64_t)S.sc->n[s]; r.off[s] = t; t += S.sc->next_id[s]; }
  r.off[PS_EION] = t;
  t += S.sc->next_id[0];
  r.total = t > 0 ? t : 1;
  r.meta_on = S.sc->meta_on;
  r.meta_tab = S.sc->meta_tab;
  return r;
}

// rank of this lane among the active lanes act
__device__ __forceinline__ unsigned long long lane_rank(unsigned long long act) {
  return (unsigned long long)__popcll(act & ((1ull << __lane_id()) - 1ull));
}

// product key k of species s from parent (ps, pid): its slot n + k, its parent key
// and bucket; -1 (and the capacity error) when the store or the key space is full
__device__ __forceinline__ int64_t place(const Sim &S, const StepCtx &cx, int s, int ps, uint32_t pid,
                                         unsigned long long k) {
  const int64_t slot = cx.n[s] + (int64_t)k;
  if (k >= (unsigned long long)S.max_products || slot >= S.cap[s]) {
    atomicOr(&S.sc->err, (uint32_t)E_CAPACITY);
    return -1;
  }
  S.pkey[s][k] = ((uint64_t)ps << 56) | ((uint64_t)pid << 24) | k;
  const int b = (int)(((cx.off[ps] + pid) * (uint64_t)NBKT) / cx.total);
  S.pbkt[s][k] = b;
  atomicAdd(&S.bcnt[s * NBKT + b], 1);
  return slot;
}

// one reservation per wave: the active lanes of this call site take consecutive keys
__device__ __forceinline__ int64_t append(const Sim &S, const StepCtx &cx, int s, int ps, uint32_t pid) {
  const unsigned long long act = __ballot(1);
  const int leader = __ffsll((long long)act) - 1;
  unsigned long long base = 0ull;
  if (__lane_id() == leader) base = atomicAdd(&S.sc->nnew[s], (unsigned long long)__popcll(act));
  base = __shfl(base, leader, 64);
  return place(S, cx, s, ps, pid, base + lane_rank(act));
}

__device__ __forceinline__ void put(const Particles &P, int64_t i, int32_t w, float off, float vx, float vy,
                                    float vz) {
  P.w[i] = w; P.off[i] = off; P.vx[i] = vx; P.vy[i] = vy; P.vz[i] = vz;
}

// ---------------------------------------------------------------- block scans
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Inclusive wave scan on DPP row shifts and row broadcasts (lanes within a row
// of 16 by 1, 2, 4, 8, then row 0's and rows 0-1's totals into the rows
// above): no LDS round trip per step, unlike the shuffle form above.  64-bit
// values move as two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ long long dpp_move(long long x) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)x, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, 0xf, 0xf, false);
  return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  return __builtin_bit_cast(double, dpp_move<CTRL>(__builtin_bit_cast(long long, x)));
}
template <typename T>
__device__ __forceinline__ T wave_incl_scan_dpp(T v) {
  const int lane = threadIdx.x & 63, rl = lane & 15;
  T x = dpp_move<0x111>(v);
  if (rl >= 1) v += x;
  x = dpp_move<0x112>(v);
  if (rl >= 2) v += x;
  x = dpp_move<0x114>(v);
  if (rl >= 4) v += x;
  x = dpp_move<0x118>(v);
  if (rl >= 8) v += x;
  x = dpp_move<0x142>(v);                          // row_bcast:15
  if ((lane & 31) >= 16) v += x;
  x = dpp_move<0x143>(v);                          // row_bcast:31
  if (lane >= 32) v += x;
  return v;
}
__device__ __forceinline__ long long wave_lane63(long long x) {
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)x, 63), hi = __builtin_amdgcn_readlane((int)(x >> 32), 63);
  return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}
__device__ __forceinline__ double wave_lane63(double x) {
  return __builtin_bit_cast(double, wave_lane63(__builtin_bit_cast(long long, x)));
}

// exclusive scan over the block (BS a multiple of 64); buf holds BS/64 entries
template <int BS, typename T>
__device__ T block_exclusive_scan(T v, T *buf, T &total) {
  constexpr int NW = BS / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const T inc = wave_incl_scan(v);
  if (lane == 63) buf[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    T x = lane < NW ? buf[lane] : T(0);
    x = wave_incl_scan(x);
    if (lane < NW) buf[lane] = x;
  }
  __syncthreads();
  const T pre = wid ? buf[wid - 1] : T(0);
  total = buf[NW - 1];
  __syncthreads();
  return pre + inc - v;
}

// ---------------------------------------------------------------- field solve
// -eps0 (phi[j-1] - 2 phi[j] + phi[j+1]) / dx^2 = rho[j], phi[0] = U sin(2 pi f t_n),
// phi[ng] = 0.  Written as D[j+1/2] = D[1/2] + sum_{m=1..j} rho[m] dx (exact int64
// prefix of the node charges), phi[j] = phi0 - (dx/eps0) sum_{m<j} D[m+1/2]; phi[ng] = 0
// fixes D[1/2].  Same linear system as the tridiagonal one, solved by two scans.
// nodes per thread of the field block, (N_g + 1) / 1024 rounded up to one of
// these (the register arrays of a solve are sized by it; 8192 cells need 9)
__host__ __device__ constexpr int field_nper(int nn) {
  return nn <= 1024 ? 1 : nn <= 2048 ? 2 : nn <= 4096 ? 4 : nn <= 5120 ? 5 : 9;
}

// What thread 0 of a field block reads for the current-density tally and the
// step count, loaded at the start of the solve so that the round trips overlap
// the charges' loads and the scans instead of following the solve one by one.
struct TallyIn {
  unsigned long long cnt[NSP], abs0[NSP], jcnt, nacc;
  double e0_prev, u_prev, jsum, jpow0, jpow1;
  int valid, ph;
};

__device__ __forceinline__ TallyIn tally_in(const Sim &S, int64_t step) {
  const Scalars *sc = S.sc;
  TallyIn ti;
  ti.ph = step >= 1 ? (int)((step - 1) % S.spc) : 0;
  ti.valid = sc->jvalid;
  for (int s = 0; s < NSP; ++s) { ti.cnt[s] = sc->cnt[C_ABS0 + s]; ti.abs0[s] = sc->abs0_prev[s]; }
  ti.e0_prev = sc->e0_prev;
  ti.u_prev = sc->u_prev;
  ti.jsum = S.jsum[ti.ph];
  ti.jcnt = S.jcnt[ti.ph];
  ti.jpow0 = S.jpow[0];
  ti.jpow1 = S.jpow[1];
  ti.nacc = S.nacc[0];
  return ti;
}

// One block solves the field.  Wave w owns nodes [w 64 per, (w + 1) 64 per), its
// lanes interleaved (round u, lane l: node w 64 per + 64 u + l), so that every
// global load and store of the solve moves 64 consecutive nodes, and both
// prefix sums are wave scans per round with a running carry plus one exchange
// of the wave totals through LDS.  COHERENT: the node charges are read with
// device-coherent loads, for a caller that runs in the same launch as the
// atomics that summed them.  NPER >= ceil((N_g + 1) / BS).
template <int BS, int NPER, bool COHERENT = false>
__device__ void field_block(const Sim &S, int64_t step, int mode) {
  constexpr int NW = BS / 64;
  __shared__ long long wI[NW];
  __shared__ double wJ[NW];
  const int ng = S.ng, nn = ng + 1, t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int per = (nn + BS - 1) / BS;
  const int base = w * 64 * per + lane;            // node of round u: base + 64 u
  const bool ion = (step % S.ksub) == 0;
  const unsigned long long *Qe = S.Q, *Qp = S.Q + nn, *Qn = S.Q + 2 * nn;
  // every load of the solve is issued here, before any store, so that they are
  // in flight together: this thread's node charges, the cycle sums they and the
  // potential are added to, and thread 0's tally inputs
  unsigned long long qe[NPER], qp[NPER], qn[NPER];
  double sq0[NPER], sq1[NPER], sq2[NPER], sph[NPER];
  long long q[NPER];
#pragma unroll
  for (int u = 0; u < NPER; ++u) {
    const int j = base + 64 * u;
    qe[u] = qp[u] = qn[u] = 0ull;
    sq0[u] = sq1[u] = sq2[u] = sph[u] = 0.0;
    if (u < per && j < nn) {
      if (COHERENT) {
        qe[u] = __hip_atomic_load(Qe + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        qp[u] = __hip_atomic_load(Qp + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        qn[u] = __hip_atomic_load(Qn + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        qe[u] = Qe[j]; qp[u] = Qp[j]; qn[u] = Qn[j];
      }
      if (mode == 0) { sq0[u] = S.sumQ[j]; sq1[u] = S.sumQ[nn + j]; sq2[u] = S.sumQ[2 * nn + j]; sph[u] = S.sumphi[j]; }
    }
  }
  // the rf phase of this solve, computed while the loads are in flight
  const double u_now = S.U * sin(2.0 * M_PI * S.f * ((double)step * S.dt));
  __shared__ TallyIn sti;
  if (t == 0 && mode == 0) sti = tally_in(S, step);
#pragma unroll
  for (int u = 0; u < NPER; ++u)
    q[u] = (long long)S.charge[0] * (long long)qe[u] + (long long)S.charge[1] * (long long)qp[u] +
           (long long)S.charge[2] * (long long)qn[u];
  if (S.flags & F_EXT_FIELD) {
#pragma unroll
    for (int u = 0; u < NPER; ++u) {
      const int j = base + 64 * u;
      if (u < per && j < nn) {
        S.E[j] = (float)(S.e_ext0 + S.e_ext1 * ((double)j * S.dx - 0.5 * S.L));
        S.phi[j] = 0.0;
      }
    }
  }
  // cycle sums of the charge this solve sees, then clear what this step rebuilds
  // (the solve works on q from here on)
  if (mode == 0) {
#pragma unroll
    for (int u = 0; u < NPER; ++u) {
      const int j = base + 64 * u;
      if (u < per && j < nn) {
        S.sumQ[j] = sq0[u] + (double)qe[u];
        S.sumQ[nn + j] = sq1[u] + (double)qp[u];
        S.sumQ[2 * nn + j] = sq2[u] + (double)qn[u];
        S.Q[j] = 0ull;
        if (ion) { S.Q[nn + j] = 0ull; S.Q[2 * nn + j] = 0ull; }
      }
    }
  }
  // I_j = sum of the interior charges q_m, 1 <= m <= j (exact, int64)
  long long icl[NPER];
  {
    long long carry = 0;
#pragma unroll
    for (int u = 0; u < NPER; ++u) {
      const int j = base + 64 * u;
      icl[u] = wave_incl_scan_dpp((u < per && j > 0 && j < ng) ? q[u] : 0ll) + carry;
      carry = wave_lane63(icl[u]);
    }
    if (lane == 63) wI[w] = carry;
  }
  __syncthreads();
  long long ipre = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k)
    if (k < w) ipre += wI[k];
  // J_j = sum_{m < j} I_m (FP64), exclusive per node
  double jex[NPER], jtot = 0.0;
  {
    double carry = 0.0;
#pragma unroll
    for (int u = 0; u < NPER; ++u) {
      const int j = base + 64 * u;
      const double jv = (u < per && j < ng) ? (double)(ipre + icl[u]) : 0.0;
      const double x = wave_incl_scan_dpp(jv) + carry;
      const double up = __shfl_up(x, 1, 64);
      jex[u] = lane == 0 ? carry : up;
      carry = wave_lane63(x);
    }
    if (lane == 63) wJ[w] = carry;
  }
  __syncthreads();
  double jpre = 0.0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const double x = wJ[k];
    if (k < w) jpre += x;
    jtot += x;
  }
  double phiv[NPER];
  double e0v = S.e_ext0 - 0.5 * S.e_ext1 * S.L;    // node-0 field (external-field mode)
#pragma unroll
  for (int u = 0; u < NPER; ++u) phiv[u] = 0.0;
  if (!(S.flags & F_EXT_FIELD)) {
    const double c = S.qcharge;            // e w 2^-32: charge per unit area per fixed-point unit
    const double phi0 = u_now;
    const double d_half = (phi0 * S.eps0 / S.dx - c * jtot) / (double)ng;
    const double k = S.dx / S.eps0;
#pragma unroll
    for (int u = 0; u < NPER; ++u) {
      const int j = base + 64 * u;
      if (u >= per || j >= nn) continue;
      const long long ij = ipre + icl[u];          // I_j
      const long long iprev = ij - ((j > 0 && j < ng) ? q[u] : 0ll);   // I_{j-1}
      const double phi = (j == ng) ? 0.0 : phi0 - k * ((double)j * d_half + c * (jpre + jex[u]));
      double e;
      if (j == 0) e = (d_half - c * (double)q[u]) / S.eps0;
      else if (j == ng) e = (d_half + c * (double)iprev + c * (double)q[u]) / S.eps0;
      else e = (2.0 * d_half + c * ((double)iprev + (double)ij)) / (2.0 * S.eps0);
      S.phi[j] = phi;
      S.E[j] = (float)e;
      phiv[u] = phi;
      if (j == 0) e0v = e;
    }
  }
  // Section 3: current density at x = 0 in +x between this solve and the previous one,
  // eps0 dE_0/dt plus the charge absorbed at x = 0 in between, summed per rf phase
  if (t == 0) {
    Scalars *sc = S.sc;
    const TallyIn ti = sti;
    if (mode == 0 && ti.valid) {
      double dq = 0.0;
      for (int s = 0; s < NSP; ++s)
        dq += (double)S.charge[s] * (double)(long long)(ti.cnt[s] - ti.abs0[s]);
      const double ew = S.qcharge * 4294967296.0;     // e w
      const double jx = S.eps0 * (e0v - ti.e0_prev) / S.dt - ew * dq / S.dt;
      S.jsum[ti.ph] = ti.jsum + jx;
      S.jcnt[ti.ph] = ti.jcnt + 1ull;
      S.jpow[0] = ti.jpow0 + 0.5 * (ti.u_prev + u_now) * jx;
      S.jpow[1] = ti.jpow1 + 1.0;
    }
    if (mode == 0) {
      sc->e0_prev = e0v;
      sc->u_prev = u_now;
      for (int s = 0; s < NSP; ++s) sc->abs0_prev[s] = ti.cnt[s];
      sc->jvalid = 1;
    } else {
      sc->jvalid = 0;
    }
  }
  if (mode != 0) return;
#pragma unroll
  for (int u = 0; u < NPER; ++u) {
    const int j = base + 64 * u;
    if (u < per && j < nn) S.sumphi[j] = sph[u] + phiv[u];
  }
  if (t == 0) S.nacc[0] = sti.nacc + 1ull;
}

// ids of the previous step's products: per species, next_id + rank of the
// parent key (parent species, parent id).  The keys were counted per bucket of
// the ordered key space when they were appended; here the buckets are scanned,
// the keys grouped by bucket and each ranked inside its (small) bucket.
template <int BS>
__device__ void fixup_block(const Sim &S, int s, int *lds) {
  const unsigned long long nnew = S.sc->nnew[s];
  if (nnew == 0) return;
  const int64_t n = (int64_t)S.sc->n[s];
  int64_t nval = (int64_t)nnew;
  if (nval > S.max_products) nval = S.max_products;
  if (nval > S.cap[s] - n) nval = S.cap[s] - n;
  int *bstart = lds, *fill = lds + NBKT;
  __shared__ long long scan_buf[BS];
  constexpr int PER = NBKT / BS;
  int *cnt = S.bcnt + s * NBKT;
  long long loc = 0;
  for (int j = 0; j < PER; ++j) loc += cnt[threadIdx.x * PER + j];
  long long tot;
  long long run = block_exclusive_scan<BS, long long>(loc, scan_buf, tot);
  for (int j = 0; j < PER; ++j) {
    const int b = threadIdx.x * PER + j;
    bstart[b] = (int)run;
    run += cnt[b];
    cnt[b] = 0;
    fill[b] = 0;
  }
  __syncthreads();
  if (tot != nval) {                 // counts and keys disagree: refuse rather than scatter out of range
    if (threadIdx.x == 0) {
      atomicOr(&S.sc->err, (uint32_t)E_CAPACITY);
      S.sc->nnew[s] = 0ull;
    }
    return;
  }
  uint64_t *tmp = S.ptmp[s];
  for (int64_t k = threadIdx.x; k < nval; k += BS) {
    const int b = S.pbkt[s][k];
    tmp[bstart[b] + atomicAdd(&fill[b], 1)] = S.pkey[s][k];
  }
  __threadfence_block();
  __syncthreads();
  const uint32_t next = S.sc->next_id[s];
  for (int64_t q = threadIdx.x; q < nval; q += BS) {
    int lo = 0, hi = NBKT - 1;                     // bucket holding position q
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (bstart[mid] <= q) lo = mid; else hi = mid - 1;
    }
    const int64_t b0 = bstart[lo], b1 = lo + 1 < NBKT ? bstart[lo + 1] : nval;
    const uint64_t key = tmp[q], parent = key >> 24;
    int64_t rank = b0;
    for (int64_t r = b0; r < b1; ++r) rank += (tmp[r] >> 24) < parent;
    S.p[s].id[n + (int64_t)(key & 0xFFFFFFull)] = next + (uint32_t)rank;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if ((uint64_t)next + (uint64_t)nval > 0xFFFFFFFFull) atomicOr(&S.sc->err, (uint32_t)E_IDOVERFLOW);
    S.sc->next_id[s] = next + (uint32_t)nval;
    S.sc->n[s] = (unsigned long long)(n + nval);
    S.sc->nnew[s] = 0ull;
  }
}

template <int BS, int NPER>
__global__ __launch_bounds__(BS) void k_field(Sim S, int64_t step, int mode) {
  extern __shared__ int dyn_fix[];
  if (blockIdx.x == 0) field_block<BS, NPER>(S, step, mode);
  else fixup_block<BS>(S, blockIdx.x - 1, dyn_fix);
}

// The electron partials into Q and, in the block that finishes last (a
// ticket), the field of the next step; NSP more blocks assign the product ids.
// One launch instead of k_reduce + k_field for the steps between two ion steps,
// where nothing else changes Q in between.  Reduction block r sums rows
// b = r / nx, r / nx + RY, ... of node column r % nx.
constexpr int RF_ROWS = 32;

template <int BS, int NPER>
__global__ __launch_bounds__(BS) void k_reduce_field(Sim S, int push_grid, int64_t next_step, int nred) {
  extern __shared__ int dyn_fix[];
  __shared__ int last;
  __shared__ int done[BS / 64];
  const int nn = S.ng + 1;
  if ((int)blockIdx.x >= nred) {
    fixup_block<BS>(S, (int)blockIdx.x - nred, dyn_fix);
    return;
  }
  const int nx = (nn + BS - 1) / BS;
  const int jx = (int)blockIdx.x % nx, y = (int)blockIdx.x / nx;
  const int j = jx * BS + threadIdx.x;
  unsigned long long old = 0ull;
  if (j < nn) {
    unsigned long long sum = 0ull;
    for (int b = y; b < push_grid; b += RF_ROWS) sum += S.part[(size_t)b * nn + j];
    if (sum) old = atomicAdd(&S.Q[j], sum);
  }
  // the returned values are used before the barrier: every add of the block has
  // been performed (device-coherently) before the ticket is taken, with no cache
  // write-back or invalidation of a release / acquire fence
  if ((threadIdx.x & 63) == 0) done[threadIdx.x >> 6] = (int)(old >> 63);
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(&S.sc->field_ticket, 1u) == (uint32_t)(nred - 1);
  __syncthreads();
  if (!last) return;
  if (threadIdx.x == 0) S.sc->field_ticket = 0u;
  field_block<BS, NPER, true>(S, next_step, 0);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_fixup(Sim S) {
  extern __shared__ int dyn_fix[];
  fixup_block<BS>(S, blockIdx.x, dyn_fix);
}

// ---------------------------------------------------------------- particle step
// A block owns a contiguous chunk of the store (a multiple of GROUP slots).  Per
// pass each thread takes GROUP (ions) or ESLOTS (electrons) consecutive particles
// with 128-bit loads and stores, keeps consecutive deposits into one cell in
// registers, and queues the slots of collision candidates in LDS; after the pass
// the block (ions) or the wave (electrons) works the queue with all its lanes.  The block's charge histogram stays in LDS and is written
// out as one partial per block; k_reduce adds the partials into the species
// histogram, so no global atomics are needed for the bulk of the charge.
constexpr int GROUP = 8;
#ifndef PICMCC_CAND_ILP
#define PICMCC_CAND_ILP 1
#endif
constexpr int CAND_ILP = PICMCC_CAND_ILP;   // candidates whose gathers a thread keeps in flight
#ifndef PICMCC_FFE_SLOTS
#define PICMCC_FFE_SLOTS 2
#endif
// electron slots per lane whose free-flight ends a wave lists before working them
constexpr int FFE_SLOTS = PICMCC_FFE_SLOTS;
// electron slots per lane in one pass (a pass's fields and the next pass's are live
// together, so the pass is half as wide as the ion one)
constexpr int ESLOTS = 4;
static_assert(GROUP % ESLOTS == 0 && ESLOTS % FFE_SLOTS == 0, "FFE_SLOTS divides ESLOTS divides GROUP");
// outcome flags of a listed free-flight end, in the (zero) cell bits of its new flight
constexpr uint32_t FFE_CAND = 1u, FFE_REDRAW = 2u;

// energies of particles absorbed at x = 0 / x = L, per block
struct WallHist { unsigned int iedf[2][NBIN]; };

struct PushShared {
  unsigned long long *Q;   // [nn] charge of this species, block-local
  float *E;                // [nn] node field
  float *N;                // [nn] O2+ node density (O- kernel)
  float *tab;              // [np][ntab]
  float *ttot;             // [ntab] sum_p scale_p sigma_p (electrons: early null test)
  unsigned short *queue;   // [GROUP BS] candidate slots relative to the pass base
  // electrons: state of the first rq_cap candidates of a pass, written by their
  // owning thread from registers so that the block does not re-read it from HBM
  int32_t *rw;
  float *roff, *rvx, *rvy, *rvz;
  uint32_t *rid;
  unsigned short *rslot;
  // electrons: free-flight ends of FFE_SLOTS slots per lane, listed per wave (id,
  // then the outcome word; squared speed, negative for a capped flight)
  uint32_t *fid;
  float *fv2;
  const StepCtx *cx;       // step-start state, in the block's LDS
};

__device__ __forceinline__ size_t align_up(size_t x) { return (x + 15) & ~(size_t)15; }

struct BlockCounts { unsigned int c[NCOUNT]; };

// per-thread tallies of the frequent outcomes, added to the block counters once
struct ThreadCounts { unsigned int push = 0u, cand = 0u, nul = 0u; };

// adds the number of active lanes to one block counter with a single LDS atomic
__device__ __forceinline__ void count_lanes(BlockCounts &bc, int idx) {
  const unsigned long long act = __ballot(1);
  if (__lane_id() == __ffsll((long long)act) - 1) atomicAdd(&bc.c[idx], (unsigned int)__popcll(act));
}

// consecutive deposits into one cell, kept in registers
struct DepRun {
  int cell;
  unsigned long long l, r;
  __device__ __forceinline__ DepRun() : cell(-1), l(0ull), r(0ull) {}
  __device__ __forceinline__ void flush(unsigned long long *sQ) {
    if (cell >= 0) { atomicAdd(&sQ[cell], l); atomicAdd(&sQ[cell + 1], r); }
    cell = -1; l = 0ull; r = 0ull;
  }
  __device__ __forceinline__ void add(unsigned long long *sQ, int c, float off) {
    const unsigned long long a = cic_a(off);
    if (c != cell) { flush(sQ); cell = c; }
    l += 4294967296ull - a;
    r += a;
  }
};

// one product of species s from parent (ps, pid)
__device__ __forceinline__ void emit(const Sim &S, const StepCtx &cx, int s, int ps, uint32_t pid, int32_t w,
                                     float off, float vx, float vy, float vz) {
  const int64_t slot = append(S, cx, s, ps, pid);
  if (slot >= 0) put(S.p[s], slot, w, off, vx, vy, vz);
}

// free flight in steps from an FP32 draw (the 1e-6 decision band covers FP32)
__device__ __forceinline__ uint32_t new_flight_f(float inv_nd, uint32_t x) {
  // tau = -ln u / (nu_max dt); inv_nd = 1 / (nu_max dt) (0 when nothing collides)
  const float tau = inv_nd > 0.0f ? -__log2f(unif(x)) * (0.69314718055994531f * inv_nd) : (float)CD_MAX;
  if (!(tau < (float)CD_MAX)) return ((uint32_t)CD_MAX << W_CD_SHIFT) | W_CAP;
  return (uint32_t)(1 + (int)tau) << W_CD_SHIFT;
}

// state of a collision candidate, gathered before any of it is used
struct Cand { int64_t i; int32_t w; uint32_t id; float off, vx, vy, vz; };

__device__ __forceinline__ Cand load_cand(const Particles &P, int64_t i) {
  Cand c;
  c.i = i; c.w = P.w[i]; c.id = P.id[i]; c.off = P.off[i]; c.vx = P.vx[i]; c.vy = P.vy[i]; c.vz = P.vz[i];
  return c;
}

// upper bound of the electron collision rate at energy ec over nu_max, times the
// relative speed g: most free-flight ends fall above it and are null collisions
__device__ __forceinline__ float electron_bound(const PushShared &sh, TabPos tp, float g) {
  return fmaf(tp.w, sh.ttot[tp.i + 1] - sh.ttot[tp.i], sh.ttot[tp.i]) * g;
}

// energy of an electron for the tables: clamped into [emin, emax], and the speed
// that goes with the clamped energy
struct ECand { float e, ec, g; bool clamped; };

__device__ __forceinline__ ECand electron_energy(const Sim &S, float v2) {
  ECand r;
  r.e = S.half_m_e[0] * v2;
  r.ec = r.e;
  r.clamped = false;
  if (r.ec < S.emin) { r.ec = S.emin; r.clamped = true; }
  else if (r.ec > S.emax) { r.ec = S.emax; r.clamped = true; }
  r.g = r.clamped ? sqrtf(S.two_e_m[0] * r.ec) : sqrtf(v2);
  return r;
}

// Electron whose free flight ended this step and whose draw fell below the
// rate bound: the channel is chosen from the tables; the new free flight is
// already in its cell word (post-push state in q).
__device__ void collide_electron(const Sim &S, int64_t step, const Cand &q, PushShared sh, BlockCounts &bc,
                                 ThreadCounts &tc) {
  const Particles &P = S.p[0];
  const int64_t i = q.i;
  const float off = q.off;
  const uint32_t id = q.id;
  const float vx = q.vx, vy = q.vy, vz = q.vz;
  const int cell = q.w & (int32_t)W_CELL;
  const U4 c = draw(S, 0, id, step, P_CAND, 0);
  const float v2 = vx * vx + vy * vy + vz * vz;
  const ECand en = electron_energy(S, v2);
  const float e = en.e, ec = en.ec, g = en.g;
  const TabPos tp = tab_pos(S, ec);
  const float target = unif(c.y);
  int chosen = -1, kind = 0;
  float eth = 0.0f, tmr = 0.0f;
  {
    float acc = 0.0f;
    const int np = S.nproc_sp[0];
    for (int k = 0; k < np; ++k) {
      const ProcDev &pd = S.proc[0][k];
      const float sg = ec < pd.e_th ? 0.0f : tab_sigma(sh.tab + k * S.ntab, tp);
      acc = fmaf(pd.scale * sg, g, acc);
      if (target < acc) { chosen = pd.tab; kind = pd.kind; eth = pd.e_th; tmr = pd.tm_ratio; break; }
    }
  }
  log_event(S, step, 0, id, chosen);
  if (chosen < 0) {
    dep_lds(sh.Q, cell, off);
    ++tc.nul;
    return;
  }
  atomicAdd(&bc.c[C_EVENT + chosen], 1u);
  if (sh.cx->meta_on && chosen == sh.cx->meta_tab) dep_global(S.meta_src, cell, off);   // an O2(a) is born here
  float d0, d1, d2;
  iso_dir(c.z, c.w, d0, d1, d2);
  float enew;
  if (kind == K_ELASTIC) {
    const float vm = sqrtf(v2);
    const float cchi = vm > 0.0f ? (vx * d0 + vy * d1 + vz * d2) / vm : 0.0f;
    enew = e * (1.0f - tmr * (1.0f - cchi));
  } else if (kind == K_EXCITE) {
    enew = e - eth;
  } else if (kind == K_IONIZE) {
    const U4 p0 = draw(S, 0, id, step, P_PROD, 0);
    const U4 p1 = draw(S, 0, id, step, P_PROD, 1);
    const float er = e - eth, r = unif(p0.x);
    enew = (1.0f - r) * er;
    // keys of both products: the two reservations are in flight together
    const unsigned long long act = __ballot(1);
    const int leader = __ffsll((long long)act) - 1;
    unsigned long long be = 0ull, bi = 0ull;
    if (__lane_id() == leader) {
      be = atomicAdd(&S.sc->nnew[0], (unsigned long long)__popcll(act));
      bi = atomicAdd(&S.sc->nnew[1], (unsigned long long)__popcll(act));
    }
    be = __shfl(be, leader, 64);
    bi = __shfl(bi, leader, 64);
    const StepCtx &cx = *sh.cx;
    {                                          // secondary electron, isotropic, energy r E_r
      float s0, s1, s2;
      iso_dir(p0.y, p0.z, s0, s1, s2);
      const float vm = sqrtf(S.two_e_m[0] * fmaxf(r * er, 0.0f));
      const int64_t slot = place(S, cx, 0, 0, id, be + lane_rank(act));
      if (slot >= 0)
        put(S.p[0], slot, cell | (int32_t)new_flight_f(S.inv_nd_ef, p0.w), off, vm * s0, vm * s1, vm * s2);
      dep_lds(sh.Q, cell, off);
      count_lanes(bc, C_BORN + 0);
    }
    {                                          // O2+ from the 300 K reservoir
      float z0, z1, z2, z3;
      normals(p1.x, p1.y, z0, z1);
      normals(p1.z, p1.w, z2, z3);
      const float vt = S.vt_gas[1];
      const int64_t slot = place(S, cx, 1, 0, id, bi + lane_rank(act));
      if (slot >= 0) put(S.p[1], slot, cell, off, vt * z0, vt * z1, vt * z2);
      dep_global(S.Q + (size_t)(S.ng + 1), cell, off);
      count_lanes(bc, C_BORN + 1);
    }
  } else {                                     // attachment: the electron becomes an O-
    const U4 p1 = draw(S, 0, id, step, P_PROD, 1);
    float z0, z1, z2, z3;
    normals(p1.x, p1.y, z0, z1);
    normals(p1.z, p1.w, z2, z3);
    const float vt = S.vt_gas[2];
    emit(S, *sh.cx, 2, 0, id, cell, off, vt * z0, vt * z1, vt * z2);
    dep_global(S.Q + (size_t)2 * (S.ng + 1), cell, off);
    count_lanes(bc, C_BORN + 2);
    P.w[i] = W_DEAD;
    return;
  }
  const float vn = sqrtf(S.two_e_m[0] * fmaxf(enew, 0.0f));
  P.vx[i] = vn * d0;
  P.vy[i] = vn * d1;
  P.vz[i] = vn * d2;
  dep_lds(sh.Q, cell, off);
}

// ion collision candidate: O2+ charge exchange; O- neutralisation against the
// O2+ grid density or associative detachment on O2(a), Eq. (1)
template <int S_>
__device__ void collide_ion(const Sim &S, int64_t step, const Cand &q, PushShared sh, BlockCounts &bc,
                            ThreadCounts &tc, float inv_numax) {
  const Particles &P = S.p[S_];
  const int64_t i = q.i;
  const int32_t w = q.w;
  const float off = q.off;
  const uint32_t id = q.id;
  const float vx = q.vx, vy = q.vy, vz = q.vz;
  const int cell = w & (int32_t)W_CELL;
  ++tc.cand;
  const U4 c = draw(S, S_, id, step, P_CAND, 0);
  const U4 t = draw(S, S_, id, step, P_TARGET, 0);
  float z0, z1, z2, z3;
  normals(t.x, t.y, z0, z1);
  normals(t.z, t.w, z2, z3);
  const float target = unif(c.y);
  float acc = 0.0f, erel_c = 0.0f, pvx = 0.0f, pvy = 0.0f, pvz = 0.0f, eth_c = 0.0f, cmf = 0.0f;
  int chosen = -1, kind = 0;
  const int np = S.nproc_sp[S_];
  for (int k = 0; k < np; ++k) {
    const ProcDev &pd = S.proc[S_][k];
    const float ux = pd.vt * z0, uy = pd.vt * z1, uz = pd.vt * z2;
    const float gx = vx - ux, gy = vy - uy, gz = vz - uz;
    const float g2 = gx * gx + gy * gy + gz * gz;
    const float erel = pd.half_mu_e * g2;                // relative kinetic energy [eV]
    float ec = erel;
    bool cl = false;
    if (ec < S.emin) { ec = S.emin; cl = true; }
    else if (ec > S.emax) { ec = S.emax; cl = true; }
    if (cl) count_lanes(bc, C_CLAMP);
    const float g = cl ? sqrtf(pd.inv_mu2 * ec) : sqrtf(g2);
    float dens;
    if (pd.target == T_GRIDPOS) dens = fmaf(off, sh.N[cell + 1] - sh.N[cell], sh.N[cell]) * inv_numax;
    else if (pd.target == T_O2A && sh.cx->meta_on)
      dens = fmaf(off, S.na_f[cell + 1] - S.na_f[cell], S.na_f[cell]) * inv_numax;
    else dens = pd.scale * (S_ == 2 ? inv_numax : 1.0f);
    const float sg = ec < pd.e_th ? 0.0f : tab_sigma(sh.tab + k * S.ntab, tab_pos(S, ec));
    acc = fmaf(dens * sg, g, acc);
    if (chosen < 0 && target < acc) {
      chosen = pd.tab; kind = pd.kind; erel_c = erel; pvx = ux; pvy = uy; pvz = uz; eth_c = pd.e_th; cmf = pd.cmf;
    }
  }
  log_event(S, step, S_, id, chosen);
  if (chosen < 0) {
    P.w[i] = cell;
    dep_lds(sh.Q, cell, off);
    ++tc.nul;
    return;
  }
  atomicAdd(&bc.c[C_EVENT + chosen], 1u);
  if (kind == K_CX) {                          // the ion leaves with the neutral's velocity
    P.w[i] = cell;
    P.vx[i] = pvx; P.vy[i] = pvy; P.vz[i] = pvz;
    dep_lds(sh.Q, cell, off);
  } else if (kind == K_ION_ELASTIC) {          // isotropic in the centre-of-mass frame (Table 1 (8))
    const U4 p0 = draw(S, S_, id, step, P_PROD, 0);
    float d0, d1, d2;
    iso_dir(p0.x, p0.y, d0, d1, d2);
    const float gx = vx - pvx, gy = vy - pvy, gz = vz - pvz;
    const float gm = sqrtf(gx * gx + gy * gy + gz * gz) * cmf;
    P.w[i] = cell;
    P.vx[i] = fmaf(gm, d0, fmaf(-cmf, gx, vx));
    P.vy[i] = fmaf(gm, d1, fmaf(-cmf, gy, vy));
    P.vz[i] = fmaf(gm, d2, fmaf(-cmf, gz, vz));
    dep_lds(sh.Q, cell, off);
  } else if (kind == K_NEUTRALIZE) {           // partner O2+ removed by the pairing rounds
    P.w[i] = W_DEAD;
    atomicAdd(&S.kleft[cell], 1);
    S.sc->pair_active = 1;
  } else {                                     // K_DETACH: electron with the relative energy above threshold
    const U4 p0 = draw(S, S_, id, step, P_PROD, 0);
    float d0, d1, d2;
    iso_dir(p0.y, p0.z, d0, d1, d2);
    const float vm = sqrtf(S.two_e_m[0] * fmaxf(erel_c - eth_c, 0.0f));
    emit(S, *sh.cx, 0, S_, id, cell | (int32_t)new_flight_f(S.inv_nd_ef, p0.w), off, vm * d0, vm * d1, vm * d2);
    dep_global(S.Q, cell, off);
    count_lanes(bc, C_BORN + 0);
    P.w[i] = W_DEAD;
  }
}

__device__ __forceinline__ int64_t push_chunk(int64_t N, int grid) {
  int64_t chunk = (N + grid - 1) / grid;
  return (chunk + GROUP - 1) / GROUP * GROUP;
}

#ifndef PICMCC_PUSH_WAVES
#define PICMCC_PUSH_WAVES 4
#endif
// block-level LDS state of a push run besides the dynamic part
struct PushLds {
  int qn[16];              // queued candidates of each wave in the current pass
  BlockCounts bc;
  WallHist wall;
  StepCtx cx;
};

// Push of the slots [begin, end) of species S_ by one block (begin a multiple of
// GROUP).  The block's charge histogram is written to part_row (ng + 1 entries).
template <int BS, int S_>
__device__ __forceinline__ void push_run(const Sim &S, int64_t step, int64_t begin, int64_t end,
                                         unsigned long long *part_row, unsigned char *smem, PushLds &pl) {
  int *qn = pl.qn;
  BlockCounts &bc = pl.bc;
  WallHist &wall = pl.wall;
  const int ng = S.ng, nn = ng + 1;
  const int np = S.nproc_sp[S_];
  PushShared sh;
  size_t o = 0;
  sh.Q = (unsigned long long *)(smem + o); o = align_up(o + sizeof(unsigned long long) * nn);
  sh.E = (float *)(smem + o); o = align_up(o + sizeof(float) * nn);
  sh.N = (float *)(smem + o); if (S_ == 2) o = align_up(o + sizeof(float) * nn);
  sh.tab = (float *)(smem + o); o = align_up(o + sizeof(float) * np * S.ntab);
  sh.ttot = (float *)(smem + o); if (S_ == 0) o = align_up(o + sizeof(float) * S.ntab);
  sh.queue = (unsigned short *)(smem + o); o = align_up(o + sizeof(unsigned short) * GROUP * BS);
  sh.fid = (uint32_t *)(smem + o); if (S_ == 0) o += sizeof(uint32_t) * FFE_SLOTS * BS;
  sh.fv2 = (float *)(smem + o); if (S_ == 0) o += sizeof(float) * FFE_SLOTS * BS;
  const int rq_cap = S_ == 0 ? S.rq_cap : 0;
  sh.rw = (int32_t *)(smem + o); o += 4 * (size_t)rq_cap;
  sh.roff = (float *)(smem + o); o += 4 * (size_t)rq_cap;
  sh.rvx = (float *)(smem + o); o += 4 * (size_t)rq_cap;
  sh.rvy = (float *)(smem + o); o += 4 * (size_t)rq_cap;
  sh.rvz = (float *)(smem + o); o += 4 * (size_t)rq_cap;
  sh.rid = (uint32_t *)(smem + o); o += 4 * (size_t)rq_cap;
  sh.rslot = (unsigned short *)(smem + o);
  for (int j = threadIdx.x; j < 2 * NBIN; j += BS) wall.iedf[j / NBIN][j % NBIN] = 0u;
  for (int j = threadIdx.x; j < nn; j += BS) {
    sh.Q[j] = 0ull;
    sh.E[j] = S.E[j];
    if (S_ == 2) sh.N[j] = S.nplus_c * ((j == 0 || j == ng) ? 2.0f : 1.0f) * (float)S.Q[nn + j];
  }
  for (int k = 0; k < np; ++k)
    for (int j = threadIdx.x; j < S.ntab; j += BS) sh.tab[k * S.ntab + j] = S.sigma[S.proc[S_][k].tab * S.ntab + j];
  if (S_ == 0)
    for (int j = threadIdx.x; j < S.ntab; j += BS) sh.ttot[j] = S.ttot_e[j];
  for (int k = threadIdx.x; k < NCOUNT; k += BS) bc.c[k] = 0u;
  if (threadIdx.x < 16) qn[threadIdx.x] = 0;
  if (threadIdx.x == 0) pl.cx = step_ctx(S);
  sh.cx = &pl.cx;
  float inv_numax = 0.0f;
  double pnull = 0.0;
  if (S_ == 1) pnull = S.pnull_pos;
  if (S_ == 2) { inv_numax = S.sc->inv_numax_neg; pnull = S.sc->pnull_neg; }
  __syncthreads();

  const Particles &P = S.p[S_];
  const float qmdt = S.qmdt[S_], dtdx = S.dtdx[S_];
  const bool nocoll = (S.flags & F_NO_COLL) != 0;
  const int lane = threadIdx.x & 63;
  // Electrons: each wave lists the free-flight ends of FFE_SLOTS slots per lane and
  // works the list on full lanes (draw, next flight, rate bound), then queues the
  // collision candidates of its own ESLOTS * 64 slots of a pass (their state as LDS
  // records while the wave's share lasts) and works them off itself, so the waves
  // of a block never wait for each other inside a run.  Ions: one queue per block,
  // worked off by all its lanes between two barriers.
  const int wv = threadIdx.x >> 6;
  unsigned short *wq = sh.queue + wv * GROUP * 64;
  const int rqw = rq_cap / (BS / 64), r0 = wv * rqw;
  ThreadCounts tc;
  DepRun run;
  if constexpr (S_ == 0) {
    const unsigned long long below = (1ull << lane) - 1ull;
    uint32_t *fid = sh.fid + wv * FFE_SLOTS * 64;
    float *fv2 = sh.fv2 + wv * FFE_SLOTS * 64;
    // A lane works ESLOTS consecutive slots per pass, and the fields of its next
    // pass are loaded before the work of this one (the pushes, the free-flight ends
    // and the wave's candidate queue all run under those loads).  Every cache line
    // of the cold fields is needed anyway (a third of the electrons end a free
    // flight each step), so they stream in with the hot ones.
    struct ESlots {
      int32_t w[ESLOTS];
      float off[ESLOTS], vx[ESLOTS], vy[ESLOTS], vz[ESLOTS];
      uint32_t id[ESLOTS];
    };
    auto load_slots = [&](const int64_t ub, ESlots &d) __attribute__((always_inline)) {
      const int64_t i0 = ub + (int64_t)ESLOTS * lane;
      const int nv = i0 < end ? (int)min((int64_t)ESLOTS, end - i0) : 0;
      if (nv > 0) {
        const int4 wa = *reinterpret_cast<const int4 *>(P.w + i0);
        const float4 oa = *reinterpret_cast<const float4 *>(P.off + i0), va = *reinterpret_cast<const float4 *>(P.vx + i0);
        const uint4 ia = *reinterpret_cast<const uint4 *>(P.id + i0);
        const float4 ya = *reinterpret_cast<const float4 *>(P.vy + i0), za = *reinterpret_cast<const float4 *>(P.vz + i0);
        d.w[0] = wa.x; d.w[1] = wa.y; d.w[2] = wa.z; d.w[3] = wa.w;
        d.off[0] = oa.x; d.off[1] = oa.y; d.off[2] = oa.z; d.off[3] = oa.w;
        d.vx[0] = va.x; d.vx[1] = va.y; d.vx[2] = va.z; d.vx[3] = va.w;
        d.id[0] = ia.x; d.id[1] = ia.y; d.id[2] = ia.z; d.id[3] = ia.w;
        d.vy[0] = ya.x; d.vy[1] = ya.y; d.vy[2] = ya.z; d.vy[3] = ya.w;
        d.vz[0] = za.x; d.vz[1] = za.y; d.vz[2] = za.z; d.vz[3] = za.w;
#pragma unroll
        for (int k = 0; k < ESLOTS; ++k)          // slots past the block's range are not its own
          if (k >= nv) d.w[k] = W_DEAD;
      } else {
#pragma unroll
        for (int k = 0; k < ESLOTS; ++k) { d.w[k] = W_DEAD; d.off[k] = d.vx[k] = d.vy[k] = d.vz[k] = 0.0f; d.id[k] = 0u; }
      }
    };
    // one wave's pass over the ESLOTS * 64 slots from ub (wave-uniform)
    auto pass = [&](const int64_t ub, const ESlots &d) __attribute__((always_inline)) {
      const int64_t i0 = ub + (int64_t)ESLOTS * lane;
      const int nv = i0 < end ? (int)min((int64_t)ESLOTS, end - i0) : 0;
      int32_t w[ESLOTS];
      float off[ESLOTS], vx[ESLOTS], vy[ESLOTS], vz[ESLOTS];
      uint32_t id[ESLOTS];
#pragma unroll
      for (int k = 0; k < ESLOTS; ++k) {
        w[k] = d.w[k]; off[k] = d.off[k]; vx[k] = d.vx[k]; vy[k] = d.vy[k]; vz[k] = d.vz[k]; id[k] = d.id[k];
      }
      int nq = 0;                                  // candidates this wave queued in this pass
#pragma unroll
      for (int k0 = 0; k0 < ESLOTS; k0 += FFE_SLOTS) {
        // push FFE_SLOTS slots; list the ones whose free flight ends
        unsigned int ended = 0u;
        int nf = 0;
#pragma unroll
        for (int k = k0; k < k0 + FFE_SLOTS; ++k) {
          bool fe = false;
          if (k < nv && w[k] >= 0) {
            ++tc.push;
            const int cell = w[k] & (int32_t)W_CELL;
            // gather (linear weighting), leapfrog velocity then position
            const float e0 = sh.E[cell], e1 = sh.E[cell + 1];
            const float v = fmaf(qmdt, fmaf(off[k], e1 - e0, e0), vx[k]);
            const float xn = fmaf(v, dtdx, off[k]);
            vx[k] = v;
            if (!(fabsf(xn) < 1.0e9f)) {
              atomicOr(&S.sc->err, (uint32_t)E_NAN);
              w[k] = W_DEAD;
            } else {
              const float fl = floorf(xn);
              int nc = cell + (int)fl;
              float no = xn - fl;
              if (no >= 1.0f) { nc += 1; no -= 1.0f; }
              off[k] = no;
              if (nc < 0 || nc >= ng) {                // absorbed by an electrode
                const int side = nc < 0 ? 0 : 1;
                const float en = S.half_m_e[0] * (v * v + vy[k] * vy[k] + vz[k] * vz[k]);
                atomicAdd(&wall.iedf[side][ebin(en)], 1u);
                atomicAdd(&bc.c[(side ? C_ABSL : C_ABS0) + 0], 1u);
                w[k] = W_DEAD;
                if (S.event_cap > 0) log_event(S, step, 0, id[k], -3);
              } else {
                const int cd = w[k] >> W_CD_SHIFT;
                const int cdn = nocoll ? cd : cd - 1;
                if (cdn > 0 || nocoll) {
                  w[k] = nc | (w[k] & (int32_t)W_CAP) | (cdn << W_CD_SHIFT);
                  run.add(sh.Q, nc, no);
                } else {                               // the free flight ends: listed
                  w[k] = nc | (w[k] & (int32_t)W_CAP);
                  fe = true;
                }
              }
            }
          }
          const unsigned long long m = __ballot(fe);
          if (fe) {
            const int e = nf + __popcll(m & below);
            fid[e] = id[k];
            fv2[e] = (w[k] & (int32_t)W_CAP) ? -1.0f : vx[k] * vx[k] + vy[k] * vy[k] + vz[k] * vz[k];
          }
          nf += __popcll(m);
          ended |= (fe ? 1u : 0u) << (k - k0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // the listed ends on full lanes: next flight, and the early null test
        // against the summed rate table (the channel is chosen after the pass)
        for (int e = lane; e < nf; e += 64) {
          const uint32_t pid = fid[e];
          const float v2 = fv2[e];
          const U4 c = draw(S, 0, pid, step, P_CAND, 0);
          uint32_t r = new_flight_f(S.inv_nd_ef, c.x);
          if (v2 < 0.0f) {                           // end of a capped flight: no collision
            r |= FFE_REDRAW;
            count_lanes(bc, C_REDRAW);
          } else {
            ++tc.cand;
            const ECand en = electron_energy(S, v2);
            if (en.clamped) count_lanes(bc, C_CLAMP);
            const TabPos tp = tab_pos(S, en.ec);
            if (unif(c.y) < electron_bound(sh, tp, en.g) * 1.000001f) r |= FFE_CAND;
          }
          fid[e] = r;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // outcomes back to the slots: null collisions deposit, candidates are queued
        int f = 0;
#pragma unroll
        for (int k = k0; k < k0 + FFE_SLOTS; ++k) {
          const bool fe = (ended >> (k - k0)) & 1u;
          const unsigned long long m = __ballot(fe);
          bool cand = false;
          if (fe) {
            const uint32_t r = fid[f + __popcll(m & below)];
            const int cell = w[k] & (int32_t)W_CELL;
            w[k] = cell | (int32_t)(r & ~W_CELL);
            if (r & FFE_CAND) {
              cand = true;
            } else {
              run.add(sh.Q, cell, off[k]);
              if (r & FFE_REDRAW) {
                if (S.event_cap > 0) log_event(S, step, 0, id[k], -2);
              } else {
                ++tc.nul;
                if (S.event_cap > 0) log_event(S, step, 0, id[k], -1);
              }
            }
          }
          f += __popcll(m);
          const unsigned long long mc = __ballot(cand);
          if (cand) {
            const int e = nq + __popcll(mc & below);
            const unsigned short slot = (unsigned short)(i0 - ub + k);
            if (e < rqw) {
              const int r = r0 + e;
              sh.rw[r] = w[k]; sh.roff[r] = off[k]; sh.rvx[r] = vx[k]; sh.rvy[r] = vy[k]; sh.rvz[r] = vz[k];
              sh.rid[r] = id[k]; sh.rslot[r] = slot;
            } else {
              wq[e - rqw] = slot;
            }
          }
          nq += __popcll(mc);
        }
        // the outcome list is read: the next slots may list theirs
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      }
      if (nv == ESLOTS) {
        *reinterpret_cast<int4 *>(P.w + i0) = make_int4(w[0], w[1], w[2], w[3]);
        *reinterpret_cast<float4 *>(P.off + i0) = make_float4(off[0], off[1], off[2], off[3]);
        *reinterpret_cast<float4 *>(P.vx + i0) = make_float4(vx[0], vx[1], vx[2], vx[3]);
      } else {
        for (int k = 0; k < nv; ++k) { P.w[i0 + k] = w[k]; P.off[i0 + k] = off[k]; P.vx[i0 + k] = vx[k]; }
      }
      // the wave's queue is complete: its LDS and global writes are visible to its lanes
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      for (int e = lane; e < nq; e += 64) {
        Cand c;
        if (e < rqw) {
          const int r = r0 + e;
          c.i = ub + sh.rslot[r]; c.w = sh.rw[r]; c.id = sh.rid[r]; c.off = sh.roff[r];
          c.vx = sh.rvx[r]; c.vy = sh.rvy[r]; c.vz = sh.rvz[r];
        } else {
          c = load_cand(P, ub + wq[e - rqw]);
        }
        collide_electron(S, step, c, sh, bc, tc);
      }
      // every lane has read its entries: the next pass may overwrite them
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    };
    // the passes of one wave: ub advances by the block's ESLOTS * BS slots
    const int64_t stride = (int64_t)ESLOTS * BS;
    int64_t ub = begin + (int64_t)wv * ESLOTS * 64;
    ESlots cur, nxt;
    if (ub < end) load_slots(ub, cur);
    for (; ub < end; ub += stride) {
      if (ub + stride < end) load_slots(ub + stride, nxt);
      pass(ub, cur);
      cur = nxt;
    }
  } else {
  int par = 0;
  for (int64_t base = begin; base < end; base += (int64_t)GROUP * BS, par ^= 1) {
    const int64_t i0 = base + (int64_t)GROUP * threadIdx.x;
    unsigned int cmask = 0u;               // candidates of this thread
    if (i0 < end) {
      const int nv = (int)min((int64_t)GROUP, end - i0);
      int32_t w[GROUP];
      float off[GROUP], vx[GROUP];
      uint32_t id[GROUP];
      {
        const int4 wa = *reinterpret_cast<const int4 *>(P.w + i0), wb = *reinterpret_cast<const int4 *>(P.w + i0 + 4);
        const float4 oa = *reinterpret_cast<const float4 *>(P.off + i0), ob = *reinterpret_cast<const float4 *>(P.off + i0 + 4);
        const float4 va = *reinterpret_cast<const float4 *>(P.vx + i0), vb = *reinterpret_cast<const float4 *>(P.vx + i0 + 4);
        w[0] = wa.x; w[1] = wa.y; w[2] = wa.z; w[3] = wa.w; w[4] = wb.x; w[5] = wb.y; w[6] = wb.z; w[7] = wb.w;
        off[0] = oa.x; off[1] = oa.y; off[2] = oa.z; off[3] = oa.w; off[4] = ob.x; off[5] = ob.y; off[6] = ob.z; off[7] = ob.w;
        vx[0] = va.x; vx[1] = va.y; vx[2] = va.z; vx[3] = va.w; vx[4] = vb.x; vx[5] = vb.y; vx[6] = vb.z; vx[7] = vb.w;
        if (!nocoll && pnull > 0.0) {
          const uint4 ia = *reinterpret_cast<const uint4 *>(P.id + i0), ib = *reinterpret_cast<const uint4 *>(P.id + i0 + 4);
          id[0] = ia.x; id[1] = ia.y; id[2] = ia.z; id[3] = ia.w; id[4] = ib.x; id[5] = ib.y; id[6] = ib.z; id[7] = ib.w;
        }
      }
#pragma unroll
      for (int k = 0; k < GROUP; ++k) {
        if (k >= nv || w[k] < 0) continue;
        ++tc.push;
        const int cell = w[k] & (int32_t)W_CELL;
        // gather (linear weighting), leapfrog velocity then position
        const float e0 = sh.E[cell], e1 = sh.E[cell + 1];
        const float v = fmaf(qmdt, fmaf(off[k], e1 - e0, e0), vx[k]);
        const float xn = fmaf(v, dtdx, off[k]);
        vx[k] = v;
        if (!(fabsf(xn) < 1.0e9f)) {
          atomicOr(&S.sc->err, (uint32_t)E_NAN);
          w[k] = W_DEAD;
          continue;
        }
        const float fl = floorf(xn);
        int nc = cell + (int)fl;
        float no = xn - fl;
        if (no >= 1.0f) { nc += 1; no -= 1.0f; }
        off[k] = no;
        if (nc < 0 || nc >= ng) {                      // absorbed by an electrode
          const int side = nc < 0 ? 0 : 1;
          const float uy = P.vy[i0 + k], uz = P.vz[i0 + k];
          const float en = S.half_m_e[S_] * (v * v + uy * uy + uz * uz);
          atomicAdd(&wall.iedf[side][ebin(en)], 1u);
          atomicAdd(&bc.c[(side ? C_ABSL : C_ABS0) + S_], 1u);
          w[k] = W_DEAD;
          if (S.event_cap > 0) log_event(S, step, S_, P.id[i0 + k], -3);
          continue;
        }
        w[k] = nc;
        bool cand = false;
        if (!nocoll && pnull > 0.0) cand = (double)unif(draw(S, S_, id[k], step, P_CAND, 0).x) < pnull;
        if (cand) cmask |= 1u << k;
        else run.add(sh.Q, nc, no);
      }
      if (nv == GROUP) {
        *reinterpret_cast<int4 *>(P.w + i0) = make_int4(w[0], w[1], w[2], w[3]);
        *reinterpret_cast<int4 *>(P.w + i0 + 4) = make_int4(w[4], w[5], w[6], w[7]);
        *reinterpret_cast<float4 *>(P.off + i0) = make_float4(off[0], off[1], off[2], off[3]);
        *reinterpret_cast<float4 *>(P.off + i0 + 4) = make_float4(off[4], off[5], off[6], off[7]);
        *reinterpret_cast<float4 *>(P.vx + i0) = make_float4(vx[0], vx[1], vx[2], vx[3]);
        *reinterpret_cast<float4 *>(P.vx + i0 + 4) = make_float4(vx[4], vx[5], vx[6], vx[7]);
      } else {
        for (int k = 0; k < nv; ++k) { P.w[i0 + k] = w[k]; P.off[i0 + k] = off[k]; P.vx[i0 + k] = vx[k]; }
      }
    }
    // queue the candidates: one LDS atomic per wave
    const int mine = __popc(cmask);
    const int incl = wave_incl_scan(mine);
    int wbase = 0;
    if (lane == 63 && incl > 0) wbase = atomicAdd(&qn[par], incl);
    wbase = __shfl(wbase, 63, 64);
    int q = wbase + incl - mine;
    for (unsigned int m = cmask; m; m &= m - 1) sh.queue[q++] = (unsigned short)(i0 - base + __ffs(m) - 1);
    __syncthreads();
    const int nq = qn[par];
    if (threadIdx.x == 0) qn[par ^ 1] = 0;   // counter of the next pass, unused since the last barrier
    for (int k = threadIdx.x; k < nq; k += CAND_ILP * BS) {
      // gathers of up to CAND_ILP candidates in flight together
      Cand c[CAND_ILP];
      bool h[CAND_ILP];
#pragma unroll
      for (int u = 0; u < CAND_ILP; ++u) {
        h[u] = k + u * BS < nq;
        if (h[u]) c[u] = load_cand(P, base + sh.queue[k + u * BS]);
      }
#pragma unroll
      for (int u = 0; u < CAND_ILP; ++u)
        if (h[u]) collide_ion<S_>(S, step, c[u], sh, bc, tc, inv_numax);
    }
    __syncthreads();
  }
  }
  __syncthreads();
  run.flush(sh.Q);
  atomicAdd(&bc.c[C_PUSH + S_], tc.push);
  if (tc.cand) atomicAdd(&bc.c[C_CAND + S_], tc.cand);
  if (tc.nul) atomicAdd(&bc.c[C_NULL + S_], tc.nul);
  __syncthreads();
  for (int j = threadIdx.x; j < nn; j += BS) part_row[j] = sh.Q[j];
  for (int j = threadIdx.x; j < 2 * NBIN; j += BS)
    if (wall.iedf[j / NBIN][j % NBIN])
      atomicAdd(&S.iedf[(size_t)S_ * 2 * NBIN + j], (unsigned long long)wall.iedf[j / NBIN][j % NBIN]);
  for (int k = threadIdx.x; k < NCOUNT; k += BS)
    if (bc.c[k]) atomicAdd(&S.sc->cnt[k], (unsigned long long)bc.c[k]);
  __syncthreads();   // the LDS may be set up for the next run
}

// Slot range [range[0], range[1]) of this block in an electron push over n slots,
// worked out by one wave.  The previous launch (other step parity) left a cost
// map: its block j spent dur[j] on the slots [begin[j], begin[j + 1]).  The cut
// points are where the cumulative cost reaches equal fractions, rounded to 512
// slots; without a map of this grid the store is cut into equal chunks.
__device__ void balanced_range(const PushBal *B, int par, int64_t n, long long *range) {
  const int G = gridDim.x, b = blockIdx.x, lane = threadIdx.x & 63, prv = par ^ 1;
  long long cut[2];
  if (B->grid[prv] != G) {
    const int64_t chunk = push_chunk(n, G);
    cut[0] = min(n, (int64_t)b * chunk);
    cut[1] = min(n, cut[0] + chunk);
  } else {
    // each lane sums a contiguous segment of the blocks' durations; a wave scan
    // gives the cumulative cost at each segment start
    const int per = (G + 63) / 64, j0 = min(G, lane * per), j1 = min(G, j0 + per);
    double own = 0.0;
    for (int j = j0; j < j1; ++j) own += (double)B->dur[prv][j];
    const double incl = wave_incl_scan(own);
    const double total = __shfl(incl, 63, 64);
    const double before = incl - own;
    for (int e = 0; e < 2; ++e) {
      const double c = total * (double)(b + e) / (double)G;
      double pos = -1.0;                     // slot where the cumulative cost reaches c
      if (b + e == G) {
        pos = (double)n;
      } else if (c >= before && c < incl) {
        double acc = before;
        for (int j = j0; j < j1; ++j) {
          const double d = (double)B->dur[prv][j];
          if (c < acc + d) {
            const double lo = (double)B->begin[prv][j], hi = (double)B->begin[prv][j + 1];
            pos = lo + (c - acc) / d * (hi - lo);
            break;
          }
          acc += d;
        }
      }
      // the one lane that found it hands it to the wave
      const unsigned long long m = __ballot(pos >= 0.0);
      const int src = m ? __ffsll((long long)m) - 1 : 0;
      pos = __shfl(pos, src, 64);
      long long x = m ? (long long)pos : (long long)n;
      x = x / (GROUP * 64) * (GROUP * 64);
      cut[e] = (b + e == G) ? (long long)n : min((long long)n, max(0ll, x));
    }
  }
  if (lane == 0) { range[0] = cut[0]; range[1] = max(cut[0], cut[1]); }
}

// one discharge: electrons in ranges balanced by the previous launch's cost,
// ions by block b pushing the b-th contiguous chunk of the store
template <int BS, int S_>
__global__ __launch_bounds__(BS, PICMCC_PUSH_WAVES) void k_push(Sim S, int64_t step) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ PushLds pl;
  const int64_t N = (int64_t)S.sc->n[S_];
  if (S_ == 0) {           // every block writes its partial row, also for an empty range
    __shared__ long long range[2];
    const long long t0 = (long long)__builtin_amdgcn_s_memrealtime();
    const int par = (int)(step & 1);
    if (threadIdx.x < 64) balanced_range(S.bal, par, N, range);
    __syncthreads();
    const int64_t begin = range[0], end = range[1];
    push_run<BS, S_>(S, step, begin, end, S.part + (size_t)blockIdx.x * (S.ng + 1), smem, pl);
    if (threadIdx.x == 0) {
      const long long t1 = (long long)__builtin_amdgcn_s_memrealtime();
      S.bal->begin[par][blockIdx.x] = begin;
      S.bal->dur[par][blockIdx.x] = max(1ll, t1 - t0);
      if (blockIdx.x == gridDim.x - 1) {
        S.bal->begin[par][gridDim.x] = end;
        S.bal->grid[par] = (int32_t)gridDim.x;
      }
    }
    return;
  }
  const int64_t chunk = push_chunk(N, gridDim.x);
  const int64_t begin = (int64_t)blockIdx.x * chunk;
  const int64_t end = min(N, begin + chunk);
  if (begin >= end) return;
  push_run<BS, S_>(S, step, begin, end, S.part + (size_t)blockIdx.x * (S.ng + 1), smem, pl);
}

// Q[s] += sum of the partial histograms of the blocks that had particles (for
// electrons every block of the push writes one)
template <int BS>
__global__ __launch_bounds__(BS) void k_reduce(Sim S, int s, int push_grid) {
  const int nn = S.ng + 1;
  const int j = blockIdx.x * BS + threadIdx.x;
  if (j >= nn) return;
  const int64_t N = (int64_t)S.sc->n[s];
  const int64_t chunk = push_chunk(N, push_grid);
  const int used = s == 0 ? push_grid : chunk > 0 ? (int)((N + chunk - 1) / chunk) : 0;
  unsigned long long sum = 0ull;
  for (int b = blockIdx.y; b < used; b += gridDim.y) sum += S.part[(size_t)b * nn + j];
  if (sum) atomicAdd(&S.Q[(size_t)s * nn + j], sum);
}

// O- bound of this ion step: nu_max = max_k sum_p n_p H_p[k], with n = the
// largest O2+ node density for neutralisation and C n(O2) for detachment
template <int BS>
__device__ void ionprep_block(const Sim &S) {
  __shared__ double red[BS];
  const int ng = S.ng, nn = ng + 1;
  double nmax = 0.0;
  const double c = (double)S.nplus_c;
  for (int j = threadIdx.x; j < nn; j += BS) {
    const double v = (double)S.Q[nn + j] * ((j == 0 || j == ng) ? 2.0 : 1.0);
    nmax = fmax(nmax, v);
  }
  red[threadIdx.x] = nmax;
  __syncthreads();
  for (int o = BS / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  nmax = red[0] * S.wd;
  __syncthreads();
  double best = 0.0;
  const int np = S.nproc_sp[2];
  for (int k = threadIdx.x; k < S.ntab - 1; k += BS) {
    double sum = 0.0;
    for (int p = 0; p < np; ++p) {
      const ProcDev &pd = S.proc[2][p];
      const double n = pd.target == T_GRIDPOS ? nmax
                     : pd.target == T_O2A ? (S.sc->meta_on ? S.sc->na_max : S.c_meta * S.n_o2) : S.n_o2;
      sum += n * S.hbound[(size_t)pd.tab * (S.ntab - 1) + k];
    }
    best = fmax(best, sum);
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int o = BS / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nu = red[0];
    S.sc->numax_neg = nu;
    S.sc->pnull_neg = 1.0 - exp(-nu * S.dti);
    S.sc->inv_numax_neg = nu > 0.0 ? (float)(1.0 / nu) : 0.0f;
    (void)c;
  }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_ionprep(Sim S) { ionprep_block<BS>(S); }

// Partners of the ion removals of an ion step (Table 1 (17) and (16): O2+, sp = 1;
// (22): O-, sp = 2).  Cell j requested k_j removals (kleft); its partners are the
// k_j ions of species sp that were in the store before the step (slot < n), are
// alive after the pushes and sit in cell j, with the smallest key (pairing draw,
// id) -- all of them when the cell holds fewer, the rest counted as a deficit.
// Exact k-smallest selection per cell in four launches over the store:
//   pair_hist    counts the candidates of flagged cells in 256 bins of the key's
//                top 8 bits (the bins order the keys),
//   pair_select  finds per cell the bin b* where the count reaches k_j: every key
//                below b* is taken, the need = k_j - (keys below b*) smallest keys
//                of bin b* are decided by rank,
//   pair_take    removes the candidates below b* and lists those of bin b*,
//   pair_rank    removes the listed keys whose rank in their cell's list is below
//                the need; its last block closes the pairing of the step.
// The list lives in the species' second particle buffer (free between re-orderings).
constexpr int PAIR_NB = 256;

__device__ __forceinline__ uint32_t pair_draw(const Sim &S, int sp, uint32_t id, int64_t step) {
  return draw(S, sp, id, step, P_PAIR, 0).x;
}

__device__ __forceinline__ int32_t *pair_active_flag(const Sim &S, int sp) {
  return sp == 1 ? &S.sc->pair_active : &S.sc->pair_active_neg;
}

// removes ion i of species sp (cell c, offset off) with its charge
__device__ __forceinline__ void pair_kill(const Sim &S, int sp, int64_t i, int c, float off) {
  unsigned long long *Qs = S.Q + (size_t)sp * (S.ng + 1);
  const unsigned long long a = cic_a(off);
  atomicAdd(&Qs[c], (unsigned long long)(-(long long)(4294967296ull - a)));
  atomicAdd(&Qs[c + 1], (unsigned long long)(-(long long)a));
  S.p[sp].w[i] = W_DEAD;
}

__device__ __forceinline__ void pair_count_kills(const Sim &S, int sp, bool killed) {
  const unsigned long long m = __ballot(killed);
  if (m && __lane_id() == __ffsll((long long)m) - 1)
    atomicAdd(&S.sc->cnt[sp == 1 ? C_PAIRED : C_PAIRED_NEG], (unsigned long long)__popcll(m));
}

// cell words of the four slots from i0 (a multiple of 4; the store's fields are
// 16-byte aligned): one 128-bit load, slots at or beyond n read as dead
__device__ __forceinline__ void load_w4(const int32_t *wp, int64_t i0, int64_t n, int32_t w[4]) {
  if (i0 + 4 <= n) {
    const int4 a = *reinterpret_cast<const int4 *>(wp + i0);
    w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      w[k] = W_DEAD;
      if (i0 + k < n) w[k] = wp[i0 + k];
    }
  }
}

template <int BS>
__device__ void pair_hist(const Sim &S, int64_t step, int sp, int bx, int gx) {
  if (!*pair_active_flag(S, sp)) return;
  if (bx == 0 && threadIdx.x == 0) S.sc->pair_nrec = 0;   // nothing reads it before pair_select
  const int32_t *kl = sp == 1 ? S.kleft : S.kleft_neg;
  const Particles &P = S.p[sp];
  const int64_t N = (int64_t)S.sc->n[sp];
  for (int64_t i0 = 4 * ((int64_t)bx * BS + threadIdx.x); i0 < N; i0 += 4 * (int64_t)gx * BS) {
    int32_t w[4];
    load_w4(P.w, i0, N, w);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (w[k] < 0) continue;
      const int c = w[k] & (int32_t)W_CELL;
      if (kl[c] <= 0) continue;
      const uint32_t x = pair_draw(S, sp, P.id[i0 + k], step);
      atomicAdd(&S.phist[(size_t)c * PAIR_NB + (x >> 24)], 1);
    }
  }
}

// one wave per cell; every cell's record is rewritten, flagged rows are cleared
template <int BS>
__device__ void pair_select(const Sim &S, int sp, int bx, int gx) {
  if (!*pair_active_flag(S, sp)) return;
  int32_t *kl = sp == 1 ? S.kleft : S.kleft_neg;
  const int lane = threadIdx.x & 63;
  const int nw = gx * (BS / 64);
  for (int c = bx * (BS / 64) + (threadIdx.x >> 6); c < S.ng; c += nw) {
    const int k = kl[c];
    PairCell rec = {0, 0, 0, 0};
    if (k > 0) {
      int32_t *row = S.phist + (size_t)c * PAIR_NB + 4 * lane;
      const int4 h4 = *reinterpret_cast<const int4 *>(row);
      const int h[4] = {h4.x, h4.y, h4.z, h4.w};
      const int sum = h[0] + h[1] + h[2] + h[3];
      const int incl = wave_incl_scan(sum);
      const int total = __shfl(incl, 63, 64);
      if (total <= k) {                        // the cell gives every candidate it has
        rec.bstar = PAIR_NB;
        if (lane == 0 && total < k)
          atomicAdd(&S.sc->cnt[sp == 1 ? C_DEFICIT : C_DEFICIT_NEG], (unsigned long long)(k - total));
      } else {
        const int excl = incl - sum;
        const bool mine = excl < k && k <= incl;       // the lane whose bins reach k
        int b = 0, need = 0, m = 0;
        if (mine) {
          int cum = excl, q = 0;
          while (cum + h[q] < k) cum += h[q++];
          b = 4 * lane + q; need = k - cum; m = h[q];
        }
        const int src = __ffsll((long long)__ballot(mine)) - 1;
        b = __shfl(b, src, 64); need = __shfl(need, src, 64); m = __shfl(m, src, 64);
        if (need == m) {                       // the whole bin is taken
          rec.bstar = b + 1;
        } else {
          rec.bstar = b;
          rec.need = need;
          int so = 0;
          if (lane == 0) so = atomicAdd(&S.sc->pair_nrec, m);
          rec.segoff = __shfl(so, 0, 64);
        }
      }
      *reinterpret_cast<int4 *>(row) = make_int4(0, 0, 0, 0);
      if (lane == 0) kl[c] = 0;
    }
    if (lane == 0) S.pcell[c] = rec;
  }
}

template <int BS>
__device__ void pair_take(const Sim &S, int64_t step, int sp, int bx, int gx) {
  if (!*pair_active_flag(S, sp)) return;
  const Particles &P = S.p[sp];
  const Particles &L = S.alt[sp];
  const int64_t N = (int64_t)S.sc->n[sp];
  // whole waves step through the slots (a wave takes 256 consecutive ones) so that
  // the kill counts are wave-aggregated
  const int64_t n_pad = (N + 255) & ~(int64_t)255;
  for (int64_t i0 = 4 * ((int64_t)bx * BS + threadIdx.x); i0 < n_pad; i0 += 4 * (int64_t)gx * BS) {
    int32_t w[4];
    load_w4(P.w, i0, N, w);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t i = i0 + k;
      bool killed = false;
      if (w[k] >= 0) {
        const int c = w[k] & (int32_t)W_CELL;
        const PairCell rec = S.pcell[c];
        if (rec.bstar > 0 || rec.need > 0) {
          const uint32_t id = P.id[i];
          const uint32_t x = pair_draw(S, sp, id, step);
          const int b = (int)(x >> 24);
          if (b < rec.bstar) {
            pair_kill(S, sp, i, c, P.off[i]);
            killed = true;
          } else if (b == rec.bstar && rec.need > 0) {
            const int e = rec.segoff + atomicAdd(&S.pcell[c].fill, 1);
            reinterpret_cast<uint32_t *>(L.vx)[e] = x;
            L.id[e] = id;
            L.w[e] = (int32_t)i;
            reinterpret_cast<int32_t *>(L.vy)[e] = c;
          }
        }
      }
      pair_count_kills(S, sp, killed);
    }
  }
}

template <int BS>
__device__ void pair_rank(const Sim &S, int sp, int bx, int gx) {
  int32_t *active = pair_active_flag(S, sp);
  if (!*active) return;
  const Particles &P = S.p[sp];
  const Particles &L = S.alt[sp];
  const int nrec = S.sc->pair_nrec;
  const int n_pad = (nrec + 63) & ~63;
  for (int e = bx * BS + threadIdx.x; e < n_pad; e += gx * BS) {
    bool killed = false;
    if (e < nrec) {
      const int c = reinterpret_cast<const int32_t *>(L.vy)[e];
      const PairCell rec = S.pcell[c];
      const uint64_t key = ((uint64_t)reinterpret_cast<const uint32_t *>(L.vx)[e] << 32) | L.id[e];
      int rank = 0;
      for (int q = rec.segoff; q < rec.segoff + rec.fill; ++q)
        rank += (((uint64_t)reinterpret_cast<const uint32_t *>(L.vx)[q] << 32) | L.id[q]) < key;
      if (rank < rec.need) {
        const int64_t i = L.w[e];
        pair_kill(S, sp, i, c, P.off[i]);
        killed = true;
      }
    }
    pair_count_kills(S, sp, killed);
  }
  // the last block to finish closes this pairing
  __shared__ bool last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(&S.sc->ticket, 1u) == (unsigned)gx - 1;
  __syncthreads();
  if (last && threadIdx.x == 0) {
    *active = 0;
    S.sc->ticket = 0u;
  }
}

// stage 0..3 = hist, select, take, rank
template <int BS>
__device__ __forceinline__ void pair_stage(const Sim &S, int64_t step, int stage, int sp, int bx, int gx) {
  if (stage == 0) pair_hist<BS>(S, step, sp, bx, gx);
  else if (stage == 1) pair_select<BS>(S, sp, bx, gx);
  else if (stage == 2) pair_take<BS>(S, step, sp, bx, gx);
  else pair_rank<BS>(S, sp, bx, gx);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_pair(Sim S, int64_t step, int stage, int sp) {
  pair_stage<BS>(S, step, stage, sp, blockIdx.x, gridDim.x);
}

// Electron-ion bound of an ion step (Table 1 (16), (22)): the O2+ and O- node
// densities of the field solve, kept before the field kernel clears the ion
// histograms, and nu_ei = max over the table intervals of sum_q n_max,q H_q
// (H: largest sigma g of the interval, the ion at rest).
template <int BS>
__device__ void eiprep_block(const Sim &S) {
  __shared__ double red[BS];
  const int ng = S.ng, nn = ng + 1;
  double nmax[2];
  for (int t = 0; t < 2; ++t) {
    double m = 0.0;
    for (int j = threadIdx.x; j < nn; j += BS) {
      const double v = (double)S.Q[(size_t)(1 + t) * nn + j] * ((j == 0 || j == ng) ? 2.0 : 1.0) * S.wd;
      S.dens_ei[(size_t)t * nn + j] = (float)v;
      m = fmax(m, v);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = BS / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
      __syncthreads();
    }
    nmax[t] = red[0];
    __syncthreads();
  }
  const int n0 = S.nproc_sp[0];
  double best = 0.0;
  for (int k = threadIdx.x; k < S.ntab - 1; k += BS) {
    double sum = 0.0;
    for (int q = 0; q < S.nei; ++q) {
      const ProcDev &pd = S.proc[0][n0 + q];
      sum += nmax[pd.target == T_GRIDPOS ? 0 : 1] * S.hbound[(size_t)pd.tab * (S.ntab - 1) + k];
    }
    best = fmax(best, sum);
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int o = BS / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nu = red[0];
    S.sc->numax_ei = nu;
    S.sc->pnull_ei = 1.0 - exp(-nu * S.dti);
    S.sc->inv_numax_ei = nu > 0.0 ? (float)(1.0 / nu) : 0.0f;
  }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_eiprep(Sim S) { eiprep_block<BS>(S); }

// Table 1 (16) e + O2+ -> O + O and (22) e + O- -> O + 2e, once per ion step after
// the electron push: every electron present at the start of the step is a
// candidate with probability 1 - exp(-nu_ei dt_i); the channel follows from
// u nu_ei against the running sum of n(x) sigma(E) g, the ion at rest (g is the
// electron speed, E its energy).  (16): the electron leaves the gap and its charge
// the histogram; an O2+ of its cell goes to the pairing.  (22): E - E_th shared
// as (1 - r, r) by the electron and a new one, both isotropic; an O- of the cell
// goes to the pairing.
template <int BS>
__device__ void eion_run(const Sim &S, int64_t step, int bx, int gx) {
  const double pnull = S.sc->pnull_ei;
  if (!(pnull > 0.0)) return;
  const float inv_nu = S.sc->inv_numax_ei;
  const Particles &P = S.p[0];
  const int64_t N = (int64_t)S.sc->n[0];
  const int nn = S.ng + 1, n0 = S.nproc_sp[0];
  for (int64_t i = (int64_t)bx * BS + threadIdx.x; i < N; i += (int64_t)gx * BS) {
    const int32_t w = P.w[i];
    if (w < 0) continue;
    const uint32_t id = P.id[i];
    const U4 c = draw(S, 0, id, step, P_EION, 0);
    if (!((double)unif(c.x) < pnull)) continue;
    atomicAdd(&S.sc->cnt[C_EICAND], 1ull);
    const int cell = w & (int32_t)W_CELL;
    const float off = P.off[i], vx = P.vx[i], vy = P.vy[i], vz = P.vz[i];
    const ECand en = electron_energy(S, vx * vx + vy * vy + vz * vz);
    if (en.clamped) atomicAdd(&S.sc->cnt[C_CLAMP], 1ull);
    const TabPos tp = tab_pos(S, en.ec);
    const float target = unif(c.y);
    float acc = 0.0f, eth = 0.0f;
    int chosen = -1, kind = 0;
    for (int q = 0; q < S.nei; ++q) {
      const ProcDev &pd = S.proc[0][n0 + q];
      const float *nd = S.dens_ei + (pd.target == T_GRIDPOS ? 0 : nn);
      const float dens = fmaf(off, nd[cell + 1] - nd[cell], nd[cell]) * inv_nu;
      const float sg = en.ec < pd.e_th ? 0.0f : tab_sigma(S.sigma + (size_t)pd.tab * S.ntab, tp);
      acc = fmaf(dens * sg, en.g, acc);
      if (target < acc) { chosen = pd.tab; kind = pd.kind; eth = pd.e_th; break; }
    }
    log_event(S, step, PS_EION, id, chosen);
    if (chosen < 0) {
      atomicAdd(&S.sc->cnt[C_EINULL], 1ull);
      continue;
    }
    atomicAdd(&S.sc->cnt[C_EVENT + chosen], 1ull);
    if (kind == K_RECOMB) {
      const unsigned long long a = cic_a(off);
      atomicAdd(&S.Q[cell], (unsigned long long)(-(long long)(4294967296ull - a)));
      atomicAdd(&S.Q[cell + 1], (unsigned long long)(-(long long)a));
      P.w[i] = W_DEAD;
      atomicAdd(&S.kleft[cell], 1);
      S.sc->pair_active = 1;
    } else {
      const U4 p0 = draw(S, 0, id, step, P_EION, 1);
      const float er = fmaxf(en.e - eth, 0.0f), r = unif(p0.x);
      float d0, d1, d2, s0, s1, s2;
      iso_dir(c.z, c.w, d0, d1, d2);
      const float vn = sqrtf(S.two_e_m[0] * ((1.0f - r) * er));
      P.vx[i] = vn * d0; P.vy[i] = vn * d1; P.vz[i] = vn * d2;
      iso_dir(p0.y, p0.z, s0, s1, s2);
      const float vm = sqrtf(S.two_e_m[0] * (r * er));
      emit(S, step_ctx(S), 0, PS_EION, id, cell | (int32_t)new_flight_f(S.inv_nd_ef, p0.w), off, vm * s0, vm * s1,
           vm * s2);
      dep_global(S.Q, cell, off);
      atomicAdd(&S.sc->cnt[C_BORN + 0], 1ull);
      atomicAdd(&S.kleft_neg[cell], 1);
      S.sc->pair_active_neg = 1;
    }
  }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_eion(Sim S, int64_t step) { eion_run<BS>(S, step, blockIdx.x, gridDim.x); }

// ---------------------------------------------------------------- O2(a1Delta_g) field
// Spatially resolved O2(a), the extension section 4 proposes for n = C n(O2) in
// Eq. (1): start from the uniform value, tally production by process tab.
template <int BS>
__global__ __launch_bounds__(BS) void k_meta_init(Sim S, int tab) {
  const int nn = S.ng + 1;
  const double n0 = S.c_meta * S.n_o2;
  for (int j = threadIdx.x; j < nn; j += BS) {
    S.na[j] = n0;
    S.na_f[j] = (float)n0;
    S.meta_src[j] = 0ull;
  }
  if (threadIdx.x == 0) {
    S.sc->meta_tab = tab;
    S.sc->na_max = n0;
    S.sc->meta_on = 1;
  }
}

// Steady D n'' - nu_q n + P = 0 on the nodes (finite volumes, half volumes at the
// electrodes, surface flux h n there), P from the events tallied over tau seconds:
// P_j = w (tally_j 2^-32) / (V_j tau).  The tridiagonal system is solved by one
// lane (Thomas, FP64, O(ng) dependent steps): it runs once per update, every
// ten to hundreds of rf cycles.
template <int BS>
__global__ __launch_bounds__(BS) void k_meta_solve(Sim S, double weight, double tau, double D, double nu_q, double h) {
  __shared__ double red[BS];
  const int ng = S.ng, nn = ng + 1;
  const double dx = S.dx;
  for (int j = threadIdx.x; j < nn; j += BS) {
    const double vol = (j == 0 || j == ng) ? 0.5 * dx : dx;
    S.na[j] = -(weight * ((double)(long long)S.meta_src[j] / 4294967296.0) / (vol * tau));   // right-hand side
    S.meta_src[j] = 0ull;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double k = D / (dx * dx);
    double *cp = S.meta_tmp, *x = S.na;
    // forward sweep: x holds the modified right-hand side
    double b = -2.0 * k - 2.0 * h / dx - nu_q, c = 2.0 * k;
    cp[0] = c / b;
    x[0] = x[0] / b;
    for (int j = 1; j < nn; ++j) {
      const double a = j == ng ? 2.0 * k : k;
      b = j == ng ? -2.0 * k - 2.0 * h / dx - nu_q : -2.0 * k - nu_q;
      c = j == ng ? 0.0 : k;
      const double m = b - a * cp[j - 1];
      cp[j] = c / m;
      x[j] = (x[j] - a * x[j - 1]) / m;
    }
    for (int j = nn - 2; j >= 0; --j) x[j] = x[j] - cp[j] * x[j + 1];
  }
  __syncthreads();
  double m = 0.0;
  for (int j = threadIdx.x; j < nn; j += BS) {
    S.na_f[j] = (float)S.na[j];
    m = fmax(m, S.na[j]);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = BS / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) S.sc->na_max = red[0];
}

// ---------------------------------------------------------------- cell sort
// Counting sort by cell, dropping dead particles.  The count and the scatter
// cut the store into the same per-block chunks.  k_sort_count counts its chunk
// per cell (runs of equal cells with one LDS atomic) and takes, per cell, a
// range for the block with one global atomic on the cell's total; k_sort_scan
// turns the totals into cell starts.  Every block then owns one contiguous
// range per cell, which its tiles fill in order, so that the lines of a range
// are written by one block in quick succession.
__device__ __forceinline__ void load_w8(const int32_t *wp, int64_t i0, int32_t w[GROUP]) {
  const int4 a = *reinterpret_cast<const int4 *>(wp + i0), b = *reinterpret_cast<const int4 *>(wp + i0 + 4);
  w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w; w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
}

template <int BS>
__device__ void count_runs(const Sim &S, int s, int64_t N, int *cnt) {
  const int64_t chunk = push_chunk(N, gridDim.x);
  const int64_t begin = (int64_t)blockIdx.x * chunk, end = min(N, begin + chunk);
  const int32_t *wp = S.p[s].w;
  for (int64_t i0 = begin + (int64_t)GROUP * threadIdx.x; i0 < end; i0 += (int64_t)GROUP * BS) {
    int32_t w[GROUP];
    load_w8(wp, i0, w);
    const int nv = (int)min((int64_t)GROUP, end - i0);
    int rc = -1, len = 0;
    for (int k = 0; k < nv; ++k) {
      if (w[k] < 0) continue;
      const int c = w[k] & (int32_t)W_CELL;
      if (c != rc) { if (len) atomicAdd(&cnt[rc], len); rc = c; len = 0; }
      ++len;
    }
    if (len) atomicAdd(&cnt[rc], len);
  }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_sort_count(Sim S, int s) {
  extern __shared__ int scnt[];
  const int ng = S.ng;
  const int64_t N = (int64_t)S.sc->n[s];
  for (int j = threadIdx.x; j < ng; j += BS) scnt[j] = 0;
  __syncthreads();
  count_runs<BS>(S, s, N, scnt);
  __syncthreads();
  int32_t *row = S.sortoff + (size_t)blockIdx.x * ng;
  for (int j = threadIdx.x; j < ng; j += BS) row[j] = scnt[j] ? atomicAdd(&S.sortcnt[j], scnt[j]) : 0;
}

template <int BS>
__global__ __launch_bounds__(BS) void k_sort_scan(Sim S, int s) {
  __shared__ long long buf[BS / 64];
  const int ng = S.ng;
  const int per = (ng + BS - 1) / BS;
  const int j0 = min((int)threadIdx.x * per, ng), j1 = min(j0 + per, ng);
  long long loc = 0;
  for (int j = j0; j < j1; ++j) loc += S.sortcnt[j];
  long long tot;
  long long run = block_exclusive_scan<BS, long long>(loc, buf, tot);
  for (int j = j0; j < j1; ++j) {
    S.sortbase[j] = (int32_t)run;
    run += S.sortcnt[j];
    S.sortcnt[j] = 0;
  }
  if (threadIdx.x == 0) {
    S.sc->nsort[s] = S.sc->n[s];
    S.sc->n[s] = (unsigned long long)tot;
  }
}

// Scatter into the other buffer, a tile of SORT_BS * G particles at a time (all six
// fields loaded with 64- or 128-bit reads; the larger the tile, the more of each
// cell's particles one tile writes together, so fewer partially written lines are
// written back).  When the live cells of a tile span at most SORT_NB cells (the usual case: between two sorts an ion crosses a few cells,
// an electron some tens), the tile is ordered by cell in LDS and written out
// with consecutive lanes on consecutive slots of the block's cell ranges.  A
// wider tile (products appended since the last sort) writes each particle
// where it goes.  Within a cell the order is that of the LDS reservations.
constexpr int SORT_BS = 1024, SORT_NB = 1024;
// LDS of one workgroup on gfx950
constexpr size_t SORT_LDS_MAX = 160 * 1024;

template <int G>   // particles per thread and tile
struct SortTile {
  static constexpr int T = SORT_BS * G;
  int32_t w[T];
  float off[T], vx[T], vy[T], vz[T];
  uint32_t id[T];
  int32_t cnt[SORT_NB], start[SORT_NB], base[SORT_NB];
  int32_t lo[SORT_BS / 64], hi[SORT_BS / 64], scan[SORT_BS / 64];
};

template <int G>
size_t sort_lds_bytes_g(const Sim &S) { return sizeof(SortTile<G>) + 2 * sizeof(int32_t) * (size_t)S.ng; }

// Electrons: tiles of 4096 where the block's LDS holds one beside the block's cell
// ranges (up to 6632 cells), else of 2048.  Ions cross a few cells between two
// sorts, so their tiles already write long runs and the smaller tile is faster.
int sort_tile_g(const Sim &S, int s) { return s == 0 && sort_lds_bytes_g<4>(S) <= SORT_LDS_MAX ? 4 : 2; }

size_t sort_lds_bytes(const Sim &S, int s) {
  return sort_tile_g(S, s) == 4 ? sort_lds_bytes_g<4>(S) : sort_lds_bytes_g<2>(S);
}

template <int G>
__global__ __launch_bounds__(SORT_BS) void k_sort_scatter(Sim S, int s, Particles dst) {
  static_assert(G == 2 || G == 4, "tiles of two or four particles per thread");
  constexpr int T = SortTile<G>::T;
  extern __shared__ __align__(16) unsigned char sort_lds[];
  SortTile<G> &t = *reinterpret_cast<SortTile<G> *>(sort_lds);
  const int ng = S.ng;
  int32_t *lbase = reinterpret_cast<int32_t *>(sort_lds + sizeof(SortTile<G>)), *lfill = lbase + ng;
  const int64_t N = (int64_t)S.sc->nsort[s];
  const int64_t chunk = push_chunk(N, gridDim.x);
  const int64_t begin = (int64_t)blockIdx.x * chunk, end = min(N, begin + chunk);
  if (begin >= end) return;
  const int32_t *row = S.sortoff + (size_t)blockIdx.x * ng;
  for (int j = threadIdx.x; j < ng; j += SORT_BS) {
    lbase[j] = S.sortbase[j] + row[j];
    lfill[j] = 0;
  }
  const Particles &P = S.p[s];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int64_t tb = begin; tb < end; tb += T) {
    const int64_t i0 = tb + (int64_t)G * threadIdx.x;
    int32_t w[G];
    float off[G], vx[G], vy[G], vz[G];
    uint32_t id[G];
#pragma unroll
    for (int k = 0; k < G; ++k) w[k] = W_DEAD;
    if (i0 < end) {
      // the chunk starts on a multiple of 8 slots and the store is padded to 256,
      // so the G slots from i0 are aligned and allocated; those past end are dead
      if constexpr (G == 4) {
        const int4 a = *reinterpret_cast<const int4 *>(P.w + i0);
        const float4 o = *reinterpret_cast<const float4 *>(P.off + i0), x = *reinterpret_cast<const float4 *>(P.vx + i0),
                     y = *reinterpret_cast<const float4 *>(P.vy + i0), z = *reinterpret_cast<const float4 *>(P.vz + i0);
        const uint4 d = *reinterpret_cast<const uint4 *>(P.id + i0);
        w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
        off[0] = o.x; off[1] = o.y; off[2] = o.z; off[3] = o.w;
        vx[0] = x.x; vx[1] = x.y; vx[2] = x.z; vx[3] = x.w;
        vy[0] = y.x; vy[1] = y.y; vy[2] = y.z; vy[3] = y.w;
        vz[0] = z.x; vz[1] = z.y; vz[2] = z.z; vz[3] = z.w;
        id[0] = d.x; id[1] = d.y; id[2] = d.z; id[3] = d.w;
      } else {
        const int2 a = *reinterpret_cast<const int2 *>(P.w + i0);
        const float2 o = *reinterpret_cast<const float2 *>(P.off + i0), x = *reinterpret_cast<const float2 *>(P.vx + i0),
                     y = *reinterpret_cast<const float2 *>(P.vy + i0), z = *reinterpret_cast<const float2 *>(P.vz + i0);
        const uint2 d = *reinterpret_cast<const uint2 *>(P.id + i0);
        w[0] = a.x; w[1] = a.y;
        off[0] = o.x; off[1] = o.y; vx[0] = x.x; vx[1] = x.y; vy[0] = y.x; vy[1] = y.y; vz[0] = z.x; vz[1] = z.y;
        id[0] = d.x; id[1] = d.y;
      }
#pragma unroll
      for (int k = 1; k < G; ++k)
        if (i0 + k >= end) w[k] = W_DEAD;
    }
    // live cell range of the tile
    int cl = 0x7FFFFFFF, ch = -1;
#pragma unroll
    for (int k = 0; k < G; ++k)
      if (w[k] >= 0) { const int c = w[k] & (int32_t)W_CELL; cl = min(cl, c); ch = max(ch, c); }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { cl = min(cl, __shfl_xor(cl, o, 64)); ch = max(ch, __shfl_xor(ch, o, 64)); }
    if (lane == 0) { t.lo[wid] = cl; t.hi[wid] = ch; }
    __syncthreads();                                  // also: lbase / lfill ready, the previous tile done
#pragma unroll
    for (int v = 0; v < SORT_BS / 64; ++v) { cl = min(cl, t.lo[v]); ch = max(ch, t.hi[v]); }
    if (ch >= 0 && ch - cl < SORT_NB) {
      const int R = ch - cl + 1;
      for (int j = threadIdx.x; j < R; j += SORT_BS) t.cnt[j] = 0;
      __syncthreads();
      int rank[G];
      if (G == 2 && w[0] >= 0 && w[1] >= 0 && ((w[0] ^ w[1]) & (int32_t)W_CELL) == 0) {
        rank[0] = atomicAdd(&t.cnt[(w[0] & (int32_t)W_CELL) - cl], 2);   // a pair in one cell: one reservation
        rank[1] = rank[0] + 1;
      } else {
#pragma unroll
        for (int k = 0; k < G; ++k)
          if (w[k] >= 0) rank[k] = atomicAdd(&t.cnt[(w[k] & (int32_t)W_CELL) - cl], 1);
      }
      __syncthreads();
      // cell starts in the tile, and where each cell's part goes in the block's range
      const int j = threadIdx.x;                      // SORT_NB == SORT_BS: one cell per thread
      const int c = j < R ? t.cnt[j] : 0;
      int tot;
      const int run = block_exclusive_scan<SORT_BS, int32_t>(c, t.scan, tot);
      if (j < R) {
        t.start[j] = run;
        t.base[j] = lbase[cl + j] + lfill[cl + j];
        lfill[cl + j] += c;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < G; ++k) {
        if (w[k] < 0) continue;
        const int pos = t.start[(w[k] & (int32_t)W_CELL) - cl] + rank[k];
        t.w[pos] = w[k]; t.off[pos] = off[k]; t.vx[pos] = vx[k]; t.vy[pos] = vy[k]; t.vz[pos] = vz[k];
        t.id[pos] = id[k];
      }
      __syncthreads();
      for (int q = threadIdx.x; q < tot; q += SORT_BS) {
        const int32_t wq = t.w[q];
        const int b = (wq & (int32_t)W_CELL) - cl;
        const int64_t d = (int64_t)t.base[b] + (q - t.start[b]);
        dst.w[d] = wq; dst.off[d] = t.off[q]; dst.vx[d] = t.vx[q]; dst.vy[d] = t.vy[q]; dst.vz[d] = t.vz[q];
        dst.id[d] = t.id[q];
      }
    } else if (ch >= 0) {
#pragma unroll
      for (int k = 0; k < G; ++k) {
        if (w[k] < 0) continue;
        const int c = w[k] & (int32_t)W_CELL;
        const int64_t d = (int64_t)lbase[c] + atomicAdd(&lfill[c], 1);
        dst.w[d] = w[k]; dst.off[d] = off[k]; dst.vx[d] = vx[k]; dst.vy[d] = vy[k]; dst.vz[d] = vz[k];
        dst.id[d] = id[k];
      }
    }
    __syncthreads();                                  // the tile's LDS is reused by the next one
  }
}

// ---------------------------------------------------------------- compaction
// Order-preserving removal of dead particles into the other buffer: per-block
// live counts, one scan, then each block writes its live particles as one
// contiguous range (all traffic 128-bit and coalesced).
template <int BS>
__device__ void compact_count_block(const Particles &P, int64_t N, long long *blk) {
  __shared__ long long buf[BS / 64];
  const int64_t chunk = push_chunk(N, gridDim.x);
  const int64_t begin = (int64_t)blockIdx.x * chunk, end = min(N, begin + chunk);
  long long live = 0;
  for (int64_t i0 = begin + (int64_t)GROUP * threadIdx.x; i0 < end; i0 += (int64_t)GROUP * BS) {
    int32_t w[GROUP];
    load_w8(P.w, i0, w);
    const int nv = (int)min((int64_t)GROUP, end - i0);
    for (int k = 0; k < nv; ++k) live += w[k] >= 0;
  }
  long long tot;
  block_exclusive_scan<BS, long long>(live, buf, tot);
  if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

// block live counts -> output offsets; the species count becomes the live count
template <int BS>
__device__ void compact_scan_block(Scalars *sc, int s, long long *blk, int nblk) {
  __shared__ long long buf[BS / 64];
  const int per = (nblk + BS - 1) / BS;
  const int b0 = min((int)threadIdx.x * per, nblk), b1 = min(b0 + per, nblk);
  long long loc = 0;
  for (int b = b0; b < b1; ++b) loc += blk[b];
  long long tot;
  long long run = block_exclusive_scan<BS, long long>(loc, buf, tot);
  for (int b = b0; b < b1; ++b) {
    const long long c = blk[b];
    blk[b] = run;
    run += c;
  }
  if (threadIdx.x == 0) {
    sc->nsort[s] = sc->n[s];
    sc->n[s] = (unsigned long long)tot;
  }
}

template <int BS>
__device__ void compact_write_block(const Particles &P, const Particles &dst, int64_t N, const long long *blk) {
  __shared__ long long buf[BS / 64];
  const int64_t chunk = push_chunk(N, gridDim.x);
  const int64_t begin = (int64_t)blockIdx.x * chunk, end = min(N, begin + chunk);
  if (begin >= end) return;
  long long out = blk[blockIdx.x];
  for (int64_t base = begin; base < end; base += (int64_t)GROUP * BS) {
    const int64_t i0 = base + (int64_t)GROUP * threadIdx.x;
    int32_t w[GROUP];
    float off[GROUP], vx[GROUP], vy[GROUP], vz[GROUP];
    uint32_t id[GROUP];
    int nv = 0, live = 0;
    if (i0 < end) {
      nv = (int)min((int64_t)GROUP, end - i0);
      load_w8(P.w, i0, w);
      const float4 *o4 = reinterpret_cast<const float4 *>(P.off + i0), *x4 = reinterpret_cast<const float4 *>(P.vx + i0),
                   *y4 = reinterpret_cast<const float4 *>(P.vy + i0), *z4 = reinterpret_cast<const float4 *>(P.vz + i0);
      const uint4 *d4 = reinterpret_cast<const uint4 *>(P.id + i0);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float4 a = o4[h], b = x4[h], c = y4[h], d = z4[h];
        const uint4 e = d4[h];
        off[4 * h] = a.x; off[4 * h + 1] = a.y; off[4 * h + 2] = a.z; off[4 * h + 3] = a.w;
        vx[4 * h] = b.x; vx[4 * h + 1] = b.y; vx[4 * h + 2] = b.z; vx[4 * h + 3] = b.w;
        vy[4 * h] = c.x; vy[4 * h + 1] = c.y; vy[4 * h + 2] = c.z; vy[4 * h + 3] = c.w;
        vz[4 * h] = d.x; vz[4 * h + 1] = d.y; vz[4 * h + 2] = d.z; vz[4 * h + 3] = d.w;
        id[4 * h] = e.x; id[4 * h + 1] = e.y; id[4 * h + 2] = e.z; id[4 * h + 3] = e.w;
      }
      for (int k = 0; k < nv; ++k) live += w[k] >= 0;
    }
    long long tot;
    long long pos = out + block_exclusive_scan<BS, long long>((long long)live, buf, tot);
    for (int k = 0; k < nv; ++k) {
      if (w[k] < 0) continue;
      dst.w[pos] = w[k]; dst.off[pos] = off[k]; dst.vx[pos] = vx[k]; dst.vy[pos] = vy[k]; dst.vz[pos] = vz[k];
      dst.id[pos] = id[k];
      ++pos;
    }
    out += tot;
  }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_compact_count(Sim S, int s) {
  compact_count_block<BS>(S.p[s], (int64_t)S.sc->n[s], S.blkcnt);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_compact_scan(Sim S, int s, int nblk) {
  compact_scan_block<BS>(S.sc, s, S.blkcnt, nblk);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_compact_write(Sim S, int s, Particles dst) {
  compact_write_block<BS>(S.p[s], dst, (int64_t)S.sc->nsort[s], S.blkcnt);
}

// ---------------------------------------------------------------- diagnostics
template <int BS>
__device__ void diag_block(const Sim &S, int s, unsigned char *dsm) {
  const int ng = S.ng;
  unsigned long long *le = (unsigned long long *)dsm;
  unsigned int *lc = (unsigned int *)(le + ng);
  unsigned int *lb = lc + ng;
  for (int j = threadIdx.x; j < ng; j += BS) { le[j] = 0ull; lc[j] = 0u; }
  for (int j = threadIdx.x; j < NBIN; j += BS) lb[j] = 0u;
  __syncthreads();
  const Particles &P = S.p[s];
  const int64_t N = (int64_t)S.sc->n[s];
  // four consecutive particles per thread and pass, with 128-bit loads (the store's
  // fields are 16-byte aligned); a ragged tail is read element by element
  for (int64_t i0 = 4 * ((int64_t)blockIdx.x * BS + threadIdx.x); i0 < N; i0 += 4 * (int64_t)gridDim.x * BS) {
    int32_t w[4];
    float vx[4], vy[4], vz[4];
    if (i0 + 4 <= N) {
      const int4 wa = *reinterpret_cast<const int4 *>(P.w + i0);
      const float4 xa = *reinterpret_cast<const float4 *>(P.vx + i0);
      const float4 ya = *reinterpret_cast<const float4 *>(P.vy + i0);
      const float4 za = *reinterpret_cast<const float4 *>(P.vz + i0);
      w[0] = wa.x; w[1] = wa.y; w[2] = wa.z; w[3] = wa.w;
      vx[0] = xa.x; vx[1] = xa.y; vx[2] = xa.z; vx[3] = xa.w;
      vy[0] = ya.x; vy[1] = ya.y; vy[2] = ya.z; vy[3] = ya.w;
      vz[0] = za.x; vz[1] = za.y; vz[2] = za.z; vz[3] = za.w;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        w[k] = -1;
        vx[k] = vy[k] = vz[k] = 0.0f;
        if (i0 + k < N) { w[k] = P.w[i0 + k]; vx[k] = P.vx[i0 + k]; vy[k] = P.vy[i0 + k]; vz[k] = P.vz[i0 + k]; }
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (w[k] < 0) continue;
      const float e = S.half_m_e[s] * (vx[k] * vx[k] + vy[k] * vy[k] + vz[k] * vz[k]);
      const int c = w[k] & (int32_t)W_CELL;
      atomicAdd(&le[c], (unsigned long long)__float2ll_rn(e * 1048576.0f));
      atomicAdd(&lc[c], 1u);
      atomicAdd(&lb[ebin(e)], 1u);
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < ng; j += BS) {
    if (lc[j]) {
      atomicAdd(&S.esum[(size_t)s * ng + j], le[j]);
      atomicAdd(&S.ecnt[(size_t)s * ng + j], (unsigned long long)lc[j]);
    }
  }
  for (int j = threadIdx.x; j < NBIN; j += BS)
    if (lb[j]) atomicAdd(&S.edf[(size_t)s * NBIN + j], (unsigned long long)lb[j]);
  if (blockIdx.x == 0 && threadIdx.x == 0 && s == 0) S.nacc[1] += 1ull;
}

template <int BS>
__global__ __launch_bounds__(BS) void k_diag(Sim S, int s) {
  extern __shared__ __align__(16) unsigned char dsm[];
  diag_block<BS>(S, s, dsm);
}

// ---------------------------------------------------------------- loading, leapfrog start, deposit
template <int BS>
__global__ __launch_bounds__(BS) void k_load(Sim S, int s, int64_t count, float vth) {
  const Particles &P = S.p[s];
  for (int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x; k < count; k += (int64_t)gridDim.x * BS) {
    const uint32_t id = (uint32_t)k;
    const U4 r0 = draw(S, s, id, 0, P_LOAD, 0);
    const U4 r1 = draw(S, s, id, 0, P_LOAD, 1);
    const uint64_t lat = (uint64_t)(r0.x >> 8) * (uint64_t)S.ng;     // point of the 2^24 lattice times ng
    const int cell = (int)(lat >> 24);
    const float off = (float)(uint32_t)(lat & 0xFFFFFFull) * 0x1p-24f;
    float z0, z1, z2, z3;
    normals(r1.x, r1.y, z0, z1);
    normals(r1.z, r1.w, z2, z3);
    const int32_t w = s == 0 ? (cell | (int32_t)new_flight(S.nd_e, r0.y)) : cell;
    put(P, k, w, off, vth * z0, vth * z1, vth * z2);
    P.id[k] = id;
  }
}

// warm-start loading: particle k of species s goes to the cell j with
// cum[j-1] <= k < cum[j], at a lattice offset, Maxwellian at vth[j]
template <int BS>
__global__ __launch_bounds__(BS) void k_load_profile(Sim S, int s, int64_t count, const long long *cum,
                                                     const float *vth) {
  const Particles &P = S.p[s];
  const int ng = S.ng;
  for (int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x; k < count; k += (int64_t)gridDim.x * BS) {
    int lo = 0, hi = ng - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (cum[mid] > k) hi = mid;
      else lo = mid + 1;
    }
    const uint32_t id = (uint32_t)k;
    const U4 r0 = draw(S, s, id, 0, P_LOAD, 0);
    const U4 r1 = draw(S, s, id, 0, P_LOAD, 1);
    const float off = (float)(r0.x >> 8) * 0x1p-24f;
    float z0, z1, z2, z3;
    normals(r1.x, r1.y, z0, z1);
    normals(r1.z, r1.w, z2, z3);
    const float v = vth[lo];
    const int32_t w = s == 0 ? (lo | (int32_t)new_flight(S.nd_e, r0.y)) : lo;
    put(P, k, w, off, v * z0, v * z1, v * z2);
    P.id[k] = id;
  }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_shift(Sim S, int s) {
  const Particles &P = S.p[s];
  const int64_t N = (int64_t)S.sc->n[s];
  const float h = -0.5f * S.qmdt[s];
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < N; i += (int64_t)gridDim.x * BS) {
    const int32_t w = P.w[i];
    if (w < 0) continue;
    const int c = w & (int32_t)W_CELL;
    const float off = P.off[i], e0 = S.E[c], e1 = S.E[c + 1];
    P.vx[i] = fmaf(h, fmaf(off, e1 - e0, e0), P.vx[i]);
  }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_deposit(Sim S, int s) {
  extern __shared__ unsigned long long dq[];
  const int nn = S.ng + 1;
  for (int j = threadIdx.x; j < nn; j += BS) dq[j] = 0ull;
  __syncthreads();
  const Particles &P = S.p[s];
  const int64_t N = (int64_t)S.sc->n[s];
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < N; i += (int64_t)gridDim.x * BS) {
    const int32_t w = P.w[i];
    if (w >= 0) dep_lds(dq, w & (int32_t)W_CELL, P.off[i]);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nn; j += BS)
    if (dq[j]) atomicAdd(&S.Q[(size_t)s * nn + j], dq[j]);
}

// ---------------------------------------------------------------- batches
// Many discharges advance in one launch per kernel: member m's Sim lives in
// device memory (its particle buffers may be swapped there by the re-ordering),
// its step is base[m] + rel, and `mask` selects the members a launch works on.
__device__ __forceinline__ bool in_mask(uint64_t mask, int m) { return (mask >> m) & 1ull; }

template <int BS, int NPER>
__global__ __launch_bounds__(BS) void k_field_b(const Sim *__restrict__ sims, const BatchDev *__restrict__ bd,
                                                 int rel) {
  extern __shared__ int dyn_fix[];
  const int m = blockIdx.y;
  if (blockIdx.x == 0) field_block<BS, NPER>(sims[m], bd->base[m] + rel, 0);
  else fixup_block<BS>(sims[m], blockIdx.x - 1, dyn_fix);
}

// block holding tile t when Tt tiles are split into G contiguous ranges
// [b Tt / G, (b + 1) Tt / G)
__device__ __forceinline__ long long block_of_tile(long long t, long long Tt, long long G) {
  return ((t + 1) * G + Tt - 1) / Tt - 1;
}

// Cut points cut[0..G] of Tt tiles over G blocks for a batched electron push,
// worked out by one wave: every block gets one tile, and the other Tt - G are
// spread where the previous launch (other parity) measured the cumulative cost
// of its blocks to reach equal fractions (its tile ranges mapped onto this
// launch's tile count).  Without a map of G blocks the ranges are equal.
__device__ void balanced_cuts(const PushBal *B, int par, long long G, long long Tt, long long *cut) {
  const int lane = threadIdx.x & 63, prv = par ^ 1;
  if (B->grid[prv] != (int)G || B->begin[prv][G] <= 0) {
    for (long long j = lane; j <= G; j += 64) cut[j] = j * Tt / G;
    return;
  }
  const int per = (int)((G + 63) / 64), k0 = (int)min(G, (long long)lane * per), k1 = (int)min(G, (long long)k0 + per);
  double own = 0.0;
  for (int k = k0; k < k1; ++k) own += (double)B->dur[prv][k];
  const double incl = wave_incl_scan(own);
  const double total = __shfl(incl, 63, 64);
  double acc = __shfl_up(incl, 1, 64);          // integer tick sums: exact in FP64
  if (lane == 0) acc = 0.0;
  const double told = (double)B->begin[prv][G], extra = (double)(Tt - G);
  for (int k = k0; k < k1; ++k) {
    const double d = (double)B->dur[prv][k], nxt = acc + d;
    // targets total j / G in [acc, nxt), each found by exactly one block k
    long long j = max(1ll, (long long)(acc / total * (double)G));
    while (j > 1 && total * (double)(j - 1) / (double)G >= acc) --j;
    while (j < G && total * (double)j / (double)G < acc) ++j;
    for (; j < G; ++j) {
      const double T = total * (double)j / (double)G;
      if (!(T < nxt)) break;
      const double lo = (double)B->begin[prv][k], hi = (double)B->begin[prv][k + 1];
      const double x = fmin(1.0, fmax(0.0, (lo + (T - acc) / d * (hi - lo)) / told));
      cut[j] = j + (long long)(x * extra);
    }
    acc = nxt;
  }
  if (lane == 0) { cut[0] = 0; cut[G] = Tt; }
}

// Persistent push over all members in the mask.  The members' stores are cut
// into tiles of one pass (GROUP * BS slots), numbered member after member; block
// b takes the contiguous tile range [cut[b], cut[b + 1]) (equal ranges of the
// min(grid, tiles) blocks, or for electrons with bal_lds the ranges balanced by
// the previous launch's cost, each at least one tile), so its work touches each
// member in at most one run.  The run's histogram goes to row (b - first block of
// the member) of the member's partials; block 0 records the number of rows per
// member for k_reduce_b.
template <int BS, int S_>
__global__ __launch_bounds__(BS, PICMCC_PUSH_WAVES) void k_push_b(const Sim *__restrict__ sims, BatchDev *bd,
                                                                  int nmem, uint64_t mask, int rel, size_t bal_lds) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ PushLds pl;
  __shared__ long long tstart[MAXBATCH + 1];
  __shared__ long long nslot[MAXBATCH];
  constexpr long long TILE = (long long)GROUP * BS;
  if (threadIdx.x < 64) {
    const int m = threadIdx.x;
    long long n = 0, t = 0;
    if (m < nmem && in_mask(mask, m)) {
      n = (long long)sims[m].sc->n[S_];
      t = (n + TILE - 1) / TILE;
    }
    nslot[m] = n;
    tstart[m + 1] = wave_incl_scan(t);
    if (m == 0) tstart[0] = 0;
  }
  __syncthreads();
  const long long ts = (long long)__builtin_amdgcn_s_memrealtime();
  const long long Tt = tstart[nmem];
  const long long G = min((long long)gridDim.x, Tt);
  const bool bal = S_ == 0 && bal_lds > 0 && G > 0;
  const int par = rel & 1;
  long long *cut = reinterpret_cast<long long *>(smem + bal_lds);   // [G + 1], past the push's LDS
  if (bal) {
    if (threadIdx.x < 64) balanced_cuts(&bd->bal, par, G, Tt, cut);
    __syncthreads();
  }
  // block whose range holds tile t
  auto block_of = [&](long long t) -> long long {
    if (!bal) return block_of_tile(t, Tt, G);
    long long lo = 0, hi = G - 1;
    while (lo < hi) {
      const long long mid = (lo + hi + 1) >> 1;
      if (cut[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
  };
  if (blockIdx.x == 0 && threadIdx.x < nmem) {
    const int m = threadIdx.x;
    int rows = 0;
    if (tstart[m + 1] > tstart[m]) rows = (int)(block_of(tstart[m + 1] - 1) - block_of(tstart[m]) + 1);
    bd->rows[S_][m] = rows;
  }
  if ((long long)blockIdx.x >= G) return;
  const long long t0 = bal ? cut[blockIdx.x] : (long long)blockIdx.x * Tt / G;
  const long long t1 = bal ? cut[blockIdx.x + 1] : ((long long)blockIdx.x + 1) * Tt / G;
  for (int m = 0; m < nmem; ++m) {
    const long long a = max(t0, tstart[m]), b = min(t1, tstart[m + 1]);
    if (a >= b) continue;
    const Sim &S = sims[m];
    const long long row = (long long)blockIdx.x - block_of(tstart[m]);
    const int64_t begin = (a - tstart[m]) * TILE, end = min((long long)nslot[m], (b - tstart[m]) * TILE);
    push_run<BS, S_>(S, bd->base[m] + rel, begin, end, S.part + (size_t)row * (S.ng + 1), smem, pl);
  }
  if (S_ == 0 && bal_lds > 0 && threadIdx.x == 0) {   // this launch's cost map for the next one
    const long long te = (long long)__builtin_amdgcn_s_memrealtime();
    bd->bal.begin[par][blockIdx.x] = t0;
    bd->bal.dur[par][blockIdx.x] = max(1ll, te - ts);
    if ((long long)blockIdx.x == G - 1) {
      bd->bal.begin[par][G] = Tt;
      bd->bal.grid[par] = (int32_t)G;
    }
  }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_reduce_b(const Sim *__restrict__ sims, const BatchDev *__restrict__ bd,
                                                  uint64_t mask, int s) {
  const int m = blockIdx.z;
  if (!in_mask(mask, m)) return;
  const Sim &S = sims[m];
  const int nn = S.ng + 1;
  const int j = blockIdx.x * BS + threadIdx.x;
  if (j >= nn) return;
  const int used = bd->rows[s][m];
  unsigned long long sum = 0ull;
  for (int b = blockIdx.y; b < used; b += gridDim.y) sum += S.part[(size_t)b * nn + j];
  if (sum) atomicAdd(&S.Q[(size_t)s * nn + j], sum);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_ionprep_b(const Sim *__restrict__ sims, uint64_t mask) {
  if (in_mask(mask, blockIdx.x)) ionprep_block<BS>(sims[blockIdx.x]);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_pair_b(const Sim *__restrict__ sims, const BatchDev *__restrict__ bd,
                                                uint64_t mask, int rel, int stage, int sp) {
  const int m = blockIdx.y;
  if (!in_mask(mask, m)) return;
  pair_stage<BS>(sims[m], bd->base[m] + rel, stage, sp, blockIdx.x, gridDim.x);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_eiprep_b(const Sim *__restrict__ sims, uint64_t mask) {
  if (in_mask(mask, blockIdx.x)) eiprep_block<BS>(sims[blockIdx.x]);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_eion_b(const Sim *__restrict__ sims, const BatchDev *__restrict__ bd,
                                               uint64_t mask, int rel) {
  const int m = blockIdx.y;
  if (in_mask(mask, m)) eion_run<BS>(sims[m], bd->base[m] + rel, blockIdx.x, gridDim.x);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_diag_b(const Sim *__restrict__ sims, uint64_t mask) {
  extern __shared__ __align__(16) unsigned char dsm[];
  const int m = blockIdx.z;
  if (in_mask(mask, m)) diag_block<BS>(sims[m], blockIdx.y, dsm);
}

// order-preserving compaction of every species of the members in the mask; the
// scan swaps the member's buffers, so the write goes from alt (old) to p (new)
template <int BS>
__global__ __launch_bounds__(BS) void k_compact_count_b(const Sim *__restrict__ sims, uint64_t mask) {
  const int s = blockIdx.y, m = blockIdx.z;
  if (!in_mask(mask, m)) return;
  const Sim &S = sims[m];
  compact_count_block<BS>(S.p[s], (int64_t)S.sc->n[s], S.blkcnt + (size_t)s * CBLK);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_compact_scan_b(Sim *sims, uint64_t mask, int nblk) {
  const int s = blockIdx.x, m = blockIdx.y;
  if (!in_mask(mask, m)) return;
  Sim &S = sims[m];
  compact_scan_block<BS>(S.sc, s, S.blkcnt + (size_t)s * CBLK, nblk);
  if (threadIdx.x == 0) {
    const Particles t = S.p[s];
    S.p[s] = S.alt[s];
    S.alt[s] = t;
  }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_compact_write_b(const Sim *__restrict__ sims, uint64_t mask) {
  const int s = blockIdx.y, m = blockIdx.z;
  if (!in_mask(mask, m)) return;
  const Sim &S = sims[m];
  compact_write_block<BS>(S.alt[s], S.p[s], (int64_t)S.sc->nsort[s], S.blkcnt + (size_t)s * CBLK);
}

__global__ void k_advance_b(BatchDev *bd, int nmem, int64_t add) {
  const int m = threadIdx.x;
  if (m < nmem) bd->base[m] += add;
}

// ---------------------------------------------------------------- launch wrappers
size_t diag_lds_bytes(const Sim &S);
constexpr int FBS = 1024;   // field / fixup / scan block
constexpr int GBS = 256;    // grid-stride helper kernels

size_t push_lds_bytes(const Sim &S, int s, int bs) {
  const size_t nn = S.ng + 1;
  size_t o = 0;
  o = (o + 8 * nn + 15) & ~(size_t)15;
  o = (o + 4 * nn + 15) & ~(size_t)15;
  if (s == 2) o = (o + 4 * nn + 15) & ~(size_t)15;
  o = (o + 4 * (size_t)S.nproc_sp[s] * S.ntab + 15) & ~(size_t)15;
  if (s == 0) o = (o + 4 * (size_t)S.ntab + 15) & ~(size_t)15;
  o = (o + sizeof(unsigned short) * GROUP * (size_t)bs + 15) & ~(size_t)15;
  if (s == 0) o += 8 * (size_t)FFE_SLOTS * bs;     // free-flight-end lists: id and squared speed
  if (s == 0) o += 26 * (size_t)S.rq_cap;          // candidate records: 6 words + a 16-bit slot
  return o;
}

int max_push_grid() { return MAXGRID; }

hipError_t launch_reduce(const Sim &S, int s, int push_grid, hipStream_t st) {
  const int nn = S.ng + 1;
  hipLaunchKernelGGL((k_reduce<256>), dim3((nn + 255) / 256, 16), dim3(256), 0, st, S, s, push_grid);
  return hipGetLastError();
}

size_t fixup_lds_bytes(const Sim &) { return 2 * sizeof(int) * NBKT; }

#define PUSH_CASE(BS_)                                                                            \
  case BS_:                                                                                       \
    if (s == 0) hipLaunchKernelGGL((k_push<BS_, 0>), dim3(grid), dim3(BS_), lds, st, S, step);    \
    else if (s == 1) hipLaunchKernelGGL((k_push<BS_, 1>), dim3(grid), dim3(BS_), lds, st, S, step); \
    else hipLaunchKernelGGL((k_push<BS_, 2>), dim3(grid), dim3(BS_), lds, st, S, step);           \
    break;

hipError_t launch_push(const Sim &S, int s, int64_t step, int grid, int block, hipStream_t st) {
  const size_t lds = push_lds_bytes(S, s, block);
  switch (block) {
    PUSH_CASE(256)
    PUSH_CASE(512)
    PUSH_CASE(1024)
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t set_lds_limits(const Sim &S, int block) {
  hipError_t e = hipSuccess;
  for (int s = 0; s < NSP && e == hipSuccess; ++s) {
    const int lds = (int)push_lds_bytes(S, s, block);
#define SETA(BS_, S__) hipFuncSetAttribute((const void *)k_push<BS_, S__>, hipFuncAttributeMaxDynamicSharedMemorySize, lds)
    if (block == 256) e = s == 0 ? SETA(256, 0) : s == 1 ? SETA(256, 1) : SETA(256, 2);
    else if (block == 512) e = s == 0 ? SETA(512, 0) : s == 1 ? SETA(512, 1) : SETA(512, 2);
    else e = s == 0 ? SETA(1024, 0) : s == 1 ? SETA(1024, 1) : SETA(1024, 2);
#undef SETA
  }
#define SET_FIELD_LDS(NP_)                                                                               \
  if (e == hipSuccess)                                                                                   \
    e = hipFuncSetAttribute((const void *)k_field<FBS, NP_>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                            (int)fixup_lds_bytes(S));                                                    \
  if (e == hipSuccess)                                                                                   \
    e = hipFuncSetAttribute((const void *)k_reduce_field<FBS, NP_>,                                      \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)fixup_lds_bytes(S));
  SET_FIELD_LDS(1) SET_FIELD_LDS(2) SET_FIELD_LDS(4) SET_FIELD_LDS(5) SET_FIELD_LDS(9)
#undef SET_FIELD_LDS
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_fixup<FBS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)fixup_lds_bytes(S));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_sort_scatter<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sort_lds_bytes_g<2>(S));
  if (e == hipSuccess && sort_tile_g(S, 0) == 4)
    e = hipFuncSetAttribute((const void *)k_sort_scatter<4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sort_lds_bytes_g<4>(S));
  return e;
}

#define FIELD_NPER_CASE(NP_, ...) \
  case NP_: __VA_ARGS__; break;
#define FIELD_NPER_SWITCH(nn_, LAUNCH_)                                                             \
  switch (field_nper(nn_)) {                                                                        \
    FIELD_NPER_CASE(1, LAUNCH_(1)) FIELD_NPER_CASE(2, LAUNCH_(2)) FIELD_NPER_CASE(4, LAUNCH_(4))     \
    FIELD_NPER_CASE(5, LAUNCH_(5)) default: LAUNCH_(9);                                              \
  }

hipError_t launch_reduce_field(const Sim &S, int push_grid, int64_t next_step, hipStream_t st) {
  const int nred = ((S.ng + 1 + FBS - 1) / FBS) * RF_ROWS;
#define RF_LAUNCH(NP_)                                                                                   \
  hipLaunchKernelGGL((k_reduce_field<FBS, NP_>), dim3(nred + NSP), dim3(FBS), fixup_lds_bytes(S), st, S, \
                     push_grid, next_step, nred)
  FIELD_NPER_SWITCH(S.ng + 1, RF_LAUNCH)
#undef RF_LAUNCH
  return hipGetLastError();
}

hipError_t launch_field(const Sim &S, int64_t step, int mode, hipStream_t st) {
#define F_LAUNCH(NP_)                                                                                     \
  hipLaunchKernelGGL((k_field<FBS, NP_>), dim3(mode == 0 ? 1 + NSP : 1), dim3(FBS), fixup_lds_bytes(S), st, S, \
                     step, mode)
  FIELD_NPER_SWITCH(S.ng + 1, F_LAUNCH)
#undef F_LAUNCH
  return hipGetLastError();
}

hipError_t launch_fixup(const Sim &S, hipStream_t st) {
  hipLaunchKernelGGL((k_fixup<FBS>), dim3(NSP), dim3(FBS), fixup_lds_bytes(S), st, S);
  return hipGetLastError();
}

hipError_t launch_ionprep(const Sim &S, hipStream_t st) {
  hipLaunchKernelGGL((k_ionprep<GBS>), dim3(1), dim3(GBS), 0, st, S);
  return hipGetLastError();
}

hipError_t launch_pair(const Sim &S, int64_t step, int stage, int sp, int grid, hipStream_t st) {
  // pair_select: one wave per cell
  const int cells = (S.ng + GBS / 64 - 1) / (GBS / 64);
  const int g = stage == 1 && cells < grid ? cells : grid;
  hipLaunchKernelGGL((k_pair<GBS>), dim3(g), dim3(GBS), 0, st, S, step, stage, sp);
  return hipGetLastError();
}

hipError_t launch_meta_init(const Sim &S, int tab, hipStream_t st) {
  hipLaunchKernelGGL((k_meta_init<GBS>), dim3(1), dim3(GBS), 0, st, S, tab);
  return hipGetLastError();
}

hipError_t launch_meta_solve(const Sim &S, double weight, double tau, double D, double nu_q, double h, hipStream_t st) {
  hipLaunchKernelGGL((k_meta_solve<GBS>), dim3(1), dim3(GBS), 0, st, S, weight, tau, D, nu_q, h);
  return hipGetLastError();
}

hipError_t launch_eiprep(const Sim &S, hipStream_t st) {
  hipLaunchKernelGGL((k_eiprep<FBS>), dim3(1), dim3(FBS), 0, st, S);
  return hipGetLastError();
}

hipError_t launch_eion(const Sim &S, int64_t step, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_eion<GBS>), dim3(grid), dim3(GBS), 0, st, S, step);
  return hipGetLastError();
}

hipError_t launch_sort(const Sim &S, int s, const Particles &dst, int grid, hipStream_t st) {
  grid = grid < SORT_GRID ? grid : SORT_GRID;      // count and scatter cut the same chunks
  hipLaunchKernelGGL((k_sort_count<FBS>), dim3(grid), dim3(FBS), sizeof(int) * S.ng, st, S, s);
  hipLaunchKernelGGL((k_sort_scan<FBS>), dim3(1), dim3(FBS), 0, st, S, s);
  const size_t lds = sort_lds_bytes(S, s);
  if (sort_tile_g(S, s) == 4) hipLaunchKernelGGL(k_sort_scatter<4>, dim3(grid), dim3(SORT_BS), lds, st, S, s, dst);
  else hipLaunchKernelGGL(k_sort_scatter<2>, dim3(grid), dim3(SORT_BS), lds, st, S, s, dst);
  return hipGetLastError();
}

hipError_t launch_compact(const Sim &S, int s, const Particles &dst, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_compact_count<GBS>), dim3(grid), dim3(GBS), 0, st, S, s);
  hipLaunchKernelGGL((k_compact_scan<FBS>), dim3(1), dim3(FBS), 0, st, S, s, grid);
  hipLaunchKernelGGL((k_compact_write<GBS>), dim3(grid), dim3(GBS), 0, st, S, s, dst);
  return hipGetLastError();
}

hipError_t launch_diag(const Sim &S, int s, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_diag<GBS>), dim3(grid), dim3(GBS), diag_lds_bytes(S), st, S, s);
  return hipGetLastError();
}

hipError_t launch_load(const Sim &S, int s, int64_t count, float vth, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_load<GBS>), dim3(grid), dim3(GBS), 0, st, S, s, count, vth);
  return hipGetLastError();
}

hipError_t launch_load_profile(const Sim &S, int s, int64_t count, const long long *cum, const float *vth, int grid,
                               hipStream_t st) {
  hipLaunchKernelGGL((k_load_profile<GBS>), dim3(grid), dim3(GBS), 0, st, S, s, count, cum, vth);
  return hipGetLastError();
}

hipError_t launch_shift(const Sim &S, int s, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_shift<GBS>), dim3(grid), dim3(GBS), 0, st, S, s);
  return hipGetLastError();
}

hipError_t launch_deposit(const Sim &S, int s, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_deposit<GBS>), dim3(grid), dim3(GBS), sizeof(unsigned long long) * (S.ng + 1), st, S, s);
  return hipGetLastError();
}

size_t max_push_lds(const Sim &S, int block) {
  size_t m = 0;
  for (int s = 0; s < NSP; ++s) m = m > push_lds_bytes(S, s, block) ? m : push_lds_bytes(S, s, block);
  return m;
}

// ---------------------------------------------------------------- batch launch wrappers
#define PUSHB_KERNEL(BS_, S__) ((const void *)k_push_b<BS_, S__>)
static const void *push_b_fn(int block, int s) {
  switch (block) {
    case 256: return s == 0 ? PUSHB_KERNEL(256, 0) : s == 1 ? PUSHB_KERNEL(256, 1) : PUSHB_KERNEL(256, 2);
    case 512: return s == 0 ? PUSHB_KERNEL(512, 0) : s == 1 ? PUSHB_KERNEL(512, 1) : PUSHB_KERNEL(512, 2);
    case 1024: return s == 0 ? PUSHB_KERNEL(1024, 0) : s == 1 ? PUSHB_KERNEL(1024, 1) : PUSHB_KERNEL(1024, 2);
    default: return nullptr;
  }
}
#undef PUSHB_KERNEL

// resident blocks per CU of the batched push (after the LDS limit is set)
hipError_t batch_push_occupancy(int block, int s, size_t lds, int *per_cu) {
  const void *fn = push_b_fn(block, s);
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  for (const void *f : {(const void *)k_field_b<FBS, 1>, (const void *)k_field_b<FBS, 2>,
                        (const void *)k_field_b<FBS, 4>, (const void *)k_field_b<FBS, 5>,
                        (const void *)k_field_b<FBS, 9>}) {
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(2 * sizeof(int) * NBKT));
    if (e != hipSuccess) return e;
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, fn, block, lds);
}

hipError_t launch_field_b(const BatchLaunch &B, int rel, hipStream_t st) {
#define FB_LAUNCH(NP_)                                                                                     \
  hipLaunchKernelGGL((k_field_b<FBS, NP_>), dim3(1 + NSP, B.nmem), dim3(FBS), 2 * sizeof(int) * NBKT, st, B.sims, \
                     B.bd, rel)
  FIELD_NPER_SWITCH(B.nn_max, FB_LAUNCH)
#undef FB_LAUNCH
  return hipGetLastError();
}

#define PUSHB_CASE(BS_)                                                                                       \
  case BS_:                                                                                                   \
    if (s == 0) hipLaunchKernelGGL((k_push_b<BS_, 0>), dim3(g), dim3(BS_), lds, st, B.sims, B.bd, B.nmem, mask, rel, B.bal_lds); \
    else if (s == 1) hipLaunchKernelGGL((k_push_b<BS_, 1>), dim3(g), dim3(BS_), lds, st, B.sims, B.bd, B.nmem, mask, rel, (size_t)0); \
    else hipLaunchKernelGGL((k_push_b<BS_, 2>), dim3(g), dim3(BS_), lds, st, B.sims, B.bd, B.nmem, mask, rel, (size_t)0); \
    break;

hipError_t launch_push_b(const BatchLaunch &B, int s, uint64_t mask, int rel, hipStream_t st) {
  const int g = B.push_grid[s];
  const size_t lds = B.push_lds[s];
  switch (B.block) {
    PUSHB_CASE(256)
    PUSHB_CASE(512)
    PUSHB_CASE(1024)
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
#undef PUSHB_CASE

hipError_t launch_reduce_b(const BatchLaunch &B, int s, uint64_t mask, hipStream_t st) {
  hipLaunchKernelGGL((k_reduce_b<256>), dim3((B.nn_max + 255) / 256, 16, B.nmem), dim3(256), 0, st, B.sims, B.bd,
                     mask, s);
  return hipGetLastError();
}

hipError_t launch_ionprep_b(const BatchLaunch &B, uint64_t mask, hipStream_t st) {
  hipLaunchKernelGGL((k_ionprep_b<GBS>), dim3(B.nmem), dim3(GBS), 0, st, B.sims, mask);
  return hipGetLastError();
}

hipError_t launch_pair_b(const BatchLaunch &B, uint64_t mask, int rel, int stage, int sp, hipStream_t st) {
  hipLaunchKernelGGL((k_pair_b<GBS>), dim3(B.pgrid, B.nmem), dim3(GBS), 0, st, B.sims, B.bd, mask, rel, stage, sp);
  return hipGetLastError();
}

hipError_t launch_eiprep_b(const BatchLaunch &B, uint64_t mask, hipStream_t st) {
  hipLaunchKernelGGL((k_eiprep_b<FBS>), dim3(B.nmem), dim3(FBS), 0, st, B.sims, mask);
  return hipGetLastError();
}

hipError_t launch_eion_b(const BatchLaunch &B, uint64_t mask, int rel, hipStream_t st) {
  hipLaunchKernelGGL((k_eion_b<GBS>), dim3(64, B.nmem), dim3(GBS), 0, st, B.sims, B.bd, mask, rel);
  return hipGetLastError();
}

hipError_t launch_diag_b(const BatchLaunch &B, uint64_t mask, hipStream_t st) {
  hipLaunchKernelGGL((k_diag_b<GBS>), dim3(B.dgrid, NSP, B.nmem), dim3(GBS), B.diag_lds, st, B.sims, mask);
  return hipGetLastError();
}

hipError_t launch_compact_b(const BatchLaunch &B, uint64_t mask, hipStream_t st) {
  hipLaunchKernelGGL((k_compact_count_b<GBS>), dim3(B.cgrid, NSP, B.nmem), dim3(GBS), 0, st, B.sims, mask);
  hipLaunchKernelGGL((k_compact_scan_b<FBS>), dim3(NSP, B.nmem), dim3(FBS), 0, st, B.sims, mask, B.cgrid);
  hipLaunchKernelGGL((k_compact_write_b<GBS>), dim3(B.cgrid, NSP, B.nmem), dim3(GBS), 0, st, B.sims, mask);
  return hipGetLastError();
}

hipError_t launch_advance_b(const BatchLaunch &B, int64_t add, hipStream_t st) {
  hipLaunchKernelGGL(k_advance_b, dim3(1), dim3(64), 0, st, B.bd, B.nmem, add);
  return hipGetLastError();
}

size_t diag_lds_bytes(const Sim &S) { return (size_t)S.ng * 12 + NBIN * 4 + 16; }

}  // namespace picmcc
