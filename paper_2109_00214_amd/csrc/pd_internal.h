// pd_internal.h -- device data layout and kernel launchers of the gfx950
// PIC-DSMC library (internal; the public boundary is include/pd.h).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace pd {

constexpr double kQE = 1.602176634e-19;    // elementary charge, C (CODATA 2018)
constexpr double kEPS0 = 8.8541878128e-12; // vacuum permittivity, F/m
constexpr double kPI = 3.14159265358979323846;
constexpr int kNS = 8;                     // species (the three Cu2+ labels apart)
constexpr int kNK = 6;                     // sort-key classes (the Cu2+ labels together)
constexpr int kNC = 10;                    // collision channels
constexpr int kCEX = 6, kNN = 7;           // Cu+ + Cu charge exchange, Cu + Cu elastic
constexpr int kCEI = 8, kCEE = 9;          // Coulomb: electron with Cu+, with an electron
// the electron channels in cumulative-sum order: EL, SI, DI, SI2, SI3, SI4,
// CEI, CEE (position q is channel q below 6, q + 2 from 6 on)
constexpr int kNEC = 8;
__host__ __device__ inline int echannel(int q) { return q < 6 ? q : q + 2; }

// sort-key class of a species: e, Cu, Cu+, Cu2+ (every label), Cu3+, Cu4+
__host__ __device__ inline uint32_t key_class(uint32_t s) {
  return s < 4u ? s : (s < 6u ? 3u : s - 2u);
}
// the label a channel's target takes: Cu+, Cu2+ (double), Cu2+ (step-wise),
// Cu3+, Cu4+ (elastic: unchanged)
__host__ __device__ inline uint32_t product_of(int ch, uint32_t sp) {
  return ch == 1 ? 2u : ch == 2 ? 4u : ch == 3 ? 3u : ch == 4 ? 6u : ch == 5 ? 7u : sp;
}

// Philox4x32-10 (Salmon et al., SC'11)
__device__ inline void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                              uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // each 32 x 32 -> 64-bit product in one instruction (both halves)
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// Chunks of a grid-stride loop in XCD order.  The dispatcher hands
// consecutive workgroups to the eight XCDs in turn, so block b runs on XCD
// b % 8 and shares that XCD's L2 with the blocks of the same residue.  The
// chunks are grouped into runs of S, and run g belongs to residue g % 8:
// blocks that share an L2 work on neighbouring chunks (the particles of a
// few rows of cells, whose records the movers read across chunks), while
// every XCD still gets runs from the whole array.  The t-th chunk of a
// residue is chunk ((t / S) * 8 + x) * S + t % S, increasing in t; every
// chunk is taken exactly once whatever the placement (with fewer than eight
// blocks, the plain order).
template <uint32_t S>
struct ChunkWalk {
  uint32_t t, step, x, n;
  // blocks blk = 0 .. nblk-1 walk the chunks; walk block blk is the
  // launch's block blk + first, whose index decides its XCD
  __device__ ChunkWalk(uint32_t nchunks, uint32_t blk, uint32_t nblk, uint32_t first)
      : n(nchunks) {
    if (nblk < 8u) {
      t = blk;
      step = nblk;
      x = 8u;  // plain order
      return;
    }
    x = (blk + first) & 7u;
    const uint32_t r0 = (x - first) & 7u;  // the first walk block of this residue
    t = (blk - r0) >> 3;
    step = (nblk - r0 + 7u) >> 3;  // walk blocks of this residue
  }
  __device__ explicit ChunkWalk(uint32_t nchunks)
      : ChunkWalk(nchunks, blockIdx.x, gridDim.x, 0u) {}
  __device__ uint32_t chunk() const {
    return x == 8u ? t : ((t / S) * 8u + x) * S + (t % S);
  }
  __device__ bool more() const { return chunk() < n; }
  __device__ void next() { t += step; }
};

// uniform in [0,1): the top 53 bits of (hi:lo) times 2^-53
__device__ inline double u53(uint32_t hi, uint32_t lo) {
  const uint64_t b = (((uint64_t)hi << 32) | (uint64_t)lo) >> 11;
  return (double)b * 0x1p-53;
}

// Device-resident counters: every launch reads the particle counts from
// here, so a step needs no host round trip and can be replayed as a graph.
struct DevState {
  uint32_t n_total;    // particles in the arrays at step start (dead ones included)
  uint32_t n_alive;    // after the sort: particles with a live key
  uint32_t n_created;  // electrons made by this step's collisions
  uint32_t next_id;    // first unused id at step start
  uint32_t step;       // step counter, the Philox counter word 2
  uint32_t sched_pos;  // next injection-schedule slot
  uint32_t sched_n;    // schedule length (steps)
  uint32_t err;        // bit 0: capacity overflow
  uint32_t heavy_now;  // this step advances the heavy species (set by the sort)
  uint32_t pad_;
  unsigned long long events[kNC];
  unsigned long long conflicts;
  unsigned long long created;
  unsigned long long pushed;   // sum over steps of the particles pushed
  unsigned long long absorbed[3 * kNS];
  // boundary physics: the gap voltage the next Poisson solve uses, the
  // emission's carried fractions (electrons, atoms) and this step's emitted
  // counts (written by the injection launch for the push's counter roll),
  // cumulative emitted counts, and sum Z absorbed at the anode at the last
  // circuit update
  double V_gap;
  double em_acc[2];
  double em_acc_next[2];
  uint32_t em_now[3];   // emitted electrons, atoms, sputtered atoms this step
  uint32_t pad2_;
  unsigned long long emitted[2];
  unsigned long long sputtered;
  long long circ_zanode;
};

// Particle store in three arrays; T = double in the FP64 deterministic form,
// float in the FP32 precision form.  The record of a particle is split in
// two: its position pair (what the deposit and the cell index need) and the
// rest (velocity, id, label: what the collisions and the push also need), so
// that a particle read out of order (a mover, a collision target) costs two
// memory transactions, not one per field; the sort key lives apart (the sort
// reads nothing else).
template <typename T>
struct alignas(2 * sizeof(T)) PosT {
  T r, z;
};
template <typename T>
struct alignas(sizeof(T) == 8 ? 16 : 8) RecT {
  T vr, vt, vz;
  uint32_t id;
  uint32_t sp;  // species / label
};
static_assert(sizeof(PosT<double>) == 16 && sizeof(RecT<double>) == 32, "FP64 record layout");
static_assert(sizeof(PosT<float>) == 8 && sizeof(RecT<float>) == 24, "FP32 record layout");
template <typename T>
struct PartsT {
  PosT<T>* x;
  RecT<T>* v;
  uint32_t* key;
  // multiplicities (unequal weights: a record stands for mu W real
  // particles), or null when every record stands for W
  uint16_t* mu = nullptr;
};
using Parts = PartsT<double>;
using PartsF = PartsT<float>;

// The records of a step: U holds them in the previous step's order (as the
// push left them, with the injected ones after); the sort gives the new
// order as perm (sorted position -> index in U) and skey (the keys in that
// order).  Collisions and the deposit read and update U through perm; the
// push reads U through perm and writes every record at its sorted position
// in S, where the collisions also put the electrons they create (after the
// live particles).  The records therefore move once per step.
template <typename T>
struct Flow {
  PartsT<T> U, S;
  const uint32_t* perm;
  const uint32_t* skey;
};

struct Grid {
  int nr, nz;
  uint32_t C;         // cells nr*nz
  uint32_t sentinel;  // key of an absorbed particle (= kNK*C)
  double dr, dz, R, L, V, dt;
  int heavy_every;    // heavy species advance every heavy_every steps (1: every step)
  double dt_heavy;    // their step, heavy_every * dt
  double W;           // particles per super-particle
  // cathode emission (em_beta == 0: off): field enhancement, tip radius,
  // work function (eV), atoms per emitted electron, their temperature, mass
  double em_beta, em_rtip, em_phi, em_ratio, em_T, em_mass;
  // external circuit (circ_C == 0: off): source, resistance, capacitance
  double circ_V0, circ_R, circ_C;
  const double* Vdev; // the gap voltage on the device when the circuit is on, else NULL
  // cathode sputtering (sput_on == 0: off): per cathode annulus the yields of
  // the ions absorbed there in units of 2^-32, and the whole atoms the
  // injection launch took this step (the push subtracts them)
  int sput_on;
  unsigned long long* sput;
  uint32_t* sput_take;
  uint32_t seed_lo, seed_hi;  // Philox key (the emission's draws)
};

struct SpeciesParams {
  int Z[kNS];
  int Zk[kNK];        // charge number of each key class
  double qmdt[kNS];   // ((Z e) / m) dt
  double m[kNS];
  double qmdt_heavy[kNS];  // ((Z e) / m) dt_heavy
};

struct CollideParams {
  double W, dt;
  uint32_t seed_lo, seed_hi;
  int enable_di;
  double ck[kNC];        // sqrt(m_r / (2 e)): relative speed -> sqrt(E/eV)
  double thr[kNC];       // thresholds, eV
  double dsq[kNC];       // table spacing in sqrt(E/eV), a power of two
  double f1[kNC], f2[kNC];
  double two_dE_mr[kNC]; // 2 (-E_th e) / m_r
  const double* tab[kNC];
  int tabn[kNC];         // 0: the channel takes no part (its table is not set)
  int chain;             // the Cu2+ -> Cu3+ or Cu3+ -> Cu4+ channel takes part
  int heavy;             // a heavy-projectile channel (CEX, NN) takes part
  int split_literal;     // the last stage of a double ionization by Eqs. 16-20
  int coulomb;           // an electron Coulomb channel (CEI, CEE) takes part
  int cee;               // the electron-electron channel takes part: every electron
                         // event then claims its projectile too
  double dt_heavy;       // their time step (the heavy step)
  const double* Vcell;   // cell volumes [nr]
};

struct Schedule {
  const int64_t* off;    // [n+1]
  int64_t max_count;     // largest per-step count (launch size)
  const double *r, *z, *vr, *vt, *vz;
  const uint8_t* sp;
};

// cell and in-cell fractions: i = min((int)(r/dr), nr-1), fr = r/dr - i,
// in the precision T of the particle record
template <typename T>
__device__ inline void cell_of(const Grid& g, T r, T z, int& i, int& j, T& fr, T& fz) {
  const T xr = r / (T)g.dr, xz = z / (T)g.dz;
  i = (int)xr;
  j = (int)xz;
  if (i > g.nr - 1) i = g.nr - 1;
  if (j > g.nz - 1) j = g.nz - 1;
  fr = xr - (T)i;
  fz = xz - (T)j;
}

// Fixed-point cloud-in-cell share of a unit charge at (r, z) (paper Eqs.
// 9-10): the 1D weights rounded to 2^-20, complementary, so the four node
// shares v[0..3] (nodes b, b+1, b+nr+1, b+nr+2) are exact integers adding
// up to 2^40.  Returns b.
template <typename T>
__device__ inline int cic_fixed(const Grid& g, T r, T z, long long v[4]) {
  int i, j;
  T fr, fz;
  cell_of<T>(g, r, z, i, j, fr, fz);
  const long long ar = (long long)floor((fr * (T)1048576) + (T)0.5), br = 1048576 - ar;
  const long long az = (long long)floor((fz * (T)1048576) + (T)0.5), bz = 1048576 - az;
  v[0] = br * bz;
  v[1] = ar * bz;
  v[2] = br * az;
  v[3] = ar * az;
  return j * (g.nr + 1) + i;
}

// deposit: weights rounded to 2^-20 per dimension, complementary, so each
// particle adds exactly Z * 2^40 to the four nodes of its cell
// The deposit covers the sorted state before this step's collisions: the
// charged species' ranges of the sorted order (the offsets give them; the
// neutral run is not read at all), each particle with the charge of the
// species in its sort key.  The collisions add what their outcomes change
// (an ionization moves charge only when the new electrons do not sit where
// the charge appeared).  Neighbouring lanes mostly share a cell: each wave
// sums the contributions of every run of equal cells (a segmented suffix
// sum over the lanes) and only the first lane of a run issues the four
// int64 atomics.  Integer addition is associative, so the node charges do
// not depend on this grouping or on the order of the collisions' additions.
// In the FP32 form the fractions come from the FP32 positions; the rounding
// to 2^-20 is the same, so the node charges stay exact integers.
// (blocks blk = 0 .. nblk-1 of a 256-thread launch share the work)
template <typename T>
__device__ inline void deposit_blocks(const Flow<T>& f, const uint32_t* __restrict__ off,
                                      const Grid& g, const SpeciesParams& spp,
                                      unsigned long long* Q, uint32_t blk, uint32_t nblk) {
  // the charged key classes' ranges laid end to end: cum[s] charged
  // particles before class s, its range starting at lo[s]
  uint32_t lo[kNK], cum[kNK + 1];
  cum[0] = 0;
#pragma unroll
  for (int s = 0; s < kNK; ++s) {
    lo[s] = off[(uint32_t)s * g.C];
    const uint32_t hi = off[(uint32_t)(s + 1) * g.C];
    cum[s + 1] = cum[s] + ((spp.Zk[s] != 0) ? hi - lo[s] : 0u);
  }
  const uint32_t n = cum[kNK];
  const int W = g.nr + 1;
  const int lane = threadIdx.x & 63;
  const uint64_t upto = (lane == 63) ? 0ull : (~0ull << (lane + 1));  // lanes above this one
  for (uint32_t q0 = blk * blockDim.x; q0 < n; q0 += nblk * blockDim.x) {
    const uint32_t q = q0 + threadIdx.x;
    int b = -1;
    long long v[4] = {0, 0, 0, 0};
    if (q < n) {
      uint32_t p = 0;
      long long Zp = 0;
#pragma unroll
      for (int s = 0; s < kNK; ++s)
        if (q >= cum[s] && q < cum[s + 1]) {
          p = lo[s] + (q - cum[s]);
          Zp = spp.Zk[s];
        }
      const uint32_t ip = f.perm[p];
      if (f.U.mu) Zp *= (long long)f.U.mu[ip];  // W_alpha of Eq. 9
      const PosT<T> x = f.U.x[ip];
      b = cic_fixed<T>(g, x.r, x.z, v);
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] *= Zp;
    }
    const int bprev = __shfl_up(b, 1, 64);
    const bool head = (lane == 0) || (b != bprev);
    const uint64_t later = __ballot(head) & upto;
    const int end = later ? (__ffsll((long long)later) - 1) : 64;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      long long t[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) t[k] = __shfl_down(v[k], o, 64);
      if (lane + o < end) {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += t[k];
      }
    }
    if (head && b >= 0) {
      if (v[0]) atomicAdd(&Q[b], (unsigned long long)v[0]);
      if (v[1]) atomicAdd(&Q[b + 1], (unsigned long long)v[1]);
      if (v[2]) atomicAdd(&Q[b + W], (unsigned long long)v[2]);
      if (v[3]) atomicAdd(&Q[b + W + 1], (unsigned long long)v[3]);
    }
  }
}

// ---- sort (k_sort.hip) ----
constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;  // 4096 keys per tile
constexpr int kMoverItems = 2;                      // movers: 512 keys per tile
constexpr int kRadixMaxBits = 10;                  // digit width of a pass
constexpr int kRadix = 1 << kRadixMaxBits;
constexpr int kScanChunk = 2048;                    // elements per scan block
constexpr int kScanMaxBlocks = 65536;

struct SortWork {
  uint32_t *k0, *k1, *v0, *v1;  // key/value ping-pong [cap]
  uint32_t* hist;               // [kRadix * tiles of 256 kMoverItems keys in cap]
  uint32_t* bsum;               // per-chunk counts: movers (sort), created electrons (collisions)
  uint32_t* skey;               // [cap] keys in the last sorted order
  uint32_t* mbits;              // [cap / 32 + 66] mover flag of each old position, 32 per word
  uint32_t* mword;              // [cap / 32 + 66] movers before each word of mbits
  uint32_t* n_mov;              // device [2]: movers of this sort, live count of the old order
  const uint32_t* msorted;      // the movers' keys in sorted order (after sort_keys)
  uint32_t* perm;               // [cap] source of every sorted position
  uint32_t* ins;                // [cap] stayers before each sorted mover
  int64_t cap;
  int heavy_every;              // the heavy-step period (the sort marks heavy steps)
};

// Stable sort of the st->n_total keys of the records by key (ties in index
// order) into w.perm (sorted position -> index) and w.skey.  The first
// st->n_alive positions hold the previous sort's order with updated keys:
// the particles whose key did not change stay in order and are merged with
// the others (radix-sorted) by (key, index), using the previous order's
// offsets off.  This places the movers; place_and_offsets places the
// stayers.
void sort_keys(const uint32_t* key, int key_bits, SortWork& w, DevState* st, const uint32_t* off,
               uint32_t sentinel, hipStream_t s);

constexpr int kScanPer = kScanChunk / 256;  // consecutive elements per thread

// exclusive scan of one value per thread over a 256-thread block (total of
// the block to *total); sh: 4 words of LDS
__device__ inline uint32_t block_scan256(uint32_t v, uint32_t* total, uint32_t* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t t = sh[w];
    wbase += (w < wid) ? t : 0u;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return wbase + x - v;
}
// Sum of c[lo .. hi) by one 256-thread block (every thread gets it): the
// launches that place items by the per-chunk counts of an earlier launch
// take their chunk's prefix this way instead of waiting for a separate scan
// launch (a few thousand counts, eight loads in flight per thread).
__device__ inline uint32_t block_range_sum(const uint32_t* __restrict__ c, uint32_t lo,
                                           uint32_t hi, uint32_t* sh) {
  uint32_t s = 0;
  for (uint32_t i0 = lo + threadIdx.x; i0 < hi; i0 += 8 * 256) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t i = i0 + (uint32_t)u * 256u;
      v[u] = (i < hi) ? c[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  uint32_t tot;
  block_scan256(s, &tot, sh);
  return tot;
}

// CSR offsets of the sorted keys (off[k] = first sorted position with key
// >= k, k < nkeys; st->n_alive = off[nkeys - 1]) from the previous order's
// offsets (off, updated in place) and the sort's movers (after sort_keys);
// the same launch clears the node charge Q.
// With the stayers' places (skey and perm for the positions that are not
// movers' places; key = the records' keys) in the same launch.
void place_and_offsets(const uint32_t* key, const SortWork& w, DevState* st, uint32_t* off,
                       uint32_t nkeys, int64_t* Q, uint32_t nnodes, hipStream_t s);

// ---- collisions (k_collide.hip) ----
struct CollideWork {
  uint8_t* choice;
  uint32_t *target, *claim;
  uint32_t* csum;  // created electrons per group of 32 chunks of 256 electrons
  int64_t cap;
};
// Q: the node charge the deposit of the sorted state goes to (NULL when
// there is no deposit): the apply adds what the outcomes change in it.
template <typename T>
void collide(const Flow<T>& f, const uint32_t* off, DevState* st, const Grid& g,
             const CollideParams& cp, const SpeciesParams& sp, int64_t* Q, CollideWork& w,
             uint32_t* bsum, int64_t cap, hipStream_t s);

// ---- particle-in-cell (k_pic.hip) ----
struct FieldWork {
  int64_t* Q;           // nodes
  double *phi, *Er, *Ez;
  float *Erf, *Ezf;     // FP32 copies of the field (FP32 form), else NULL
  double* f;            // [(nz-1) * (nr+1)] right-hand side, interior rows, r fastest
  double* fh;           // [(nz-1) * (nr+1)] transformed, per mode, r fastest
  double* g;            // [(nz-1) * (nr+1)] per-mode solutions, r fastest
  const double* T;      // [2 nz] DST-I entries by (k j) mod 2 nz
  const double* Sm;     // [(nz-1) * (nz-1)] DST-I matrix sin(pi (b+1)(c+1) / nz)
  const double* tinv;   // [(nz-1) * (nr+1)] Thomas reciprocals, per mode, r fastest
  const double* tcp;    // [(nz-1) * (nr+1)] Thomas upper factors, per mode, r fastest
  const double* ra;     // [nr+1] radial lower coefficients
  const double* rc;     // [nr+1] radial upper coefficients
  const double* twinv;  // [(nz-1) * (nr+1)] the same systems eliminated from both ends:
  const double* twcp;   //   pivot reciprocals and factors toward the middle row nr / 2
  const double* Vnode;  // [nr+1]
  double qunit;
  // the right-hand-side scale of the matrix-core form of the direct solve
  const double* coef;   // [nr+1] -qunit / (V_node eps0)
};
// Node charge of the sorted state: every particle of a charged species with
// the species of its sort key (before this step's collisions), through perm.
template <typename T>
void deposit(const Flow<T>& f, const uint32_t* off, const Grid& g, const SpeciesParams& sp,
             int64_t* Q, int64_t cap, hipStream_t s);
void poisson_direct(const Grid& g, FieldWork& fw, hipStream_t s);
bool direct_fits(int nr, int nz);
// the same solve with the transforms on the FP64 matrix cores and the
// tridiagonal recurrences as wave scans (k_spectral.hip)
void poisson_spectral(const Grid& g, FieldWork& fw, hipStream_t s);
bool spectral_fits(int nr, int nz);

// ---- multigrid-preconditioned CG with FP64 refinement (k_mgpcg.hip) ----
constexpr int kMGBlock = 256;
constexpr int kMGParts = 1024;          // most blocks of a reducing launch
constexpr int kMGMaxLevels = 12;
constexpr int kMGCoarseNodes = 3072;    // nodes of the levels the one-workgroup cycle takes

// one grid level: nodes (nr+1) x (nz+1), rows 0 and nz are the (zero)
// Dirichlet rows; operator coefficients per radial node
struct MGLevel {
  int nr, nz;
  float* x;              // V-cycle result (level 0: the preconditioned residual z)
  const float* b;        // right-hand side (level 0: the CG residual r)
  const float *ew, *ee, *ez, *dinv;
};
// level-0 operator in FP64 for the refinement residual
struct MGOp64 {
  int nr, nz;
  const double *ew, *ee, *ez, *dg, *w, *Vnode;
  double qunit;
};
// device scalars of a solve
struct MGScal {
  double rnorm, rel, rtol;  // ||b - A phi||, its ratio to ||b||, target ratio
  float tol2;               // inner stop: ||r||^2 of the scaled correction solve
  float rz[2];              // r.z of the last two CG iterations (slot it & 1)
  int done, conv;           // CG stopped; refinement converged
  int iters, outer;         // cumulative CG iterations and refinements
  int it_last;              // CG iterations of the latest refinement
};
constexpr int kMGCoarsestDense = 64;    // coarsest unknowns solved by a dense inverse
struct MGWork {
  int nlev, lc, coarse_sweeps;
  const float* coarsest_inv;  // [n x n] or NULL (then coarse_sweeps sweeps)
  MGLevel lev[kMGMaxLevels];
  MGOp64 op;
  float *xc, *s, *p, *q;  // CG solution, A z, search direction, A p
  float* part;            // [kMGParts * 5]: CG partials (4 dots, then r.r)
  double* part64;         // [kMGParts * 2]
  MGScal* sc;
};
size_t mg_coarse_lds_bytes(const MGWork& w);
void mg_configure(MGWork& w);
// sc->rnorm, rel, conv of phi for the node charge Q
void mg_residual(const MGWork& w, const double* phi, const int64_t* Q, hipStream_t s);
// one refinement: FP32 PCG (at most `inner` iterations) on the scaled FP64
// residual, phi += correction, new residual
void mg_outer(MGWork& w, double* phi, const int64_t* Q, int inner, hipStream_t s);
void field(const Grid& g, FieldWork& fw, hipStream_t s);
// the field, the same launch appending this step's scheduled particles to P
// (after alive + created)
template <typename T>
void field_and_inject(const Grid& g, FieldWork& fw, const PartsT<T>& P, DevState* st,
                      const SpeciesParams& spp, const Schedule& sc, int64_t cap, hipStream_t s);
// gather + push into f.S; its first thread rolls the step counters (the
// injection above included)
template <typename T>
void push(const Flow<T>& f, DevState* st, const Grid& g, const SpeciesParams& sp,
          const FieldWork& fw, const Schedule& sc, int64_t cap, hipStream_t s);
template <typename T>
void append(const PartsT<T>& P, DevState* st, const Grid& g, const PartsT<T>& src, uint32_t n,
            hipStream_t s);
// snapshot reductions: per-block partial counts, KE sums, spectrum bins
constexpr int kDiagBlocks = 512;
template <typename T>
void diag_snapshot(const PartsT<T>& P, const DevState* st, const Grid& g, const SpeciesParams& sp,
                   const double* edges, unsigned long long* counts /*[kDiagBlocks*kNS]*/,
                   double* ke /*[kDiagBlocks*kNS]*/, unsigned long long* spec /*[3*66]*/,
                   unsigned long long* real /*[kDiagBlocks*kNS]: sums of multiplicities*/,
                   hipStream_t s);
// ---- learned Poisson part: U-Net on the BF16 matrix cores (k_unet.hip) ----
struct Unet;
Unet* unet_create(int nr, int nz, int levels, int base, int batch, int64_t dataset_cap,
                  std::string& err);
void unet_destroy(Unet* u);
int64_t unet_nparams(const Unet* u);
int unet_height(const Unet* u);
int unet_width(const Unet* u);
int64_t unet_samples(const Unet* u);
int unet_set_weights(Unet* u, const float* host, hipStream_t s);
int unet_get_weights(const Unet* u, float* host);
// host [n][2][H][W] FP32 -> host [n][H][W] FP32
int unet_forward_host(Unet* u, int n, const float* x, float* out, hipStream_t s);
// gradient of sum(dout * out) with respect to the weights (flat FP32)
int unet_gradient_host(Unet* u, int n, const float* x, const float* dout, float* dw, hipStream_t s);
// the (b, phi_p) pair of the node charge Q and potential phi into the training set
int unet_add_sample(Unet* u, const MGOp64& op, const double* phi, const int64_t* Q, double V,
                    hipStream_t s);
int unet_train(Unet* u, int epochs, int batch, double lr, uint64_t seed, double* loss, hipStream_t s);
// preconditioner: z (level-0 x) = net(r) for CG iteration it (gated on sc)
void unet_apply(Unet* u, const MGLevel& m, MGScal* sc, const float* part_rr, int nb, int it,
                hipStream_t s);
// one refinement with flexible CG: first direction from the network, the
// rest preconditioned by the V-cycle
void mg_outer_learned(MGWork& w, Unet* u, double* phi, const int64_t* Q, int inner, hipStream_t s);

void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s);

}  // namespace pd
