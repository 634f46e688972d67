// k_sort.hip -- per-cell particle lists: stable LSD radix sort of the
// (species, cell) keys, the payload permutation and the CSR offsets.
//
// The pairing of DSMC collisions needs the particles of every cell (paper
// Sec. 2.1: a projectile and a target are chosen in the same cell each
// step).  Keys are species-major: key = species * nr * nz + j * nr + i; an
// absorbed particle carries the sentinel 6 * nr * nz and sorts last.
//
// A pass over a digit of D <= 10 bits:
//   up   -- per-tile digit histogram (wave ballots, one LDS update per
//           distinct digit), tile-major in memory (each tile one row);
//   scan -- per digit, exclusive prefix over the tiles (in place) and the
//           digit totals (one launch, one lane per digit);
//   down -- start of every digit from the totals, plus the tile's prefix;
//           stable ranking inside the tile: each wave walks its contiguous
//           quarter of the tile 64 keys at a time, finds the lanes holding the same digit
//           with one ballot per digit bit, ranks by popcount under the lane
//           mask and carries a per-wave count per digit in LDS; a prefix
//           over waves and digits then places every key at its tile-local
//           sorted position in LDS, and the tile is written out in that
//           order, so the stores of one digit run are contiguous.
// Between steps the order changes little: the particles are still sorted
// as the last sort left them, with the keys the push recomputed.  A
// particle whose key did not change (a stayer) keeps its order relative to
// the other stayers; only the others (movers: key changed, created,
// injected, absorbed) are radix-sorted, by (key, index).  The two sorted
// sequences are then merged by (key, index): a stayer's place is its rank
// among stayers plus the movers before it (binary search over the sorted
// movers); a mover's place is its rank among movers plus the stayers before
// it, read off the previous order's per-key offsets and the count of movers
// before each old position (kept as one flag bit per old position and a
// prefix per 32 of them).  The result is the stable sort of all keys: the
// permutation (sorted position -> index) and the sorted keys; the push
// moves the records.  The cell offsets follow from the old ones and the
// sorted movers.  No kernel waits on another block: every launch finishes
// for any input.
#include "pd_internal.h"

namespace pd {

static inline int grid_for(int64_t n, int block = 256) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (int)g;
}


// ---------------------------------------------------------------------------
// Stable digit ranking of 64 keys held one per lane: the lanes with the same
// digit are found with one ballot per digit bit; returns the rank of this
// lane among them and (in *cnt) their number.
template <int DB>
__device__ inline uint32_t match_rank(uint32_t d, bool valid, uint64_t lt, uint32_t* cnt) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < DB; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  *cnt = (uint32_t)__popcll(peers);
  return (uint32_t)__popcll(peers & lt);
}

// Tiles are taken in a grid-stride loop by a grid of at most a few blocks
// per CU: launching one block per possible tile of the capacity would
// dispatch many empty blocks, each reserving its LDS.
static inline int tile_grid(int64_t cap, int per_cu, int tile) {
  int64_t tiles = (cap + tile - 1) / tile;
  int64_t lim = 256 * per_cu;
  if (tiles < 1) tiles = 1;
  return (int)(tiles < lim ? tiles : lim);
}

// Keys per thread of a radix tile (tiles of 256 * items keys), chosen from
// the number of movers n alone, so that every launch of a sort agrees: short
// tiles when the movers are few (the usual step: many blocks), long ones
// when most particles moved (the first steps: the per-tile digit rows, and
// the column scan over them, stay few).
constexpr int kMoverItemsMax = 16;
__device__ inline int mover_items(uint32_t n) {
  return (n > (1u << 20)) ? 16 : ((n > (1u << 18)) ? 8 : kMoverItems);
}

// per-tile digit histogram: every key adds one to its digit's count in LDS
// (integer counts, the same in any order; keys of one digit in one wave
// instruction are added one after another by the LDS, which the near order
// of the movers makes common but still cheaper than ranking every key)
template <int DB, int ITM, int NT>  // NT threads per block, a multiple of 256
__global__ void __launch_bounds__(NT) k_radix_up(const uint32_t* __restrict__ keys,
                                                 const uint32_t* np, int shift,
                                                 uint32_t* __restrict__ hist) {
  constexpr int R = 1 << DB;
  constexpr int IT = (256 * ITM + NT - 1) / NT;  // keys per thread in the longest tile
  __shared__ uint32_t wh[R];
  const uint32_t n = *np;
  const int itn = mover_items(n);
  const uint32_t tsz = 256u * (uint32_t)itn;
  const uint32_t ntiles = (n + tsz - 1) / tsz;
  constexpr uint32_t mask = (uint32_t)R - 1u;
  const int t = threadIdx.x;
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    for (int d = t; d < R; d += NT) wh[d] = 0;
    const uint32_t base = tile * tsz;
    uint32_t dd[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      if ((uint32_t)(it * NT + t) < tsz) {
        const uint32_t idx = base + it * NT + t;
        dd[it] = (keys[(idx < n) ? idx : n - 1] >> shift) & mask;  // clamped, unconditional
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it)
      if ((uint32_t)(it * NT + t) < tsz && base + it * NT + t < n) atomicAdd(&wh[dd[it]], 1u);
    __syncthreads();
    for (int d = t; d < R; d += NT) hist[(size_t)tile * R + d] = wh[d];
    __syncthreads();
  }
}

// Per digit (32 digits per block): hist[t][d] <- sum of hist[t'][d] over
// t' < t, and tot[d] <- the sum over all tiles.  The 16 waves of a block
// take consecutive runs of tiles, and a wave's two halves (lanes 0-31 and
// 32-63, the same 32 digits) the two halves of its run; the half sums meet
// through a lane exchange, the wave sums in LDS, then each half rewrites
// its part of the run.
constexpr int kColWaves = 16;
constexpr uint32_t kColHeld = 16;  // tiles per lane held in registers
template <int R>
__global__ void __launch_bounds__(64 * kColWaves) k_radix_colscan(uint32_t* __restrict__ hist,
                                                                  uint32_t* __restrict__ tot,
                                                                  const uint32_t* np) {
  __shared__ uint32_t part[kColWaves][32];
  const uint32_t n = *np;
  const uint32_t tsz = 256u * (uint32_t)mover_items(n);
  const uint32_t ntiles = (n + tsz - 1) / tsz;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int dl = lane & 31, hf = lane >> 5;
  const int d = blockIdx.x * 32 + dl;
  const uint32_t ch = (ntiles + kColWaves - 1) / kColWaves;
  const uint32_t t0 = (uint32_t)w * ch;
  const uint32_t t1 = (t0 + ch < ntiles) ? t0 + ch : ntiles;
  const uint32_t hc = (ch + 1) / 2;  // the first half's tiles
  const uint32_t tm = (t0 + hc < t1) ? t0 + hc : t1;
  const uint32_t a0 = hf ? tm : t0, a1 = hf ? t1 : tm;  // this lane's tiles
  const bool held = hc <= kColHeld;  // the usual case: the part loaded once
  uint32_t v[kColHeld];
  uint32_t s = 0;
  if (held) {
#pragma unroll
    for (int u = 0; u < kColHeld; ++u)
      v[u] = (a0 + u < a1) ? hist[(size_t)(a0 + u) * R + d] : 0u;
#pragma unroll
    for (int u = 0; u < kColHeld; ++u) s += v[u];
  } else {
    for (uint32_t tb = a0; tb < a1; tb += 8) {
      uint32_t x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = (tb + u < a1) ? hist[(size_t)(tb + u) * R + d] : 0u;
#pragma unroll
      for (int u = 0; u < 8; ++u) s += x[u];
    }
  }
  const uint32_t so = __shfl_xor(s, 32, 64);  // the other half's sum
  if (hf == 0) part[w][dl] = s + so;
  __syncthreads();
  uint32_t run = 0;
  for (int q = 0; q < w; ++q) run += part[q][dl];
  if (w == kColWaves - 1 && hf == 0) tot[d] = run + s + so;
  if (hf) run += so;  // the first half's tiles come before
  if (held) {
#pragma unroll
    for (int u = 0; u < kColHeld; ++u) {
      if (a0 + u < a1) hist[(size_t)(a0 + u) * R + d] = run;
      run += v[u];
    }
    return;
  }
  for (uint32_t tb = a0; tb < a1; tb += 8) {
    uint32_t x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = (tb + u < a1) ? hist[(size_t)(tb + u) * R + d] : 0u;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (tb + u < a1) hist[(size_t)(tb + u) * R + d] = run;
      run += x[u];
    }
  }
}

// Movers among the old positions [0, i): the word prefix of the flag bits
// and the bits of i's own word below it (i <= n, the arrays written by the
// classification up to the word of position n).
__device__ inline uint32_t movers_before(const uint32_t* __restrict__ mbits,
                                         const uint32_t* __restrict__ mword, uint32_t i) {
  const uint32_t w = i >> 5;
  return mword[w] + __popc(mbits[w] & ((1u << (i & 31)) - 1u));
}

// What the last pass over the movers needs to place them: a mover of
// sorted rank r with (key k, index i) goes to ins + r, ins = stayers before
// it = p - movers_before(p) with p = i clamped to the old run of key k
// [off_prev[k], off_prev[k+1]] (all stayers for the sentinel key).  ins is
// kept per rank (non-decreasing) for the stayers' searches.
struct MoverPlace {
  const uint32_t* off_prev;
  const uint32_t* mbits;
  const uint32_t* mword;
  const DevState* st;
  uint32_t sentinel;
  uint32_t* skey;
  uint32_t* perm;
  uint32_t* ins;
};

__device__ inline uint32_t stayers_before(const MoverPlace& mp, uint32_t n_prev, uint32_t k,
                                          uint32_t i) {
  if (n_prev == 0) return 0;
  if (k >= mp.sentinel) return n_prev - movers_before(mp.mbits, mp.mword, n_prev);
  const uint32_t lo = mp.off_prev[k], hi = mp.off_prev[k + 1];
  const uint32_t p = (i < lo) ? lo : ((i > hi) ? hi : i);
  return p - movers_before(mp.mbits, mp.mword, p);
}

template <int DB, int ITM, bool FIRST>  // FIRST: the values are the source indices
__global__ void __launch_bounds__(256) k_radix_down(const uint32_t* __restrict__ kin,
                                                    const uint32_t* __restrict__ vin,
                                                    uint32_t* __restrict__ kout,
                                                    uint32_t* __restrict__ vout,
                                                    const uint32_t* np, int shift,
                                                    const uint32_t* __restrict__ hist,
                                                    const uint32_t* __restrict__ tot,
                                                    MoverPlace mp) {
  constexpr int R = 1 << DB;
  constexpr uint32_t mask = (uint32_t)R - 1u;
  constexpr int PER = (R + 255) / 256;
  constexpr int kStage = 256 * ITM;  // every tile is reordered in LDS
  __shared__ uint32_t wh[4][R];
  __shared__ uint32_t gofs[R];
  __shared__ uint32_t dbase[R];
  __shared__ uint32_t tkey[kStage];
  __shared__ uint32_t tval[kStage];
  __shared__ uint32_t tins[kStage];  // last pass: stayers before each mover
  __shared__ uint32_t sh[4];
  const uint32_t n = *np;
  const int itn = mover_items(n);
  const uint32_t tsz = 256u * (uint32_t)itn;
  const uint32_t ntiles = (n + tsz - 1) / tsz;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const bool last = mp.skey != nullptr;
  const uint32_t n_prev = last ? mp.st->n_alive : 0u;
  bool have_base = false;
  // tiles in runs of eight per XCD: the digit runs of neighbouring tiles
  // are neighbours in the output, and their partial lines meet in one L2
  for (ChunkWalk<8> cw(ntiles); cw.more(); cw.next()) {
    const uint32_t tile = cw.chunk();
    const uint32_t tile0 = tile * tsz;
    const uint32_t base = tile0 + w * (tsz / 4);
    // everything the tile reads from memory is requested first: its keys
    // and values, its prefix of every digit over the earlier tiles, and (in
    // the last pass) the stayers before each mover, so that the reads are in
    // flight together
    uint32_t kk[ITM], vv[ITM], rk[ITM], cc[ITM], hh[PER], in[ITM];
#pragma unroll
    for (int it = 0; it < ITM; ++it) {
      if (it < itn) {
        const uint32_t idx = base + it * 64 + lane;
        const bool valid = idx < n;
        const uint32_t ic = valid ? idx : n - 1;  // clamped, unconditional loads
        kk[it] = kin[ic];
        vv[it] = FIRST ? idx : vin[ic];
      }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int d = t * PER + q;
      hh[q] = (d < R) ? hist[(size_t)tile * R + d] : 0u;
    }
    if (last) {
#pragma unroll
      for (int it = 0; it < ITM; ++it)
        if (it < itn) in[it] = stayers_before(mp, n_prev, kk[it], vv[it]);
    }
    if (!have_base) {
      // global start of every digit: exclusive scan of the digit totals
      have_base = true;
      uint32_t c[PER];
      uint32_t s = 0;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int d = t * PER + q;
        c[q] = (d < R) ? tot[d] : 0u;
        s += c[q];
      }
      uint32_t total;
      uint32_t run = block_scan256(s, &total, sh);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int d = t * PER + q;
        if (d < R) dbase[d] = run;
        run += c[q];
      }
    }
    for (int d = t; d < R; d += 256) wh[0][d] = wh[1][d] = wh[2][d] = wh[3][d] = 0;
#pragma unroll
    for (int it = 0; it < ITM; ++it)
      if (it < itn)
        rk[it] = match_rank<DB>((kk[it] >> shift) & mask, base + it * 64 + lane < n, lt, &cc[it]);
    __syncthreads();
    // carry the per-digit counts of earlier iterations (in-order per wave)
#pragma unroll
    for (int it = 0; it < ITM; ++it) {
      if (it < itn) {
        const uint32_t d = (kk[it] >> shift) & mask;
        const uint32_t old = wh[w][d];
        if (base + it * 64 + lane < n && rk[it] == 0) wh[w][d] = old + cc[it];
        rk[it] += old;
      }
    }
    __syncthreads();
    // tile-local start of every digit, start of each wave's share, and
    // global minus local start
    {
      uint32_t cnt[PER];
      uint32_t s = 0;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int d = t * PER + q;
        cnt[q] = (d < R) ? (wh[0][d] + wh[1][d] + wh[2][d] + wh[3][d]) : 0u;
        s += cnt[q];
      }
      uint32_t tot;
      uint32_t run = block_scan256(s, &tot, sh);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int d = t * PER + q;
        if (d < R) {
          const uint32_t a0 = wh[0][d], a1 = wh[1][d], a2 = wh[2][d];
          gofs[d] = dbase[d] + hh[q] - run;
          wh[0][d] = run;
          wh[1][d] = run + a0;
          wh[2][d] = run + a0 + a1;
          wh[3][d] = run + a0 + a1 + a2;
        }
        run += cnt[q];
      }
    }
    __syncthreads();
    {
      // the tile reordered in LDS, so that the stores of a digit run are
      // contiguous
#pragma unroll
      for (int it = 0; it < ITM; ++it) {
        if (it < itn && base + it * 64 + lane < n) {
          const uint32_t lp = wh[w][(kk[it] >> shift) & mask] + rk[it];
          tkey[lp] = kk[it];
          tval[lp] = vv[it];
          if (last) tins[lp] = in[it];
        }
      }
      __syncthreads();
      const uint32_t cnt = (n - tile0 < tsz) ? (n - tile0) : tsz;
      if (!last) {
#pragma unroll 4
        for (uint32_t q = t; q < cnt; q += 256) {
          const uint32_t k = tkey[q];
          const uint32_t p = gofs[(k >> shift) & mask] + q;
          kout[p] = k;
          vout[p] = tval[q];
        }
      } else {
        // last pass: place the movers (p = final rank among the movers)
#pragma unroll 4
        for (uint32_t q = t; q < cnt; q += 256) {
          const uint32_t k = tkey[q], i = tval[q], ins = tins[q];
          const uint32_t p = gofs[(k >> shift) & mask] + q;
          kout[p] = k;  // the movers' keys in order (for the offsets)
          mp.ins[p] = ins;
          mp.skey[ins + p] = k;
          mp.perm[ins + p] = i;
        }
      }
    }
    __syncthreads();
  }
}

// one pass over the movers' tiles (their length chosen on the device from the
// number of movers, mover_items)
template <int DB>
static void radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                       int shift, SortWork& w, const uint32_t* np, const MoverPlace& mp,
                       hipStream_t s) {
  constexpr int R = 1 << DB;
  constexpr int ITM = kMoverItemsMax;
  const int grid = tile_grid(w.cap, 2, 256 * kMoverItems);
  // the histograms with four times the threads per tile: more loads in
  // flight per CU (the tiles are few)
  k_radix_up<DB, ITM, 1024><<<grid, 1024, 0, s>>>(kin, np, shift, w.hist);
  k_radix_colscan<R><<<R / 32, 64 * kColWaves, 0, s>>>(w.hist, w.bsum, np);
  if (!vin)
    k_radix_down<DB, ITM, true><<<grid, 256, 0, s>>>(kin, vin, kout, vout, np, shift, w.hist,
                                                     w.bsum, mp);
  else
    k_radix_down<DB, ITM, false><<<grid, 256, 0, s>>>(kin, vin, kout, vout, np, shift, w.hist,
                                                      w.bsum, mp);
}

// ---- stayers and movers ---------------------------------------------------
// position i is a mover unless it lies in the previous sorted prefix
// (i < n_prev) with its key unchanged.  A thread takes kScanPer consecutive
// positions, read as two 16-byte vectors when all of them are in range.
__device__ inline void mover_flags(uint32_t base, uint32_t n, uint32_t n_prev,
                                   const uint32_t* __restrict__ key,
                                   const uint32_t* __restrict__ kprev, uint32_t* f,
                                   uint32_t* kv) {
  static_assert(kScanPer == 8, "two 16-byte vectors per thread");
  if (base + 8 <= n) {
    const uint4 a0 = *(const uint4*)(key + base), a1 = *(const uint4*)(key + base + 4);
    kv[0] = a0.x; kv[1] = a0.y; kv[2] = a0.z; kv[3] = a0.w;
    kv[4] = a1.x; kv[5] = a1.y; kv[6] = a1.z; kv[7] = a1.w;
    if (base + 8 <= n_prev) {
      const uint4 b0 = *(const uint4*)(kprev + base), b1 = *(const uint4*)(kprev + base + 4);
      const uint32_t pv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
      for (int k = 0; k < 8; ++k) f[k] = (kv[k] != pv[k]) ? 1u : 0u;
      return;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) kv[k] = (base + k < n) ? key[base + k] : 0u;
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t i = base + k;
    f[k] = (i >= n) ? 0u : ((i >= n_prev) ? 1u : ((kv[k] != kprev[i]) ? 1u : 0u));
  }
}

// movers per chunk of kScanChunk positions
__global__ void __launch_bounds__(256) k_cls_count(const uint32_t* __restrict__ key,
                                                   const uint32_t* __restrict__ kprev,
                                                   const DevState* st, uint32_t* __restrict__ bsum,
                                                   uint32_t* __restrict__ mbits) {
  __shared__ uint32_t sh[4];
  const uint32_t n = st->n_total, n_prev = st->n_alive;
  const uint32_t nb = n / kScanChunk + 1;  // the chunks up to position n itself
  if (blockIdx.x >= nb) return;
  const uint32_t base = blockIdx.x * kScanChunk + threadIdx.x * kScanPer;
  uint32_t f[kScanPer], kv[kScanPer];
  mover_flags(base, n, n_prev, key, kprev, f, kv);
  uint32_t acc = 0, m = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    acc += f[k];
    m |= f[k] << k;
  }
  // four threads' eight flags make one word of 32 positions
  const uint32_t m1 = __shfl_down(m, 1, 64), m2 = __shfl_down(m, 2, 64),
                 m3 = __shfl_down(m, 3, 64);
  if ((threadIdx.x & 3) == 0)
    mbits[(base >> 5)] = m | (m1 << 8) | (m2 << 16) | (m3 << 24);
  uint32_t tot;
  block_scan256(acc, &tot, sh);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// The movers' (key, index) in index order to mk, mi, and mword[w] = movers
// before position 32 w, so that movers_before(i) = mword[i/32] + the flags
// of mbits[i/32] below i.
// (bsum: the movers of every chunk; each block adds up those of the chunks
// before its own, block 0 all of them into n_mov)
__global__ void __launch_bounds__(256) k_cls_compact(const uint32_t* __restrict__ key,
                                                     const DevState* st,
                                                     const uint32_t* __restrict__ bsum,
                                                     const uint32_t* __restrict__ mbits,
                                                     uint32_t* __restrict__ mword,
                                                     uint32_t* __restrict__ mk,
                                                     uint32_t* __restrict__ mi,
                                                     uint32_t* __restrict__ n_mov,
                                                     int heavy_every,
                                                     uint32_t* __restrict__ heavy_now) {
  __shared__ uint32_t sh[4];
  __shared__ uint32_t sk[kScanChunk], si[kScanChunk];
  const uint32_t n = st->n_total, n_prev = st->n_alive;
  const uint32_t nb = n / kScanChunk + 1;
  if (blockIdx.x == 0) {
    const uint32_t all = block_range_sum(bsum, 0, nb, sh);
    if (threadIdx.x == 0) {
      n_mov[0] = all;
      n_mov[1] = n_prev;  // the old order's live count, for the offsets
      // whether this step's push advances the heavy species (the push itself
      // cannot read the step counter: its first thread advances it)
      *heavy_now = (heavy_every <= 1 || (st->step % (uint32_t)heavy_every) == 0u) ? 1u : 0u;
    }
  }
  if (blockIdx.x >= nb) return;
  const uint32_t base = blockIdx.x * kScanChunk + threadIdx.x * kScanPer;
  const uint32_t m = (mbits[base >> 5] >> (8 * (threadIdx.x & 3))) & 0xFFu;
  uint32_t kv[kScanPer];
  if (m) {  // the keys only where there are movers
    if (base + 8 <= n) {
      const uint4 a0 = *(const uint4*)(key + base), a1 = *(const uint4*)(key + base + 4);
      kv[0] = a0.x; kv[1] = a0.y; kv[2] = a0.z; kv[3] = a0.w;
      kv[4] = a1.x; kv[5] = a1.y; kv[6] = a1.z; kv[7] = a1.w;
    } else {
#pragma unroll
      for (int k = 0; k < kScanPer; ++k) kv[k] = (base + k < n) ? key[base + k] : 0u;
    }
  }
  const uint32_t before = block_range_sum(bsum, 0, blockIdx.x, sh);
  uint32_t tot;
  uint32_t run = block_scan256(__popc(m), &tot, sh);
  if ((threadIdx.x & 3) == 0) mword[base >> 5] = before + run;
  // the chunk's movers are the run [before, before + tot) of the output:
  // gathered in LDS in order, then written with consecutive lanes on
  // consecutive words
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if ((m >> k) & 1u) {
      sk[run] = kv[k];
      si[run] = base + k;
      ++run;
    }
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < tot; j += 256) {
    mk[before + j] = sk[j];
    mi[before + j] = si[j];
  }
}

// first j in [lo, hi) with ins[j] > s (the movers placed before the stayer
// of rank s)
__device__ inline uint32_t movers_upto(const uint32_t* __restrict__ ins, uint32_t lo, uint32_t hi,
                                       uint32_t s) {
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (ins[mid] <= s) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}
// Stayers' places, in chunks of kPlaceChunk old positions: the stayer of
// rank s goes to s + (movers with ins <= s).  Chunk ch holds the stayer
// ranks [s0(ch), s0(ch+1)), s0(ch) = base - movers_before(base), so the movers it
// needs are those of ranks [bound(ch), bound(ch+1)), bound(ch) = the count
// for s0(ch): two searches per chunk, then the chunk searches only its own
// movers, staged in LDS.
constexpr int kPlaceChunk = 1024;
constexpr int kPlaceLds = 2048;

// movers m with ins[m] <= s (ins is non-decreasing): the whole wave, a
// 64-way search (each step probes 64 places, about log_65(nm) steps of one
// load)
__device__ inline uint32_t movers_upto_wave(const uint32_t* __restrict__ ins, uint32_t nm,
                                            uint32_t s, int lane) {
  uint32_t lo = 0, hi = nm;  // the answer is in [lo, hi]
  while (hi > lo) {
    const uint64_t r = hi - lo;
    const uint32_t p = lo + (uint32_t)((r * (uint64_t)(lane + 1)) / 65u);  // < hi
    const unsigned long long bt = __ballot(ins[p] > s);
    if (bt == 0ull) {
      lo = __shfl(p, 63, 64) + 1u;
    } else {
      const int f = __ffsll((long long)bt) - 1;
      const uint32_t pf = __shfl(p, f, 64);
      const uint32_t pb = __shfl(p, f > 0 ? f - 1 : 0, 64);
      hi = pf;
      if (f > 0) lo = pb + 1u;
    }
  }
  return lo;
}

// Each block finds its chunk's mover range itself: waves 0 and 1 search for
// the movers placed before the chunk's first stayer and before the next
// chunk's (s0 = the chunk start minus the movers before it).
// (blocks blk = 0 .. nblk-1 of a 256-thread launch share the chunks; the old
// order's live count comes from n_mov[1], as the same launch computes the
// new one)
__device__ inline void place_blocks(const uint32_t* __restrict__ key,
                                    const uint32_t* __restrict__ mbits,
                                    const uint32_t* __restrict__ mword,
                                    const uint32_t* __restrict__ ins,
                                    const uint32_t* __restrict__ n_mov,
                                    uint32_t* __restrict__ skey, uint32_t* __restrict__ perm,
                                    uint32_t blk, uint32_t nblk, uint32_t* sm) {
  uint32_t* lins = sm;             // [kPlaceLds]
  uint32_t* cb = sm + kPlaceLds;   // [2]
  const uint32_t nm = n_mov[0], n_prev = n_mov[1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const uint32_t nch = (n_prev + kPlaceChunk - 1) / kPlaceChunk;
  for (uint32_t ch = blk; ch < nch; ch += nblk) {
    const uint32_t base = ch * kPlaceChunk;
    const uint32_t end = (base + kPlaceChunk < n_prev) ? base + kPlaceChunk : n_prev;
    constexpr int U = kPlaceChunk / 256;
    uint32_t wb[U], wp[U], kv[U];  // mover flags and movers before, by words of 32
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = base + u * 256 + t;
      const uint32_t ic = (i < end) ? i : base;
      wb[u] = mbits[ic >> 5];
      wp[u] = mword[ic >> 5];
      kv[u] = key[ic];
    }
    if (w < 2) {
      const uint32_t b = (w == 0) ? base : end;  // end = the next chunk's start, or n_prev
      const uint32_t v = movers_upto_wave(ins, nm, b - movers_before(mbits, mword, b), lane);
      if (lane == 0) cb[w] = v;
    }
    __syncthreads();
    const uint32_t c0 = cb[0], c1 = cb[1];
    const bool in_lds = (c1 - c0) <= (uint32_t)kPlaceLds;
    if (in_lds)
      for (uint32_t j = c0 + t; j < c1; j += 256) lins[j - c0] = ins[j];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = base + u * 256 + t;
      const uint32_t below = (1u << (i & 31)) - 1u;
      if (i >= end || ((wb[u] >> (i & 31)) & 1u)) continue;  // past the chunk, or a mover
      const uint32_t sr = i - (wp[u] + __popc(wb[u] & below));
      uint32_t cnt;
      if (in_lds) {
        uint32_t lo = 0, hi = c1 - c0;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (lins[mid] <= sr) lo = mid + 1;
          else hi = mid;
        }
        cnt = c0 + lo;
      } else {
        cnt = movers_upto(ins, c0, c1, sr);
      }
      const uint32_t pos = sr + cnt;
      skey[pos] = kv[u];
      perm[pos] = i;
    }
    __syncthreads();
  }
}

// key_bits <= 20: two passes of ceil(key_bits/2) bits (at most 10);
// wider keys: passes of 10 bits
void sort_keys(const uint32_t* key, int key_bits, SortWork& w, DevState* st, const uint32_t* off,
               uint32_t sentinel, hipStream_t s) {
  int passes = (key_bits + kRadixMaxBits - 1) / kRadixMaxBits;
  if (passes < 2) passes = 2;
  const int dbits = (key_bits + passes - 1) / passes;
  const int nb = (int)(w.cap / kScanChunk + 1);
  {
    // classify, count and compact the movers (key, index) into k0/v0
    k_cls_count<<<nb, 256, 0, s>>>(key, w.skey, st, w.bsum, w.mbits);
    k_cls_compact<<<nb, 256, 0, s>>>(key, st, w.bsum, w.mbits, w.mword, w.k0, w.v0, w.n_mov,
                                     w.heavy_every, &st->heavy_now);
    // stable radix sort of the movers
    const uint32_t* kin = w.k0;
    const uint32_t* vin = w.v0;
    const MoverPlace none{};
    const MoverPlace last{off, w.mbits, w.mword, st, sentinel, w.skey, w.perm, w.ins};
    for (int p = 0; p < passes; ++p) {
      uint32_t* kout = (p & 1) ? w.k0 : w.k1;
      uint32_t* vout = (p & 1) ? w.v0 : w.v1;
      const int shift = p * dbits;
      const MoverPlace& mp = (p == passes - 1) ? last : none;
      if (dbits <= 8) radix_pass<8>(kin, vin, kout, vout, shift, w, w.n_mov, mp, s);
      else radix_pass<10>(kin, vin, kout, vout, shift, w, w.n_mov, mp, s);
      kin = kout;
      vin = vout;
    }
    w.msorted = kin;  // the last pass's keys: the movers' keys in sorted order
  }
}

// ---------------------------------------------------------------------------
// off[k] = first sorted position whose key >= k, for k = 0 .. nkeys-1;
// off[sentinel] is the number of live particles.  The same launch clears the
// node charge for the deposit that follows.
//
// off[k] = (stayers with key < k) + (movers with key < k).  A stayer keeps
// its old key and the old order is sorted, so the stayers with key < k are
// those at old positions below off_prev[k]: off_prev[k] -
// movers_before(off_prev[k]); each key reads its own old entry
// and overwrites it.  The movers' count is the merge of their sorted keys
// A[0..nm) with the key list 0..nkeys-1 (a key before the A entries equal
// to it): in the merged order A[i] stands at i + A[i] + 1 and key k at
// k + (movers below k).  Each block takes an equal share of the nm + nkeys
// merged places, finds the A entries of its share by a 64-way search of the
// strictly increasing i + A[i] + 1, stages them in LDS and searches them for
// each of its keys.
constexpr int kOffMax = 4096;  // merged places per block at most

// smallest i in [0, n] with i == n or i + A[i] + 1 >= d; the whole wave
// (each step probes 64 places, so about log_65(n) steps of one load)
__device__ inline uint32_t merged_split(const uint32_t* __restrict__ A, uint32_t n, uint32_t d,
                                        int lane) {
  uint32_t lo = 0, hi = n;
  while (hi > lo) {
    const uint64_t r = hi - lo;
    const uint32_t p = lo + (uint32_t)((r * (uint64_t)(lane + 1)) / 65u);
    const bool pred = (uint64_t)p + A[p] + 1u >= d;  // p < hi <= n
    const unsigned long long bt = __ballot(pred);
    if (bt == 0ull) {
      lo = __shfl(p, 63, 64) + 1u;
    } else {
      const int f = __ffsll((long long)bt) - 1;
      const uint32_t pf = __shfl(p, f, 64);
      const uint32_t pb = __shfl(p, f > 0 ? f - 1 : 0, 64);
      hi = pf;
      if (f > 0) lo = pb + 1u;
    }
  }
  return lo;
}

// (blocks blk = 0 .. nblk-1 of a 256-thread launch)
__device__ inline void offsets_blocks(const uint32_t* __restrict__ A,
                                      const uint32_t* __restrict__ n_mov,
                                      const uint32_t* __restrict__ mbits,
                                      const uint32_t* __restrict__ mword, DevState* st,
                                      uint32_t* __restrict__ off, uint32_t nkeys,
                                      int64_t* __restrict__ Q, uint32_t nnodes, uint32_t blk,
                                      uint32_t nblk, uint32_t* sm) {
  uint32_t* As = sm;              // [kOffMax]
  uint32_t* split = sm + kOffMax;  // [2]
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const uint32_t stride = nblk * blockDim.x;
  for (uint32_t b = blk * blockDim.x + t; b < nnodes; b += stride) Q[b] = 0;
  const uint32_t n = n_mov[0], n_prev = n_mov[1];
  const uint32_t tot = n + nkeys;
  const uint32_t D = (tot + nblk - 1) / nblk;  // <= kOffMax by the launch
  const uint32_t d0 = blk * D;
  if (d0 >= tot) return;  // whole block
  const uint32_t d1 = (tot - d0 < D) ? tot : d0 + D;
  if (w < 2) {
    const uint32_t v = merged_split(A, n, w == 0 ? d0 : d1, lane);
    if (lane == 0) split[w] = v;
  }
  __syncthreads();
  const uint32_t ia = split[0], ib = split[1];
  const uint32_t na = ib - ia;  // <= D
  for (uint32_t i = t; i < na; i += blockDim.x) As[i] = A[ia + i];
  __syncthreads();
  const uint32_t j0 = d0 - ia, j1 = d1 - ib;
  const uint32_t c = (j1 - j0 + blockDim.x - 1) / blockDim.x;  // keys per thread
  const uint32_t ja = j0 + t * c;
  const uint32_t je = (ja + c < j1) ? ja + c : j1;
  for (uint32_t k = ja; k < je; ++k) {
    uint32_t stay = 0;
    if (n_prev) {
      const uint32_t x = off[k];  // <= n_prev
      stay = x - movers_before(mbits, mword, x);
    }
    uint32_t lo = 0, hi = na;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (As[mid] < k) lo = mid + 1;
      else hi = mid;
    }
    const uint32_t o = stay + ia + lo;
    off[k] = o;
    if (k == nkeys - 1) st->n_alive = o;
  }
}

// The stayers' placement and the offsets read nothing the other writes
// (both take the old order's live count from n_mov[1]): one launch, the
// offsets' blocks first (their chains of dependent reads are the longer).
__global__ void __launch_bounds__(256) k_place_offsets(
    const uint32_t* __restrict__ key, const uint32_t* __restrict__ mbits,
    const uint32_t* __restrict__ mword, const uint32_t* __restrict__ ins,
    const uint32_t* __restrict__ n_mov, uint32_t* __restrict__ skey, uint32_t* __restrict__ perm,
    const uint32_t* __restrict__ A, DevState* st, uint32_t* __restrict__ off, uint32_t nkeys,
    int64_t* __restrict__ Q, uint32_t nnodes, uint32_t npl) {
  // one LDS buffer for either kind of block (the larger need: the offsets')
  static_assert(kPlaceLds <= kOffMax, "placement staging fits the offsets' buffer");
  __shared__ uint32_t sm[kOffMax + 2];
  const uint32_t nof = gridDim.x - npl;  // the offsets' blocks come first
  if (blockIdx.x >= nof)
    place_blocks(key, mbits, mword, ins, n_mov, skey, perm, blockIdx.x - nof, npl, sm);
  else
    offsets_blocks(A, n_mov, mbits, mword, st, off, nkeys, Q, nnodes, blockIdx.x, nof, sm);
}

void place_and_offsets(const uint32_t* key, const SortWork& w, DevState* st, uint32_t* off,
                       uint32_t nkeys, int64_t* Q, uint32_t nnodes, hipStream_t s) {
  const int64_t nch = (w.cap + kPlaceChunk - 1) / kPlaceChunk;
  int pg = (int)(nch < 4096 ? nch : 4096);
  if (pg < 1) pg = 1;
  const int64_t places = w.cap + (int64_t)nkeys;
  int64_t gr = (places + kOffMax - 1) / kOffMax;
  if (gr < 1024) gr = 1024;  // a fuller chip for small runs
  k_place_offsets<<<pg + (int)gr, 256, 0, s>>>(key, w.mbits, w.mword, w.ins, w.n_mov, w.skey,
                                                w.perm, w.msorted, st, off, nkeys, Q, nnodes,
                                                (uint32_t)pg);
}

}  // namespace pd
