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
//           distinct digit), digit-major in memory;
//   scan -- exclusive scan of that histogram: global start of every
//           (digit, tile) run;
//   down -- stable ranking inside the tile: each wave walks its contiguous
//           1024 keys 64 at a time, finds the lanes holding the same digit
//           with one ballot per digit bit, ranks by popcount under the lane
//           mask and carries a per-wave count per digit in LDS; a prefix
//           over waves and digits then places every key at its tile-local
//           sorted position in LDS, and the tile is written out in that
//           order, so the stores of one digit run are contiguous.
// The particle records then move once, gathered by the source index with
// contiguous stores.  No kernel waits on another block: every launch
// finishes for any input.
#include "pd_internal.h"

namespace pd {

static inline int grid_for(int64_t n, int block = 256) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (int)g;
}

// exclusive scan of one value per thread over a 256-thread block
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

// ---------------------------------------------------------------------------
// exclusive scan of *len_p u32 values; chunks of kScanChunk = 256 x 8
constexpr int kScanPer = kScanChunk / 256;

__global__ void __launch_bounds__(256) k_scan_reduce(const uint32_t* __restrict__ in,
                                                     const uint32_t* len_p,
                                                     uint32_t* __restrict__ bsum) {
  __shared__ uint32_t sh[4];
  const uint32_t len = *len_p;
  const uint32_t nb = (len + kScanChunk - 1) / kScanChunk;
  if (blockIdx.x >= nb) return;
  const uint32_t base = blockIdx.x * kScanChunk + threadIdx.x * kScanPer;
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const uint32_t x = in[(base + k < len) ? base + k : len - 1];  // no branch around the load
    acc += (base + k < len) ? x : 0u;
  }
  uint32_t tot;
  block_scan256(acc, &tot, sh);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of the block sums by one 1024-thread block (<= 65536 sums).
// With a guard state, the total is the number of electrons a collision step
// creates: if they do not fit (capacity, 32-bit ids) or an error is already
// flagged, the error is flagged and the total forced to 0, so every later
// launch of the step touches only the live particles.
__global__ void __launch_bounds__(1024) k_scan_bsums(uint32_t* bsum, const uint32_t* len_p,
                                                     uint32_t* total, DevState* guard,
                                                     uint32_t cap) {
  __shared__ uint32_t sh[16];
  const uint32_t len = *len_p;
  const uint32_t nb = (len + kScanChunk - 1) / kScanChunk;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const uint32_t per = (nb + 1023) / 1024;
  const uint32_t b0 = t * per;
  uint32_t s = 0;
  for (uint32_t k = 0; k < per; ++k) s += (b0 + k < nb) ? bsum[b0 + k] : 0u;
  uint32_t x = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
  for (int w = 0; w < 16; ++w) {
    wbase += (w < wid) ? sh[w] : 0u;
    tot += sh[w];
  }
  uint32_t run = wbase + x - s;
  for (uint32_t k = 0; k < per; ++k) {
    if (b0 + k < nb) {
      const uint32_t v = bsum[b0 + k];
      bsum[b0 + k] = run;
      run += v;
    }
  }
  if (t == 0 && total) {
    if (guard && (guard->err || (uint64_t)guard->n_alive + tot > cap ||
                  (uint64_t)guard->next_id + tot > 0xFFFFFFFFull)) {
      guard->err |= 1u;
      tot = 0;
    }
    *total = tot;
  }
}

__global__ void __launch_bounds__(256) k_scan_down(const uint32_t* in, uint32_t* out,
                                                   const uint32_t* len_p,
                                                   const uint32_t* __restrict__ bsum) {
  __shared__ uint32_t sh[4];
  const uint32_t len = *len_p;
  const uint32_t nb = (len + kScanChunk - 1) / kScanChunk;
  if (blockIdx.x >= nb) return;
  const uint32_t base = blockIdx.x * kScanChunk + threadIdx.x * kScanPer;
  uint32_t v[kScanPer];
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const uint32_t x = in[(base + k < len) ? base + k : len - 1];
    v[k] = (base + k < len) ? x : 0u;
    acc += v[k];
  }
  uint32_t tot;
  uint32_t run = bsum[blockIdx.x] + block_scan256(acc, &tot, sh);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < len) out[base + k] = run;
    run += v[k];
  }
}

void scan_exclusive(const uint32_t* in, uint32_t* out, const uint32_t* len, uint32_t* total,
                    uint32_t* bsum, int64_t max_len, hipStream_t s, DevState* guard,
                    uint32_t cap) {
  int nb = (int)((max_len + kScanChunk - 1) / kScanChunk);
  if (nb < 1) nb = 1;
  k_scan_reduce<<<nb, 256, 0, s>>>(in, len, bsum);
  k_scan_bsums<<<1, 1024, 0, s>>>(bsum, len, total, guard, cap);
  k_scan_down<<<nb, 256, 0, s>>>(in, out, len, bsum);
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
static inline int tile_grid(int64_t cap, int per_cu) {
  int64_t tiles = (cap + kSortTile - 1) / kSortTile;
  int64_t lim = 256 * per_cu;
  if (tiles < 1) tiles = 1;
  return (int)(tiles < lim ? tiles : lim);
}

// per-tile digit histogram: each wave ranks its contiguous 1024 keys 64 at a
// time (all 16 rankings first, so their ballot chains overlap), then adds
// one count per distinct digit to its LDS row (no atomics)
template <int DB>
__global__ void __launch_bounds__(256) k_radix_up(const uint32_t* __restrict__ keys,
                                                  const DevState* st, int shift,
                                                  uint32_t* __restrict__ hist,
                                                  uint32_t* __restrict__ scan_len) {
  constexpr int R = 1 << DB;
  __shared__ uint32_t wh[4][R];
  const uint32_t n = st->n_total;
  const uint32_t ntiles = (n + kSortTile - 1) / kSortTile;
  constexpr uint32_t mask = (uint32_t)R - 1u;
  if (blockIdx.x == 0 && threadIdx.x == 0) *scan_len = (uint32_t)R * ntiles;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    for (int d = t; d < R; d += 256) wh[0][d] = wh[1][d] = wh[2][d] = wh[3][d] = 0;
    const uint32_t base = tile * kSortTile + w * (kSortTile / 4);
    uint32_t dd[kSortItems], rr[kSortItems], cc[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
      const uint32_t idx = base + it * 64 + lane;
      dd[it] = (keys[(idx < n) ? idx : n - 1] >> shift) & mask;  // clamped, unconditional
    }
#pragma unroll
    for (int it = 0; it < kSortItems; ++it)
      rr[it] = match_rank<DB>(dd[it], base + it * 64 + lane < n, lt, &cc[it]);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSortItems; ++it)
      if (base + it * 64 + lane < n && rr[it] == 0) wh[w][dd[it]] += cc[it];
    __syncthreads();
    for (int d = t; d < R; d += 256)
      hist[(size_t)d * ntiles + tile] = wh[0][d] + wh[1][d] + wh[2][d] + wh[3][d];
    __syncthreads();
  }
}

template <int DB, bool FIRST>  // FIRST: the values are the source indices
__global__ void __launch_bounds__(256) k_radix_down(const uint32_t* __restrict__ kin,
                                                    const uint32_t* __restrict__ vin,
                                                    uint32_t* __restrict__ kout,
                                                    uint32_t* __restrict__ vout,
                                                    const DevState* st, int shift,
                                                    const uint32_t* __restrict__ hist) {
  constexpr int R = 1 << DB;
  constexpr uint32_t mask = (uint32_t)R - 1u;
  __shared__ uint32_t wh[4][R];
  __shared__ uint32_t gofs[R];
  __shared__ uint32_t tkey[kSortTile];
  __shared__ uint32_t tval[kSortTile];
  __shared__ uint32_t sh[4];
  const uint32_t n = st->n_total;
  const uint32_t ntiles = (n + kSortTile - 1) / kSortTile;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    for (int d = t; d < R; d += 256) wh[0][d] = wh[1][d] = wh[2][d] = wh[3][d] = 0;
    const uint32_t tile0 = tile * kSortTile;
    const uint32_t base = tile0 + w * (kSortTile / 4);
    uint32_t kk[kSortItems], vv[kSortItems], rk[kSortItems], cc[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
      const uint32_t idx = base + it * 64 + lane;
      const bool valid = idx < n;
      const uint32_t ic = valid ? idx : n - 1;  // clamped, unconditional loads
      kk[it] = kin[ic];
      vv[it] = FIRST ? idx : vin[ic];
    }
#pragma unroll
    for (int it = 0; it < kSortItems; ++it)
      rk[it] = match_rank<DB>((kk[it] >> shift) & mask, base + it * 64 + lane < n, lt, &cc[it]);
    __syncthreads();
    // carry the per-digit counts of earlier iterations (in-order per wave)
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
      const uint32_t d = (kk[it] >> shift) & mask;
      const uint32_t old = wh[w][d];
      if (base + it * 64 + lane < n && rk[it] == 0) wh[w][d] = old + cc[it];
      rk[it] += old;
    }
    __syncthreads();
    // tile-local start of every digit, start of each wave's share, and
    // global minus local start
    {
      constexpr int PER = (R + 255) / 256;
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
          gofs[d] = hist[(size_t)d * ntiles + tile] - run;
          wh[0][d] = run;
          wh[1][d] = run + a0;
          wh[2][d] = run + a0 + a1;
          wh[3][d] = run + a0 + a1 + a2;
        }
        run += cnt[q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
      if (base + it * 64 + lane < n) {
        const uint32_t lp = wh[w][(kk[it] >> shift) & mask] + rk[it];
        tkey[lp] = kk[it];
        tval[lp] = vv[it];
      }
    }
    __syncthreads();
    const uint32_t cnt = (n - tile0 < (uint32_t)kSortTile) ? (n - tile0) : (uint32_t)kSortTile;
#pragma unroll 4
    for (uint32_t q = t; q < cnt; q += 256) {
      const uint32_t k = tkey[q];
      const uint32_t p = gofs[(k >> shift) & mask] + q;
      kout[p] = k;
      vout[p] = tval[q];
    }
    __syncthreads();
  }
}

// payload permutation: dst[p] = src[perm[p]] for the live particles; every
// sorted key (the sentinel ones included) goes to dst.key
constexpr int kGatherPer = 4;
template <typename T>
__global__ void __launch_bounds__(256) k_gather(PartsT<T> src, PartsT<T> dst,
                                                const uint32_t* __restrict__ skeys,
                                                const uint32_t* __restrict__ perm,
                                                const DevState* st, uint32_t sentinel) {
  const uint32_t n = st->n_total;
  const uint32_t stride = gridDim.x * blockDim.x * kGatherPer;
  // every load uses a valid index (clamped position; perm holds source
  // indices < n), so all of a thread's loads are in flight together; only
  // the stores are guarded
  for (uint32_t p0 = blockIdx.x * blockDim.x * kGatherPer + threadIdx.x; p0 < n; p0 += stride) {
    uint32_t k[kGatherPer], q[kGatherPer];
#pragma unroll
    for (int u = 0; u < kGatherPer; ++u) {
      const uint32_t p = p0 + u * blockDim.x;
      const uint32_t pc = (p < n) ? p : n - 1;
      k[u] = skeys[pc];
      q[u] = perm[pc];
    }
    T r[kGatherPer], z[kGatherPer], vr[kGatherPer], vt[kGatherPer], vz[kGatherPer];
    uint32_t id[kGatherPer];
    uint8_t sp[kGatherPer];
#pragma unroll
    for (int u = 0; u < kGatherPer; ++u) {
      // an absorbed particle's record is not written: read the (contiguous)
      // record at its own position instead of its scattered source
      const uint32_t p = p0 + u * blockDim.x;
      const uint32_t s = (k[u] == sentinel) ? ((p < n) ? p : n - 1) : q[u];
      r[u] = src.r[s];
      z[u] = src.z[s];
      vr[u] = src.vr[s];
      vt[u] = src.vt[s];
      vz[u] = src.vz[s];
      sp[u] = src.sp[s];
      id[u] = src.id[s];
    }
#pragma unroll
    for (int u = 0; u < kGatherPer; ++u) {
      const uint32_t p = p0 + u * blockDim.x;
      if (p >= n) continue;
      dst.key[p] = k[u];
      if (k[u] == sentinel) continue;
      dst.r[p] = r[u];
      dst.z[p] = z[u];
      dst.vr[p] = vr[u];
      dst.vt[p] = vt[u];
      dst.vz[p] = vz[u];
      dst.sp[p] = sp[u];
      dst.id[p] = id[u];
    }
  }
}

template <int DB>
static void radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                       int shift, SortWork& w, DevState* st, hipStream_t s) {
  const int tiles = (int)((w.cap + kSortTile - 1) / kSortTile);
  k_radix_up<DB><<<tile_grid(w.cap, 4), 256, 0, s>>>(kin, st, shift, w.hist, w.scan_len);
  scan_exclusive(w.hist, w.hist, w.scan_len, nullptr, w.bsum,
                 (int64_t)(1 << DB) * (tiles < 1 ? 1 : tiles), s, nullptr, 0);
  if (!vin)
    k_radix_down<DB, true><<<tile_grid(w.cap, 3), 256, 0, s>>>(kin, vin, kout, vout, st, shift,
                                                               w.hist);
  else
    k_radix_down<DB, false><<<tile_grid(w.cap, 3), 256, 0, s>>>(kin, vin, kout, vout, st, shift,
                                                                w.hist);
}

// key_bits <= 20: two passes of ceil(key_bits/2) bits (at most 10);
// wider keys: passes of 10 bits
template <typename T>
void sort_particles(const PartsT<T>& src, const PartsT<T>& dst, int key_bits, SortWork& w,
                    DevState* st, uint32_t sentinel, int part, hipStream_t s) {
  int passes = (key_bits + kRadixMaxBits - 1) / kRadixMaxBits;
  if (passes < 2) passes = 2;
  const int dbits = (key_bits + passes - 1) / passes;
  if (part == 0) {
    const uint32_t* kin = src.key;
    const uint32_t* vin = nullptr;
    for (int p = 0; p < passes; ++p) {
      uint32_t* kout = (p & 1) ? w.k1 : w.k0;
      uint32_t* vout = (p & 1) ? w.v1 : w.v0;
      const int shift = p * dbits;
      if (dbits <= 8) radix_pass<8>(kin, vin, kout, vout, shift, w, st, s);
      else radix_pass<10>(kin, vin, kout, vout, shift, w, st, s);
      kin = kout;
      vin = vout;
    }
  } else {
    const uint32_t* skeys = ((passes - 1) & 1) ? w.k1 : w.k0;
    const uint32_t* perm = ((passes - 1) & 1) ? w.v1 : w.v0;
    int64_t gb = (w.cap + 256 * kGatherPer - 1) / (256 * kGatherPer);
    if (gb < 1) gb = 1;
    if (gb > 2048) gb = 2048;
    k_gather<T><<<(int)gb, 256, 0, s>>>(src, dst, skeys, perm, st, sentinel);
  }
}
template void sort_particles<double>(const Parts&, const Parts&, int, SortWork&, DevState*,
                                     uint32_t, int, hipStream_t);
template void sort_particles<float>(const PartsF&, const PartsF&, int, SortWork&, DevState*,
                                    uint32_t, int, hipStream_t);

// ---------------------------------------------------------------------------
// off[k] = first sorted position whose key >= k, for k = 0 .. nkeys-1;
// off[sentinel] is the number of live particles.  The same launch clears the
// node charge for the deposit that follows.
__global__ void __launch_bounds__(256) k_offsets(const uint32_t* __restrict__ skeys, DevState* st,
                                                 uint32_t* __restrict__ off, uint32_t nkeys,
                                                 int64_t* __restrict__ Q, uint32_t nnodes) {
  const uint32_t n = st->n_total;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nkeys; k += stride) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
      const uint32_t mid = lo + ((hi - lo) >> 1);
      if (skeys[mid] < k) lo = mid + 1;
      else hi = mid;
    }
    off[k] = lo;
    if (k == nkeys - 1) st->n_alive = lo;
  }
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < nnodes; b += stride) Q[b] = 0;
}

void build_offsets(const uint32_t* skeys, DevState* st, uint32_t* off, uint32_t nkeys,
                   int64_t* Q, uint32_t nnodes, hipStream_t s) {
  k_offsets<<<grid_for(nkeys), 256, 0, s>>>(skeys, st, off, nkeys, Q, nnodes);
}

}  // namespace pd
