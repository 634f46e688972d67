// k_sort.hip -- per-cell particle lists: stable LSD radix sort of the
// (species, cell) keys, CSR offsets, and the payload permutation.
//
// The pairing of DSMC collisions needs the particles of every cell (paper
// Sec. 2.1: a projectile and a target are chosen in the same cell each
// step).  Keys are species-major: key = species * nr * nz + j * nr + i; an
// absorbed particle carries the sentinel 6 * nr * nz and sorts last.
//
// Radix pass = upsweep (per-tile digit histogram, LDS atomics) -> exclusive
// scan of the digit-major histogram -> downsweep.  The downsweep ranks keys
// stably with wave ballots: the lanes holding equal digits are found with
// one ballot per digit bit, the rank inside the wave is a popcount under
// the lane mask, and a per-wave LDS counter per digit carries the rank
// across the 16 iterations of a wave's contiguous 1024-key chunk; a
// cross-wave prefix per digit then fixes the order between the four waves.
// No spin waits anywhere: every kernel finishes for any input.
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
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    uint32_t t = sh[w];
    wbase += (w < wid) ? t : 0u;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return wbase + x - v;
}

__global__ void __launch_bounds__(256) k_scan_reduce(const uint32_t* in, const uint32_t* len_p,
                                                     uint32_t* bsum) {
  __shared__ uint32_t sh[4];
  const uint32_t len = *len_p;
  const uint32_t nb = (len + kScanChunk - 1) / kScanChunk;
  if (blockIdx.x >= nb) return;
  const uint32_t base = blockIdx.x * kScanChunk;
  uint32_t acc = 0;
  for (int it = 0; it < kScanChunk / 256; ++it) {
    uint32_t idx = base + it * 256 + threadIdx.x;
    acc += (idx < len) ? in[idx] : 0u;
  }
  uint32_t tot;
  block_scan256(acc, &tot, sh);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// exclusive scan of the block sums (<= 16384 of them) by one 1024-thread block
__global__ void __launch_bounds__(1024) k_scan_bsums(uint32_t* bsum, const uint32_t* len_p,
                                                     uint32_t* total) {
  __shared__ uint32_t sh[16];
  const uint32_t len = *len_p;
  const uint32_t nb = (len + kScanChunk - 1) / kScanChunk;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  uint32_t v[16];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    uint32_t idx = t * 16 + k;
    v[k] = (idx < nb) ? bsum[idx] : 0u;
    s += v[k];
  }
  uint32_t x = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
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
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    uint32_t idx = t * 16 + k;
    if (idx < nb) bsum[idx] = run;
    run += v[k];
  }
  if (t == 0 && total) *total = tot;
}

__global__ void __launch_bounds__(256) k_scan_down(const uint32_t* in, uint32_t* out,
                                                   const uint32_t* len_p, const uint32_t* bsum) {
  __shared__ uint32_t sh[4];
  const uint32_t len = *len_p;
  const uint32_t nb = (len + kScanChunk - 1) / kScanChunk;
  if (blockIdx.x >= nb) return;
  uint32_t run = bsum[blockIdx.x];
  const uint32_t base = blockIdx.x * kScanChunk;
  for (int it = 0; it < kScanChunk / 256; ++it) {
    uint32_t idx = base + it * 256 + threadIdx.x;
    uint32_t v = (idx < len) ? in[idx] : 0u;
    uint32_t tot;
    uint32_t ex = block_scan256(v, &tot, sh);
    if (idx < len) out[idx] = run + ex;
    run += tot;
  }
}

void scan_exclusive(const uint32_t* in, uint32_t* out, const uint32_t* len, uint32_t* total,
                    uint32_t* bsum, int64_t max_len, hipStream_t s) {
  int nb = (int)((max_len + kScanChunk - 1) / kScanChunk);
  if (nb < 1) nb = 1;
  k_scan_reduce<<<nb, 256, 0, s>>>(in, len, bsum);
  k_scan_bsums<<<1, 1024, 0, s>>>(bsum, len, total);
  k_scan_down<<<nb, 256, 0, s>>>(in, out, len, bsum);
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_radix_up(const uint32_t* keys, const DevState* st,
                                                  int shift, uint32_t* hist, uint32_t* scan_len) {
  __shared__ uint32_t h[kRadix];
  const uint32_t n = st->n_total;
  const uint32_t ntiles = (n + kSortTile - 1) / kSortTile;
  if (blockIdx.x == 0 && threadIdx.x == 0) *scan_len = kRadix * ntiles;
  if (blockIdx.x >= ntiles) return;
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kSortTile;
#pragma unroll 4
  for (int it = 0; it < kSortItems; ++it) {
    uint32_t idx = base + it * kSortBlock + threadIdx.x;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & (kRadix - 1)], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(256) k_radix_down(const uint32_t* kin, const uint32_t* vin,
                                                    uint32_t* kout, uint32_t* vout,
                                                    const DevState* st, int shift,
                                                    const uint32_t* hist) {
  __shared__ uint32_t wh[4][kRadix];
  const uint32_t n = st->n_total;
  const uint32_t ntiles = (n + kSortTile - 1) / kSortTile;
  if (blockIdx.x >= ntiles) return;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const uint32_t gb = hist[t * ntiles + blockIdx.x];
#pragma unroll
  for (int q = 0; q < 4; ++q) wh[q][t] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint32_t base = blockIdx.x * kSortTile + w * (kSortTile / 4);
  uint32_t kk[kSortItems], vv[kSortItems], rk[kSortItems];
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const uint32_t idx = base + it * 64 + lane;
    const bool valid = idx < n;
    const uint32_t k = valid ? kin[idx] : 0u;
    const uint32_t v = valid ? (vin ? vin[idx] : idx) : 0u;
    const uint32_t d = (k >> shift) & (kRadix - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t r = (uint32_t)__popcll(peers & lt);
    const uint32_t old = wh[w][d];
    if (valid && r == 0) wh[w][d] = old + (uint32_t)__popcll(peers);
    kk[it] = k;
    vv[it] = v;
    rk[it] = old + r;
  }
  __syncthreads();
  {
    const uint32_t a0 = wh[0][t], a1 = wh[1][t], a2 = wh[2][t];
    wh[0][t] = gb;
    wh[1][t] = gb + a0;
    wh[2][t] = gb + a0 + a1;
    wh[3][t] = gb + a0 + a1 + a2;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const uint32_t idx = base + it * 64 + lane;
    if (idx < n) {
      const uint32_t d = (kk[it] >> shift) & (kRadix - 1);
      const uint32_t dst = wh[w][d] + rk[it];
      kout[dst] = kk[it];
      vout[dst] = vv[it];
    }
  }
}

void sort_keys(const uint32_t* keys, int key_bits, SortWork& w, DevState* st, uint32_t** skeys,
               uint32_t** perm, hipStream_t s) {
  const int tiles_cap = (int)((w.cap + kSortTile - 1) / kSortTile);
  const int g = tiles_cap < 1 ? 1 : tiles_cap;
  const uint32_t* kin = keys;
  const uint32_t* vin = nullptr;
  int passes = (key_bits + kRadixBits - 1) / kRadixBits;
  if (passes < 1) passes = 1;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * kRadixBits;
    uint32_t* kout = (p & 1) ? w.k1 : w.k0;
    uint32_t* vout = (p & 1) ? w.v1 : w.v0;
    k_radix_up<<<g, 256, 0, s>>>(kin, st, shift, w.hist, w.scan_len);
    scan_exclusive(w.hist, w.hist, w.scan_len, nullptr, w.bsum, (int64_t)kRadix * g, s);
    k_radix_down<<<g, 256, 0, s>>>(kin, vin, kout, vout, st, shift, w.hist);
    kin = kout;
    vin = vout;
  }
  *skeys = const_cast<uint32_t*>(kin);
  *perm = const_cast<uint32_t*>(vin);
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_gather(Parts src, Parts dst, const uint32_t* skeys,
                                                const uint32_t* perm, const DevState* st,
                                                uint32_t sentinel) {
  const uint32_t n = st->n_total;
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    const uint32_t k = skeys[p];
    if (k == sentinel) continue;
    const uint32_t q = perm[p];
    dst.r[p] = src.r[q];
    dst.z[p] = src.z[q];
    dst.vr[p] = src.vr[q];
    dst.vt[p] = src.vt[q];
    dst.vz[p] = src.vz[q];
    dst.sp[p] = src.sp[q];
    dst.id[p] = src.id[q];
    dst.key[p] = k;
  }
}

void gather_sorted(const Parts& src, const Parts& dst, const uint32_t* skeys, const uint32_t* perm,
                   const DevState* st, uint32_t sentinel, int64_t cap, hipStream_t s) {
  k_gather<<<grid_for(cap), 256, 0, s>>>(src, dst, skeys, perm, st, sentinel);
}

// off[k] = first sorted position whose key >= k, for k = 0 .. nkeys-1;
// off[sentinel] is the number of live particles.
__global__ void __launch_bounds__(256) k_offsets(const uint32_t* skeys, DevState* st,
                                                 uint32_t* off, uint32_t nkeys) {
  const uint32_t n = st->n_total;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nkeys; k += gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
      uint32_t mid = lo + ((hi - lo) >> 1);
      if (skeys[mid] < k) lo = mid + 1;
      else hi = mid;
    }
    off[k] = lo;
    if (k == nkeys - 1) st->n_alive = lo;
  }
}

void build_offsets(const uint32_t* skeys, DevState* st, uint32_t* off, uint32_t nkeys,
                   hipStream_t s) {
  k_offsets<<<grid_for(nkeys), 256, 0, s>>>(skeys, st, off, nkeys);
}

}  // namespace pd
