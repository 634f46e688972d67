// k_poisson.hip -- direct FP64 solve of the cylindrical Poisson equation
// (paper Eq. 8, read as lap(phi) = -rho/eps0) on the node grid.
//
// phi = phi_vac + phi_p, phi_vac linear between the electrodes; phi_p by a
// sine transform (DST-I) over the interior z nodes, one tridiagonal solve per
// sine mode across r (the finite-volume radial operator plus the mode's
// eigenvalue of the 3-point d2/dz2), and the inverse transform.  Every sum of
// the transforms runs over its index in ascending order and every recurrence
// in its natural order, with no contraction: the result is the exact binary64
// value of the written expressions, independent of the launch geometry.
#include "pd_internal.h"

namespace pd {

// The right-hand side on the interior rows: f[c][a] = -(rho / eps0) at row
// c+1, radial node a, rho = Q qunit / V_node; the electrode rows of phi take
// the vacuum values (the sine series is zero there).
// The same launch reads the sine table once per XCD (every eighth block,
// in block order, takes one slice of it), so that the forward transform that
// follows finds it in its XCD's L2 rather than in memory: its scalar reads
// of the table are not prefetched and wait for every group of terms.
__global__ void __launch_bounds__(256) k_rhs(const int64_t* __restrict__ Q,
                                             const double* __restrict__ Vnode, double qunit,
                                             int nr, int nz, double V, const double* Vp,
                                             double* __restrict__ f,
                                             double* __restrict__ phi,
                                             const double* __restrict__ Sm,
                                             double* __restrict__ sink) {
  const int W = nr + 1, M = nz - 1;
  const int n = M * W;
  if (Vp) V = *Vp;  // the circuit's gap voltage
  {
    // slice blockIdx.x / 8 of gridDim.x / 8 slices: one word of every
    // 128-byte line of the slice
    const size_t words = (size_t)M * (size_t)M;
    const uint32_t nsl = gridDim.x / 8u > 0u ? gridDim.x / 8u : 1u;
    const size_t per = (words + nsl - 1) / nsl;
    const size_t lo = (size_t)(blockIdx.x / 8u) * per;
    const size_t hi = (lo + per < words) ? lo + per : words;
    double acc = 0.0;
    for (size_t i = lo + 16 * (size_t)threadIdx.x; i < hi; i += 16 * 256) acc += Sm[i];
    if (acc == 1.0e300) sink[0] = acc;  // keeps the reads
  }
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const int a = t % W;
    const double rho = ((double)Q[(size_t)t + W] * qunit) / Vnode[a];
    f[t] = -(rho / kEPS0);
    if (t < W) {
      phi[t] = ((-V) + (V * (0.0 / (double)nz))) + 0.0;
      phi[(size_t)nz * W + t] = ((-V) + (V * ((double)nz / (double)nz))) + 0.0;
    }
  }
}

// Sine transform with every sum in ascending order of its index:
//   Out[b][a] = sum_{c = 0 .. M-1} X[c][a] Sm[b][c], from +0.0, c ascending,
// Sm[b][c] = sin(pi (b+1)(c+1) / nz) (the DST-I matrix, symmetric; a host
// table).
//   FWD: X = f (c = interior row, a = radial node), Out -> fh[b][a] (b = mode)
//   INV: X = G (c = mode),                          Out -> phi[b+1][a], with
//        phi_vac added and the factor 2/nz.
// Each output is one chain of dependent additions.  A wave's lanes take
// consecutive radial nodes a (the radial extent split into equal groups of at
// most 64) and three b, the same for every lane: a term costs one vector load
// of a row of X (coalesced; the four waves of a block read the same rows) and
// the three sine entries come as scalar operands, eight consecutive c of a
// table row per scalar load.  No LDS: with one wave per SIMD every
// instruction takes an issue slot, and the operands need no staging.  The
// row loads are requested kFoAhead terms ahead, as buffer loads from the
// lane's byte offset of each of the kFoAhead rows (fixed for the kernel) and
// one scalar offset per block of rows, so that a term costs no address
// arithmetic; a half block's eight rows are requested after its eight terms,
// and one wait at the start of a half covers them all.  No contraction: each
// term is the product rounded, then the sum rounded, as written.
constexpr int kFoWaves = 4, kFoRb = 3, kFoAhead = 16;
constexpr int kFoB = kFoWaves * kFoRb;  // b per block
constexpr int kFoWait = ((kFoAhead - 8) & 0xF) | (((kFoAhead - 8) >> 4) << 14) | 0x70 | 0xF00;

template <bool FWD>
__global__ void __launch_bounds__(256, 1) k_sine_fo(const double* __restrict__ X,
                                                    const double* __restrict__ Sm, int nr,
                                                    int nz, int ag, double V, const double* Vp,
                                                    double* __restrict__ out) {
  const int W = nr + 1, M = nz - 1;
  if (!FWD && Vp) V = *Vp;  // the circuit's gap voltage
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int a = (int)blockIdx.x * ag + lane;
  const bool live = lane < ag && a < W;
  const int ac = live ? a : 0;
  const int bw = (int)blockIdx.y * kFoB + w * kFoRb;  // this wave's first b
  const double* __restrict__ sr[kFoRb];
#pragma unroll
  for (int q = 0; q < kFoRb; ++q) sr[q] = Sm + (size_t)((bw + q < M) ? bw + q : M - 1) * M;
  double acc[kFoRb];
#pragma unroll
  for (int q = 0; q < kFoRb; ++q) acc[q] = 0.0;
  // ring of row values requested kFoAhead terms ahead
  const uint32_t last = (uint32_t)(M - 1) * (uint32_t)W + (uint32_t)ac;
  double xr[kFoAhead];
#pragma unroll
  for (int u = 0; u < kFoAhead; ++u) {
    const uint32_t o = (uint32_t)u * (uint32_t)W + (uint32_t)ac;
    xr[u] = X[(o < last) ? o : last];
  }
  const int mfull = (M / kFoAhead) * kFoAhead;
  int c0 = 0;
  // the terms of a half block (its sine entries, three table rows of eight
  // words, are loaded just before it, which keeps them within the scalar
  // registers)
  auto half = [&](int h) {
    double sv[kFoRb][8];
#pragma unroll
    for (int q = 0; q < kFoRb; ++q)
#pragma unroll
      for (int u = 0; u < 8; ++u) sv[q][u] = sr[q][c0 + h + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      double p[kFoRb];
#pragma unroll
      for (int q = 0; q < kFoRb; ++q) p[q] = xr[h + u] * sv[q][u];
#pragma unroll
      for (int q = 0; q < kFoRb; ++q) acc[q] = acc[q] + p[q];
    }
  };
  // the blocks whose look-ahead rows all exist: the byte offsets of a block's
  // rows from its first row's, per lane, and the buffer over X
  __amdgpu_buffer_rsrc_t rx =
      __builtin_amdgcn_make_buffer_rsrc((void*)X, (short)0, (int)((size_t)M * W * 8), 0x00020000);
  int voff[kFoAhead];
#pragma unroll
  for (int u = 0; u < kFoAhead; ++u) voff[u] = (ac + u * W) * 8;
  for (; c0 + 2 * kFoAhead <= M; c0 += kFoAhead) {
    const int sob = (c0 + kFoAhead) * W * 8;  // the next block's first row
#pragma unroll
    for (int h = 0; h < kFoAhead; h += 8) {
      // this group's rows were requested before the other groups': at most
      // their kFoAhead - 8 loads are still in flight (s_waitcnt vmcnt, split
      // into bits 3:0 and 15:14; the other counters at their maximum)
      __builtin_amdgcn_s_waitcnt(kFoWait);
      half(h);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(rx, voff[h + u], sob, 0);
        __builtin_memcpy(&xr[h + u], &v, sizeof(double));
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // then the last full block, whose look-ahead rows are clamped to the last
  // row, then the remaining rows (already in the ring)
  for (; c0 < mfull; c0 += kFoAhead) {
#pragma unroll
    for (int h = 0; h < kFoAhead; h += 8) {
      half(h);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t o = (uint32_t)(c0 + kFoAhead + h + u) * (uint32_t)W + (uint32_t)ac;
        xr[h + u] = X[(o < last) ? o : last];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int u = 0; u < kFoAhead; ++u) {  // unrolled: the ring stays in registers
    if (c0 + u < M) {
#pragma unroll
      for (int q = 0; q < kFoRb; ++q) acc[q] = acc[q] + (xr[u] * sr[q][c0 + u]);
    }
  }
  if (!live) return;
#pragma unroll
  for (int q = 0; q < kFoRb; ++q) {
    const int b = bw + q;
    if (b >= M) break;
    if (FWD) {
      out[(size_t)b * W + a] = acc[q];
    } else {
      const int j = b + 1;
      const double vac = (-V) + (V * ((double)j / (double)nz));
      out[(size_t)j * W + a] = vac + (acc[q] * (2.0 / (double)nz));
    }
  }
}

// Tridiagonal solve per sine mode, eliminated from both ends with the
// host-factored pivot reciprocals (tinv) and factors toward the middle row
// m = nr / 2 (tcp), both [mode][i]:
//   rows s = 0 .. m-1 from the axis:  d_s = (f_s - a_s d_{s-1}) inv_s,
//   rows i = nr .. m+1 from the wall: d_i = (f_i - c_i d_{i+1}) inv_i,
//   x_m = ((f_m - a_m d_{m-1}) - c_m d_{m+1}) inv_m,
//   x_s = d_s - cp_s x_{s+1} above m, x_i = d_i - cp_i x_{i-1} below.
// Each half is one chain of dependent operations, so two lanes per mode,
// each with half the chain; the time is the chain's: a single wave per SIMD
// waits out every dependent FP64 operation, so what matters is that nothing
// else is on the chain.  The block stages its modes' inputs in LDS half by
// half, the wall's half reversed, so that both lanes of a mode run the same
// instructions on ascending rows (s = i above, s = nr - i below; each half
// thomas_pitch(nr) words apart with kThomasPad padding rows at each end),
// all loads in flight at once; each lane then sweeps its own rows at fixed
// offsets from one address, kThomasAhead rows read ahead into registers
// with no bounds checks (the reads past either end land in the padding and
// are never used).  The two lanes meet in row m through a lane exchange and
// compute it alike; the back substitution writes x straight to G[mode][i],
// the layout the inverse transform reads.  Meanwhile the block's other
// three waves read the sine table once per XCD, as the right-hand side does
// for the forward transform, so that the inverse transform finds it in its
// XCD's L2.
constexpr int kThomasAhead = 8;
constexpr int kThomasStage = 12;  // staged words per thread and input array
constexpr int kThomasPad = 2 * kThomasAhead;

static int thomas_pitch(int nr) {
  int P = (nr - nr / 2 + 1) + 2 * kThomasPad;  // rows of the longer half, middle included
  return (P & 1) ? P : P + 1;  // odd: the lanes' rows fall in different banks
}

__global__ void __launch_bounds__(256) k_thomas_fo(const double* __restrict__ fh,
                                                  const double* __restrict__ tinv,
                                                  const double* __restrict__ tcp,
                                                  const double* __restrict__ ra,
                                                  const double* __restrict__ rc, int nr, int nz,
                                                  int mpb, int P, double* __restrict__ G,
                                                  const double* __restrict__ Sm,
                                                  double* __restrict__ sink) {
  extern __shared__ double sh[];
  constexpr int K = kThomasAhead, H = kThomasPad;
  const int M = nz - 1, W = nr + 1, m = nr / 2;
  const int L = 2 * mpb;                  // lanes: a mode's two halves
  double* fL = sh;                        // [lane][P]: rhs, then d
  double* iL = sh + (size_t)L * P;        // pivot reciprocals
  double* cL = sh + (size_t)2 * L * P;    // factors toward the middle
  double* oL = sh + (size_t)3 * L * P;    // [half][P] a (axis half), c (wall half)
  const int t = threadIdx.x;
  const int k0 = (int)blockIdx.x * mpb;
  const int nm = (M - k0 < mpb) ? M - k0 : mpb;  // modes of this block
  const int nL = nm * W;
  const size_t g0 = (size_t)k0 * W;  // the block's modes are contiguous in fh, tinv, tcp, G
  for (int i = t; i < W; i += 256) {
    if (i <= m) oL[H + i] = ra[i];
    if (i >= m) oL[P + H + (nr - i)] = rc[i];
  }
  // every load in flight at once (mpb * W <= kThomasStage * 256 by the
  // choice of mpb), then the stores; row m goes to both halves
  double fv[kThomasStage], iv[kThomasStage], cv[kThomasStage];
#pragma unroll
  for (int u = 0; u < kThomasStage; ++u) {
    int e = 256 * u + t;
    e = (e < nL) ? e : nL - 1;
    fv[u] = fh[g0 + e];
    iv[u] = tinv[g0 + e];
    cv[u] = tcp[g0 + e];
  }
#pragma unroll
  for (int u = 0; u < kThomasStage; ++u) {
    const int e = 256 * u + t;
    if (e < nL) {
      const int kk = e / W, i = e - kk * W;
      if (i <= m) {
        const int o = (2 * kk) * P + H + i;
        fL[o] = fv[u];
        iL[o] = iv[u];
        cL[o] = cv[u];
      }
      if (i >= m) {
        const int o = (2 * kk + 1) * P + H + (nr - i);
        fL[o] = fv[u];
        iL[o] = iv[u];
        cL[o] = cv[u];
      }
    }
  }
  __syncthreads();
  if (t >= 2 * nm) {
    if (t >= 64) {
      // slice blockIdx.x / 8 of gridDim.x / 8 slices: one word of every
      // 128-byte line of the slice
      const size_t words = (size_t)M * (size_t)M;
      const uint32_t nsl = gridDim.x / 8u > 0u ? gridDim.x / 8u : 1u;
      const size_t per = (words + nsl - 1) / nsl;
      const size_t lo = (size_t)(blockIdx.x / 8u) * per;
      const size_t hi = (lo + per < words) ? lo + per : words;
      double acc = 0.0;
      for (size_t i = lo + 16 * (size_t)(t - 64); i < hi; i += 16 * 192) acc += Sm[i];
      if (acc == 1.0e300) sink[0] = acc;  // keeps the reads
    }
    return;
  }
  const int half = t & 1, kk = t >> 1;
  const int len = half ? nr - m : m;  // rows this lane eliminates: s = 0 .. len-1
  double* fr = fL + t * P + H;        // row s of this lane's half at fr[s]
  const double* ir = iL + t * P + H;
  const double* cr = cL + t * P + H;
  const double* ar = oL + half * P + H;
  double* gr = G + g0 + (size_t)kk * W;
  // elimination toward the middle: runs of K rows, the next run read while
  // this one is computed; the last two runs are checked against len - 1
  const int last = len - 1;
  double dp = 0.0;
  if (len > 0) {
    dp = fr[0] * ir[0];
    fr[0] = dp;
  }
  {
    double fa[K], ia[K], aa[K], fb[K], ib[K], ab[K];
    auto rd = [&](double* f, double* iv, double* a, int i0) {
#pragma unroll
      for (int u = 0; u < K; ++u) {
        f[u] = fr[i0 + u];
        iv[u] = ir[i0 + u];
        a[u] = ar[i0 + u];
      }
    };
    auto run = [&](const double* f, const double* iv, const double* a, int i0, bool check) {
#pragma unroll
      for (int u = 0; u < K; ++u) {
        if (!check || i0 + u <= last) {
          dp = (f[u] - (a[u] * dp)) * iv[u];
          fr[i0 + u] = dp;
        }
      }
    };
    int i = 1;
    rd(fa, ia, aa, 1);
    for (; i + 2 * K - 1 <= last; i += 2 * K) {
      rd(fb, ib, ab, i + K);
      run(fa, ia, aa, i, false);
      rd(fa, ia, aa, i + 2 * K);  // rows up to last + K
      run(fb, ib, ab, i + K, false);
    }
    rd(fb, ib, ab, i + K);  // i <= last + 1: rows up to last + 2K
    run(fa, ia, aa, i, true);
    run(fb, ib, ab, i + K, true);
  }
  // row m from both halves' last eliminated rows, the same arithmetic on
  // both lanes (the axis half's first, as in the elimination order)
  const int ta = t & ~1;
  const double da = __shfl(dp, ta, 64), dw = __shfl(dp, ta | 1, 64);
  double num = fL[ta * P + H + m];
  if (m > 0) num = num - (oL[H + m] * da);
  if (m < nr) num = num - (oL[P + H + (nr - m)] * dw);
  double x = num * iL[ta * P + H + m];
  if (half == 0) gr[m] = x;
  // back substitution from row m outwards: x_s = d_s - cp_s x_{s+1}, s from
  // len - 1 down to 0; G at i = s (axis half) or i = nr - s (wall half)
  double* gx = half ? gr + nr : gr;
  const int gs = half ? -1 : 1;
  {
    double da_[K], ca[K], db[K], cb[K];
    auto rd = [&](double* d, double* c, int i0) {
#pragma unroll
      for (int u = 0; u < K; ++u) {
        d[u] = fr[i0 - u];
        c[u] = cr[i0 - u];
      }
    };
    auto run = [&](const double* d, const double* c, int i0, bool check) {
#pragma unroll
      for (int u = 0; u < K; ++u) {
        if (!check || i0 - u >= 0) {
          x = d[u] - (c[u] * x);
          gx[gs * (i0 - u)] = x;
        }
      }
    };
    int i = len - 1;
    rd(da_, ca, len - 1);
    for (; i - 2 * K + 1 >= 0; i -= 2 * K) {
      rd(db, cb, i - K);
      run(da_, ca, i, false);
      rd(da_, ca, i - 2 * K);  // rows down to -K
      run(db, cb, i - K, false);
    }
    rd(db, cb, i - K);  // i >= -1: rows down to -2K
    run(da_, ca, i, true);
    run(db, cb, i - K, true);
  }
}

// modes per tridiagonal block: two (the sweeps take the same time for any
// number of lanes, and a small block stages its inputs sooner), one where
// two do not fit in 64 KB of LDS or the staging registers
static int thomas_modes(int nr) {
  const size_t P = (size_t)thomas_pitch(nr);
  int mpb = 2;
  while (mpb > 1 && (((size_t)6 * mpb + 2) * P * sizeof(double) > 65536 ||
                     (size_t)mpb * (size_t)(nr + 1) > (size_t)kThomasStage * 256))
    mpb >>= 1;
  return mpb;
}

void poisson_direct(const Grid& g, FieldWork& fw, hipStream_t s) {
  const int nr = g.nr, nz = g.nz, M = nz - 1, W = nr + 1;
  int gr = (M * W + 255) / 256;
  if (gr > 4096) gr = 4096;
  k_rhs<<<gr, 256, 0, s>>>(fw.Q, fw.Vnode, fw.qunit, nr, nz, g.V, g.Vdev, fw.f, fw.phi, fw.Sm,
                           fw.g);
  // the radial nodes in equal groups of at most 64 (one group per lane set)
  const int ngrp = (W + 63) / 64, ag = (W + ngrp - 1) / ngrp;
  const dim3 grid(ngrp, (M + kFoB - 1) / kFoB);
  k_sine_fo<true><<<grid, 256, 0, s>>>(fw.f, fw.Sm, nr, nz, ag, g.V, nullptr, fw.fh);
  const int mpb = thomas_modes(nr), P = thomas_pitch(nr);
  k_thomas_fo<<<(M + mpb - 1) / mpb, 256, sizeof(double) * ((size_t)6 * mpb + 2) * P, s>>>(
      fw.fh, fw.twinv, fw.twcp, fw.ra, fw.rc, nr, nz, mpb, P, fw.g, fw.Sm, fw.f);
  k_sine_fo<false><<<grid, 256, 0, s>>>(fw.g, fw.Sm, nr, nz, ag, g.V, g.Vdev, fw.phi);
}

// the direct solve's limits: the full sine table (nz-1)^2 words; the
// tridiagonal inputs of at least one mode, with the padding rows, in 64 KB
// of LDS
bool direct_fits(int nr, int nz) {
  return nz - 1 <= 2048 && (size_t)8 * (size_t)thomas_pitch(nr) * sizeof(double) <= 65536 &&
         (size_t)(nr + 1) <= (size_t)kThomasStage * 256;
}

}  // namespace pd
