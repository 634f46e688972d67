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
// most 64) and two b, the same for every lane: a term costs one vector load
// of a row of X (coalesced; the four waves of a block read the same rows) and
// the two sine entries come as scalar operands, eight consecutive c of a
// table row per scalar load.  No LDS: with one wave per SIMD every
// instruction takes an issue slot, and the operands need no staging.  The
// row loads are requested kFoAhead terms ahead; no contraction: each term is
// the product rounded, then the sum rounded, as written.
constexpr int kFoWaves = 4, kFoRb = 3, kFoAhead = 16;
constexpr int kFoB = kFoWaves * kFoRb;  // b per block

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
  const double* __restrict__ xp = X + (size_t)kFoAhead * W + ac;
  const int mfull = (M / kFoAhead) * kFoAhead;
  int c0 = 0;
  // a block of kFoAhead terms in two halves; each half's sine entries (three
  // table rows, eight words each) are loaded just before it, which keeps
  // them within the scalar registers
  auto block = [&](bool clamp) {
#pragma unroll
    for (int h = 0; h < kFoAhead; h += 8) {
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
        if (clamp) {
          const uint32_t o = (uint32_t)(c0 + kFoAhead + h + u) * (uint32_t)W + (uint32_t)ac;
          xr[h + u] = X[(o < last) ? o : last];
        } else {
          xr[h + u] = xp[(size_t)(h + u) * W];
        }
#pragma unroll
        for (int q = 0; q < kFoRb; ++q) acc[q] = acc[q] + p[q];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    xp += (size_t)kFoAhead * W;
  };
  // the blocks whose look-ahead rows all exist, then the last full block,
  // then the remaining rows (already in the ring)
  for (; c0 + 2 * kFoAhead <= M; c0 += kFoAhead) block(false);
  for (; c0 < mfull; c0 += kFoAhead) block(true);
  for (int u = 0; c0 + u < M; ++u) {
#pragma unroll
    for (int q = 0; q < kFoRb; ++q) acc[q] = acc[q] + (xr[u] * sr[q][c0 + u]);
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

// Tridiagonal solve per sine mode with the host-factored reciprocals (tinv)
// and upper factors (tcp), both [mode][i]: dp_0 = f_0 inv_0,
// dp_i = (f_i - a_i dp_{i-1}) inv_i; x_nr = dp_nr, x_i = dp_i - cp_i x_{i+1}.
// Each mode is one chain of dependent operations, so one lane per mode.  The
// block first stages every input of its modes in LDS with all loads in
// flight at once (one memory latency), then each lane runs its two sweeps
// from LDS with the next kThomasAhead rows read ahead into registers (dp
// and then x overwrite the right-hand side in place).  The result is
// written [mode][i], the layout the inverse transform reads.
constexpr int kThomasAhead = 8;
constexpr int kThomasStage = 12;  // staged words per thread and input array

__global__ void __launch_bounds__(256) k_thomas_fo(const double* __restrict__ fh,
                                                  const double* __restrict__ tinv,
                                                  const double* __restrict__ tcp,
                                                  const double* __restrict__ ra, int nr, int nz,
                                                  int mpb, double* __restrict__ G) {
  extern __shared__ double sh[];
  const int M = nz - 1, W = nr + 1;
  const int nL = W * mpb;
  double* fL = sh;            // [W][mpb] rhs, then dp
  double* iL = sh + nL;       // reciprocals
  double* cL = sh + 2 * nL;   // upper factors
  double* aL = sh + 3 * nL;   // [W] lower coefficients
  const int t = threadIdx.x;
  const int k0 = (int)blockIdx.x * mpb;
  for (int i = t; i < W; i += 256) aL[i] = ra[i];
  // every load in flight at once (mpb * W <= kThomasStage * 256 by the
  // choice of mpb), then the stores; element e = (mode kk, row i), i fastest
  double fv[kThomasStage], iv[kThomasStage], cv[kThomasStage];
#pragma unroll
  for (int u = 0; u < kThomasStage; ++u) {
    int e = 256 * u + t;
    e = (e < nL) ? e : nL - 1;
    const int kk = e / W, i = e % W;
    const int k = (k0 + kk < M) ? k0 + kk : M - 1;
    const size_t q = (size_t)k * W + i;
    fv[u] = fh[q];
    iv[u] = tinv[q];
    cv[u] = tcp[q];
  }
#pragma unroll
  for (int u = 0; u < kThomasStage; ++u) {
    const int e = 256 * u + t;
    if (e < nL) {
      const int kk = e / W, i = e % W;
      fL[i * mpb + kk] = fv[u];
      iL[i * mpb + kk] = iv[u];
      cL[i * mpb + kk] = cv[u];
    }
  }
  __syncthreads();
  // the two sweeps, one lane per mode: full runs of kThomasAhead rows with no
  // bounds checks (the rows of the next run are read while this one is
  // computed), then the remaining rows one at a time
  if (t < mpb) {
    double dp = fL[t] * iL[t];
    fL[t] = dp;
    {
      double fa[kThomasAhead], ia[kThomasAhead], aa[kThomasAhead];
      double fb[kThomasAhead], ib[kThomasAhead], ab[kThomasAhead];
      auto rd = [&](double* f, double* iv, double* a, int i0) {
#pragma unroll
        for (int u = 0; u < kThomasAhead; ++u) {
          const int i = (i0 + u <= nr) ? i0 + u : nr;
          f[u] = fL[i * mpb + t];
          iv[u] = iL[i * mpb + t];
          a[u] = aL[i];
        }
      };
      auto run = [&](const double* f, const double* iv, const double* a, int i0) {
#pragma unroll
        for (int u = 0; u < kThomasAhead; ++u) {
          dp = (f[u] - (a[u] * dp)) * iv[u];
          fL[(i0 + u) * mpb + t] = dp;
        }
      };
      int i = 1;
      rd(fa, ia, aa, 1);
      for (; i + 2 * kThomasAhead - 1 <= nr; i += 2 * kThomasAhead) {
        rd(fb, ib, ab, i + kThomasAhead);
        run(fa, ia, aa, i);
        rd(fa, ia, aa, i + 2 * kThomasAhead);
        run(fb, ib, ab, i + kThomasAhead);
      }
      if (i + kThomasAhead - 1 <= nr) {
        run(fa, ia, aa, i);
        i += kThomasAhead;
      }
      for (; i <= nr; ++i) {
        dp = (fL[i * mpb + t] - (aL[i] * dp)) * iL[i * mpb + t];
        fL[i * mpb + t] = dp;
      }
    }
    // backward sweep from x_nr = dp_nr; x overwrites dp in LDS
    double x = dp;
    {
      double da[kThomasAhead], ca[kThomasAhead], db[kThomasAhead], cb[kThomasAhead];
      auto rd = [&](double* d, double* c, int i0) {
#pragma unroll
        for (int u = 0; u < kThomasAhead; ++u) {
          const int i = (i0 - u >= 0) ? i0 - u : 0;
          d[u] = fL[i * mpb + t];
          c[u] = cL[i * mpb + t];
        }
      };
      auto run = [&](const double* d, const double* c, int i0) {
#pragma unroll
        for (int u = 0; u < kThomasAhead; ++u) {
          x = d[u] - (c[u] * x);
          fL[(i0 - u) * mpb + t] = x;
        }
      };
      int i = nr - 1;
      rd(da, ca, nr - 1);
      for (; i - 2 * kThomasAhead + 1 >= 0; i -= 2 * kThomasAhead) {
        rd(db, cb, i - kThomasAhead);
        run(da, ca, i);
        rd(da, ca, i - 2 * kThomasAhead);
        run(db, cb, i - kThomasAhead);
      }
      if (i - kThomasAhead + 1 >= 0) {
        run(da, ca, i);
        i -= kThomasAhead;
      }
      for (; i >= 0; --i) {
        x = fL[i * mpb + t] - (cL[i * mpb + t] * x);
        fL[i * mpb + t] = x;
      }
    }
  }
  __syncthreads();
  // the block's solutions to G[mode][i], coalesced over the rows
  for (int e = t; e < nL; e += 256) {
    const int kk = e / W, i = e % W, k = k0 + kk;
    if (k < M) G[(size_t)k * W + i] = fL[i * mpb + kk];
  }
}

// modes per Thomas block: the block's three input columns per mode and the
// lower coefficients in 64 KB of LDS
static int thomas_modes(int nr) {
  int mpb = 64;
  while (mpb > 1 && (((size_t)3 * mpb + 1) * (size_t)(nr + 1) * sizeof(double) > 65536 ||
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
  const int mpb = thomas_modes(nr);
  k_thomas_fo<<<(M + mpb - 1) / mpb, 256, sizeof(double) * ((size_t)3 * mpb + 1) * W, s>>>(
      fw.fh, fw.tinv, fw.tcp, fw.ra, nr, nz, mpb, fw.g);
  k_sine_fo<false><<<grid, 256, 0, s>>>(fw.g, fw.Sm, nr, nz, ag, g.V, g.Vdev, fw.phi);
}

// the direct solve's limits: the full sine table (nz-1)^2 words; the
// tridiagonal inputs of at least one mode in 64 KB of LDS
bool direct_fits(int nr, int nz) {
  return nz - 1 <= 2048 && (size_t)4 * (size_t)(nr + 1) * sizeof(double) <= 65536 &&
         (size_t)(nr + 1) <= (size_t)kThomasStage * 256;
}

}  // namespace pd
