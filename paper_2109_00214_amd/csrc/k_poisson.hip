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

// f[c][a] = -(rho / eps0) at interior row c+1, node a, rho = Q qunit / V_node;
// the electrode rows of phi take the vacuum values (the sine series is zero).
__global__ void __launch_bounds__(256) k_rhs(const int64_t* __restrict__ Q,
                                             const double* __restrict__ Vnode, double qunit,
                                             int nr, int nz, double V, double* __restrict__ f,
                                             double* __restrict__ phi) {
  const int W = nr + 1, M = nz - 1;
  const int n = M * W;
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

// Out[a][b] = sum_c X[c][a] S[c][b], c ascending, S[c][b] the DST-I entry of
// sine index k = b+1 (resp. c+1) and node j = c+1 (resp. b+1).  The entry
// depends only on m = ((c+1)(b+1)) mod 2nz, so it is looked up in a table T
// of 2nz values (built on the host with the same formula as the entries
// themselves) held in LDS; m advances by b+1 per term.  Block = 4 waves
// covering 64 b (lanes) x 8 a (2 per wave: two independent accumulation
// chains per lane); the block's X columns (all c) sit in LDS too.  No global
// traffic in the loop and no barriers.
//   FWD: X = f (rows = interior z nodes), Out -> fh[a][b] (a = r node, b = mode)
//   INV: X = G (rows = modes),            Out -> phi[b+1][a] with phi_vac, 2/nz
constexpr int kSineA = 4, kSineWaves = 4, kSineAPW = kSineA / kSineWaves;

template <bool FWD>
__global__ void __launch_bounds__(64 * kSineWaves) k_sine(const double* __restrict__ X,
                                                          const double* __restrict__ T, int nr,
                                                          int nz, double V,
                                                          double* __restrict__ out) {
  extern __shared__ double lds[];
  constexpr int NT = 64 * kSineWaves;
  const int W = nr + 1, M = nz - 1, N2 = 2 * nz;
  const int nA = W, nB = M, nC = M;
  double* Tsh = lds;             // [2 nz]
  double* Xsh = lds + N2;        // [nC][kSineA]
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int b = blockIdx.x * 64 + lane;
  const int bl = (b < nB) ? b : nB - 1;
  const int a0 = blockIdx.y * kSineA;
  // loads use clamped (always valid) indices and no branches, so that a
  // thread's loads are all in flight together
  for (int i0 = 0; i0 < N2; i0 += NT * 4) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + NT * u + t;
      v[u] = T[(i < N2) ? i : N2 - 1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + NT * u + t < N2) Tsh[i0 + NT * u + t] = v[u];
  }
  const int nX = nC * kSineA;
  for (int i0 = 0; i0 < nX; i0 += NT * 4) {
    double v[4];
    int ix[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ix[u] = i0 + NT * u + t;
      const int idx = (ix[u] < nX) ? ix[u] : nX - 1;
      const int c = idx / kSineA, a = a0 + idx % kSineA;
      v[u] = X[(size_t)c * W + ((a < nA) ? a : nA - 1)];
      if (a >= nA) v[u] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (ix[u] < nX) Xsh[ix[u]] = v[u];
  }
  __syncthreads();
  double acc[kSineAPW];
#pragma unroll
  for (int q = 0; q < kSineAPW; ++q) acc[q] = 0.0;
  const double* x0 = Xsh + kSineAPW * w;
  const int step = bl + 1;
  int m = step;  // (c+1)(b+1) mod 2nz at c = 0
  const int nfull = (nC / 8) * 8;
  for (int c0 = 0; c0 < nfull; c0 += 8) {
    double s[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      s[u] = Tsh[m];
      m += step;
      if (m >= N2) m -= N2;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int q = 0; q < kSineAPW; ++q)
        acc[q] = acc[q] + (x0[(c0 + u) * kSineA + q] * s[u]);
    }
  }
  for (int c = nfull; c < nC; ++c) {
    const double s = Tsh[m];
    m += step;
    if (m >= N2) m -= N2;
#pragma unroll
    for (int q = 0; q < kSineAPW; ++q) acc[q] = acc[q] + (x0[c * kSineA + q] * s);
  }
  if (b >= nB) return;
#pragma unroll
  for (int q = 0; q < kSineAPW; ++q) {
    const int a = a0 + kSineAPW * w + q;
    if (a >= nA) break;
    if (FWD) {
      out[(size_t)a * M + b] = acc[q];
    } else {
      const int j = b + 1;
      const double vac = (-V) + (V * ((double)j / (double)nz));
      out[(size_t)j * W + a] = vac + (acc[q] * (2.0 / (double)nz));
    }
  }
}

// Tridiagonal solve per sine mode with the host-factored reciprocals
// (tinv) and upper factors (tcp): dp_0 = f_0 inv_0, dp_i = (f_i - a_i
// dp_{i-1}) inv_i; x_nr = dp_nr, x_i = dp_i - cp_i x_{i+1}.  A block takes
// kThomasModes modes; their columns are staged in LDS with coalesced loads;
// the upper factors are staged by the idle waves while the first wave runs
// the forward sweep.  Each sweep fetches the next 8 rows from LDS while it
// computes the current 8.  The result is written mode-major (G[k][i]) for
// the inverse transform.
constexpr int kThomasModes = 8;

__global__ void __launch_bounds__(256) k_thomas_lds(const double* __restrict__ fh,
                                                   const double* __restrict__ tinv,
                                                   const double* __restrict__ tcp,
                                                   const double* __restrict__ ra, int nr, int nz,
                                                   double* __restrict__ G) {
  extern __shared__ double sh[];
  const int W = nr + 1, M = nz - 1;
  const int nL = W * kThomasModes;
  double* fL = sh;                 // [W][kThomasModes]: rhs, then dp, then x
  double* tL = sh + nL;            // reciprocals
  double* cL = sh + 2 * nL;        // upper factors
  double* aL = sh + 3 * nL;        // [W] lower coefficients
  const int k0 = blockIdx.x * kThomasModes;
  const int t = threadIdx.x;
  for (int i = t; i < W; i += 256) aL[i] = ra[i];
  // clamped indices, no branches around the loads (all in flight together)
  for (int j0 = 0; j0 < nL; j0 += 256 * 4) {
    double fv[4], tv[4];
    int ix[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ix[u] = j0 + 256 * u + t;
      const int idx = (ix[u] < nL) ? ix[u] : nL - 1;
      const int i = idx / kThomasModes, k = k0 + idx % kThomasModes;
      const size_t q = (size_t)i * M + ((k < M) ? k : M - 1);
      fv[u] = fh[q];
      tv[u] = tinv[q];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (ix[u] < nL) {
        fL[ix[u]] = fv[u];
        tL[ix[u]] = tv[u];
      }
  }
  __syncthreads();
  const bool act = (t < kThomasModes) && (k0 + t < M);
  double dp = 0.0;
  if (t < 64) {
    if (act) {
      dp = fL[t] * tL[t];
      fL[t] = dp;
      double fa[8], ia[8], aa[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = (1 + u <= nr) ? 1 + u : nr;
        fa[u] = fL[i * kThomasModes + t];
        ia[u] = tL[i * kThomasModes + t];
        aa[u] = aL[i];
      }
      for (int i0 = 1; i0 <= nr; i0 += 8) {
        double fb[8], ib[8], ab[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = (i0 + 8 + u <= nr) ? i0 + 8 + u : nr;
          fb[u] = fL[i * kThomasModes + t];
          ib[u] = tL[i * kThomasModes + t];
          ab[u] = aL[i];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (i0 + u <= nr) {
            dp = (fa[u] - (aa[u] * dp)) * ia[u];
            fL[(i0 + u) * kThomasModes + t] = dp;
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          fa[u] = fb[u];
          ia[u] = ib[u];
          aa[u] = ab[u];
        }
      }
    }
  } else {
    for (int j0 = 0; j0 < nL; j0 += 192 * 4) {
      double cv[4];
      int ix[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ix[u] = j0 + 192 * u + (t - 64);
        const int idx = (ix[u] < nL) ? ix[u] : nL - 1;
        const int i = idx / kThomasModes, k = k0 + idx % kThomasModes;
        cv[u] = tcp[(size_t)i * M + ((k < M) ? k : M - 1)];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (ix[u] < nL) cL[ix[u]] = cv[u];
    }
  }
  __syncthreads();
  if (act) {
    double x = dp;
    double fa[8], ca[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = (nr - 1 - u >= 0) ? nr - 1 - u : 0;
      fa[u] = fL[i * kThomasModes + t];
      ca[u] = cL[i * kThomasModes + t];
    }
    for (int i0 = nr - 1; i0 >= 0; i0 -= 8) {
      double fb[8], cb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = (i0 - 8 - u >= 0) ? i0 - 8 - u : 0;
        fb[u] = fL[i * kThomasModes + t];
        cb[u] = cL[i * kThomasModes + t];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (i0 - u >= 0) {
          x = fa[u] - (ca[u] * x);
          fL[(i0 - u) * kThomasModes + t] = x;
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        fa[u] = fb[u];
        ca[u] = cb[u];
      }
    }
  }
  __syncthreads();
#pragma unroll 8
  for (int idx = t; idx < nL; idx += 256) {
    const int kk = idx / W, i = idx % W, k = k0 + kk;
    if (k < M) G[(size_t)k * W + i] = fL[i * kThomasModes + kk];
  }
}

void poisson_direct(const Grid& g, FieldWork& fw, hipStream_t s) {
  const int nr = g.nr, nz = g.nz, M = nz - 1, W = nr + 1;
  int gr = (M * W + 255) / 256;
  if (gr > 4096) gr = 4096;
  k_rhs<<<gr, 256, 0, s>>>(fw.Q, fw.Vnode, fw.qunit, nr, nz, g.V, fw.f, fw.phi);
  const dim3 grid((M + 63) / 64, (W + kSineA - 1) / kSineA);
  const size_t xlds = sizeof(double) * ((size_t)M * kSineA + 2 * (size_t)nz);
  k_sine<true><<<grid, 64 * kSineWaves, xlds, s>>>(fw.f, fw.T, nr, nz, g.V, fw.fh);
  k_thomas_lds<<<(M + kThomasModes - 1) / kThomasModes, 256, poisson_lds_bytes(nr, nz), s>>>(
      fw.fh, fw.tinv, fw.tcp, fw.ra, nr, nz, fw.g);
  k_sine<false><<<grid, 64 * kSineWaves, xlds, s>>>(fw.g, fw.T, nr, nz, g.V, fw.phi);
}

// the larger of the two dynamic LDS needs (Thomas columns, transform rows)
size_t poisson_lds_bytes(int nr, int nz) {
  const size_t th = sizeof(double) * (3 * (size_t)kThomasModes + 1) * (size_t)(nr + 1);
  const size_t tr = sizeof(double) * ((size_t)(nz - 1) * kSineA + 2 * (size_t)nz);
  return th > tr ? th : tr;
}

}  // namespace pd
