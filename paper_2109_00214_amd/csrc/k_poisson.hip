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

// Out[a][b] = sum_c X[c][a] S[c][b], c ascending.  Block = 4 waves, tile =
// 64 b (lanes) x 16 a (4 per wave, 4 independent accumulation chains per
// lane).  c advances in chunks of 32: the next chunk is fetched into
// registers while the current one is consumed from LDS (two LDS buffers,
// one barrier per chunk), so global latency overlaps the arithmetic.
//   FWD: X = f (rows = interior z nodes), Out -> fh[a][b] (a = r node, b = mode)
//   INV: X = G (rows = modes),            Out -> phi[b+1][a] with phi_vac, 2/nz
constexpr int kSineB = 64, kSineA = 16, kSineC = 32;

template <bool FWD>
__global__ void __launch_bounds__(256) k_sine(const double* __restrict__ X,
                                              const double* __restrict__ S, int nr, int nz,
                                              double V, double* __restrict__ out) {
  __shared__ double Ssh[2][kSineC][kSineB];
  __shared__ double Xsh[2][kSineC][kSineA];
  const int W = nr + 1, M = nz - 1;
  const int nA = W, nB = M, nC = M;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int b0 = blockIdx.x * kSineB, a0 = blockIdx.y * kSineA;
  // staging roles: S rows (t>>6) + 4q, column lane; X row t>>4 (+16), column t&15
  double sreg[8], xreg[2];
  auto fetch = [&](int c0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int c = c0 + (t >> 6) + 4 * q, b = b0 + lane;
      sreg[q] = (c < nC && b < nB) ? S[(size_t)c * M + b] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int c = c0 + (t >> 4) + 16 * q, a = a0 + (t & 15);
      xreg[q] = (c < nC && a < nA) ? X[(size_t)c * W + a] : 0.0;
    }
  };
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  fetch(0);
  int buf = 0;
  for (int c0 = 0; c0 < nC; c0 += kSineC, buf ^= 1) {
#pragma unroll
    for (int q = 0; q < 8; ++q) Ssh[buf][(t >> 6) + 4 * q][lane] = sreg[q];
#pragma unroll
    for (int q = 0; q < 2; ++q) Xsh[buf][(t >> 4) + 16 * q][t & 15] = xreg[q];
    __syncthreads();
    if (c0 + kSineC < nC) fetch(c0 + kSineC);
    if (nC - c0 >= kSineC) {
#pragma unroll 8
      for (int cc = 0; cc < kSineC; ++cc) {
        const double s = Ssh[buf][cc][lane];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = acc[q] + (Xsh[buf][cc][4 * w + q] * s);
      }
    } else {
      for (int cc = 0; cc < nC - c0; ++cc) {
        const double s = Ssh[buf][cc][lane];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = acc[q] + (Xsh[buf][cc][4 * w + q] * s);
      }
    }
  }
  const int b = b0 + lane;
  if (b >= nB) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int a = a0 + 4 * w + q;
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
// kThomasModes modes; their columns are staged in LDS with coalesced loads
// so the dependent sweeps read LDS instead of waiting on memory; the result
// is written mode-major (G[k][i]) for the inverse transform.
constexpr int kThomasModes = 8;

__global__ void __launch_bounds__(256) k_thomas_lds(const double* __restrict__ fh,
                                                   const double* __restrict__ tinv,
                                                   const double* __restrict__ tcp,
                                                   const double* __restrict__ ra, int nr, int nz,
                                                   double* __restrict__ G) {
  extern __shared__ double sh[];
  const int W = nr + 1, M = nz - 1;
  double* fL = sh;                       // [W][kThomasModes]
  double* tL = sh + (size_t)W * kThomasModes;
  const int k0 = blockIdx.x * kThomasModes;
  const int t = threadIdx.x;
  const int nL = W * kThomasModes;
#pragma unroll 4
  for (int idx = t; idx < nL; idx += 256) {
    const int i = idx / kThomasModes, kk = idx % kThomasModes, k = k0 + kk;
    fL[idx] = (k < M) ? fh[(size_t)i * M + k] : 0.0;
    tL[idx] = (k < M) ? tinv[(size_t)i * M + k] : 0.0;
  }
  __syncthreads();
  const bool act = (t < kThomasModes) && (k0 + t < M);
  double dp = 0.0;
  if (act) {
    dp = fL[t] * tL[t];
    fL[t] = dp;
    for (int i0 = 1; i0 <= nr; i0 += 8) {
      double fv[8], iv[8], av[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = (i0 + u <= nr) ? i0 + u : nr;
        fv[u] = fL[i * kThomasModes + t];
        iv[u] = tL[i * kThomasModes + t];
        av[u] = ra[i];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (i0 + u <= nr) {
          dp = (fv[u] - (av[u] * dp)) * iv[u];
          fL[(i0 + u) * kThomasModes + t] = dp;
        }
      }
    }
  }
  __syncthreads();
#pragma unroll 4
  for (int idx = t; idx < nL; idx += 256) {
    const int i = idx / kThomasModes, kk = idx % kThomasModes, k = k0 + kk;
    tL[idx] = (k < M) ? tcp[(size_t)i * M + k] : 0.0;
  }
  __syncthreads();
  if (act) {
    double x = dp;
    for (int i0 = nr - 1; i0 >= 0; i0 -= 8) {
      double fv[8], cv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = (i0 - u >= 0) ? i0 - u : 0;
        fv[u] = fL[i * kThomasModes + t];
        cv[u] = tL[i * kThomasModes + t];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (i0 - u >= 0) {
          x = fv[u] - (cv[u] * x);
          fL[(i0 - u) * kThomasModes + t] = x;
        }
      }
    }
  }
  __syncthreads();
#pragma unroll 4
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
  const dim3 grid((M + kSineB - 1) / kSineB, (W + kSineA - 1) / kSineA);
  k_sine<true><<<grid, 256, 0, s>>>(fw.f, fw.S, nr, nz, g.V, fw.fh);
  const size_t lds = sizeof(double) * 2 * (size_t)W * kThomasModes;
  k_thomas_lds<<<(M + kThomasModes - 1) / kThomasModes, 256, lds, s>>>(fw.fh, fw.tinv, fw.tcp,
                                                                     fw.ra, nr, nz, fw.g);
  k_sine<false><<<grid, 256, 0, s>>>(fw.g, fw.S, nr, nz, g.V, fw.phi);
}

size_t poisson_lds_bytes(int nr) { return sizeof(double) * 2 * (size_t)(nr + 1) * kThomasModes; }

}  // namespace pd
