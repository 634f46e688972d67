// k_spectral.hip -- the direct FP64 Poisson solve of k_poisson.hip (sine
// transform in z, one tridiagonal system per sine mode in r, inverse
// transform; paper Eq. 8 read as lap(phi) = -rho/eps0) evaluated for speed
// instead of for a fixed rounding order:
//
//   transforms  -- dense products D[b][a] = sum_c S[c][b] X[c][a] on the FP64
//                  matrix cores (v_mfma_f64_16x16x4f64): one 16 x 16 output
//                  tile per block, the c range split over its four waves and
//                  their partial tiles added in LDS in a fixed order;
//   tridiagonal -- each mode's recurrences dp_i = u_i - w_i dp_{i-1} and
//                  x_i = dp_i - c_i x_{i+1} as scans of affine maps over one
//                  wave (each lane composes a run of rows, the lanes combine
//                  by shuffles in log2(64) steps, each lane then replays its
//                  run from the value entering it).
//
// Same equations, tables and factorisation as the sequential solve; only the
// order of the floating-point operations differs, so the potential agrees
// with the sequential solve to rounding.  Every launch is deterministic.
#include "pd_internal.h"

namespace pd {
namespace {

typedef double dx4 __attribute__((ext_vector_type(4)));

// D[b][a] (b: output row of the transform, a: radial node) for the 16 x 16
// tile (blockIdx.y, blockIdx.x).  FWD: X[c][a] = Q[c+1][a] coef[a] (the
// right-hand side -rho/eps0 at interior row c+1), out = fh[b][a].  INV:
// X[c][a] = G[c][a] (mode c), out = phi[b+1][a] = vac + (2/nz) D and the
// electrode rows.  Operand layout of the 16x16x4 product: lane l holds
// A[l%16][l/16] and B[l/16][l%16]; result register r of lane l is
// D[4r + l/16][l%16].
constexpr int kDstSteps = 16;  // k-steps of 4 loaded ahead of their products

// At most 128 registers a lane, so that four waves share a SIMD: the 16 x 16
// tiles of a 256 x 512 grid (544 blocks) then run in one round.
template <bool FWD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_dst_mfma(const int64_t* __restrict__ Q, const double* __restrict__ coef,
           const double* __restrict__ G, const double* __restrict__ T, int nr, int nz, double V,
           const double* Vp, double* __restrict__ out) {
  extern __shared__ double Ts[];  // the sine table, 2 nz entries (dynamic LDS)
  __shared__ double red[3][4][64];
  const int W = nr + 1, M = nz - 1, N2 = 2 * nz;
  if (Vp) V = *Vp;  // the circuit's gap voltage
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // the operand entries are scattered over the table: served from LDS, a
  // gather from the vector cache costs one tag lookup per lane
  for (int i0 = 0; i0 < N2; i0 += 4 * 256) {
    double tv[4];  // four loads in flight, then the four stores
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * 256 + t;
      tv[u] = T[(i < N2) ? i : 0];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * 256 + t;
      if (i < N2) Ts[i] = tv[u];
    }
  }
  const int li = lane & 15, lk = lane >> 4;
  const int a0 = blockIdx.x * 16, b0 = blockIdx.y * 16;
  const int a = a0 + li, ac = (a < W) ? a : W - 1;
  const int bA = b0 + li, bc = (bA < M) ? bA : M - 1;  // row of the A operand
  const int KW = (((M + 3) / 4 + 3) / 4) * 4;           // c per wave, multiple of 4
  const int cw0 = w * KW;
  const int nsteps = KW / 4;
  const int sb = bc + 1;
  const int dm = (4 * sb) % N2;  // products below nz^2 <= 2^26: 32-bit
  int c = cw0 + lk;
  int m = ((c + 1) * sb) % N2;
  dx4 acc = {0.0, 0.0, 0.0, 0.0};
  const double cf = FWD ? coef[ac] : 1.0;
  __syncthreads();
  for (int s0 = 0; s0 < nsteps; s0 += kDstSteps) {
    // every load of the chunk first (clamped, unconditional), then the
    // products, so that the loads are in flight together
    int mi[kDstSteps];
#pragma unroll
    for (int u = 0; u < kDstSteps; ++u) {
      mi[u] = m;
      m += dm;
      if (m >= N2) m -= N2;
    }
    double av[kDstSteps], bv[kDstSteps];
    int64_t qv[kDstSteps];
#pragma unroll
    for (int u = 0; u < kDstSteps; ++u) {
      const int cu = c + 4 * u;
      const int cl = (cu < M) ? cu : M - 1;
      av[u] = Ts[mi[u]];
      if (FWD) qv[u] = Q[(size_t)(cl + 1) * W + ac];
      else bv[u] = G[(size_t)cl * W + ac];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep every load of the chunk ahead
#pragma unroll
    for (int u = 0; u < kDstSteps; ++u) {
      const int cu = c + 4 * u;
      const bool ok = (s0 + u < nsteps) && (cu < M);
      const double x = FWD ? (double)qv[u] * cf : bv[u];
      bv[u] = ok ? x : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kDstSteps; ++u)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    c += 4 * kDstSteps;
  }
  if (w > 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) red[w - 1][r][lane] = acc[r];
  }
  __syncthreads();
  if (w > 0) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double v = ((acc[r] + red[0][r][lane]) + red[1][r][lane]) + red[2][r][lane];
    const int b = b0 + 4 * r + lk;
    if (b >= M || a >= W) continue;
    if (FWD) {
      out[(size_t)b * W + a] = v;
    } else {
      const int j = b + 1;
      const double vac = (-V) + (V * ((double)j / (double)nz));
      out[(size_t)j * W + a] = vac + (v * (2.0 / (double)nz));
    }
  }
  if (!FWD && blockIdx.y == 0 && lane < 16 && a < W) {
    out[a] = ((-V) + (V * (0.0 / (double)nz))) + 0.0;
    out[(size_t)nz * W + a] = ((-V) + (V * ((double)nz / (double)nz))) + 0.0;
  }
}

// affine map y -> al + be y; compose(p, q) = p after q
struct Aff {
  double al, be;
};
__device__ inline Aff after(Aff p, Aff q) { return {p.al + p.be * q.al, p.be * q.be}; }

__device__ inline double shfl_up_f64(double v, int o) {
  return __shfl_up(v, o, 64);
}
__device__ inline double shfl_down_f64(double v, int o) {
  return __shfl_down(v, o, 64);
}

// One wave per sine mode k: fh[k][i] -> G[k][i] by the factored tridiagonal
// solve (invT = the pivots' reciprocals, cT = the upper factors, ra = the
// radial lower coefficients), lane l holding rows l P .. l P + P - 1
// (P <= PM).  Every load comes first, then the scans.
constexpr int kTriMaxP = 16;  // rows per lane: nr + 1 <= 1024

template <int PM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2)))
k_tri_scan(const double* __restrict__ fh, const double* __restrict__ invT,
           const double* __restrict__ cT, const double* __restrict__ ra, int nr, int nz,
           double* __restrict__ G) {
  const int W = nr + 1, M = nz - 1;
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= M) return;  // whole wave
  const int P = (W + 63) / 64;
  const size_t base = (size_t)k * W;
  double fv[PM], iv[PM], rv[PM], cv[PM];
#pragma unroll
  for (int p = 0; p < PM; ++p) {
    const int i = lane * P + p;
    const int ic = (p < P && i < W) ? i : 0;  // clamped, unconditional loads
    fv[p] = fh[base + ic];
    iv[p] = invT[base + ic];
    rv[p] = ra[ic];
    cv[p] = cT[base + ic];
  }
  double y[PM];
  Aff f[PM];
  // forward: dp_i = u_i - w_i dp_{i-1}, u_i = f_i inv_i, w_i = a_i inv_i (w_0 = 0)
  Aff run = {0.0, 1.0};
#pragma unroll
  for (int p = 0; p < PM; ++p) {
    const int i = lane * P + p;
    const bool ok = (p < P) && (i < W);
    const double u = fv[p] * iv[p];
    const double wv = (i == 0) ? 0.0 : rv[p] * iv[p];
    f[p] = ok ? Aff{u, -wv} : Aff{0.0, 1.0};
    run = after(f[p], run);
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const Aff q = {shfl_up_f64(run.al, o), shfl_up_f64(run.be, o)};
    if (lane >= o) run = after(run, q);
  }
  double v = shfl_up_f64(run.al, 1);
  if (lane == 0) v = 0.0;
#pragma unroll
  for (int p = 0; p < PM; ++p) {
    v = f[p].al + f[p].be * v;
    y[p] = v;
  }
  // backward: x_{W-1} = dp_{W-1}, x_i = dp_i - c_i x_{i+1}
  run = {0.0, 1.0};
#pragma unroll
  for (int p = PM - 1; p >= 0; --p) {
    const int i = lane * P + p;
    const bool ok = (p < P) && (i < W);
    const double c = (i == W - 1) ? 0.0 : cv[p];
    f[p] = ok ? Aff{y[p], -c} : Aff{0.0, 1.0};
    run = after(f[p], run);
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const Aff q = {shfl_down_f64(run.al, o), shfl_down_f64(run.be, o)};
    if (lane + o < 64) run = after(run, q);
  }
  v = shfl_down_f64(run.al, 1);
  if (lane == 63) v = 0.0;
#pragma unroll
  for (int p = PM - 1; p >= 0; --p) {
    v = f[p].al + f[p].be * v;
    const int i = lane * P + p;
    if (p < P && i < W) G[base + i] = v;
  }
}

}  // namespace

void poisson_spectral(const Grid& g, FieldWork& fw, hipStream_t s) {
  const int nr = g.nr, nz = g.nz, M = nz - 1, W = nr + 1;
  const dim3 grid((W + 15) / 16, (M + 15) / 16);
  const size_t lds = (size_t)2 * nz * sizeof(double);
  k_dst_mfma<true><<<grid, 256, lds, s>>>(fw.Q, fw.coef, nullptr, fw.T, nr, nz, g.V, nullptr,
                                           fw.fh);
  const int P = (W + 63) / 64;
  if (P <= 4) k_tri_scan<4><<<(M + 3) / 4, 256, 0, s>>>(fw.fh, fw.tinv, fw.tcp, fw.ra, nr, nz, fw.g);
  else if (P <= 8) k_tri_scan<8><<<(M + 3) / 4, 256, 0, s>>>(fw.fh, fw.tinv, fw.tcp, fw.ra, nr, nz, fw.g);
  else k_tri_scan<kTriMaxP><<<(M + 3) / 4, 256, 0, s>>>(fw.fh, fw.tinv, fw.tcp, fw.ra, nr, nz, fw.g);
  k_dst_mfma<false><<<grid, 256, lds, s>>>(nullptr, nullptr, fw.g, fw.T, nr, nz, g.V, g.Vdev,
                                            fw.phi);
}

// rows per lane of the scan; the sine table (2 nz doubles) within 64 KiB of LDS
bool spectral_fits(int nr, int nz) {
  return nr + 1 <= 64 * kTriMaxP && nz >= 2 && (size_t)2 * nz * sizeof(double) <= 65536;
}

}  // namespace pd
