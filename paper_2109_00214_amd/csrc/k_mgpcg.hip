// k_mgpcg.hip -- Poisson solve of the precision form: conjugate gradients in
// FP32, preconditioned by one symmetric geometric-multigrid V-cycle, inside
// an FP64 iterative refinement (FP64 residual, FP64 update of phi).
//
// The system is the node equation of the cylindrical Poisson equation
// (paper Eq. 8, lap(phi) = -rho/eps0) multiplied by the node's control volume
// A_i dz (A_i = integral of r dr over [r_{i-1/2}, r_{i+1/2}] clipped to
// [0, R]), which makes it symmetric positive definite:
//   (A phi)_ij = dg_i phi_ij - ew_i phi_{i-1,j} - ee_i phi_{i+1,j}
//                - ez_i (phi_{i,j-1} + phi_{i,j+1}),
//   ew_i = r_{i-1/2} dz/dr, ee_i = r_{i+1/2} dz/dr, ez_i = A_i/dz,
//   dg_i = ew_i + ee_i + 2 ez_i,  b_ij = A_i dz rho_ij / eps0,
// over the interior z rows; the electrode rows (Dirichlet) enter b.  The
// relative residual is ||b - A phi||_2 / ||b||_2 with the electrode values
// included in b.
//
// V-cycle (levels l = 0..L-1, grid halved in r and z): one red-black
// Gauss-Seidel sweep (red = (i+j) even first) from zero, residual, full
// weighting (the transpose of bilinear prolongation), recursion, bilinear
// correction, one sweep in the reverse colour order.  The coarse operators
// are the same discretisation on the coarse grid; the coarsest grid takes a
// palindromic sequence of sweeps.  Every step is linear and the sequence is
// its own adjoint, so the V-cycle is a symmetric preconditioner.
//   With one sweep from zero, a red value after the pre-sweep is b/dg and a
//   black value depends only on its red neighbours, so only red nodes carry
//   residual; after the correction, the post-sweep's black values depend only
//   on corrected red values and its red values only on the new black ones.
//   Each fine level therefore takes two kernels, each over LDS tiles with a
//   halo: DOWN (pre-sweep, residual and restriction from b alone) and UP
//   (correction and post-sweep); the coarse levels run in one workgroup out
//   of LDS.
//
// Reductions (dot products, norms) write one partial per block; the next
// kernel sums the partials in every block in the same fixed order, so the
// result does not depend on timing and needs no device-wide fence.
#include "pd_internal.h"


namespace pd {

namespace {

constexpr int kB = kMGBlock;
constexpr int kCoarseThreads = 512;
// DOWN tile: 32 x 8 coarse nodes; fine region with a 3-node halo
constexpr int kDI = 32, kDJ = 8, kDW = 2 * kDI + 5, kDH = 2 * kDJ + 5;
// UP tile: 64 x 16 fine nodes with a 2-node halo
constexpr int kUI = 64, kUJ = 16, kUW = kUI + 4, kUH = kUJ + 4;

// ---- reductions ---------------------------------------------------------------
// Sum over the block of v (any blockDim that is a multiple of 64, at most
// 1024); every thread receives the total.
template <typename T>
__device__ T block_total(T v) {
  __shared__ T sh[16];
  __shared__ T res;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    T a = sh[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) a += sh[w];
    res = a;
  }
  __syncthreads();
  return res;
}

// sum of part[0..nb) in a fixed order (same value in every block)
template <typename T>
__device__ T sum_parts(const T* part, int nb) {
  T a = T(0);
  for (int b = threadIdx.x; b < nb; b += blockDim.x) a += part[b];
  return block_total<T>(a);
}

__device__ __forceinline__ bool block0() {
  return blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0;
}

// Iteration gate of the first kernel of CG iteration it (part_rr != NULL):
// the launch stops when the solve has stopped or the previous iteration's
// r.r partials meet the tolerance.  The loads are issued at kernel entry
// together with the kernel's own data; the decision is block-uniform.
struct Gate {
  const float* part_rr;  // NULL: no gate (not the first kernel of an iteration)
  int nb, it;
};

__device__ __forceinline__ float gate_partial(const Gate& g) {
  float a = 0.f;
  if (g.part_rr && g.it > 0)
    for (int b = threadIdx.x; b < g.nb; b += blockDim.x) a += g.part_rr[b];
  return a;
}

// after a barrier that published done (read by thread 0): whether to run
__device__ bool gate_decide(MGScal* sc, const Gate& g, int done, float part) {
  if (done) return false;
  if (g.part_rr) {
    if (g.it > 0) {
      const float rr = block_total<float>(part);
      if (!(rr > sc->tol2)) {
        if (block0()) sc->done = 1;
        return false;
      }
    }
    if (block0()) {
      sc->iters += 1;
      sc->it_last = g.it + 1;
    }
  }
  return true;
}

// bilinear prolongation of the coarse correction to fine node (i, j); the
// coarse Dirichlet rows hold zero
__device__ __forceinline__ float prolong(const float* xc, int Wc, int i, int j) {
  const int I = i >> 1, J = j >> 1;
  const float* p = xc + J * Wc + I;
  if (!(i & 1) && !(j & 1)) return p[0];
  if ((i & 1) && !(j & 1)) return 0.5f * (p[0] + p[1]);
  if (!(i & 1)) return 0.5f * (p[0] + p[Wc]);
  return 0.25f * ((p[0] + p[1]) + (p[Wc] + p[Wc + 1]));
}

// coefficients of the tile's radial columns i0 .. i0+n-1 (clamped) into LDS
__device__ __forceinline__ void stage_coef(const MGLevel& L, int i0, int n, float* cw, float* ce,
                                           float* cz, float* cd) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    int i = i0 + t;
    i = i < 0 ? 0 : (i > L.nr ? L.nr : i);
    cw[t] = L.ew[i];
    ce[t] = L.ee[i];
    cz[t] = L.ez[i];
    cd[t] = L.dinv[i];
  }
}

// DOWN: coarse right-hand side = full weighting of the fine residual after
// the pre-sweep from zero.  Red values are b/dg, black values follow from
// their red neighbours, only red nodes keep a residual (so the
// 1/2-weighted edge neighbours of the restriction drop out).
__global__ void __launch_bounds__(kB) k_mg_down(MGLevel F, MGLevel C, MGScal* sc, Gate gate) {
  __shared__ float Bs[kDH][kDW], Xs[kDH][kDW];
  __shared__ float cw[kDW], ce[kDW], cz[kDW], cd[kDW];
  __shared__ int sdone;
  const int W = F.nr + 1;
  const int I0 = blockIdx.x * kDI, J0 = 1 + blockIdx.y * kDJ;
  const int i0 = 2 * I0 - 3, j0 = 2 * J0 - 3;
  if (threadIdx.x == 0) sdone = sc->done;
  const float gp = gate_partial(gate);
  for (int t = threadIdx.x; t < kDH * kDW; t += kB) {
    const int lj = t / kDW, li = t % kDW, i = i0 + li, j = j0 + lj;
    const bool in = i >= 0 && i <= F.nr && j >= 1 && j < F.nz;
    Bs[lj][li] = in ? F.b[j * W + i] : 0.f;
  }
  stage_coef(F, i0, kDW, cw, ce, cz, cd);
  __syncthreads();
  if (!gate_decide(sc, gate, sdone, gp)) return;
  for (int t = threadIdx.x; t < kDH * kDW; t += kB) {
    const int lj = t / kDW, li = t % kDW, i = i0 + li, j = j0 + lj;
    const bool in = i >= 0 && i <= F.nr && j >= 1 && j < F.nz;
    Xs[lj][li] = (in && !((i + j) & 1)) ? Bs[lj][li] * cd[li] : 0.f;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < (kDH - 2) * (kDW - 2); t += kB) {
    const int lj = 1 + t / (kDW - 2), li = 1 + t % (kDW - 2), i = i0 + li, j = j0 + lj;
    if (i >= 0 && i <= F.nr && j >= 1 && j < F.nz && ((i + j) & 1)) {
      float s = Bs[lj][li];
      if (i > 0) s += cw[li] * Xs[lj][li - 1];
      if (i < F.nr) s += ce[li] * Xs[lj][li + 1];
      s += cz[li] * (Xs[lj - 1][li] + Xs[lj + 1][li]);
      Xs[lj][li] = s * cd[li];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < (kDH - 4) * (kDW - 4); t += kB) {
    const int lj = 2 + t / (kDW - 4), li = 2 + t % (kDW - 4), i = i0 + li, j = j0 + lj;
    if (!((i + j) & 1)) {
      float s = 0.f;
      if (i >= 0 && i <= F.nr && j >= 1 && j < F.nz) {
        if (i > 0) s += cw[li] * Xs[lj][li - 1];
        if (i < F.nr) s += ce[li] * Xs[lj][li + 1];
        s += cz[li] * (Xs[lj - 1][li] + Xs[lj + 1][li]);
      }
      Bs[lj][li] = s;
    }
  }
  __syncthreads();
  {
    const int I = I0 + threadIdx.x % kDI, J = J0 + threadIdx.x / kDI;
    if (I <= C.nr && J < C.nz) {
      const int li = 2 * (I - I0) + 3, lj = 2 * (J - J0) + 3;
      const float d = (Bs[lj - 1][li - 1] + Bs[lj - 1][li + 1]) + (Bs[lj + 1][li - 1] + Bs[lj + 1][li + 1]);
      const_cast<float*>(C.b)[J * (C.nr + 1) + I] = Bs[lj][li] + 0.25f * d;
    }
  }
}

// UP: correction and post-sweep.  Red values b/dg + P(coarse x) feed the
// black half-sweep; the red half-sweep then reads the new black values.
__global__ void __launch_bounds__(kB) k_mg_up(MGLevel F, MGLevel C, const MGScal* sc) {
  __shared__ float Bs[kUH][kUW], Xs[kUH][kUW];
  __shared__ float cw[kUW], ce[kUW], cz[kUW], cd[kUW];
  __shared__ int sdone;
  const int W = F.nr + 1, Wc = C.nr + 1;
  const int i0 = blockIdx.x * kUI - 2, j0 = 1 + blockIdx.y * kUJ - 2;
  if (threadIdx.x == 0) sdone = sc->done;
  for (int t = threadIdx.x; t < kUH * kUW; t += kB) {
    const int lj = t / kUW, li = t % kUW, i = i0 + li, j = j0 + lj;
    const bool in = i >= 0 && i <= F.nr && j >= 1 && j < F.nz;
    const float b = in ? F.b[j * W + i] : 0.f;
    Bs[lj][li] = b;
    Xs[lj][li] = (in && !((i + j) & 1)) ? b * F.dinv[i] + prolong(C.x, Wc, i, j) : 0.f;
  }
  stage_coef(F, i0, kUW, cw, ce, cz, cd);
  __syncthreads();
  if (sdone) return;
  for (int t = threadIdx.x; t < (kUH - 2) * (kUW - 2); t += kB) {
    const int lj = 1 + t / (kUW - 2), li = 1 + t % (kUW - 2), i = i0 + li, j = j0 + lj;
    if (i >= 0 && i <= F.nr && j >= 1 && j < F.nz && ((i + j) & 1)) {
      float s = Bs[lj][li];
      if (i > 0) s += cw[li] * Xs[lj][li - 1];
      if (i < F.nr) s += ce[li] * Xs[lj][li + 1];
      s += cz[li] * (Xs[lj - 1][li] + Xs[lj + 1][li]);
      Xs[lj][li] = s * cd[li];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kUI * kUJ; t += kB) {
    const int lj = 2 + t / kUI, li = 2 + t % kUI, i = i0 + li, j = j0 + lj;
    if (i > F.nr || j >= F.nz) continue;
    float x;
    if ((i + j) & 1) {
      x = Xs[lj][li];
    } else {
      float s = Bs[lj][li];
      if (i > 0) s += cw[li] * Xs[lj][li - 1];
      if (i < F.nr) s += ce[li] * Xs[lj][li + 1];
      s += cz[li] * (Xs[lj - 1][li] + Xs[lj + 1][li]);
      x = s * cd[li];
    }
    F.x[j * W + i] = x;
  }
}

// Coarse levels lc..nlev-1 in one workgroup: the same V-cycle with the
// intermediate values and the coefficients held in LDS.  The coarsest
// grid is solved exactly with its inverse (host-computed) when it has at
// most kMGCoarsestDense unknowns, else by palindromic sweeps.
struct CoarseArgs {
  int lc, nlev, sweeps;
  const float* inv;  // [n x n] inverse of the coarsest operator, or NULL
  MGLevel lev[kMGMaxLevels];
};

// one level in LDS: values X, right-hand side B, coefficients by radial node
struct LdsLev {
  int nr, nz;
  float *X, *B, *ew, *ee, *ez, *dinv;
};

__device__ __forceinline__ float relax(const LdsLev& m, int i, int j) {
  const int W = m.nr + 1, q = j * W + i;
  float s = m.B[q];
  if (i > 0) s += m.ew[i] * m.X[q - 1];
  if (i < m.nr) s += m.ee[i] * m.X[q + 1];
  s += m.ez[i] * (m.X[q - W] + m.X[q + W]);
  return s * m.dinv[i];
}

// Work over the nodes of one colour, flattened (hw = nodes of the colour per
// row at most) and four per thread in flight: every load of a pass is
// issued before its stores, which touch only the other colour's inputs.
constexpr int kCU = 4;

// op 0: X = b/dg (pre-sweep red from zero); 1: relax; 2: X += P(coarse X)
template <int OP>
__device__ __forceinline__ void colour_pass(const LdsLev& m, int colour, const LdsLev* c) {
  const int W = m.nr + 1, hw = (W + 1) >> 1, total = hw * (m.nz - 1);
  for (int k0 = threadIdx.x; k0 < total; k0 += kCU * kCoarseThreads) {
    float v[kCU];
    int q[kCU];
#pragma unroll
    for (int u = 0; u < kCU; ++u) {
      const int k = k0 + u * kCoarseThreads;
      const int r = k / hw, j = 1 + r, i = 2 * (k - r * hw) + ((j + colour) & 1);
      q[u] = (k < total && i <= m.nr) ? j * W + i : -1;
      v[u] = 0.f;
      if (q[u] >= 0) {
        if (OP == 0) v[u] = m.B[q[u]] * m.dinv[i];
        if (OP == 1) v[u] = relax(m, i, j);
        if (OP == 2) v[u] = m.X[q[u]] + prolong(c->X, c->nr + 1, i, j);
      }
    }
#pragma unroll
    for (int u = 0; u < kCU; ++u)
      if (q[u] >= 0) m.X[q[u]] = v[u];
  }
  __syncthreads();
}

__device__ __forceinline__ void sweep_colour(const LdsLev& m, int colour) {
  colour_pass<1>(m, colour, nullptr);
}

__device__ __forceinline__ LdsLev lds_level(const CoarseArgs& a, float* lds, int l) {
  size_t o = 0;
  for (int k = a.lc; k < l; ++k)
    o += 2 * (size_t)(a.lev[k].nr + 1) * (a.lev[k].nz + 1) + 4 * (size_t)(a.lev[k].nr + 1);
  const int W = a.lev[l].nr + 1, nn = W * (a.lev[l].nz + 1);
  float* p = lds + o;
  return LdsLev{a.lev[l].nr, a.lev[l].nz, p, p + nn, p + 2 * nn, p + 2 * nn + W,
                p + 2 * nn + 2 * W, p + 2 * nn + 3 * W};
}

__global__ void __launch_bounds__(kCoarseThreads) k_mg_coarse(CoarseArgs a, MGScal* sc, Gate gate) {
  extern __shared__ float lds[];
  __shared__ int sdone;
  if (threadIdx.x == 0) sdone = sc->done;
  const float gp = gate_partial(gate);
  // zero the values, stage the coefficients and the first level's b
  for (int l = a.lc; l < a.nlev; ++l) {
    const LdsLev m = lds_level(a, lds, l);
    const MGLevel& g = a.lev[l];
    const int W = m.nr + 1, nn = W * (m.nz + 1);
    for (int t = threadIdx.x; t < nn; t += blockDim.x) {
      m.X[t] = 0.f;
      m.B[t] = (l == a.lc && t >= W && t < nn - W) ? g.b[t] : 0.f;
    }
    for (int t = threadIdx.x; t < W; t += blockDim.x) {
      m.ew[t] = g.ew[t];
      m.ee[t] = g.ee[t];
      m.ez[t] = g.ez[t];
      m.dinv[t] = g.dinv[t];
    }
    if (l == a.nlev - 1 && a.inv) {
      const int n = W * (m.nz - 1);
      for (int t = threadIdx.x; t < n * n; t += blockDim.x) m.dinv[W + t] = a.inv[t];
    }
  }
  __syncthreads();
  if (!gate_decide(sc, gate, sdone, gp)) return;
  for (int l = a.lc; l < a.nlev - 1; ++l) {
    const LdsLev m = lds_level(a, lds, l), c = lds_level(a, lds, l + 1);
    const int W = m.nr + 1;
    // pre-sweep from zero: red = b / dg, then black
    colour_pass<0>(m, 0, nullptr);
    sweep_colour(m, 1);
    // residual at the red nodes, full weighting into the coarse b
    auto rred = [&](int i, int j) -> float {
      if (i < 0 || i > m.nr || j <= 0 || j >= m.nz) return 0.f;
      const int q = j * W + i;
      float s = 0.f;
      if (i > 0) s += m.ew[i] * m.X[q - 1];
      if (i < m.nr) s += m.ee[i] * m.X[q + 1];
      s += m.ez[i] * (m.X[q - W] + m.X[q + W]);
      return s;
    };
    const int Wc = c.nr + 1, nc = Wc * (c.nz - 1);
    for (int t = threadIdx.x; t < nc; t += kCoarseThreads) {
      const int J = 1 + t / Wc, I = t - (J - 1) * Wc, i = 2 * I, j = 2 * J;
      const float d = (rred(i - 1, j - 1) + rred(i + 1, j - 1)) + (rred(i - 1, j + 1) + rred(i + 1, j + 1));
      c.B[J * Wc + I] = rred(i, j) + 0.25f * d;
    }
    __syncthreads();
  }
  {
    const LdsLev m = lds_level(a, lds, a.nlev - 1);
    if (a.inv) {
      // exact: x = A^-1 b over the interior unknowns (row-major, r fastest);
      // the inverse was staged in LDS after the last level
      const int W = m.nr + 1, n = W * (m.nz - 1);
      const float* inv = m.dinv + W;
      for (int r = threadIdx.x; r < n; r += blockDim.x) {
        float acc = 0.f;
        for (int k = 0; k < n; ++k) acc += inv[r * n + k] * m.B[W + k];
        m.X[W + r] = acc;
      }
      __syncthreads();
    } else {
      // palindromic red-black / black-red sweeps from zero
      for (int s = 0; s < a.sweeps; ++s) {
        sweep_colour(m, 0);
        sweep_colour(m, 1);
      }
      for (int s = 0; s < a.sweeps; ++s) {
        sweep_colour(m, 1);
        sweep_colour(m, 0);
      }
    }
  }
  for (int l = a.nlev - 2; l >= a.lc; --l) {
    const LdsLev m = lds_level(a, lds, l), c = lds_level(a, lds, l + 1);
    // correct the red values (the black ones are overwritten next)
    colour_pass<2>(m, 0, &c);
    sweep_colour(m, 1);
    sweep_colour(m, 0);
  }
  {
    const LdsLev m = lds_level(a, lds, a.lc);
    const int W = m.nr + 1, n = W * (m.nz - 1);
    float* x = a.lev[a.lc].x;
    for (int t = threadIdx.x; t < n; t += kCoarseThreads) x[W + t] = m.X[W + t];
  }
}

// ---- conjugate gradients (level-0 vectors) ---------------------------------
__device__ __forceinline__ float apply_A(const MGLevel& m, const float* v, int i, int j) {
  const int W = m.nr + 1, q = j * W + i;
  float s = (m.ew[i] + m.ee[i] + 2.f * m.ez[i]) * v[q];
  if (i > 0) s -= m.ew[i] * v[q - 1];
  if (i < m.nr) s -= m.ee[i] * v[q + 1];
  s -= m.ez[i] * (v[q - W] + v[q + W]);
  return s;
}

// s = A z and the block partials of r.z, z.s, z.q, p.q (p, q: the previous
// direction and A times it)
__global__ void __launch_bounds__(kB) k_cg_s(MGLevel m, const float* r, float* s, const float* p,
                                             const float* q, const MGScal* sc, float* part4) {
  if (sc->done) return;
  const int W = m.nr + 1, n = W * (m.nz - 1);
  const float* z = m.x;
  float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f;
  for (int t = blockIdx.x * kB + threadIdx.x; t < n; t += gridDim.x * kB) {
    const int i = t % W, j = 1 + t / W, k = W + t;
    const float sz = apply_A(m, z, i, j);
    s[k] = sz;
    const float zk = z[k];
    v0 += r[k] * zk;
    v1 += zk * sz;
    v2 += zk * q[k];
    v3 += p[k] * q[k];
  }
  v0 = block_total<float>(v0);
  v1 = block_total<float>(v1);
  v2 = block_total<float>(v2);
  v3 = block_total<float>(v3);
  if (threadIdx.x == 0) {
    part4[0 * gridDim.x + blockIdx.x] = v0;
    part4[1 * gridDim.x + blockIdx.x] = v1;
    part4[2 * gridDim.x + blockIdx.x] = v2;
    part4[3 * gridDim.x + blockIdx.x] = v3;
  }
}

// beta = r.z / r.z(previous); p = z + beta p, q = s + beta q (= A p), so
// p.Ap = z.s + 2 beta z.q + beta^2 p.q; alpha = r.z / p.Ap;
// x += alpha p, r -= alpha q; block partials of r.r
// (flex: flexible CG with one stored direction for a nonlinear
// preconditioner, beta = -z.q / p.q of the previous direction)
__global__ void __launch_bounds__(kB) k_cg_x(MGLevel m, float* r, const float* s, float* p, float* q,
                                             float* x, MGScal* sc, const float* part4, float* part_rr,
                                             int it, int flex) {
  if (sc->done) return;
  const int nb = gridDim.x;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  for (int b = threadIdx.x; b < nb; b += kB) {
    a0 += part4[b];
    a1 += part4[nb + b];
    a2 += part4[2 * nb + b];
    a3 += part4[3 * nb + b];
  }
  const float prev = sc->rz[(it + 1) & 1];
  const float rz = block_total<float>(a0);
  const float zs = block_total<float>(a1);
  const float zq = block_total<float>(a2);
  const float pq = block_total<float>(a3);
  float beta;
  if (flex) beta = (it == 0 || !(pq > 0.f)) ? 0.f : -zq / pq;
  else beta = (it == 0 || !(prev > 0.f)) ? 0.f : rz / prev;
  const float pap = (zs + 2.f * beta * zq) + (beta * beta) * pq;
  // (a breakdown leaves x and r unchanged; the next gate sees the same r.r)
  const float alpha = (pap > 0.f) ? rz / pap : 0.f;
  if (block0()) sc->rz[it & 1] = rz;
  const int W = m.nr + 1, n = W * (m.nz - 1);
  const float* z = m.x;
  float v = 0.f;
  for (int t = blockIdx.x * kB + threadIdx.x; t < n; t += gridDim.x * kB) {
    const int k = W + t;
    const float pk = z[k] + beta * p[k];
    const float qk = s[k] + beta * q[k];
    p[k] = pk;
    q[k] = qk;
    x[k] += alpha * pk;
    const float rk = r[k] - alpha * qk;
    r[k] = rk;
    v += rk * rk;
  }
  v = block_total<float>(v);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = v;
}

// ---- FP64 refinement -------------------------------------------------------
__device__ __forceinline__ void res64(const MGOp64& o, const double* phi, const int64_t* Q, int i, int j,
                                      double& r, double& bf) {
  const int W = o.nr + 1, q = j * W + i;
  const double b = o.w[i] * ((((double)Q[q] * o.qunit) / o.Vnode[i]) / kEPS0);
  double ax = o.dg[i] * phi[q];
  if (i > 0) ax -= o.ew[i] * phi[q - 1];
  if (i < o.nr) ax -= o.ee[i] * phi[q + 1];
  ax -= o.ez[i] * (phi[q - W] + phi[q + W]);
  r = b - ax;
  bf = b;
  if (j == 1) bf += o.ez[i] * phi[i];
  if (j == o.nz - 1) bf += o.ez[i] * phi[(size_t)o.nz * W + i];
}

// block partials of ||b - A phi||^2 and ||b||^2 (electrode values in b)
__global__ void __launch_bounds__(kB) k_res64(MGOp64 o, const double* phi, const int64_t* Q,
                                              double* part64) {
  const int W = o.nr + 1, n = W * (o.nz - 1);
  double v0 = 0.0, v1 = 0.0;
  for (int t = blockIdx.x * kB + threadIdx.x; t < n; t += gridDim.x * kB) {
    double r, bf;
    res64(o, phi, Q, t % W, 1 + t / W, r, bf);
    v0 += r * r;
    v1 += bf * bf;
  }
  v0 = block_total<double>(v0);
  v1 = block_total<double>(v1);
  if (threadIdx.x == 0) {
    part64[blockIdx.x] = v0;
    part64[gridDim.x + blockIdx.x] = v1;
  }
}

// the norms, the relative residual, convergence, and the scale of the next
// FP32 correction solve; stops any CG iterations still queued
__global__ void __launch_bounds__(kB) k_res64_fin(const double* part64, int nb, MGScal* sc) {
  const double rr = sum_parts<double>(part64, nb);
  const double bb = sum_parts<double>(part64 + nb, nb);
  if (threadIdx.x == 0) {
    const double rn = sqrt(rr), bn = sqrt(bb);
    sc->rnorm = rn;
    sc->rel = bn > 0.0 ? rn / bn : rn;
    sc->conv = (rn <= sc->rtol * bn) ? 1 : 0;
    sc->done = 1;
  }
}

// FP32 right-hand side of the correction solve: r = (b - A phi) / ||.||
__global__ void __launch_bounds__(kB) k_cg_init(MGOp64 o, const double* phi, const int64_t* Q,
                                                MGLevel m, float* x, float* p, float* q, MGScal* sc) {
  if (sc->conv) return;
  const int W = o.nr + 1, n = W * (o.nz - 1);
  const double inv = 1.0 / sc->rnorm;
  float* r = const_cast<float*>(m.b);
  for (int t = blockIdx.x * kB + threadIdx.x; t < n; t += gridDim.x * kB) {
    double rr, bf;
    res64(o, phi, Q, t % W, 1 + t / W, rr, bf);
    r[W + t] = (float)(rr * inv);
    x[W + t] = 0.f;
    p[W + t] = 0.f;
    q[W + t] = 0.f;
  }
  if (block0()) {
    sc->done = 0;
    sc->it_last = 0;
  }
}

// phi += ||r|| x on the interior rows
__global__ void __launch_bounds__(kB) k_phi_update(int nr, int nz, const float* x, double* phi,
                                                   MGScal* sc) {
  if (sc->conv) return;
  const int W = nr + 1, n = W * (nz - 1);
  const double s = sc->rnorm;
  for (int t = blockIdx.x * kB + threadIdx.x; t < n; t += gridDim.x * kB)
    phi[W + t] += (double)x[W + t] * s;
  if (block0()) sc->outer += 1;
}

int grid_for(int n) {
  int g = (n + kB - 1) / kB;
  return g < 1 ? 1 : (g > kMGParts ? kMGParts : g);
}

}  // namespace

size_t mg_coarse_lds_bytes(const MGWork& w) {
  size_t o = 0;
  for (int l = w.lc; l < w.nlev; ++l)
    o += 2 * (size_t)(w.lev[l].nr + 1) * (w.lev[l].nz + 1) + 4 * (size_t)(w.lev[l].nr + 1);
  if (w.coarsest_inv) {
    const MGLevel& m = w.lev[w.nlev - 1];
    const size_t n = (size_t)(m.nr + 1) * (m.nz - 1);
    o += n * n;  // the inverse, after the last level's coefficients
  }
  return o * sizeof(float);
}

void mg_configure(MGWork& w) {
  (void)hipFuncSetAttribute((const void*)k_mg_coarse, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)mg_coarse_lds_bytes(w));
}

static void vcycle(MGWork& w, const Gate& first, hipStream_t s) {
  const Gate none{nullptr, 0, 0};
  for (int l = 0; l < w.lc; ++l) {
    const MGLevel& c = w.lev[l + 1];
    dim3 grid((c.nr + 1 + kDI - 1) / kDI, (c.nz - 1 + kDJ - 1) / kDJ);
    k_mg_down<<<grid, kB, 0, s>>>(w.lev[l], c, w.sc, l == 0 ? first : none);
  }
  CoarseArgs a{};
  a.lc = w.lc;
  a.nlev = w.nlev;
  a.sweeps = w.coarse_sweeps;
  a.inv = w.coarsest_inv;
  for (int l = 0; l < w.nlev; ++l) a.lev[l] = w.lev[l];
  k_mg_coarse<<<1, kCoarseThreads, mg_coarse_lds_bytes(w), s>>>(a, w.sc, w.lc == 0 ? first : none);
  for (int l = w.lc - 1; l >= 0; --l) {
    const MGLevel& f = w.lev[l];
    dim3 grid((f.nr + 1 + kUI - 1) / kUI, (f.nz - 1 + kUJ - 1) / kUJ);
    k_mg_up<<<grid, kB, 0, s>>>(f, w.lev[l + 1], w.sc);
  }
}

void mg_residual(const MGWork& w, const double* phi, const int64_t* Q, hipStream_t s) {
  const int g = grid_for((w.op.nr + 1) * (w.op.nz - 1));
  k_res64<<<g, kB, 0, s>>>(w.op, phi, Q, w.part64);
  k_res64_fin<<<1, kB, 0, s>>>(w.part64, g, w.sc);
}

void mg_outer(MGWork& w, double* phi, const int64_t* Q, int inner, hipStream_t s) {
  const MGLevel& m = w.lev[0];
  const int n = (m.nr + 1) * (m.nz - 1), g = grid_for(n);
  k_cg_init<<<g, kB, 0, s>>>(w.op, phi, Q, m, w.xc, w.p, w.q, w.sc);
  float* part4 = w.part;
  float* part_rr = w.part + 4 * kMGParts;
  for (int it = 0; it < inner; ++it) {
    vcycle(w, Gate{part_rr, g, it}, s);
    k_cg_s<<<g, kB, 0, s>>>(m, m.b, w.s, w.p, w.q, w.sc, part4);
    k_cg_x<<<g, kB, 0, s>>>(m, const_cast<float*>(m.b), w.s, w.p, w.q, w.xc, w.sc, part4, part_rr, it,
                            0);
  }
  k_phi_update<<<g, kB, 0, s>>>(m.nr, m.nz, w.xc, phi, w.sc);
  mg_residual(w, phi, Q, s);
}

void mg_outer_learned(MGWork& w, Unet* u, double* phi, const int64_t* Q, int inner, hipStream_t s) {
  const MGLevel& m = w.lev[0];
  const int n = (m.nr + 1) * (m.nz - 1), g = grid_for(n);
  k_cg_init<<<g, kB, 0, s>>>(w.op, phi, Q, m, w.xc, w.p, w.q, w.sc);
  float* part4 = w.part;
  float* part_rr = w.part + 4 * kMGParts;
  for (int it = 0; it < inner; ++it) {
    // the network gives the first direction (its input is then the
    // right-hand side it was trained on: charge, or the change of charge
    // since the last solve); the V-cycle preconditions the rest, and the
    // flexible recurrence keeps each direction A-orthogonal to the last
    if (it == 0) unet_apply(u, m, w.sc, part_rr, g, it, s);
    else vcycle(w, Gate{part_rr, g, it}, s);
    k_cg_s<<<g, kB, 0, s>>>(m, m.b, w.s, w.p, w.q, w.sc, part4);
    k_cg_x<<<g, kB, 0, s>>>(m, const_cast<float*>(m.b), w.s, w.p, w.q, w.xc, w.sc, part4, part_rr, it,
                            1);
  }
  k_phi_update<<<g, kB, 0, s>>>(m.nr, m.nz, w.xc, phi, w.sc);
  mg_residual(w, phi, Q, s);
}

}  // namespace pd
