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
//   Each fine level therefore takes two kernels: DOWN (pre-sweep, residual
//   and restriction, evaluated on the fly from b) and UP (correction and
//   post-sweep); the coarse levels run in one workgroup out of LDS.
#include "pd_internal.h"

namespace pd {

namespace {

constexpr int kB = kMGBlock;

struct Lev {
  int nr, nz;
  float* x;
  const float* b;
  const float *ew, *ee, *ez, *dinv;
};

inline Lev lev_of(const MGLevel& m) { return Lev{m.nr, m.nz, m.x, m.b, m.ew, m.ee, m.ez, m.dinv}; }

// ---- block reductions and the last-block pattern ---------------------------
template <typename T, int NV>
__device__ void block_sum(T (&v)[NV]) {
  __shared__ T sh[NV][kB / 64];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    T x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      T a = sh[k][0];
      for (int w = 1; w < kB / 64; ++w) a += sh[k][w];
      v[k] = a;
    }
  }
}

// Publishes the block's sums; in the last block to finish returns true with
// the grid totals in tot (thread 0), summed in a fixed order.
template <typename T, int NV>
__device__ bool grid_sum(T (&v)[NV], T* part, unsigned* ticket, T (&tot)[NV]) {
  __shared__ bool last;
  block_sum<T, NV>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) part[(size_t)k * gridDim.x + blockIdx.x] = v[k];
    __threadfence();
    last = atomicAdd(ticket, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  T a[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) a[k] = T(0);
  for (int b = threadIdx.x; b < (int)gridDim.x; b += kB)
#pragma unroll
    for (int k = 0; k < NV; ++k) a[k] += __builtin_nontemporal_load(&part[(size_t)k * gridDim.x + b]);
  block_sum<T, NV>(a);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) tot[k] = a[k];
    *ticket = 0u;
  }
  return true;
}

// ---- level operators --------------------------------------------------------
// red value after the pre-sweep from zero (b / dg); zero off the grid and on
// the Dirichlet rows
__device__ __forceinline__ float xr_pre(const Lev& L, int i, int j) {
  if (i < 0 || i > L.nr || j <= 0 || j >= L.nz) return 0.f;
  return L.b[j * (L.nr + 1) + i] * L.dinv[i];
}
// black value after the pre-sweep
__device__ __forceinline__ float xb_pre(const Lev& L, int i, int j) {
  if (j <= 0 || j >= L.nz) return 0.f;
  float s = L.b[j * (L.nr + 1) + i];
  if (i > 0) s += L.ew[i] * xr_pre(L, i - 1, j);
  if (i < L.nr) s += L.ee[i] * xr_pre(L, i + 1, j);
  s += L.ez[i] * (xr_pre(L, i, j - 1) + xr_pre(L, i, j + 1));
  return s * L.dinv[i];
}
// residual at a red node after the pre-sweep (b - dg b/dg = 0 exactly in
// real arithmetic, so only the black neighbours remain)
__device__ __forceinline__ float res_red(const Lev& L, int i, int j) {
  if (i < 0 || i > L.nr || j <= 0 || j >= L.nz) return 0.f;
  float s = 0.f;
  if (i > 0) s += L.ew[i] * xb_pre(L, i - 1, j);
  if (i < L.nr) s += L.ee[i] * xb_pre(L, i + 1, j);
  s += L.ez[i] * (xb_pre(L, i, j - 1) + xb_pre(L, i, j + 1));
  return s;
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
// corrected red value entering the post-sweep
__device__ __forceinline__ float xr_cor(const Lev& L, const Lev& C, int i, int j) {
  if (i < 0 || i > L.nr || j <= 0 || j >= L.nz) return 0.f;
  return L.b[j * (L.nr + 1) + i] * L.dinv[i] + prolong(C.x, C.nr + 1, i, j);
}
// black value after the post-sweep's black half
__device__ __forceinline__ float xb_post(const Lev& L, const Lev& C, int i, int j) {
  if (j <= 0 || j >= L.nz) return 0.f;
  float s = L.b[j * (L.nr + 1) + i];
  if (i > 0) s += L.ew[i] * xr_cor(L, C, i - 1, j);
  if (i < L.nr) s += L.ee[i] * xr_cor(L, C, i + 1, j);
  s += L.ez[i] * (xr_cor(L, C, i, j - 1) + xr_cor(L, C, i, j + 1));
  return s * L.dinv[i];
}

// DOWN: coarse right-hand side = full weighting of the fine residual after
// the pre-sweep (black residuals vanish, so the 1/2-weighted edge
// neighbours drop out).
__global__ void __launch_bounds__(kB) k_mg_down(Lev F, Lev C, const MGScal* sc) {
  if (sc->done) return;
  const int Wc = C.nr + 1, n = Wc * (C.nz - 1);
  float* bc = const_cast<float*>(C.b);
  for (int t = blockIdx.x * kB + threadIdx.x; t < n; t += gridDim.x * kB) {
    const int I = t % Wc, J = 1 + t / Wc, i = 2 * I, j = 2 * J;
    const float d = (res_red(F, i - 1, j - 1) + res_red(F, i + 1, j - 1)) +
                    (res_red(F, i - 1, j + 1) + res_red(F, i + 1, j + 1));
    bc[J * Wc + I] = res_red(F, i, j) + 0.25f * d;
  }
}

// UP: correction and post-sweep; black nodes first half, red nodes second
// half (their black neighbours recomputed in registers).
__global__ void __launch_bounds__(kB) k_mg_up(Lev F, Lev C, const MGScal* sc) {
  if (sc->done) return;
  const int W = F.nr + 1, n = W * (F.nz - 1);
  for (int t = blockIdx.x * kB + threadIdx.x; t < n; t += gridDim.x * kB) {
    const int i = t % W, j = 1 + t / W;
    float x;
    if ((i + j) & 1) {
      x = xb_post(F, C, i, j);
    } else {
      float s = F.b[j * W + i];
      if (i > 0) s += F.ew[i] * xb_post(F, C, i - 1, j);
      if (i < F.nr) s += F.ee[i] * xb_post(F, C, i + 1, j);
      s += F.ez[i] * (xb_post(F, C, i, j - 1) + xb_post(F, C, i, j + 1));
      x = s * F.dinv[i];
    }
    F.x[j * W + i] = x;
  }
}

// Coarse levels lc..nlev-1 in one workgroup: the same V-cycle with the
// intermediate values held in LDS.
struct CoarseArgs {
  int lc, nlev, sweeps;
  MGLevel lev[kMGMaxLevels];
};

__device__ __forceinline__ void sweep_colour(float* X, const float* B, const MGLevel& m, int colour) {
  const int W = m.nr + 1, n = W * (m.nz - 1);
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const int i = t % W, j = 1 + t / W;
    if (((i + j) & 1) != colour) continue;
    const int q = j * W + i;
    float s = B[q];
    if (i > 0) s += m.ew[i] * X[q - 1];
    if (i < m.nr) s += m.ee[i] * X[q + 1];
    s += m.ez[i] * (X[q - W] + X[q + W]);
    X[q] = s * m.dinv[i];
  }
  __syncthreads();
}

__global__ void __launch_bounds__(1024) k_mg_coarse(CoarseArgs a, const MGScal* sc) {
  if (sc->done) return;
  extern __shared__ float lds[];
  __shared__ float* X[kMGMaxLevels];
  __shared__ float* B[kMGMaxLevels];
  size_t total = 0;
  for (int l = a.lc; l < a.nlev; ++l) {
    const int nn = (a.lev[l].nr + 1) * (a.lev[l].nz + 1);
    if (threadIdx.x == 0) {
      X[l] = lds + total;
      B[l] = lds + total + nn;
    }
    total += 2 * (size_t)nn;
  }
  for (size_t t = threadIdx.x; t < total; t += blockDim.x) lds[t] = 0.f;
  __syncthreads();
  {
    const MGLevel& m = a.lev[a.lc];
    const int W = m.nr + 1, n = W * (m.nz - 1);
    for (int t = threadIdx.x; t < n; t += blockDim.x) B[a.lc][W + t] = m.b[W + t];
  }
  __syncthreads();
  for (int l = a.lc; l < a.nlev - 1; ++l) {
    const MGLevel& m = a.lev[l];
    const MGLevel& c = a.lev[l + 1];
    const int W = m.nr + 1, n = W * (m.nz - 1);
    // pre-sweep from zero: red = b / dg, then black
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      const int i = t % W, j = 1 + t / W;
      if (!((i + j) & 1)) X[l][W + t] = B[l][W + t] * m.dinv[i];
    }
    __syncthreads();
    sweep_colour(X[l], B[l], m, 1);
    // residual at the red nodes, full weighting into the coarse b
    const int Wc = c.nr + 1, nc = Wc * (c.nz - 1);
    auto rred = [&](int i, int j) -> float {
      if (i < 0 || i > m.nr || j <= 0 || j >= m.nz) return 0.f;
      const int q = j * W + i;
      float s = 0.f;
      if (i > 0) s += m.ew[i] * X[l][q - 1];
      if (i < m.nr) s += m.ee[i] * X[l][q + 1];
      s += m.ez[i] * (X[l][q - W] + X[l][q + W]);
      return s;
    };
    for (int t = threadIdx.x; t < nc; t += blockDim.x) {
      const int I = t % Wc, J = 1 + t / Wc, i = 2 * I, j = 2 * J;
      const float d = (rred(i - 1, j - 1) + rred(i + 1, j - 1)) + (rred(i - 1, j + 1) + rred(i + 1, j + 1));
      B[l + 1][J * Wc + I] = rred(i, j) + 0.25f * d;
    }
    __syncthreads();
  }
  {
    // coarsest grid: palindromic red-black / black-red sweeps from zero
    const int l = a.nlev - 1;
    for (int s = 0; s < a.sweeps; ++s) {
      sweep_colour(X[l], B[l], a.lev[l], 0);
      sweep_colour(X[l], B[l], a.lev[l], 1);
    }
    for (int s = 0; s < a.sweeps; ++s) {
      sweep_colour(X[l], B[l], a.lev[l], 1);
      sweep_colour(X[l], B[l], a.lev[l], 0);
    }
  }
  for (int l = a.nlev - 2; l >= a.lc; --l) {
    const MGLevel& m = a.lev[l];
    const MGLevel& c = a.lev[l + 1];
    const int W = m.nr + 1, n = W * (m.nz - 1);
    // correct the red values (the black ones are overwritten next)
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      const int i = t % W, j = 1 + t / W;
      if (!((i + j) & 1)) X[l][W + t] += prolong(X[l + 1], c.nr + 1, i, j);
    }
    __syncthreads();
    sweep_colour(X[l], B[l], m, 1);
    sweep_colour(X[l], B[l], m, 0);
  }
  {
    const MGLevel& m = a.lev[a.lc];
    const int W = m.nr + 1, n = W * (m.nz - 1);
    for (int t = threadIdx.x; t < n; t += blockDim.x) m.x[W + t] = X[a.lc][W + t];
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

// s = A z; r.z, z.s, z.q, p.q -> beta, p.Ap of p = z + beta p, alpha
__global__ void __launch_bounds__(kB) k_cg_s(MGLevel m, const float* r, float* s, const float* p,
                                             const float* q, MGScal* sc, float* part) {
  if (sc->done) return;
  const int W = m.nr + 1, n = W * (m.nz - 1);
  const float* z = m.x;
  float v[4] = {0.f, 0.f, 0.f, 0.f};
  for (int t = blockIdx.x * kB + threadIdx.x; t < n; t += gridDim.x * kB) {
    const int i = t % W, j = 1 + t / W, k = W + t;
    const float sz = apply_A(m, z, i, j);
    s[k] = sz;
    const float zk = z[k];
    v[0] += r[k] * zk;
    v[1] += zk * sz;
    v[2] += zk * q[k];
    v[3] += p[k] * q[k];
  }
  float tot[4];
  if (grid_sum<float, 4>(v, part, &sc->ticket[0], tot) && threadIdx.x == 0) {
    const float rz = tot[0];
    const float beta = (sc->it == 0 || !(sc->rz_old > 0.f)) ? 0.f : rz / sc->rz_old;
    const float pq = (tot[1] + 2.f * beta * tot[2]) + (beta * beta) * tot[3];
    sc->beta = beta;
    sc->alpha = (pq > 0.f) ? rz / pq : 0.f;
    sc->rz_old = rz;
  }
}

// p = z + beta p, q = s + beta q, x += alpha p, r -= alpha q; r.r -> stop test
__global__ void __launch_bounds__(kB) k_cg_x(MGLevel m, float* r, const float* s, float* p,
                                             float* q, float* x, MGScal* sc, float* part) {
  if (sc->done) return;
  const int W = m.nr + 1, n = W * (m.nz - 1);
  const float alpha = sc->alpha, beta = sc->beta;
  const float* z = m.x;
  float v[1] = {0.f};
  for (int t = blockIdx.x * kB + threadIdx.x; t < n; t += gridDim.x * kB) {
    const int k = W + t;
    const float pk = z[k] + beta * p[k];
    const float qk = s[k] + beta * q[k];
    p[k] = pk;
    q[k] = qk;
    x[k] += alpha * pk;
    const float rk = r[k] - alpha * qk;
    r[k] = rk;
    v[0] += rk * rk;
  }
  float tot[1];
  if (grid_sum<float, 1>(v, part, &sc->ticket[1], tot) && threadIdx.x == 0) {
    sc->it += 1;
    sc->iters += 1;
    if (!(tot[0] > sc->tol2) || sc->it >= sc->inner_max || !(sc->alpha > 0.f)) sc->done = 1;
  }
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

// ||b - A phi||^2 and ||b||^2 (electrode values in b); decides convergence
// and the scale of the next FP32 correction solve
__global__ void __launch_bounds__(kB) k_res64(MGOp64 o, const double* phi, const int64_t* Q, MGScal* sc,
                                              double* part) {
  const int W = o.nr + 1, n = W * (o.nz - 1);
  double v[2] = {0.0, 0.0};
  for (int t = blockIdx.x * kB + threadIdx.x; t < n; t += gridDim.x * kB) {
    double r, bf;
    res64(o, phi, Q, t % W, 1 + t / W, r, bf);
    v[0] += r * r;
    v[1] += bf * bf;
  }
  double tot[2];
  if (grid_sum<double, 2>(v, part, &sc->ticket[2], tot) && threadIdx.x == 0) {
    const double rn = sqrt(tot[0]), bn = sqrt(tot[1]);
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
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->it = 0;
    sc->rz_old = 0.f;
    sc->done = 0;
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
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->outer += 1;
}

int grid_for(int n) {
  int g = (n + kB - 1) / kB;
  return g < 1 ? 1 : (g > kMGParts ? kMGParts : g);
}

}  // namespace

size_t mg_coarse_lds_bytes(const MGWork& w) {
  size_t o = 0;
  for (int l = w.lc; l < w.nlev; ++l) o += 2 * (size_t)(w.lev[l].nr + 1) * (w.lev[l].nz + 1);
  return o * sizeof(float);
}

void mg_configure(MGWork& w) {
  (void)hipFuncSetAttribute((const void*)k_mg_coarse, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)mg_coarse_lds_bytes(w));
}

static void vcycle(MGWork& w, hipStream_t s) {
  for (int l = 0; l < w.lc; ++l) {
    const MGLevel& c = w.lev[l + 1];
    k_mg_down<<<grid_for((c.nr + 1) * (c.nz - 1)), kB, 0, s>>>(lev_of(w.lev[l]), lev_of(c), w.sc);
  }
  CoarseArgs a{};
  a.lc = w.lc;
  a.nlev = w.nlev;
  a.sweeps = w.coarse_sweeps;
  for (int l = 0; l < w.nlev; ++l) a.lev[l] = w.lev[l];
  k_mg_coarse<<<1, 1024, mg_coarse_lds_bytes(w), s>>>(a, w.sc);
  for (int l = w.lc - 1; l >= 0; --l) {
    const MGLevel& f = w.lev[l];
    k_mg_up<<<grid_for((f.nr + 1) * (f.nz - 1)), kB, 0, s>>>(lev_of(f), lev_of(w.lev[l + 1]), w.sc);
  }
}

void mg_residual(const MGWork& w, const double* phi, const int64_t* Q, hipStream_t s) {
  const int n = (w.op.nr + 1) * (w.op.nz - 1);
  k_res64<<<grid_for(n), kB, 0, s>>>(w.op, phi, Q, w.sc, w.part64);
}

void mg_outer(MGWork& w, double* phi, const int64_t* Q, int inner, hipStream_t s) {
  const MGLevel& m = w.lev[0];
  const int n = (m.nr + 1) * (m.nz - 1), g = grid_for(n);
  k_cg_init<<<g, kB, 0, s>>>(w.op, phi, Q, m, w.xc, w.p, w.q, w.sc);
  for (int it = 0; it < inner; ++it) {
    vcycle(w, s);
    k_cg_s<<<g, kB, 0, s>>>(m, m.b, w.s, w.p, w.q, w.sc, w.part);
    k_cg_x<<<g, kB, 0, s>>>(m, const_cast<float*>(m.b), w.s, w.p, w.q, w.xc, w.sc, w.part);
  }
  k_phi_update<<<g, kB, 0, s>>>(m.nr, m.nz, w.xc, phi, w.sc);
  mg_residual(w, phi, Q, s);
}

}  // namespace pd
