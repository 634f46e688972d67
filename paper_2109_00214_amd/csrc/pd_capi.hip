// pd_capi.hip -- host engine and C ABI (include/pd.h) of the gfx950
// PIC-DSMC library.  Owns the device memory of a context, builds the host
// tables of the method (node and cell volumes, the finite-volume radial
// operator, the sine table and the per-mode tridiagonal factors), and
// enqueues the kernels of one step on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <new>
#include <string>
#include <vector>

#include "../../include/pd.h"
#include "pd_internal.h"

using namespace pd;

struct pd_ctx {
  pd_domain dom;
  pd_opts opts;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  bool poisoned = false;
  bool weighted = false;  // the records carry multiplicities (A.mu, B.mu)

  Grid g{};
  SpeciesParams spp{};
  CollideParams cpar{};
  bool species_set = false;
  bool xs_set[kNC] = {};
  double xs_thr[kNC] = {};
  double qunit = 0;
  int key_bits = 0;
  int64_t cap = 0;

  // device memory
  std::vector<void*> allocs;
  Parts A{}, B{};    // FP64 form: the particles (A) and the sort's destination
  PartsF Af{}, Bf{};  // FP32 form
  bool fp32 = false;
  SortWork sw{};
  CollideWork cw{};
  FieldWork fw{};
  DevState* st = nullptr;
  uint32_t* off = nullptr;
  double* d_xs[kNC] = {};
  double* d_edges = nullptr;
  unsigned long long* d_dcount = nullptr;
  unsigned long long* d_dreal = nullptr;  // per-block sums of multiplicities
  double* d_dke = nullptr;
  unsigned long long* d_spec = nullptr;
  unsigned long long* sput = nullptr;  // cathode sputtering: yields per annulus (2^-32 units)
  uint32_t* sput_take = nullptr;

  // injection schedule
  Schedule sched{};
  std::vector<void*> sched_allocs;
  std::vector<std::array<int64_t, kNS>> sched_species;
  int64_t sched_n = 0, host_sched_pos = 0;

  // host-side bookkeeping
  int64_t host_step = 0;
  int64_t injected[kNS] = {};

  // Poisson: FP64 residual operator (every solver) and the multigrid-CG work
  MGWork mg{};
  MGScal* h_sc = nullptr;  // pinned host copy of the solve scalars
  bool mg_on = false;
  bool learned = false;
  bool spectral = false;  // direct solve on the matrix cores
  bool timing_used = false;  // stage timing was on at some point
  int in_ensemble = 0;    // the ensemble's graph holds this context's buffers
  struct pd_unet* net = nullptr;
  int mg_inner = 8, mg_inner_max = 16, mg_outer_max = 8;
  int64_t p_solves = 0, p_fallbacks = 0;
  double p_call_ms = 0.0;  // device time of the solves made by pd_poisson
  int device = -1;         // the HIP device the context was created on

  // timing
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::vector<hipEvent_t>> ev_pending;
  double t_ms[PD_NTIMERS] = {0};
  int64_t t_steps = 0;
};

struct pd_unet {
  pd::Unet* u = nullptr;
  hipStream_t stream = nullptr;
  std::string err;
};

struct pd_ensemble {
  std::vector<pd_ctx*> m;
  hipStream_t s0 = nullptr;           // launch stream of the graph
  std::vector<hipStream_t> ws;        // worker streams of the capture
  std::vector<hipEvent_t> ev;         // K joins, fork, member ordering
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool owns = false;                  // members marked as in this ensemble
  std::string err;
};

// Scratch of pd_poisson_noalloc, the entry point that allocates nothing: the
// direct solve's right-hand side, transformed right-hand side and per-mode
// solutions, 3 (nz-1)(nr+1) words.  Each GPU the library runs on holds one
// copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchWords = (size_t)1 << 19;  // 4 MiB
static __device__ __align__(256) double scratch[kScratchWords];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// the scratch address on the current device, looked up once per device
// (at context creation); nullptr if the lookup fails
double* scratch_on_current_device(int* dev_out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  if (dev_out) *dev_out = dev;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

namespace {

thread_local std::string g_create_err;
thread_local std::string g_unet_err;
thread_local std::string g_ens_err;

pd::Unet* unet_of(pd_unet* n) { return n->u; }

pd_status set_err(pd_ctx* c, pd_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return s;
}

#define HIPCHK(ctx, call)                                                                 \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return set_err(ctx, PD_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));           \
  } while (0)

template <class T>
pd_status dalloc(pd_ctx* c, T** p, size_t n) {
  void* q = nullptr;
  size_t bytes = n * sizeof(T);
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return set_err(c, PD_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
  }
  c->allocs.push_back(q);
  *p = (T*)q;
  return PD_OK;
}

template <class T>
pd_status alloc_parts(pd_ctx* c, PartsT<T>& P, int64_t n) {
  pd_status s;
  if ((s = dalloc(c, &P.x, n)) || (s = dalloc(c, &P.v, n)) || (s = dalloc(c, &P.key, n)))
    return s;
  return PD_OK;
}

// the first n records of P on the host, in the device layout
template <class T>
pd_status pull_records(pd_ctx* c, const PartsT<T>& P, size_t n, std::vector<PosT<T>>& x,
                       std::vector<RecT<T>>& v, std::vector<uint32_t>& key) {
  x.resize(n);
  v.resize(n);
  key.resize(n);
  if (n == 0) return PD_OK;
  HIPCHK(c, hipMemcpy(x.data(), P.x, sizeof(PosT<T>) * n, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(v.data(), P.v, sizeof(RecT<T>) * n, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(key.data(), P.key, 4 * n, hipMemcpyDeviceToHost));
  return PD_OK;
}

bool finite_all(int64_t n, const double* a) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

pd_status check_particles(pd_ctx* c, int64_t n, const double* r, const double* z, const double* vr,
                          const double* vt, const double* vz, const uint8_t* sp) {
  if (n > 0 && (!r || !z || !vr || !vt || !vz || !sp))
    return set_err(c, PD_EINVAL, "null particle array");
  if (!finite_all(n, r) || !finite_all(n, z) || !finite_all(n, vr) || !finite_all(n, vt) ||
      !finite_all(n, vz))
    return set_err(c, PD_EINVAL, "non-finite particle value");
  for (int64_t p = 0; p < n; ++p) {
    if (!(r[p] >= 0.0) || !(r[p] < c->dom.R) || !(z[p] >= 0.0) || !(z[p] < c->dom.L))
      return set_err(c, PD_EINVAL, "particle %lld outside the domain", (long long)p);
    if (sp[p] >= kNS) return set_err(c, PD_EINVAL, "particle %lld: species %d", (long long)p, sp[p]);
  }
  return PD_OK;
}

// Host tables of the method.  Every expression is the binary64 value of the
// formula as parenthesised (compiled without contraction).
void build_tables(pd_ctx* c, std::vector<double>& Vnode, std::vector<double>& Vcell,
                  std::vector<double>& ra, std::vector<double>& S, std::vector<double>& tinv,
                  std::vector<double>& tcp, std::vector<double>& edges, std::vector<double>& rcv,
                  std::vector<double>& twinv, std::vector<double>& twcp) {
  const int nr = c->dom.nr, nz = c->dom.nz, M = nz - 1;
  const double R = c->dom.R, dr = c->g.dr, dz = c->g.dz;
  Vnode.assign(nr + 1, 0.0);
  Vcell.assign(nr, 0.0);
  // node volumes of linear weighting in r (the hat function's volume
  // integral) and the cell volumes
  Vnode[0] = ((kPI * (dr * dr)) * dz) / 3.0;
  for (int i = 1; i < nr; ++i) Vnode[i] = (((2.0 * kPI) * ((double)i * dr)) * dr) * dz;
  Vnode[nr] = (kPI * dz) * ((R * dr) - ((dr * dr) / 3.0));
  for (int i = 0; i < nr; ++i) {
    const double a = (double)i * dr, b = (double)(i + 1) * dr;
    Vcell[i] = (kPI * ((b * b) - (a * a))) * dz;
  }
  // radial finite-volume operator: flux r dphi/dr through the faces of
  // [r_{i-1/2}, r_{i+1/2}] clipped to [0, R], none through r = 0 and r = R
  std::vector<double> rb(nr + 1), rc(nr + 1);
  ra.assign(nr + 1, 0.0);
  for (int i = 0; i <= nr; ++i) {
    double area;
    if (i == 0) area = (dr * dr) / 8.0;
    else if (i == nr) area = ((R * dr) / 2.0) - ((dr * dr) / 8.0);
    else area = ((double)i * dr) * dr;
    const double lo = (i == 0) ? 0.0 : ((double)i - 0.5) * dr;
    const double hi = (i == nr) ? 0.0 : ((double)i + 0.5) * dr;
    ra[i] = lo / (dr * area);
    rc[i] = hi / (dr * area);
    rb[i] = -(ra[i] + rc[i]);
  }
  // DST-I entries sin(pi k j / nz): they depend only on m = (k j) mod 2 nz,
  // reduced exactly to [0, nz/2] by the symmetries of sin (sign restored)
  S.assign((size_t)2 * nz, 0.0);
  for (int m0 = 0; m0 < 2 * nz; ++m0) {
    long long m = m0;
    bool neg = false;
    if (m >= nz) {
      m -= nz;
      neg = true;
    }
    if (2 * m > nz) m = nz - m;
    const double v = (m == 0) ? 0.0 : std::sin((kPI * (double)m) / (double)nz);
    S[m0] = neg ? -v : v;
  }
  // per-mode tridiagonal factors of (D_r + mu_k), mu_k the eigenvalue of
  // the 3-point d2/dz2 on sin(pi k j / nz)
  tinv.assign((size_t)(nr + 1) * M, 0.0);  // [mode][i], i fastest
  tcp.assign((size_t)(nr + 1) * M, 0.0);
  for (int k = 1; k <= M; ++k) {
    const double h = std::sin((kPI * (double)k) / (2.0 * (double)nz));
    const double mu = -(4.0 * (h * h)) / (dz * dz);
    double inv = 1.0 / (rb[0] + mu);
    double cp = rc[0] * inv;
    tinv[(size_t)(k - 1) * (nr + 1) + 0] = inv;
    tcp[(size_t)(k - 1) * (nr + 1) + 0] = cp;
    for (int i = 1; i <= nr; ++i) {
      const double den = (rb[i] + mu) - (ra[i] * cp);
      inv = 1.0 / den;
      cp = rc[i] * inv;
      tinv[(size_t)(k - 1) * (nr + 1) + i] = inv;
      tcp[(size_t)(k - 1) * (nr + 1) + i] = cp;
    }
  }
  // the same systems eliminated from both ends (rows 0 .. m-1 from the axis,
  // nr .. m+1 from the wall, m = nr / 2): each row's pivot reciprocal and
  // its factor toward the middle ([mode][i]; row m: the middle pivot's
  // reciprocal and no factor), in the order the direct solve uses them
  const int m = nr / 2;
  twinv.assign((size_t)(nr + 1) * M, 0.0);
  twcp.assign((size_t)(nr + 1) * M, 0.0);
  for (int k = 1; k <= M; ++k) {
    const double h = std::sin((kPI * (double)k) / (2.0 * (double)nz));
    const double mu = -(4.0 * (h * h)) / (dz * dz);
    double* iv = &twinv[(size_t)(k - 1) * (nr + 1)];
    double* cv = &twcp[(size_t)(k - 1) * (nr + 1)];
    for (int i = 0; i < m; ++i) {
      double den = rb[i] + mu;
      if (i > 0) den = den - (ra[i] * cv[i - 1]);
      iv[i] = 1.0 / den;
      cv[i] = rc[i] * iv[i];
    }
    for (int i = nr; i > m; --i) {
      double den = rb[i] + mu;
      if (i < nr) den = den - (rc[i] * cv[i + 1]);
      iv[i] = 1.0 / den;
      cv[i] = ra[i] * iv[i];
    }
    double den = rb[m] + mu;
    if (m > 0) den = den - (ra[m] * cv[m - 1]);
    if (m < nr) den = den - (rc[m] * cv[m + 1]);
    iv[m] = 1.0 / den;
  }
  rcv = rc;
  edges.assign(65, 0.0);
  for (int b = 0; b <= 64; ++b) edges[b] = std::pow(10.0, (3.0 * (double)b) / 64.0);
}

// Coefficients of the volume-weighted symmetric operator on a grid of
// nr x nz cells: ew_i = r_{i-1/2} dz/dr, ee_i = r_{i+1/2} dz/dr,
// ez_i = A_i/dz, w_i = A_i dz, A_i = integral of r dr over the node's radial
// control interval clipped to [0, R].
void weighted_operator(int nr, int nz, double R, double L, std::vector<double>& ew,
                       std::vector<double>& ee, std::vector<double>& ez, std::vector<double>& w) {
  const double dr = R / (double)nr, dz = L / (double)nz;
  ew.assign(nr + 1, 0.0);
  ee.assign(nr + 1, 0.0);
  ez.assign(nr + 1, 0.0);
  w.assign(nr + 1, 0.0);
  for (int i = 0; i <= nr; ++i) {
    double area;
    if (i == 0) area = (dr * dr) / 8.0;
    else if (i == nr) area = ((R * dr) / 2.0) - ((dr * dr) / 8.0);
    else area = ((double)i * dr) * dr;
    const double lo = (i == 0) ? 0.0 : ((double)i - 0.5) * dr;
    const double hi = (i == nr) ? 0.0 : ((double)i + 0.5) * dr;
    ew[i] = (lo * dz) / dr;
    ee[i] = (hi * dz) / dr;
    ez[i] = area / dz;
    w[i] = area * dz;
  }
}

// FP64 residual operator, solve scalars and, for the iterative solver, the
// multigrid hierarchy (levels halve nr and nz while both stay even and >= 4;
// the coarsest levels that fit kMGCoarseLds run in one workgroup).
pd_status build_mg(pd_ctx* c, const double* dVnode) {
  const int nr = c->dom.nr, nz = c->dom.nz;
  MGWork& w = c->mg;
  pd_status s;
  std::vector<double> ew, ee, ez, wt;
  weighted_operator(nr, nz, c->dom.R, c->dom.L, ew, ee, ez, wt);
  std::vector<double> dg(nr + 1);
  for (int i = 0; i <= nr; ++i) dg[i] = (ew[i] + ee[i]) + (2.0 * ez[i]);
  double *d[5];
  const std::vector<double>* h[5] = {&ew, &ee, &ez, &dg, &wt};
  for (int k = 0; k < 5; ++k) {
    if ((s = dalloc(c, &d[k], nr + 1))) return s;
    if (hipMemcpy(d[k], h[k]->data(), 8 * (nr + 1), hipMemcpyHostToDevice) != hipSuccess)
      return set_err(c, PD_EDEVICE, "upload");
  }
  w.op = MGOp64{nr, nz, d[0], d[1], d[2], d[3], d[4], dVnode, c->qunit};
  if ((s = dalloc(c, &w.sc, 1)) || (s = dalloc(c, &w.part, (size_t)kMGParts * 5)) ||
      (s = dalloc(c, &w.part64, (size_t)kMGParts * 2)))
    return s;
  if (hipHostMalloc((void**)&c->h_sc, sizeof(MGScal), 0) != hipSuccess)
    return set_err(c, PD_ENOMEM, "pinned host memory");
  MGScal h0{};
  h0.rtol = c->opts.poisson_rtol > 0 ? c->opts.poisson_rtol : 1e-8;
  h0.tol2 = 1e-10f;  // inner solve: ||r|| / ||r0|| <= 1e-5 (||r0|| = 1)
  h0.done = 1;
  if (hipMemcpy(w.sc, &h0, sizeof h0, hipMemcpyHostToDevice) != hipSuccess)
    return set_err(c, PD_EDEVICE, "upload");
  if (!c->mg_on) return PD_OK;

  int nl = 1;
  while (nl < kMGMaxLevels && ((nr >> (nl - 1)) % 2 == 0) && ((nz >> (nl - 1)) % 2 == 0) &&
         (nr >> (nl - 1)) >= 4 && (nz >> (nl - 1)) >= 4)
    ++nl;
  w.nlev = nl;
  w.coarse_sweeps = 4;
  w.lc = -1;
  for (int l = 0; l < nl && w.lc < 0; ++l) {
    size_t b = 0;
    for (int k = l; k < nl; ++k) b += (size_t)((nr >> k) + 1) * ((nz >> k) + 1);
    if (b <= (size_t)kMGCoarseNodes) w.lc = l;
  }
  if (w.lc < 0)
    return set_err(c, PD_EINVAL, "multigrid: grid %dx%d does not coarsen to %d nodes", nr, nz,
                   kMGCoarseNodes);
  for (int l = 0; l < nl; ++l) {
    const int a = nr >> l, b = nz >> l;
    const size_t nn = (size_t)(a + 1) * (b + 1);
    MGLevel& m = w.lev[l];
    m.nr = a;
    m.nz = b;
    std::vector<double> lew, lee, lez, lw;
    weighted_operator(a, b, c->dom.R, c->dom.L, lew, lee, lez, lw);
    std::vector<float> tab(4 * (size_t)(a + 1));
    for (int i = 0; i <= a; ++i) {
      tab[i] = (float)lew[i];
      tab[(a + 1) + i] = (float)lee[i];
      tab[2 * (a + 1) + i] = (float)lez[i];
      tab[3 * (a + 1) + i] = (float)(1.0 / ((lew[i] + lee[i]) + (2.0 * lez[i])));
    }
    float *dt, *x, *bb;
    if ((s = dalloc(c, &dt, tab.size())) || (s = dalloc(c, &x, nn)) || (s = dalloc(c, &bb, nn)))
      return s;
    if (hipMemcpy(dt, tab.data(), 4 * tab.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(x, 0, 4 * nn) != hipSuccess || hipMemset(bb, 0, 4 * nn) != hipSuccess)
      return set_err(c, PD_EDEVICE, "upload");
    m.x = x;
    m.b = bb;
    m.ew = dt;
    m.ee = dt + (a + 1);
    m.ez = dt + 2 * (a + 1);
    m.dinv = dt + 3 * (a + 1);
  }
  // exact coarsest solve: the inverse of the coarsest operator (FP64
  // Gauss-Jordan with partial pivoting, stored in FP32)
  w.coarsest_inv = nullptr;
  {
    const int a = nr >> (nl - 1), b = nz >> (nl - 1), W = a + 1, n = W * (b - 1);
    if (n <= kMGCoarsestDense) {
      std::vector<double> lew, lee, lez, lw, A((size_t)n * n, 0.0), I((size_t)n * n, 0.0);
      weighted_operator(a, b, c->dom.R, c->dom.L, lew, lee, lez, lw);
      for (int j = 1; j < b; ++j)
        for (int i = 0; i <= a; ++i) {
          const int k = (j - 1) * W + i;
          A[(size_t)k * n + k] = (lew[i] + lee[i]) + (2.0 * lez[i]);
          if (i > 0) A[(size_t)k * n + k - 1] = -lew[i];
          if (i < a) A[(size_t)k * n + k + 1] = -lee[i];
          if (j > 1) A[(size_t)k * n + k - W] = -lez[i];
          if (j < b - 1) A[(size_t)k * n + k + W] = -lez[i];
          I[(size_t)k * n + k] = 1.0;
        }
      for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
          if (std::fabs(A[(size_t)r * n + col]) > std::fabs(A[(size_t)piv * n + col])) piv = r;
        for (int k = 0; k < n; ++k) {
          std::swap(A[(size_t)col * n + k], A[(size_t)piv * n + k]);
          std::swap(I[(size_t)col * n + k], I[(size_t)piv * n + k]);
        }
        const double d = A[(size_t)col * n + col];
        for (int k = 0; k < n; ++k) {
          A[(size_t)col * n + k] /= d;
          I[(size_t)col * n + k] /= d;
        }
        for (int r = 0; r < n; ++r) {
          if (r == col) continue;
          const double f = A[(size_t)r * n + col];
          if (f == 0.0) continue;
          for (int k = 0; k < n; ++k) {
            A[(size_t)r * n + k] -= f * A[(size_t)col * n + k];
            I[(size_t)r * n + k] -= f * I[(size_t)col * n + k];
          }
        }
      }
      std::vector<float> inv((size_t)n * n);
      for (size_t k = 0; k < inv.size(); ++k) inv[k] = (float)I[k];
      float* d;
      if ((s = dalloc(c, &d, inv.size()))) return s;
      if (hipMemcpy(d, inv.data(), 4 * inv.size(), hipMemcpyHostToDevice) != hipSuccess)
        return set_err(c, PD_EDEVICE, "upload");
      w.coarsest_inv = d;
    }
  }
  const size_t n0 = (size_t)(nr + 1) * (nz + 1);
  float** v[4] = {&w.xc, &w.s, &w.p, &w.q};
  for (int k = 0; k < 4; ++k) {
    if ((s = dalloc(c, v[k], n0))) return s;
    if (hipMemset(*v[k], 0, 4 * n0) != hipSuccess) return set_err(c, PD_EDEVICE, "memset");
  }
  mg_configure(w);
  return PD_OK;
}

pd_status read_mg(pd_ctx* c) {
  if (hipMemcpyAsync(c->h_sc, c->mg.sc, sizeof(MGScal), hipMemcpyDeviceToHost, c->stream) !=
          hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    c->poisoned = true;
    return set_err(c, PD_EDEVICE, "Poisson scalars");
  }
  return PD_OK;
}

// The step's Poisson solve: direct, or multigrid CG from the current phi
// with FP64 refinement until the relative residual reaches rtol (the direct
// solve takes over if it does not within mg_outer_max refinements).
pd_status solve_poisson(pd_ctx* c) {
  hipStream_t s = c->stream;
  c->p_solves += 1;
  if (c->spectral) {
    poisson_spectral(c->g, c->fw, s);
    return PD_OK;
  }
  if (!c->mg_on || (c->learned && !c->net)) {
    poisson_direct(c->g, c->fw, s);
    return PD_OK;
  }
  // the first refinement is enqueued without waiting: a warm start that
  // already meets the tolerance turns it into no-ops on the device
  mg_residual(c->mg, c->fw.phi, c->fw.Q, s);
  for (int o = 0;; ++o) {
    if (c->learned) mg_outer_learned(c->mg, unet_of(c->net), c->fw.phi, c->fw.Q, c->mg_inner, s);
    else mg_outer(c->mg, c->fw.phi, c->fw.Q, c->mg_inner, s);
    pd_status st = read_mg(c);
    if (st) return st;
    // CG iterations for the next refinement: one more than the last took
    const int used = c->h_sc->it_last;
    c->mg_inner = std::min(c->mg_inner_max, std::max(2, used + (used >= c->mg_inner ? 2 : 1)));
    if (c->h_sc->conv) break;
    if (o + 1 == c->mg_outer_max) {
      poisson_direct(c->g, c->fw, s);
      c->p_fallbacks += 1;
      break;
    }
  }
  return PD_OK;
}

void derive_pairs(pd_ctx* c) {
  // projectile: electron, Cu+ (CEX) or Cu (NN); target: Cu (EL, SI, DI,
  // CEX, NN), Cu+ (SI2), Cu2+ of any label (SI3: the labels share the Cu2+
  // mass) or Cu3+ (SI4)
  const int tgt[kNC] = {PD_CU, PD_CU, PD_CU, PD_CU1, PD_CU2_STEP, PD_CU3, PD_CU, PD_CU,
                        PD_CU1, PD_E};
  const int prj[kNC] = {PD_E, PD_E, PD_E, PD_E, PD_E, PD_E, PD_CU1, PD_CU, PD_E, PD_E};
  for (int k = 0; k < kNC; ++k) {
    const double m1 = c->spp.m[prj[k]], m2 = c->spp.m[tgt[k]];
    const double mr = (m1 * m2) / (m1 + m2);
    c->cpar.f1[k] = mr / m1;
    c->cpar.f2[k] = mr / m2;
    c->cpar.ck[k] = std::sqrt(mr / (2.0 * kQE));
    // energy lost: the ionization thresholds; the other channels are elastic
    c->cpar.two_dE_mr[k] =
        (k >= PD_SI && k <= PD_SI4) ? (2.0 * (-(c->xs_thr[k] * kQE))) / mr : 0.0;
  }
}

pd_status sync(pd_ctx* c) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    c->poisoned = true;
    return set_err(c, PD_EDEVICE, "stream: %s", hipGetErrorString(e));
  }
  return PD_OK;
}

pd_status read_state(pd_ctx* c, DevState* h) {
  pd_status s = sync(c);
  if (s) return s;
  HIPCHK(c, hipMemcpy(h, c->st, sizeof(DevState), hipMemcpyDeviceToHost));
  if (h->err) {
    c->poisoned = true;
    return set_err(c, PD_ECAPACITY, "particle capacity (%lld) or id space exhausted on the device",
                   (long long)c->cap);
  }
  return PD_OK;
}

hipEvent_t get_event(pd_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void harvest_timing(pd_ctx* c) {
  for (auto& set : c->ev_pending) {
    // a null entry repeats the boundary before it
    for (size_t k = 1; k < set.size(); ++k)
      if (!set[k]) set[k] = set[k - 1];
    for (int k = 0; k < PD_NTIMERS; ++k) {
      float ms = 0.f;
      if (set[k] != set[k + 1] && hipEventElapsedTime(&ms, set[k], set[k + 1]) == hipSuccess)
        c->t_ms[k] += ms;
    }
    c->t_steps += 1;
    for (size_t k = 0; k < set.size(); ++k)
      if (k == 0 || set[k] != set[k - 1]) c->ev_pool.push_back(set[k]);
  }
  c->ev_pending.clear();
}

// host-side bookkeeping of one step (injected counts from the schedule)
void host_after_step(pd_ctx* c) {
  if (c->host_sched_pos < c->sched_n) {
    for (int k = 0; k < kNS; ++k) c->injected[k] += c->sched_species[c->host_sched_pos][k];
    c->host_sched_pos += 1;
  }
  c->host_step += 1;
}

// host arrays -> staging buffers (converted to the record's precision) ->
// appended after the particles held now
template <class T>
pd_status stage_append(pd_ctx* c, const PartsT<T>& A, const PartsT<T>& B, int64_t n,
                              const double* r, const double* z, const double* vr,
                              const double* vt, const double* vz, const uint8_t* sp,
                              const uint16_t* mu) {
  std::vector<PosT<T>> x((size_t)n);
  std::vector<RecT<T>> v((size_t)n);
  for (int64_t p = 0; p < n; ++p) {
    x[p] = PosT<T>{(T)r[p], (T)z[p]};
    v[p] = RecT<T>{(T)vr[p], (T)vt[p], (T)vz[p], 0u, (uint32_t)sp[p]};  // ids set on the device
  }
  HIPCHK(c, hipMemcpy(B.x, x.data(), sizeof(PosT<T>) * n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(B.v, v.data(), sizeof(RecT<T>) * n, hipMemcpyHostToDevice));
  if (B.mu) {
    std::vector<uint16_t> m((size_t)n, (uint16_t)1);
    if (mu) std::memcpy(m.data(), mu, sizeof(uint16_t) * (size_t)n);
    HIPCHK(c, hipMemcpy(B.mu, m.data(), sizeof(uint16_t) * n, hipMemcpyHostToDevice));
  }
  append(A, c->st, c->g, B, (uint32_t)n, c->stream);
  HIPCHK(c, hipGetLastError());
  return PD_OK;
}

// one step on the context's stream: sort -> offsets -> collide (+ deposit)
// -> Poisson -> field (+ inject) -> push (mark() records the stage boundaries; the
// records stay in A, in the previous order, until the push writes them
// sorted into B, which then becomes A)
template <class T, class Mark>
pd_status enqueue_step(pd_ctx* c, PartsT<T>& A, PartsT<T>& B, int64_t nn, Mark& mark) {
  hipStream_t s = c->stream;
  mark();
  sort_keys(A.key, c->key_bits, c->sw, c->st, c->off, c->g.sentinel, s);
  mark();
  mark(true);  // no separate record permutation: the push moves the records
  place_and_offsets(A.key, c->sw, c->st, c->off, c->g.sentinel + 1, c->fw.Q, (uint32_t)nn, s);
  const Flow<T> f{A, B, c->sw.perm, c->sw.skey};
  mark();
  // The deposit reads only what the collisions leave alone (positions, the
  // sort's keys and permutation), and the collisions add their charge
  // changes with integer atomics: with collisions, the deposit runs as extra
  // blocks of the collision decisions' launch (which is bound by latency,
  // not by bandwidth), otherwise on its own.
  int64_t* Qd = c->opts.deposit_off ? nullptr : c->fw.Q;
  if (!c->opts.collisions_off)
    collide(f, c->off, c->st, c->g, c->cpar, c->spp, Qd, c->cw, c->sw.bsum, c->cap, s);
  mark();
  if (c->opts.collisions_off && !c->opts.deposit_off) {
    deposit(f, c->off, c->g, c->spp, c->fw.Q, c->cap, s);
    mark();
  } else {
    mark(true);  // inside the collisions' stage
  }
  pd_status ps = solve_poisson(c);
  if (ps) return ps;
  mark();
  field_and_inject(c->g, c->fw, B, c->st, c->spp, c->sched, c->cap, s);
  mark();
  push(f, c->st, c->g, c->spp, c->fw, c->sched, c->cap, s);
  mark();
  std::swap(A, B);
  mark(true);  // the injection ran with the field
  return PD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

pd_status pd_create(const pd_domain* dom, const pd_opts* opts, pd_ctx** out) {
  if (!dom || !opts || !out) return PD_EINVAL;
  *out = nullptr;
  pd_ctx* c = new (std::nothrow) pd_ctx();
  if (!c) return PD_ENOMEM;
  c->dom = *dom;
  c->opts = *opts;
  auto fail = [&](pd_status s) {
    g_create_err = c->err;
    pd_destroy(c);
    return s;
  };
  if (dom->nr < 2 || dom->nz < 2 || dom->nz > 8192 ||
      (opts->poisson != PD_POISSON_SPECTRAL && !direct_fits(dom->nr, dom->nz)) ||
      (int64_t)dom->nr * dom->nz * kNK >= (1LL << 31) || !(dom->R > 0) || !(dom->L > 0) ||
      !(dom->dt > 0) || !(dom->weight > 0) || !std::isfinite(dom->V_cathode) ||
      !std::isfinite(dom->R) || !std::isfinite(dom->L) || dom->capacity < 1 ||
      dom->capacity > (int64_t)kScanChunk * kScanMaxBlocks)
    return fail(set_err(c, PD_EINVAL, "invalid domain"));
  if ((opts->precision != PD_FP64_DET && opts->precision != PD_FP32_MIXED) ||
      (opts->poisson != PD_POISSON_DIRECT64 && opts->poisson != PD_POISSON_MGPCG &&
       opts->poisson != PD_POISSON_LEARNED && opts->poisson != PD_POISSON_SPECTRAL) ||
      (opts->poisson == PD_POISSON_SPECTRAL && !spectral_fits(dom->nr, dom->nz)) ||
      !(opts->poisson_rtol >= 0.0) || !std::isfinite(opts->poisson_rtol))
    return fail(set_err(c, PD_EINVAL, "unsupported precision or Poisson mode"));
  c->spectral = opts->poisson == PD_POISSON_SPECTRAL;
  c->timing_used = opts->timing != 0;
  c->mg_on = opts->poisson != PD_POISSON_DIRECT64 && !c->spectral;
  c->learned = opts->poisson == PD_POISSON_LEARNED;
  c->fp32 = opts->precision == PD_FP32_MIXED;
  if (!scratch_on_current_device(&c->device))
    return fail(set_err(c, PD_EDEVICE, "scratch address of the current device"));
  if (opts->stream) {
    c->stream = (hipStream_t)opts->stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) return fail(set_err(c, PD_EDEVICE, "stream"));
    c->own_stream = true;
  }
  const int nr = dom->nr, nz = dom->nz;
  c->cap = dom->capacity;
  c->g.nr = nr;
  c->g.nz = nz;
  c->g.C = (uint32_t)(nr * nz);
  c->g.sentinel = (uint32_t)kNK * c->g.C;
  c->g.dr = dom->R / (double)nr;
  c->g.dz = dom->L / (double)nz;
  c->g.R = dom->R;
  c->g.L = dom->L;
  c->g.V = dom->V_cathode;
  c->g.dt = dom->dt;
  c->g.W = dom->weight;
  c->g.seed_lo = (uint32_t)dom->seed;
  c->g.seed_hi = (uint32_t)(dom->seed >> 32);
  c->g.heavy_every = 1;
  c->g.dt_heavy = dom->dt;
  c->cpar.dt_heavy = dom->dt;
  c->sw.heavy_every = 1;
  c->qunit = (kQE * dom->weight) * 0x1p-40;
  {
    int b = 0;
    while ((1u << b) <= c->g.sentinel) ++b;
    c->key_bits = b;
  }
  const int Zd[kNS] = {-1, 0, 1, 2, 2, 2, 3, 4};
  for (int k = 0; k < kNS; ++k) c->spp.Z[k] = Zd[k];
  for (int k = 0; k < kNS; ++k) c->spp.Zk[key_class((uint32_t)k)] = Zd[k];
  c->cpar.W = dom->weight;
  c->cpar.dt = dom->dt;
  c->cpar.seed_lo = (uint32_t)dom->seed;
  c->cpar.seed_hi = (uint32_t)(dom->seed >> 32);
  c->cpar.enable_di = opts->enable_di ? 1 : 0;

  const int64_t cap = c->cap;
  const int64_t nn = (int64_t)(nr + 1) * (nz + 1);
  const int M = nz - 1;
  const int64_t tiles = (cap + kSortBlock * kMoverItems - 1) / (kSortBlock * kMoverItems);
  pd_status s;
  if ((c->fp32 ? ((s = alloc_parts(c, c->Af, cap)) || (s = alloc_parts(c, c->Bf, cap)) ||
                  (s = dalloc(c, &c->fw.Erf, nn)) || (s = dalloc(c, &c->fw.Ezf, nn)))
               : ((s = alloc_parts(c, c->A, cap)) || (s = alloc_parts(c, c->B, cap)))) ||
      (s = dalloc(c, &c->sw.k0, cap)) || (s = dalloc(c, &c->sw.k1, cap)) ||
      (s = dalloc(c, &c->sw.v0, cap)) || (s = dalloc(c, &c->sw.v1, cap)) ||
      (s = dalloc(c, &c->sw.hist, (size_t)kRadix * (tiles < 1 ? 1 : tiles))) ||
      (s = dalloc(c, &c->sw.bsum, std::max<int64_t>(kScanMaxBlocks, cap / 256 + 1))) ||
      (s = dalloc(c, &c->sw.skey, cap)) || (s = dalloc(c, &c->sw.mbits, cap / 32 + 66)) ||
      (s = dalloc(c, &c->sw.mword, cap / 32 + 66)) ||
      (s = dalloc(c, &c->sw.n_mov, 2)) || (s = dalloc(c, &c->sw.perm, cap)) ||
      (s = dalloc(c, &c->sw.ins, cap)) ||
      (s = dalloc(c, &c->cw.choice, cap)) || (s = dalloc(c, &c->cw.target, cap)) ||
      (s = dalloc(c, &c->cw.claim, cap)) || (s = dalloc(c, &c->cw.csum, (cap / 256 + 1) / 32 + 2)) ||
      (s = dalloc(c, &c->fw.Q, nn)) || (s = dalloc(c, &c->fw.phi, nn)) ||
      (s = dalloc(c, &c->fw.Er, nn)) || (s = dalloc(c, &c->fw.Ez, nn)) ||
      (s = dalloc(c, &c->fw.fh, (size_t)M * (nr + 1))) ||
      (s = dalloc(c, &c->fw.f, (size_t)M * (nr + 1))) ||
      (s = dalloc(c, &c->fw.g, (size_t)M * (nr + 1))) || (s = dalloc(c, &c->st, 1)) ||
      (s = dalloc(c, &c->off, (size_t)c->g.sentinel + 1)) || (s = dalloc(c, &c->d_edges, 65)) ||
      (s = dalloc(c, &c->d_dcount, (size_t)kDiagBlocks * kNS)) ||
      (s = dalloc(c, &c->d_dreal, (size_t)kDiagBlocks * kNS)) ||
      (s = dalloc(c, &c->d_dke, (size_t)kDiagBlocks * kNS)) ||
      (s = dalloc(c, &c->d_spec, 3 * 66)) || (s = dalloc(c, &c->sput, (size_t)nr + 1)) ||
      (s = dalloc(c, &c->sput_take, (size_t)nr + 1)))
    return fail(s);
  if (hipMemset(c->sput, 0, sizeof(unsigned long long) * ((size_t)nr + 1)) != hipSuccess ||
      hipMemset(c->sput_take, 0, sizeof(uint32_t) * ((size_t)nr + 1)) != hipSuccess)
    return fail(set_err(c, PD_EDEVICE, "clearing the sputtering counters failed"));
  c->g.sput = c->sput;
  c->g.sput_take = c->sput_take;
  c->sw.cap = cap;
  c->cw.cap = cap;

  std::vector<double> Vnode, Vcell, ra, S, tinv, tcp, edges, rcv, twinv, twcp;
  build_tables(c, Vnode, Vcell, ra, S, tinv, tcp, edges, rcv, twinv, twcp);
  double *dVn, *dVc, *dra, *dS, *dti, *dtc, *drc, *dwi, *dwc;
  if ((s = dalloc(c, &dVn, Vnode.size())) || (s = dalloc(c, &dVc, Vcell.size())) ||
      (s = dalloc(c, &dra, ra.size())) || (s = dalloc(c, &dS, S.size())) ||
      (s = dalloc(c, &dti, tinv.size())) || (s = dalloc(c, &dtc, tcp.size())) ||
      (s = dalloc(c, &drc, rcv.size())) || (s = dalloc(c, &dwi, twinv.size())) ||
      (s = dalloc(c, &dwc, twcp.size())))
    return fail(s);
  auto up = [&](void* d, const void* h, size_t b) {
    return hipMemcpy(d, h, b, hipMemcpyHostToDevice) == hipSuccess;
  };
  if (!up(dVn, Vnode.data(), Vnode.size() * 8) || !up(dVc, Vcell.data(), Vcell.size() * 8) ||
      !up(dra, ra.data(), ra.size() * 8) || !up(dS, S.data(), S.size() * 8) ||
      !up(dti, tinv.data(), tinv.size() * 8) || !up(dtc, tcp.data(), tcp.size() * 8) ||
      !up(drc, rcv.data(), rcv.size() * 8) || !up(dwi, twinv.data(), twinv.size() * 8) ||
      !up(dwc, twcp.data(), twcp.size() * 8) ||
      !up(c->d_edges, edges.data(), 65 * 8))
    return fail(set_err(c, PD_EDEVICE, "table upload failed"));
  c->fw.Vnode = dVn;
  c->fw.ra = dra;
  c->fw.T = dS;
  c->fw.tinv = dti;
  c->fw.tcp = dtc;
  c->fw.rc = drc;
  c->fw.twinv = dwi;
  c->fw.twcp = dwc;
  c->fw.qunit = c->qunit;
  if (!c->spectral) {
    // the whole DST-I matrix for the fixed-order transforms (its entries are
    // the reduced table's, by (c+1)(b+1) mod 2 nz)
    std::vector<double> Sm((size_t)M * M);
    for (int cc = 0; cc < M; ++cc)
      for (int b = 0; b < M; ++b)
        Sm[(size_t)cc * M + b] = S[((size_t)(cc + 1) * (size_t)(b + 1)) % (size_t)(2 * nz)];
    double* dSm;
    if ((s = dalloc(c, &dSm, Sm.size()))) return fail(s);
    if (!up(dSm, Sm.data(), Sm.size() * 8)) return fail(set_err(c, PD_EDEVICE, "table upload failed"));
    c->fw.Sm = dSm;
  }
  if (c->spectral) {
    // the right-hand-side scale of the matrix-core form
    const int W = nr + 1;
    std::vector<double> coef(W);
    for (int i = 0; i < W; ++i) coef[i] = -(c->qunit / (Vnode[i] * kEPS0));
    double* dcoef;
    if ((s = dalloc(c, &dcoef, coef.size()))) return fail(s);
    if (!up(dcoef, coef.data(), coef.size() * 8))
      return fail(set_err(c, PD_EDEVICE, "table upload failed"));
    c->fw.coef = dcoef;
  }
  c->cpar.Vcell = dVc;
  if ((s = build_mg(c, dVn))) return fail(s);

  DevState h{};
  h.V_gap = dom->V_cathode;  // every Poisson solve reads the gap voltage here
  c->g.Vdev = &c->st->V_gap;
  if (hipMemcpy(c->st, &h, sizeof h, hipMemcpyHostToDevice) != hipSuccess)
    return fail(set_err(c, PD_EDEVICE, "state upload failed"));
  fill_u32(c->cw.claim, 0xFFFFFFFFu, cap, c->stream);
  fill_i64(c->fw.Q, 0, nn, c->stream);
  // vacuum potential and field until the first solve
  {
    std::vector<double> phi(nn), er(nn, 0.0), ez(nn);
    for (int j = 0; j <= nz; ++j) {
      const double vac = (-dom->V_cathode) + (dom->V_cathode * ((double)j / (double)nz));
      for (int i = 0; i <= nr; ++i) phi[(size_t)j * (nr + 1) + i] = vac;
    }
    if (!up(c->fw.phi, phi.data(), nn * 8)) return fail(set_err(c, PD_EDEVICE, "upload"));
    field(c->g, c->fw, c->stream);
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return fail(set_err(c, PD_EDEVICE, "initialisation failed"));
  *out = c;
  return PD_OK;
}

pd_status pd_set_species(pd_ctx* c, int n, const int32_t* Z, const double* mass) {
  if (!c) return PD_EINVAL;
  if (n != kNS || !Z || !mass) return set_err(c, PD_EINVAL, "need %d species", kNS);
  for (int k = 0; k < n; ++k)
    if (!(mass[k] > 0) || !std::isfinite(mass[k]) || Z[k] < -8 || Z[k] > 8)
      return set_err(c, PD_EINVAL, "species %d: bad charge or mass", k);
  // the Cu2+ labels share a key class (one charge) and the SI3 pair (one mass)
  for (int k = PD_CU2_DOUBLE; k <= PD_CU2_INIT; ++k)
    if (Z[k] != Z[PD_CU2_STEP] || mass[k] != mass[PD_CU2_STEP])
      return set_err(c, PD_EINVAL, "the Cu2+ labels must share one charge and mass");
  c->g.em_mass = mass[PD_CU];
  for (int k = 0; k < n; ++k) {
    c->spp.Z[k] = Z[k];
    c->spp.Zk[key_class((uint32_t)k)] = Z[k];
    c->spp.m[k] = mass[k];
    c->spp.qmdt[k] = (((double)Z[k] * kQE) / mass[k]) * c->dom.dt;
    c->spp.qmdt_heavy[k] = (((double)Z[k] * kQE) / mass[k]) * c->g.dt_heavy;
  }
  c->species_set = true;
  derive_pairs(c);
  return PD_OK;
}

pd_status pd_set_cross_section(pd_ctx* c, int ch, double thr, int n, double dsq, const double* sig) {
  if (!c) return PD_EINVAL;
  if (ch < 0 || ch >= kNC) return set_err(c, PD_EINVAL, "channel %d", ch);
  if (n < 2 || !sig || !(dsq > 0) || !std::isfinite(dsq) || !(thr >= 0) || !std::isfinite(thr))
    return set_err(c, PD_EINVAL, "bad cross-section table");
  int ex;
  if (std::frexp(dsq, &ex) != 0.5) return set_err(c, PD_EINVAL, "dsqrtE must be a power of 2");
  for (int i = 0; i < n; ++i)
    if (!(sig[i] >= 0) || !std::isfinite(sig[i])) return set_err(c, PD_EINVAL, "sigma[%d]", i);
  pd_status s = sync(c);
  if (s) return s;
  double* d = nullptr;
  if ((s = dalloc(c, &d, (size_t)n))) return s;
  HIPCHK(c, hipMemcpy(d, sig, sizeof(double) * n, hipMemcpyHostToDevice));
  c->d_xs[ch] = d;
  c->cpar.tab[ch] = d;
  c->cpar.tabn[ch] = n;
  c->cpar.thr[ch] = thr;
  c->cpar.dsq[ch] = dsq;
  c->xs_thr[ch] = thr;
  c->xs_set[ch] = true;
  c->cpar.chain = (c->xs_set[PD_SI3] || c->xs_set[PD_SI4]) ? 1 : 0;
  c->cpar.heavy = (c->xs_set[PD_CEX] || c->xs_set[PD_NN]) ? 1 : 0;
  c->cpar.coulomb = (c->xs_set[PD_CEI] || c->xs_set[PD_CEE]) ? 1 : 0;
  c->cpar.cee = c->xs_set[PD_CEE] ? 1 : 0;
  if (c->species_set) derive_pairs(c);
  return PD_OK;
}

pd_status pd_set_heavy_subcycle(pd_ctx* c, int32_t every) {
  if (!c) return PD_EINVAL;
  if (c->in_ensemble) return set_err(c, PD_ESTATE, "the ensemble's graph holds the step period");
  if (every < 1 || every > 1000) return set_err(c, PD_EINVAL, "every must be in 1..1000");
  pd_status s = sync(c);
  if (s) return s;
  c->g.heavy_every = every;
  c->g.dt_heavy = (double)every * c->dom.dt;
  c->cpar.dt_heavy = c->g.dt_heavy;
  c->sw.heavy_every = every;
  for (int k = 0; k < kNS; ++k)
    c->spp.qmdt_heavy[k] = (((double)c->spp.Z[k] * kQE) / c->spp.m[k]) * c->g.dt_heavy;
  return PD_OK;
}

pd_status pd_set_emission(pd_ctx* c, double beta, double r_tip, double phi_w, double neutral_ratio,
                          double T) {
  if (!c) return PD_EINVAL;
  if (c->in_ensemble) return set_err(c, PD_ESTATE, "the ensemble's graph holds the emission");
  if (!(beta >= 0.0) || !std::isfinite(beta) || !(r_tip >= 0.0) || !(r_tip <= c->dom.R) ||
      (beta > 0.0 && !(phi_w > 0.0)) || !std::isfinite(phi_w) || !(neutral_ratio >= 0.0) ||
      !std::isfinite(neutral_ratio) || !(T >= 0.0) || !std::isfinite(T))
    return set_err(c, PD_EINVAL, "bad emission parameters");
  if (beta > 0.0 && (r_tip / c->g.dr) + 0.5 >= 1023.0)
    return set_err(c, PD_EINVAL, "the tip spans more than 1023 radial nodes");
  pd_status s = sync(c);
  if (s) return s;
  c->g.em_beta = beta;
  c->g.em_rtip = r_tip;
  c->g.em_phi = phi_w;
  c->g.em_ratio = neutral_ratio;
  c->g.em_T = T;
  return PD_OK;
}

pd_status pd_set_sputtering(pd_ctx* c, int32_t on) {
  if (!c) return PD_EINVAL;
  if (c->in_ensemble) return set_err(c, PD_ESTATE, "the ensemble's graph holds the sputtering");
  if (on && c->g.nr + 1 > 4096) return set_err(c, PD_EINVAL, "more than 4096 cathode annuli");
  pd_status s = sync(c);
  if (s) return s;
  c->g.sput_on = on ? 1 : 0;
  return PD_OK;
}

pd_status pd_set_split_literal(pd_ctx* c, int32_t on) {
  if (!c) return PD_EINVAL;
  if (c->in_ensemble) return set_err(c, PD_ESTATE, "the ensemble's graph holds the split");
  pd_status s = sync(c);
  if (s) return s;
  c->cpar.split_literal = on ? 1 : 0;
  return PD_OK;
}

pd_status pd_set_circuit(pd_ctx* c, double V0, double R, double C) {
  if (!c) return PD_EINVAL;
  if (c->in_ensemble) return set_err(c, PD_ESTATE, "the ensemble's graph holds the circuit");
  if (!std::isfinite(V0) || !(R > 0.0) || !std::isfinite(R) || !(C >= 0.0) || !std::isfinite(C))
    return set_err(c, PD_EINVAL, "bad circuit parameters");
  if (C > 0.0 && c->mg_on)
    return set_err(c, PD_ESTATE, "the circuit needs a direct Poisson solve");
  if (C > 0.0 && c->weighted)
    return set_err(c, PD_EINVAL, "the circuit counts super-particles; no multiplicities with it");
  DevState h;
  pd_status s = read_state(c, &h);
  if (s) return s;
  // the anode charge counted so far is not current of the circuit
  long long za = 0;
  for (int k = 0; k < kNS; ++k) za += (long long)c->spp.Z[k] * (long long)h.absorbed[kNS + k];
  HIPCHK(c, hipMemcpy((char*)c->st + offsetof(DevState, circ_zanode), &za, sizeof za,
                      hipMemcpyHostToDevice));
  c->g.circ_V0 = V0;
  c->g.circ_R = R;
  c->g.circ_C = C;
  return PD_OK;
}

pd_status pd_inject(pd_ctx* c, int64_t n, const double* r, const double* z, const double* vr,
                    const double* vt, const double* vz, const uint8_t* sp) {
  if (!c) return PD_EINVAL;
  if (c->poisoned) return set_err(c, PD_ESTATE, "context unusable after an earlier error");
  if (n < 0) return set_err(c, PD_EINVAL, "n < 0");
  pd_status s = check_particles(c, n, r, z, vr, vt, vz, sp);
  if (s) return s;
  if (n == 0) return PD_OK;
  DevState h;
  if ((s = read_state(c, &h))) return s;
  if ((int64_t)h.n_total + n > c->cap) return set_err(c, PD_ECAPACITY, "capacity %lld", (long long)c->cap);
  if ((int64_t)h.next_id + n > (int64_t)0xFFFFFFFFLL) return set_err(c, PD_ECAPACITY, "id space");
  // stage through the sort's destination buffers (scratch between steps)
  if (c->fp32) s = stage_append(c, c->Af, c->Bf, n, r, z, vr, vt, vz, sp, nullptr);
  else s = stage_append(c, c->A, c->B, n, r, z, vr, vt, vz, sp, nullptr);
  if (s) return s;
  if ((s = sync(c))) return s;
  for (int64_t p = 0; p < n; ++p) c->injected[sp[p]] += 1;
  return PD_OK;
}

pd_status pd_set_weighted(pd_ctx* c, int32_t on) {
  if (!c) return PD_EINVAL;
  if (!on) return c->weighted ? set_err(c, PD_EINVAL, "multiplicities cannot be turned off")
                              : PD_OK;
  if (c->weighted) return PD_OK;
  if (c->poisoned) return set_err(c, PD_ESTATE, "context unusable after an earlier error");
  if (c->in_ensemble) return set_err(c, PD_ESTATE, "context is in an ensemble");
  if (c->fp32) return set_err(c, PD_EINVAL, "multiplicities need the FP64 record");
  if (c->g.circ_C > 0.0)
    return set_err(c, PD_EINVAL, "the circuit counts super-particles; no multiplicities with it");
  pd_status s;
  if ((s = sync(c))) return s;
  if ((s = dalloc(c, &c->A.mu, c->cap)) || (s = dalloc(c, &c->B.mu, c->cap))) return s;
  std::vector<uint16_t> one((size_t)c->cap, (uint16_t)1);
  HIPCHK(c, hipMemcpy(c->A.mu, one.data(), sizeof(uint16_t) * c->cap, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->B.mu, one.data(), sizeof(uint16_t) * c->cap, hipMemcpyHostToDevice));
  c->weighted = true;
  return PD_OK;
}

pd_status pd_inject_weighted(pd_ctx* c, int64_t n, const double* r, const double* z,
                             const double* vr, const double* vt, const double* vz,
                             const uint8_t* sp, const uint16_t* mu) {
  if (!c) return PD_EINVAL;
  if (c->poisoned) return set_err(c, PD_ESTATE, "context unusable after an earlier error");
  if (!c->weighted) return set_err(c, PD_ESTATE, "multiplicities not enabled (pd_set_weighted)");
  if (n < 0) return set_err(c, PD_EINVAL, "n < 0");
  if (n > 0 && !mu) return set_err(c, PD_EINVAL, "mu is NULL");
  for (int64_t p = 0; p < n; ++p)
    if (mu[p] < 1) return set_err(c, PD_EINVAL, "multiplicity of particle %lld below 1", (long long)p);
  pd_status s = check_particles(c, n, r, z, vr, vt, vz, sp);
  if (s) return s;
  if (n == 0) return PD_OK;
  DevState h;
  if ((s = read_state(c, &h))) return s;
  if ((int64_t)h.n_total + n > c->cap) return set_err(c, PD_ECAPACITY, "capacity %lld", (long long)c->cap);
  if ((int64_t)h.next_id + n > (int64_t)0xFFFFFFFFLL) return set_err(c, PD_ECAPACITY, "id space");
  if ((s = stage_append(c, c->A, c->B, n, r, z, vr, vt, vz, sp, mu))) return s;
  if ((s = sync(c))) return s;
  for (int64_t p = 0; p < n; ++p) c->injected[sp[p]] += 1;
  return PD_OK;
}

pd_status pd_schedule_injection(pd_ctx* c, int nsteps, const int64_t* offs, const double* r,
                                const double* z, const double* vr, const double* vt,
                                const double* vz, const uint8_t* sp) {
  if (!c) return PD_EINVAL;
  if (c->in_ensemble) return set_err(c, PD_ESTATE, "schedule is fixed while in an ensemble");
  if (c->poisoned) return set_err(c, PD_ESTATE, "context unusable after an earlier error");
  if (nsteps < 0 || (nsteps > 0 && !offs) || (nsteps > 0 && offs[0] != 0))
    return set_err(c, PD_EINVAL, "bad schedule offsets");
  int64_t maxc = 0;
  for (int k = 0; k < nsteps; ++k) {
    if (offs[k + 1] < offs[k]) return set_err(c, PD_EINVAL, "schedule offsets decrease");
    maxc = std::max<int64_t>(maxc, offs[k + 1] - offs[k]);
  }
  const int64_t tot = nsteps ? offs[nsteps] : 0;
  pd_status s = check_particles(c, tot, r, z, vr, vt, vz, sp);
  if (s) return s;
  if ((s = sync(c))) return s;
  for (void* p : c->sched_allocs) (void)hipFree(p);
  c->sched_allocs.clear();
  c->sched = Schedule{};
  c->sched_species.clear();
  auto dup = [&](const void* h, size_t bytes) -> void* {
    void* d = nullptr;
    if (hipMalloc(&d, bytes ? bytes : 16) != hipSuccess) return nullptr;
    c->sched_allocs.push_back(d);
    if (bytes && hipMemcpy(d, h, bytes, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return d;
  };
  if (nsteps > 0) {
    Schedule sc{};
    sc.off = (const int64_t*)dup(offs, sizeof(int64_t) * (nsteps + 1));
    sc.r = (const double*)dup(r, 8 * tot);
    sc.z = (const double*)dup(z, 8 * tot);
    sc.vr = (const double*)dup(vr, 8 * tot);
    sc.vt = (const double*)dup(vt, 8 * tot);
    sc.vz = (const double*)dup(vz, 8 * tot);
    sc.sp = (const uint8_t*)dup(sp, tot);
    sc.max_count = maxc;
    if (!sc.off || !sc.r || !sc.z || !sc.vr || !sc.vt || !sc.vz || !sc.sp)
      return set_err(c, PD_ENOMEM, "schedule upload failed");
    c->sched = sc;
    c->sched_species.resize(nsteps);
    for (int k = 0; k < nsteps; ++k) {
      std::array<int64_t, kNS> a{};
      for (int64_t p = offs[k]; p < offs[k + 1]; ++p) a[sp[p]] += 1;
      c->sched_species[k] = a;
    }
  }
  c->sched_n = nsteps;
  c->host_sched_pos = 0;
  uint32_t v[2] = {0u, (uint32_t)nsteps};
  HIPCHK(c, hipMemcpy((char*)c->st + offsetof(DevState, sched_pos), v, sizeof v,
                      hipMemcpyHostToDevice));
  return PD_OK;
}

pd_status pd_step(pd_ctx* c, int nsteps) {
  if (!c) return PD_EINVAL;
  if (c->in_ensemble) return set_err(c, PD_ESTATE, "context steps through its ensemble");
  if (c->poisoned) return set_err(c, PD_ESTATE, "context unusable after an earlier error");
  if (nsteps < 0) return set_err(c, PD_EINVAL, "nsteps < 0");
  if (!c->species_set) return set_err(c, PD_ESTATE, "species not set");
  if (!c->opts.collisions_off)
    for (int k = 0; k <= PD_SI2; ++k)
      if (!c->xs_set[k]) return set_err(c, PD_ESTATE, "cross section %d not set", k);
  hipStream_t s = c->stream;
  const int64_t nn = (int64_t)(c->g.nr + 1) * (c->g.nz + 1);
  for (int t = 0; t < nsteps; ++t) {
    std::vector<hipEvent_t> ev;
    // same: the boundary coincides with the previous one (an empty stage,
    // kept as a null entry, no event recorded)
    auto mark = [&](bool same = false) {
      if (c->opts.timing) {
        if (same && !ev.empty()) {
          ev.push_back(nullptr);
          return;
        }
        hipEvent_t e = get_event(c);
        (void)hipEventRecord(e, s);
        ev.push_back(e);
      }
    };
    pd_status ps = c->fp32 ? enqueue_step(c, c->Af, c->Bf, nn, mark)
                           : enqueue_step(c, c->A, c->B, nn, mark);
    if (ps) return ps;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      c->poisoned = true;
      return set_err(c, PD_EDEVICE, "launch failed: %s", hipGetErrorString(e));
    }
    host_after_step(c);
    if (c->opts.timing) {
      c->ev_pending.push_back(ev);
      if (c->ev_pending.size() >= 512) {
        pd_status st = sync(c);
        if (st) return st;
        harvest_timing(c);
      }
    }
  }
  return PD_OK;
}

pd_status pd_synchronize(pd_ctx* c) {
  if (!c) return PD_EINVAL;
  DevState h;
  return read_state(c, &h);
}

static pd_status snapshot(pd_ctx* c, DevState& h, int64_t counts[kNS], double ke[kNS],
                          int64_t spec[3][66], int64_t real[kNS]) {
  pd_status s = read_state(c, &h);
  if (s) return s;
  HIPCHK(c, hipMemsetAsync(c->d_spec, 0, sizeof(unsigned long long) * 3 * 66, c->stream));
  if (c->fp32)
    diag_snapshot(c->Af, c->st, c->g, c->spp, c->d_edges, c->d_dcount, c->d_dke, c->d_spec,
                  c->d_dreal, c->stream);
  else
    diag_snapshot(c->A, c->st, c->g, c->spp, c->d_edges, c->d_dcount, c->d_dke, c->d_spec,
                  c->d_dreal, c->stream);
  HIPCHK(c, hipGetLastError());
  if ((s = sync(c))) return s;
  std::vector<unsigned long long> hc((size_t)kDiagBlocks * kNS), hs(3 * 66),
      hr((size_t)kDiagBlocks * kNS);
  std::vector<double> hk((size_t)kDiagBlocks * kNS);
  HIPCHK(c, hipMemcpy(hc.data(), c->d_dcount, hc.size() * 8, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(hr.data(), c->d_dreal, hr.size() * 8, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(hk.data(), c->d_dke, hk.size() * 8, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(hs.data(), c->d_spec, hs.size() * 8, hipMemcpyDeviceToHost));
  for (int k = 0; k < kNS; ++k) {
    counts[k] = 0;
    real[k] = 0;
    ke[k] = 0.0;
  }
  for (int b = 0; b < kDiagBlocks; ++b)
    for (int k = 0; k < kNS; ++k) {
      counts[k] += (int64_t)hc[(size_t)b * kNS + k];
      real[k] += (int64_t)hr[(size_t)b * kNS + k];
      ke[k] += hk[(size_t)b * kNS + k];
    }
  for (int t = 0; t < 3; ++t)
    for (int b = 0; b < 66; ++b) spec[t][b] = (int64_t)hs[t * 66 + b];
  return PD_OK;
}

pd_status pd_get_diagnostics(pd_ctx* c, pd_diag* out) {
  if (!c || !out) return PD_EINVAL;
  DevState h;
  int64_t counts[kNS], real[kNS];
  double ke[kNS];
  int64_t spec[3][66];
  pd_status s = snapshot(c, h, counts, ke, spec, real);
  if (s) return s;
  std::memset(out, 0, sizeof *out);
  for (int k = 0; k < kNS; ++k) out->real[k] = real[k];
  out->step = c->host_step;
  out->next_id = h.next_id;
  int64_t n = 0;
  for (int k = 0; k < kNS; ++k) {
    out->count[k] = counts[k];
    out->ke_J[k] = ke[k];
    n += counts[k];
    out->injected[k] = c->injected[k];
    out->charge_alive += counts[k] * c->spp.Z[k];
    out->charge_injected += c->injected[k] * c->spp.Z[k];
  }
  out->n_alive = n;
  for (int k = 0; k < kNC; ++k) out->events[k] = (int64_t)h.events[k];
  out->conflicts = (int64_t)h.conflicts;
  out->particle_steps = (int64_t)h.pushed;
  out->created = (int64_t)h.created;
  for (int b = 0; b < 3; ++b)
    for (int k = 0; k < kNS; ++k) {
      out->absorbed[b][k] = (int64_t)h.absorbed[b * kNS + k];
      out->charge_absorbed += out->absorbed[b][k] * c->spp.Z[k];
    }
  mg_residual(c->mg, c->fw.phi, c->fw.Q, c->stream);
  if ((s = read_mg(c))) return s;
  out->poisson_rel_res = c->h_sc->rel;
  out->poisson_solves = c->p_solves;
  out->poisson_iters = c->h_sc->iters;
  out->poisson_refinements = c->h_sc->outer;
  out->poisson_fallbacks = c->p_fallbacks;
  out->poisson_seconds = c->p_call_ms * 1e-3;
  // Eq. 21 over the charge states 0..4 (N_2: every Cu2+ label) of the real
  // particle numbers (in units of W), integer sums, one division each
  const int64_t N[5] = {real[PD_CU], real[PD_CU1],
                        real[PD_CU2_STEP] + real[PD_CU2_DOUBLE] + real[PD_CU2_INIT],
                        real[PD_CU3], real[PD_CU4]};
  const int64_t ions = N[1] + N[2] + N[3] + N[4];
  const int64_t qsum = N[1] + 2 * N[2] + 3 * N[3] + 4 * N[4];
  out->gamma = (ions + N[0]) > 0 ? (double)ions / (double)(ions + N[0]) : 0.0;
  out->qbar = ions > 0 ? (double)qsum / (double)ions : 0.0;
  out->V_gap = h.V_gap;
  out->emitted[0] = (int64_t)h.emitted[0];
  out->emitted[1] = (int64_t)h.emitted[1];
  out->sputtered = (int64_t)h.sputtered;
  // the emitted and sputtered particles enter like injected ones
  out->injected[PD_E] += out->emitted[0];
  out->injected[PD_CU] += out->emitted[1] + out->sputtered;
  out->charge_injected += out->emitted[0] * c->spp.Z[PD_E] + out->emitted[1] * c->spp.Z[PD_CU];
  return PD_OK;
}

pd_status pd_get_spectrum(pd_ctx* c, int tag, int64_t out[66]) {
  if (!c || !out) return PD_EINVAL;
  if (tag < 0 || tag > 2) return set_err(c, PD_EINVAL, "tag %d", tag);
  DevState h;
  int64_t counts[kNS], real[kNS];
  double ke[kNS];
  int64_t spec[3][66];
  pd_status s = snapshot(c, h, counts, ke, spec, real);
  if (s) return s;
  for (int b = 0; b < 66; ++b) out[b] = spec[tag][b];
  return PD_OK;
}

pd_status pd_get_count(pd_ctx* c, int64_t* n) {
  if (!c || !n) return PD_EINVAL;
  DevState h;
  pd_status s = read_state(c, &h);
  if (s) return s;
  int64_t a = 0;
  for (int k = 0; k < 3 * kNS; ++k) a += (int64_t)h.absorbed[k];
  int64_t inj = 0;
  for (int k = 0; k < kNS; ++k) inj += c->injected[k];
  *n = inj + (int64_t)h.emitted[0] + (int64_t)h.emitted[1] + (int64_t)h.sputtered +
       (int64_t)h.created - a;
  return PD_OK;
}

pd_status pd_get_particles(pd_ctx* c, int64_t cap, double* r, double* z, double* vr, double* vt,
                           double* vz, uint8_t* sp, uint32_t* id, uint32_t* key) {
  if (!c) return PD_EINVAL;
  DevState h;
  pd_status s = read_state(c, &h);
  if (s) return s;
  const int64_t n = h.n_total;
  auto out = [&](const auto& P) -> pd_status {
    using T = std::remove_reference_t<decltype(P.x[0].r)>;
    std::vector<PosT<T>> x;
    std::vector<RecT<T>> v;
    std::vector<uint32_t> k;
    pd_status s = pull_records(c, P, (size_t)n, x, v, k);
    if (s) return s;
    int64_t alive = 0;
    for (int64_t p = 0; p < n; ++p) alive += (k[p] != c->g.sentinel);
    if (cap < alive)
      return set_err(c, PD_EINVAL, "cap %lld < %lld particles", (long long)cap, (long long)alive);
    // FP32 records are widened to double
    int64_t w = 0;
    for (int64_t p = 0; p < n; ++p) {
      if (k[p] == c->g.sentinel) continue;
      if (r) r[w] = (double)x[p].r;
      if (z) z[w] = (double)x[p].z;
      if (vr) vr[w] = (double)v[p].vr;
      if (vt) vt[w] = (double)v[p].vt;
      if (vz) vz[w] = (double)v[p].vz;
      if (sp) sp[w] = (uint8_t)v[p].sp;
      if (id) id[w] = v[p].id;
      if (key) key[w] = k[p];
      ++w;
    }
    return PD_OK;
  };
  return c->fp32 ? out(c->Af) : out(c->A);
}

pd_status pd_get_weights(pd_ctx* c, int64_t cap, uint16_t* mu) {
  if (!c || !mu) return PD_EINVAL;
  DevState h;
  pd_status s = read_state(c, &h);
  if (s) return s;
  const size_t n = h.n_total;
  std::vector<uint32_t> k(n);
  std::vector<uint16_t> m(n, (uint16_t)1);
  const uint32_t* dkey = c->fp32 ? c->Af.key : c->A.key;
  if (n) {
    HIPCHK(c, hipMemcpy(k.data(), dkey, 4 * n, hipMemcpyDeviceToHost));
    if (c->weighted) HIPCHK(c, hipMemcpy(m.data(), c->A.mu, 2 * n, hipMemcpyDeviceToHost));
  }
  int64_t alive = 0;
  for (size_t p = 0; p < n; ++p) alive += (k[p] != c->g.sentinel);
  if (cap < alive)
    return set_err(c, PD_EINVAL, "cap %lld < %lld particles", (long long)cap, (long long)alive);
  int64_t w = 0;
  for (size_t p = 0; p < n; ++p)
    if (k[p] != c->g.sentinel) mu[w++] = m[p];
  return PD_OK;
}

pd_status pd_get_field(pd_ctx* c, double* phi, double* Er, double* Ez, int64_t* Q) {
  if (!c) return PD_EINVAL;
  pd_status s = sync(c);
  if (s) return s;
  const size_t nn = (size_t)(c->g.nr + 1) * (c->g.nz + 1);
  if (phi) HIPCHK(c, hipMemcpy(phi, c->fw.phi, 8 * nn, hipMemcpyDeviceToHost));
  if (Er) HIPCHK(c, hipMemcpy(Er, c->fw.Er, 8 * nn, hipMemcpyDeviceToHost));
  if (Ez) HIPCHK(c, hipMemcpy(Ez, c->fw.Ez, 8 * nn, hipMemcpyDeviceToHost));
  if (Q) HIPCHK(c, hipMemcpy(Q, c->fw.Q, 8 * nn, hipMemcpyDeviceToHost));
  return PD_OK;
}

pd_status pd_poisson(pd_ctx* c, const int64_t* Q, double* phi, int32_t* iters, double* rel_res) {
  if (!c) return PD_EINVAL;
  if (c->poisoned) return set_err(c, PD_ESTATE, "context unusable after an earlier error");
  if (!Q) return set_err(c, PD_EINVAL, "Q is NULL");
  pd_status s = sync(c);
  if (s) return s;
  const size_t nn = (size_t)(c->g.nr + 1) * (c->g.nz + 1);
  HIPCHK(c, hipMemcpy(c->fw.Q, Q, 8 * nn, hipMemcpyHostToDevice));
  if ((s = read_mg(c))) return s;
  const int it0 = c->h_sc->iters;
  hipEvent_t e0 = get_event(c), e1 = get_event(c);
  HIPCHK(c, hipEventRecord(e0, c->stream));
  if ((s = solve_poisson(c))) return s;
  HIPCHK(c, hipEventRecord(e1, c->stream));
  field(c->g, c->fw, c->stream);
  mg_residual(c->mg, c->fw.phi, c->fw.Q, c->stream);
  HIPCHK(c, hipGetLastError());
  if ((s = read_mg(c))) return s;
  {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) c->p_call_ms += ms;
    c->ev_pool.push_back(e0);
    c->ev_pool.push_back(e1);
  }
  if (iters) *iters = c->h_sc->iters - it0;
  if (rel_res) *rel_res = c->h_sc->rel;
  if (phi) HIPCHK(c, hipMemcpy(phi, c->fw.phi, 8 * nn, hipMemcpyDeviceToHost));
  return PD_OK;
}

// ---- checkpoint: the whole state between two steps in one file -----------
// Layout (host byte order, this library's struct layouts): the magic, the
// version, sizeof of the saved structs; the domain and the options that
// shape the state; species and cross-section tables; the device counters;
// the particle records in the order the next sort receives them (native
// precision); the last sort's keys and cell offsets (the next sort starts
// from them); the node charge, potential and field; the injection schedule
// with its read position; the host-side counters; the solver's scalars; the
// magic again.
static const char kSaveMagic[8] = {'P', 'D', 'S', 'T', 'A', 'T', 'E', '1'};
constexpr uint32_t kSaveVersion = 5;

struct SaveHead {
  char magic[8];
  uint32_t version, sz_domain, sz_state, sz_mgscal;
  pd_domain dom;
  int32_t precision, poisson, enable_di, deposit_off, collisions_off, heavy_every;
};

struct SaveBoundary {
  double em_beta, em_rtip, em_phi, em_ratio, em_T, circ_V0, circ_R, circ_C;
  int32_t split_literal, sput_on, weighted, pad;
};

struct SaveHost {
  int64_t injected[kNS];
  int64_t host_step, host_sched_pos, sched_n, p_solves, p_fallbacks;
  int32_t mg_inner, pad;
};

pd_status pd_save(pd_ctx* c, const char* path) {
  if (!c) return PD_EINVAL;
  if (!path) return set_err(c, PD_EINVAL, "path is NULL");
  if (c->poisoned) return set_err(c, PD_ESTATE, "context unusable after an earlier error");
  if (c->in_ensemble) return set_err(c, PD_ESTATE, "context is in an ensemble");
  if (!c->species_set) return set_err(c, PD_ESTATE, "species not set");
  DevState st;
  pd_status s = read_state(c, &st);
  if (s) return s;
  std::vector<unsigned char> out;
  auto put = [&](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    out.insert(out.end(), b, b + n);
  };
  auto putd = [&](const void* dev, size_t n) -> pd_status {
    const size_t o = out.size();
    out.resize(o + n);
    if (n) HIPCHK(c, hipMemcpy(out.data() + o, dev, n, hipMemcpyDeviceToHost));
    return PD_OK;
  };
  SaveHead h{};
  std::memcpy(h.magic, kSaveMagic, 8);
  h.version = kSaveVersion;
  h.sz_domain = sizeof(pd_domain);
  h.sz_state = sizeof(DevState);
  h.sz_mgscal = sizeof(MGScal);
  h.dom = c->dom;
  h.precision = c->opts.precision;
  h.poisson = c->opts.poisson;
  h.enable_di = c->opts.enable_di;
  h.deposit_off = c->opts.deposit_off;
  h.collisions_off = c->opts.collisions_off;
  h.heavy_every = c->g.heavy_every;
  put(&h, sizeof h);
  const SaveBoundary sb{c->g.em_beta, c->g.em_rtip, c->g.em_phi, c->g.em_ratio,
                        c->g.em_T,    c->g.circ_V0, c->g.circ_R, c->g.circ_C,
                        c->cpar.split_literal, c->g.sput_on, c->weighted ? 1 : 0, 0};
  put(&sb, sizeof sb);
  put(c->spp.Z, sizeof c->spp.Z);
  put(c->spp.m, sizeof c->spp.m);
  for (int k = 0; k < kNC; ++k) {
    const int32_t set = c->xs_set[k] ? 1 : 0;
    const int32_t n = set ? c->cpar.tabn[k] : 0;
    put(&set, 4);
    put(&n, 4);
    put(&c->cpar.thr[k], 8);
    put(&c->cpar.dsq[k], 8);
    if (set && (s = putd(c->d_xs[k], 8 * (size_t)n))) return s;
  }
  put(&st, sizeof st);
  const size_t n = st.n_total;
  const size_t nn = (size_t)(c->g.nr + 1) * (c->g.nz + 1);
  // the records in the device layout (position pairs, then the rest), keys
  if (c->fp32) {
    if ((s = putd(c->Af.x, sizeof(PosT<float>) * n)) ||
        (s = putd(c->Af.v, sizeof(RecT<float>) * n)) || (s = putd(c->Af.key, 4 * n)))
      return s;
  } else {
    if ((s = putd(c->A.x, sizeof(PosT<double>) * n)) ||
        (s = putd(c->A.v, sizeof(RecT<double>) * n)) || (s = putd(c->A.key, 4 * n)))
      return s;
    if (c->weighted && (s = putd(c->A.mu, sizeof(uint16_t) * n))) return s;
  }
  if ((s = putd(c->sw.skey, 4 * (size_t)st.n_alive)) ||
      (s = putd(c->off, 4 * ((size_t)c->g.sentinel + 1))) || (s = putd(c->fw.Q, 8 * nn)) ||
      (s = putd(c->fw.phi, 8 * nn)) || (s = putd(c->fw.Er, 8 * nn)) ||
      (s = putd(c->fw.Ez, 8 * nn)) ||
      (s = putd(c->sput, sizeof(unsigned long long) * ((size_t)c->g.nr + 1))))
    return s;
  const int64_t sn = c->sched_n;
  put(&sn, 8);
  if (sn > 0) {
    std::vector<int64_t> off(sn + 1);
    HIPCHK(c, hipMemcpy(off.data(), c->sched.off, 8 * (sn + 1), hipMemcpyDeviceToHost));
    put(off.data(), 8 * (sn + 1));
    const size_t tot = (size_t)off[sn];
    const double* a[5] = {c->sched.r, c->sched.z, c->sched.vr, c->sched.vt, c->sched.vz};
    for (int k = 0; k < 5; ++k)
      if ((s = putd(a[k], 8 * tot))) return s;
    if ((s = putd(c->sched.sp, tot))) return s;
  }
  SaveHost hh{};
  for (int k = 0; k < kNS; ++k) hh.injected[k] = c->injected[k];
  hh.host_step = c->host_step;
  hh.host_sched_pos = c->host_sched_pos;
  hh.sched_n = c->sched_n;
  hh.p_solves = c->p_solves;
  hh.p_fallbacks = c->p_fallbacks;
  hh.mg_inner = c->mg_inner;
  put(&hh, sizeof hh);
  if ((s = putd(c->mg.sc, sizeof(MGScal)))) return s;
  put(kSaveMagic, 8);
  FILE* f = std::fopen(path, "wb");
  if (!f) return set_err(c, PD_EINVAL, "cannot open %s for writing", path);
  const size_t w = std::fwrite(out.data(), 1, out.size(), f);
  const int cl = std::fclose(f);
  if (w != out.size() || cl != 0) return set_err(c, PD_EINVAL, "short write to %s", path);
  return PD_OK;
}

pd_status pd_load(pd_ctx* c, const char* path) {
  if (!c) return PD_EINVAL;
  if (!path) return set_err(c, PD_EINVAL, "path is NULL");
  if (c->poisoned) return set_err(c, PD_ESTATE, "context unusable after an earlier error");
  if (c->in_ensemble) return set_err(c, PD_ESTATE, "context is in an ensemble");
  std::vector<unsigned char> in;
  {
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_err(c, PD_EINVAL, "cannot open %s", path);
    unsigned char buf[1 << 16];
    size_t r;
    while ((r = std::fread(buf, 1, sizeof buf, f)) > 0) in.insert(in.end(), buf, buf + r);
    std::fclose(f);
  }
  // parse and check everything before the context is touched
  size_t pos = 0;
  bool ok = true;
  auto get = [&](void* p, size_t n) {
    if (!ok || n > in.size() - pos) {
      ok = false;
      return;
    }
    std::memcpy(p, in.data() + pos, n);
    pos += n;
  };
  auto span = [&](size_t n) -> const unsigned char* {
    if (!ok || n > in.size() - pos) {
      ok = false;
      return nullptr;
    }
    const unsigned char* p = in.data() + pos;
    pos += n;
    return p;
  };
  SaveHead h{};
  get(&h, sizeof h);
  if (!ok || std::memcmp(h.magic, kSaveMagic, 8) != 0 || h.version != kSaveVersion ||
      h.sz_domain != sizeof(pd_domain) || h.sz_state != sizeof(DevState) ||
      h.sz_mgscal != sizeof(MGScal))
    return set_err(c, PD_EINVAL, "%s: not a state file of this library version", path);
  const pd_domain& d = h.dom;
  if (d.nr != c->dom.nr || d.nz != c->dom.nz || d.R != c->dom.R || d.L != c->dom.L ||
      d.V_cathode != c->dom.V_cathode || d.dt != c->dom.dt || d.weight != c->dom.weight ||
      d.seed != c->dom.seed || h.precision != c->opts.precision ||
      h.enable_di != c->opts.enable_di || h.deposit_off != c->opts.deposit_off ||
      h.collisions_off != c->opts.collisions_off || h.heavy_every < 1 || h.heavy_every > 1000)
    return set_err(c, PD_EINVAL, "%s: domain or options differ from the context's", path);
  SaveBoundary sb{};
  get(&sb, sizeof sb);
  int32_t Z[kNS];
  double m[kNS];
  get(Z, sizeof Z);
  get(m, sizeof m);
  int32_t xset[kNC], xn[kNC];
  double xthr[kNC], xdsq[kNC];
  const double* xsig[kNC];
  for (int k = 0; k < kNC; ++k) {
    get(&xset[k], 4);
    get(&xn[k], 4);
    get(&xthr[k], 8);
    get(&xdsq[k], 8);
    xsig[k] = nullptr;
    if (ok && xset[k]) {
      if (xn[k] < 2 || xn[k] > (1 << 24)) ok = false;
      else xsig[k] = (const double*)span(8 * (size_t)xn[k]);
    }
  }
  DevState st{};
  get(&st, sizeof st);
  if (!ok) return set_err(c, PD_EINVAL, "%s: truncated", path);
  if ((int64_t)st.n_total > c->cap || st.n_alive > st.n_total || st.err != 0)
    return set_err(c, PD_EINVAL, "%s: %u particles do not fit the capacity %lld", path,
                   st.n_total, (long long)c->cap);
  const size_t n = st.n_total;
  const size_t nn = (size_t)(c->g.nr + 1) * (c->g.nz + 1);
  const size_t xsz = c->fp32 ? sizeof(PosT<float>) : sizeof(PosT<double>);
  const size_t vsz = c->fp32 ? sizeof(RecT<float>) : sizeof(RecT<double>);
  const size_t sp_at = c->fp32 ? offsetof(RecT<float>, sp) : offsetof(RecT<double>, sp);
  const unsigned char* xrec = span(xsz * n);
  const unsigned char* vrec = span(vsz * n);
  const unsigned char* key = span(4 * n);
  if (ok && sb.weighted && c->fp32) ok = false;
  const unsigned char* mu = sb.weighted ? span(sizeof(uint16_t) * n) : nullptr;
  const unsigned char* skey = span(4 * (size_t)st.n_alive);
  const unsigned char* off = span(4 * ((size_t)c->g.sentinel + 1));
  const unsigned char* Q = span(8 * nn);
  const unsigned char* phi = span(8 * nn);
  const unsigned char* Er = span(8 * nn);
  const unsigned char* Ez = span(8 * nn);
  const unsigned char* sput = span(sizeof(unsigned long long) * ((size_t)c->g.nr + 1));
  int64_t sn = 0;
  get(&sn, 8);
  std::vector<int64_t> soff;
  const unsigned char* sarr[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  if (ok && (sn < 0 || sn > (1 << 26))) ok = false;
  if (ok && sn > 0) {
    soff.resize(sn + 1);
    get(soff.data(), 8 * (sn + 1));
    if (ok && soff[0] != 0) ok = false;
    for (int64_t k = 0; ok && k < sn; ++k)
      if (soff[k + 1] < soff[k]) ok = false;
    if (ok) {
      const size_t tot = (size_t)soff[sn];
      for (int k = 0; k < 5; ++k) sarr[k] = span(8 * tot);
      sarr[5] = span(tot);
    }
  }
  SaveHost hh{};
  get(&hh, sizeof hh);
  const unsigned char* sc = span(sizeof(MGScal));
  char tail[8] = {0};
  get(tail, 8);
  if (!ok || pos != in.size() || std::memcmp(tail, kSaveMagic, 8) != 0)
    return set_err(c, PD_EINVAL, "%s: truncated or malformed", path);
  if (hh.sched_n != sn || hh.host_sched_pos < 0 || hh.host_sched_pos > sn ||
      st.sched_n != (uint32_t)sn || st.sched_pos > (uint32_t)sn)
    return set_err(c, PD_EINVAL, "%s: inconsistent injection schedule", path);
  for (size_t p = 0; p < n; ++p) {
    uint32_t sp;
    std::memcpy(&sp, vrec + vsz * p + sp_at, 4);
    if (sp >= kNS) return set_err(c, PD_EINVAL, "%s: species out of range", path);
  }
  for (int64_t p = 0; p < (sn > 0 ? soff[sn] : 0); ++p)
    if (sarr[5][p] >= kNS) return set_err(c, PD_EINVAL, "%s: schedule species out of range", path);
  for (size_t p = 0; mu && p < n; ++p) {
    uint16_t m;
    std::memcpy(&m, mu + 2 * p, 2);
    if (m < 1) return set_err(c, PD_EINVAL, "%s: multiplicity below 1", path);
  }
  if (sb.weighted && sb.circ_C > 0.0)
    return set_err(c, PD_EINVAL, "%s: multiplicities with the circuit", path);
  // apply: tables, then the device state
  pd_status s = pd_set_species(c, kNS, Z, m);
  if (s) return s;
  if ((s = pd_set_heavy_subcycle(c, h.heavy_every))) return s;
  if ((s = pd_set_emission(c, sb.em_beta, sb.em_rtip, sb.em_phi, sb.em_ratio, sb.em_T))) return s;
  if (sb.circ_C > 0.0 && c->mg_on)
    return set_err(c, PD_EINVAL, "%s: a circuit state for an iterative Poisson solve", path);
  // (the saved device counters below carry the circuit's anode charge)
  c->g.circ_V0 = sb.circ_V0;
  c->g.circ_R = sb.circ_R;
  c->g.circ_C = sb.circ_C;
  c->cpar.split_literal = sb.split_literal ? 1 : 0;
  c->g.sput_on = sb.sput_on ? 1 : 0;
  for (int k = 0; k < kNC; ++k)
    if (xset[k] && (s = pd_set_cross_section(c, k, xthr[k], xn[k], xdsq[k], xsig[k]))) return s;
  if (sn > 0) {
    std::vector<double> a[5];
    for (int k = 0; k < 5; ++k) {
      a[k].resize((size_t)soff[sn]);
      std::memcpy(a[k].data(), sarr[k], 8 * a[k].size());
    }
    if ((s = pd_schedule_injection(c, (int)sn, soff.data(), a[0].data(), a[1].data(),
                                   a[2].data(), a[3].data(), a[4].data(), sarr[5])))
      return s;
  } else if ((s = pd_schedule_injection(c, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                                        nullptr, nullptr))) {
    return s;
  }
  if (sb.weighted && (s = pd_set_weighted(c, 1))) return s;
  if ((s = sync(c))) return s;
  void* dx = c->fp32 ? (void*)c->Af.x : (void*)c->A.x;
  void* dv = c->fp32 ? (void*)c->Af.v : (void*)c->A.v;
  uint32_t* dkey = c->fp32 ? c->Af.key : c->A.key;
  auto up = [&](void* dst, const void* src, size_t bytes) -> pd_status {
    if (bytes) HIPCHK(c, hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return PD_OK;
  };
  if ((s = up(dx, xrec, xsz * n)) || (s = up(dv, vrec, vsz * n)) || (s = up(dkey, key, 4 * n)) ||
      (s = up(c->sw.skey, skey, 4 * (size_t)st.n_alive)) ||
      (s = up(c->off, off, 4 * ((size_t)c->g.sentinel + 1))) || (s = up(c->fw.Q, Q, 8 * nn)) ||
      (s = up(c->fw.phi, phi, 8 * nn)) || (s = up(c->fw.Er, Er, 8 * nn)) ||
      (s = up(c->fw.Ez, Ez, 8 * nn)) ||
      (s = up(c->sput, sput, sizeof(unsigned long long) * ((size_t)c->g.nr + 1))) ||
      (s = up(c->st, &st, sizeof st)) ||
      (s = up(c->mg.sc, sc, sizeof(MGScal))))
    return s;
  if (c->weighted) {
    // a file without multiplicities: every record stands for W
    std::vector<uint16_t> m(n, (uint16_t)1);
    if (mu) std::memcpy(m.data(), mu, 2 * n);
    if ((s = up(c->A.mu, m.data(), 2 * n))) return s;
  }
  for (int k = 0; k < kNS; ++k) c->injected[k] = hh.injected[k];
  c->host_step = hh.host_step;
  c->host_sched_pos = hh.host_sched_pos;
  c->p_solves = hh.p_solves;
  c->p_fallbacks = hh.p_fallbacks;
  c->mg_inner = hh.mg_inner;
  if (c->fp32) {
    // the FP32 copies of the field follow the FP64 field
    field(c->g, c->fw, c->stream);
    HIPCHK(c, hipGetLastError());
  }
  return sync(c);
}

pd_status pd_poisson_noalloc(pd_ctx* c, const int64_t* Q, double* phi, void* stream) {
  if (!c) return PD_EINVAL;
  if (c->poisoned) return set_err(c, PD_ESTATE, "context unusable after an earlier error");
  if (!Q || !phi) return set_err(c, PD_EINVAL, "Q or phi is NULL");
  if (c->spectral)
    return set_err(c, PD_EINVAL, "the context has no fixed-order solve (created with PD_POISSON_SPECTRAL)");
  const size_t words = (size_t)3 * (size_t)(c->g.nz - 1) * (size_t)(c->g.nr + 1);
  if (words > kScratchWords)
    return set_err(c, PD_EINVAL, "grid %dx%d needs %zu scratch words, more than the %zu held",
                   c->g.nr, c->g.nz, words, kScratchWords);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device)
    return set_err(c, PD_EDEVICE, "current device %d is not the context's device %d", dev,
                   c->device);
  double* sp;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    sp = g_scratch_ptr[dev];
  }
  if (!sp) return set_err(c, PD_EDEVICE, "no scratch address for device %d", dev);
  const size_t part = (size_t)(c->g.nz - 1) * (size_t)(c->g.nr + 1);
  FieldWork fw = c->fw;
  fw.Q = const_cast<int64_t*>(Q);
  fw.phi = phi;
  fw.f = sp;
  fw.fh = sp + part;
  fw.g = sp + 2 * part;
  poisson_direct(c->g, fw, stream ? (hipStream_t)stream : c->stream);
  HIPCHK(c, hipGetLastError());
  return PD_OK;
}

pd_status pd_ensemble_create(int32_t n, pd_ctx* const* members, int32_t nstreams,
                             pd_ensemble** out) {
  if (!out || n < 1 || !members || nstreams < 1) return PD_EINVAL;
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    pd_ctx* c = members[i];
    if (!c || c->poisoned || !c->species_set || c->mg_on || c->opts.timing) {
      g_ens_err = "member %d: missing, unusable, iterative Poisson solver or timing on";
      g_ens_err.replace(g_ens_err.find("%d"), 2, std::to_string(i));
      return PD_EINVAL;
    }
    if (!c->opts.collisions_off)
      for (int k = 0; k <= PD_SI2; ++k)
        if (!c->xs_set[k]) {
          g_ens_err = "member " + std::to_string(i) + ": cross section not set";
          return PD_ESTATE;
        }
    for (int j = 0; j < i; ++j)
      if (members[j] == c) {
        g_ens_err = "a context appears twice";
        return PD_EINVAL;
      }
  }
  pd_ensemble* e = new (std::nothrow) pd_ensemble();
  if (!e) return PD_ENOMEM;
  e->m.assign(members, members + n);
  auto fail = [&](pd_status st, const char* msg) {
    g_ens_err = msg;
    pd_ensemble_destroy(e);
    return st;
  };
  for (pd_ctx* c : e->m)
    if (sync(c)) return fail(PD_EDEVICE, "member stream");
  const int K = std::min(nstreams, n);
  if (hipStreamCreate(&e->s0) != hipSuccess) return fail(PD_EDEVICE, "stream");
  e->ws.assign(K, nullptr);
  e->ev.assign(K + 2, nullptr);
  for (int k = 0; k < K; ++k)
    if (hipStreamCreate(&e->ws[k]) != hipSuccess) return fail(PD_EDEVICE, "stream");
  for (auto& v : e->ev)
    if (hipEventCreateWithFlags(&v, hipEventDisableTiming) != hipSuccess)
      return fail(PD_EDEVICE, "event");
  // capture two steps of every member, member i on worker stream i % K
  std::vector<hipStream_t> own(n);
  for (int i = 0; i < n; ++i) own[i] = e->m[i]->stream;
  bool ok = hipStreamBeginCapture(e->s0, hipStreamCaptureModeRelaxed) == hipSuccess &&
            hipEventRecord(e->ev[K], e->s0) == hipSuccess;
  for (int k = 0; ok && k < K; ++k) ok = hipStreamWaitEvent(e->ws[k], e->ev[K], 0) == hipSuccess;
  auto nomark = [](bool = false) {};
  for (int i = 0; ok && i < n; ++i) {
    pd_ctx* c = e->m[i];
    c->stream = e->ws[i % K];
    const int64_t nn = (int64_t)(c->g.nr + 1) * (c->g.nz + 1);
    for (int t = 0; ok && t < 2; ++t) {
      const pd_status ps = c->fp32 ? enqueue_step(c, c->Af, c->Bf, nn, nomark)
                                   : enqueue_step(c, c->A, c->B, nn, nomark);
      ok = ps == PD_OK && hipGetLastError() == hipSuccess;
    }
  }
  for (int k = 0; ok && k < K; ++k)
    ok = hipEventRecord(e->ev[k], e->ws[k]) == hipSuccess &&
         hipStreamWaitEvent(e->s0, e->ev[k], 0) == hipSuccess;
  hipGraph_t g = nullptr;
  const bool ended = hipStreamEndCapture(e->s0, &g) == hipSuccess;
  for (int i = 0; i < n; ++i) {
    e->m[i]->stream = own[i];
    e->m[i]->p_solves -= 2;  // counted at replay
  }
  e->graph = g;
  if (!ok || !ended || !g) return fail(PD_EDEVICE, "graph capture failed");
  if (hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0) != hipSuccess)
    return fail(PD_EDEVICE, "graph instantiation failed");
  for (pd_ctx* c : e->m) c->in_ensemble += 1;
  e->owns = true;
  *out = e;
  return PD_OK;
}

pd_status pd_ensemble_step(pd_ensemble* e, int32_t nsteps) {
  if (!e) return PD_EINVAL;
  if (nsteps < 0 || nsteps % 2) {
    e->err = "nsteps must be even and >= 0";
    return PD_EINVAL;
  }
  const int K = (int)e->ws.size();
  // order after each member's own pending work
  for (pd_ctx* c : e->m) {
    if (c->poisoned) {
      e->err = "a member is unusable";
      return PD_ESTATE;
    }
    if (hipEventRecord(e->ev[K + 1], c->stream) != hipSuccess ||
        hipStreamWaitEvent(e->s0, e->ev[K + 1], 0) != hipSuccess) {
      e->err = "event";
      return PD_EDEVICE;
    }
  }
  for (int t = 0; t < nsteps; t += 2) {
    if (hipGraphLaunch(e->exec, e->s0) != hipSuccess) {
      e->err = "graph launch failed";
      for (pd_ctx* c : e->m) c->poisoned = true;
      return PD_EDEVICE;
    }
    for (pd_ctx* c : e->m) {
      host_after_step(c);
      host_after_step(c);
      c->p_solves += 2;
    }
  }
  // each member's later work waits for the ensemble's
  if (hipEventRecord(e->ev[K + 1], e->s0) != hipSuccess) return PD_EDEVICE;
  for (pd_ctx* c : e->m)
    if (hipStreamWaitEvent(c->stream, e->ev[K + 1], 0) != hipSuccess) return PD_EDEVICE;
  return PD_OK;
}

pd_status pd_ensemble_synchronize(pd_ensemble* e) {
  if (!e) return PD_EINVAL;
  if (hipStreamSynchronize(e->s0) != hipSuccess) {
    e->err = "device error";
    return PD_EDEVICE;
  }
  for (pd_ctx* c : e->m) {
    pd_status s = pd_synchronize(c);
    if (s) {
      e->err = c->err;
      return s;
    }
  }
  return PD_OK;
}

const char* pd_ensemble_last_error(const pd_ensemble* e) {
  return e ? e->err.c_str() : g_ens_err.c_str();
}

void pd_ensemble_destroy(pd_ensemble* e) {
  if (!e) return;
  if (e->s0) (void)hipStreamSynchronize(e->s0);
  if (e->owns)
    for (pd_ctx* c : e->m) c->in_ensemble -= 1;
  if (e->exec) (void)hipGraphExecDestroy(e->exec);
  if (e->graph) (void)hipGraphDestroy(e->graph);
  for (auto v : e->ev)
    if (v) (void)hipEventDestroy(v);
  for (auto st : e->ws)
    if (st) (void)hipStreamDestroy(st);
  if (e->s0) (void)hipStreamDestroy(e->s0);
  delete e;
}

pd_status pd_unet_create(int32_t nr, int32_t nz, int32_t levels, int32_t base, int32_t batch,
                         int64_t dataset_capacity, pd_unet** out) {
  if (!out) return PD_EINVAL;
  *out = nullptr;
  pd_unet* n = new (std::nothrow) pd_unet();
  if (!n) return PD_ENOMEM;
  std::string err;
  n->u = unet_create(nr, nz, levels, base, batch, dataset_capacity, err);
  if (!n->u) {
    g_unet_err = err;
    delete n;
    return err.find("alloc") != std::string::npos ? PD_ENOMEM : PD_EINVAL;
  }
  if (hipStreamCreate(&n->stream) != hipSuccess) {
    unet_destroy(n->u);
    delete n;
    g_unet_err = "stream";
    return PD_EDEVICE;
  }
  std::vector<float> zero((size_t)unet_nparams(n->u), 0.f);
  unet_set_weights(n->u, zero.data(), n->stream);
  *out = n;
  return PD_OK;
}

pd_status pd_unet_info(const pd_unet* n, int64_t* np, int32_t* H, int32_t* W) {
  if (!n) return PD_EINVAL;
  if (np) *np = unet_nparams(n->u);
  if (H) *H = unet_height(n->u);
  if (W) *W = unet_width(n->u);
  return PD_OK;
}

pd_status pd_unet_set_weights(pd_unet* n, const float* w) {
  if (!n || !w) return PD_EINVAL;
  const int64_t np = unet_nparams(n->u);
  for (int64_t k = 0; k < np; ++k)
    if (!std::isfinite(w[k])) {
      n->err = "non-finite weight";
      return PD_EINVAL;
    }
  if (unet_set_weights(n->u, w, n->stream)) {
    n->err = "device error";
    return PD_EDEVICE;
  }
  return PD_OK;
}

pd_status pd_unet_get_weights(const pd_unet* n, float* w) {
  if (!n || !w) return PD_EINVAL;
  return unet_get_weights(n->u, w) ? PD_EDEVICE : PD_OK;
}

pd_status pd_unet_forward(pd_unet* n, int32_t k, const float* x, float* out) {
  if (!n || !x || !out || k < 1) return PD_EINVAL;
  if (unet_forward_host(n->u, k, x, out, n->stream)) {
    n->err = "batch too large or device error";
    return PD_EINVAL;
  }
  return PD_OK;
}

pd_status pd_unet_gradient(pd_unet* n, int32_t k, const float* x, const float* dout, float* dw) {
  if (!n || !x || !dout || !dw || k < 1) return PD_EINVAL;
  if (unet_gradient_host(n->u, k, x, dout, dw, n->stream)) {
    n->err = "batch too large or device error";
    return PD_EINVAL;
  }
  return PD_OK;
}

pd_status pd_unet_add_sample(pd_unet* n, pd_ctx* c) {
  if (!n || !c) return PD_EINVAL;
  pd_status s = sync(c);
  if (s) return s;
  const int rc = unet_add_sample(n->u, c->mg.op, c->fw.phi, c->fw.Q, c->dom.V_cathode, c->stream);
  if (rc == -1) {
    n->err = "training set full";
    return PD_ECAPACITY;
  }
  if (rc) {
    n->err = "grid of the context differs from the network's";
    return PD_EINVAL;
  }
  return sync(c);
}

pd_status pd_unet_train(pd_unet* n, int32_t epochs, int32_t batch, double lr, uint64_t seed,
                        double* loss) {
  if (!n || epochs < 1 || batch < 1 || !(lr > 0)) return PD_EINVAL;
  if (unet_train(n->u, epochs, batch, lr, seed, loss, n->stream)) {
    n->err = "empty training set, batch too large, or device error";
    return PD_EINVAL;
  }
  return PD_OK;
}

pd_status pd_set_unet(pd_ctx* c, pd_unet* n) {
  if (!c) return PD_EINVAL;
  if (n && !c->learned) return set_err(c, PD_ESTATE, "context not created with PD_POISSON_LEARNED");
  if (n && (unet_height(n->u) < c->g.nz + 1 || unet_width(n->u) < c->g.nr + 1))
    return set_err(c, PD_EINVAL, "network grid smaller than the context's");
  pd_status s = sync(c);
  if (s) return s;
  if (n && hipStreamSynchronize(n->stream) != hipSuccess) return set_err(c, PD_EDEVICE, "network");
  c->net = n;
  return PD_OK;
}

const char* pd_unet_last_error(const pd_unet* n) { return n ? n->err.c_str() : g_unet_err.c_str(); }

void pd_unet_destroy(pd_unet* n) {
  if (!n) return;
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  unet_destroy(n->u);
  if (n->stream) (void)hipStreamDestroy(n->stream);
  delete n;
}

pd_status pd_set_timing(pd_ctx* c, int on) {
  if (!c) return PD_EINVAL;
  if (c->in_ensemble) return set_err(c, PD_ESTATE, "context belongs to an ensemble");
  c->opts.timing = on ? 1 : 0;
  if (on) c->timing_used = true;
  return PD_OK;
}

pd_status pd_get_timing(pd_ctx* c, double* ms, int64_t* steps, int reset) {
  if (!c) return PD_EINVAL;
  if (!c->opts.timing && !c->timing_used)
    return set_err(c, PD_ESTATE, "timing was not enabled");
  pd_status s = sync(c);
  if (s) return s;
  harvest_timing(c);
  if (ms)
    for (int k = 0; k < PD_NTIMERS; ++k) ms[k] = c->t_ms[k];
  if (steps) *steps = c->t_steps;
  if (reset) {
    for (int k = 0; k < PD_NTIMERS; ++k) c->t_ms[k] = 0.0;
    c->t_steps = 0;
  }
  return PD_OK;
}

const char* pd_last_error(const pd_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

void pd_destroy(pd_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  // the pending steps' events go back to the pool once each (their null
  // entries repeat the boundary before them)
  harvest_timing(c);
  for (auto e : c->ev_pool)
    if (e) (void)hipEventDestroy(e);
  for (void* p : c->sched_allocs) (void)hipFree(p);
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->h_sc) (void)hipHostFree(c->h_sc);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

}  // extern "C"
