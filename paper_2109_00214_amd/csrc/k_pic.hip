// k_pic.hip -- particle-in-cell part of the step (paper Sec. 2.1):
// fixed-point cloud-in-cell deposit (Eqs. 9-10), the cylindrical Poisson
// solve (Eq. 8) by a sine transform in z and tridiagonal solves in r, the
// nodal field E = -grad(phi), gather + leapfrog push in 2D3V, absorption,
// injection, and the snapshot reductions.
#include "pd_internal.h"

namespace pd {

static inline int grid_for(int64_t n, int block = 256) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (int)g;
}

// ---------------------------------------------------------------------------
// deposit on its own (no collisions this step); with collisions the same
// blocks run inside the decisions' launch
template <typename T>
__global__ void __launch_bounds__(256) k_deposit(Flow<T> f, const uint32_t* __restrict__ off,
                                                 Grid g, SpeciesParams spp,
                                                 unsigned long long* Q) {
  deposit_blocks<T>(f, off, g, spp, Q, blockIdx.x, gridDim.x);
}

__global__ void k_fill_i64(int64_t* p, int64_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s) {
  k_fill_i64<<<grid_for(n), 256, 0, s>>>(p, v, n);
}
void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  k_fill_u32<<<grid_for(n), 256, 0, s>>>(p, v, n);
}

template <typename T>
void deposit(const Flow<T>& f, const uint32_t* off, const Grid& g, const SpeciesParams& sp,
             int64_t* Q, int64_t cap, hipStream_t s) {
  // Q was cleared by the offsets launch
  k_deposit<T><<<grid_for(cap), 256, 0, s>>>(f, off, g, sp, (unsigned long long*)Q);
}
template void deposit<double>(const Flow<double>&, const uint32_t*, const Grid&,
                              const SpeciesParams&, int64_t*, int64_t, hipStream_t);
template void deposit<float>(const Flow<float>&, const uint32_t*, const Grid&,
                             const SpeciesParams&, int64_t*, int64_t, hipStream_t);

// E = -grad(phi): central differences, second-order one-sided at the
// electrodes, E_r = 0 on the axis and at the wall; FP32 copies for the FP32
// push when Erf is not NULL
// (blocks blk = 0 .. nblk-1 of a 256-thread launch share the nodes)
__device__ inline void field_nodes(const double* phi, int nr, int nz, double dr, double dz,
                                   double* Er, double* Ez, float* Erf, float* Ezf, int blk,
                                   int nblk) {
  const int W = nr + 1;
  const int n = (nz + 1) * W;
  const double tdz = 2.0 * dz, tdr = 2.0 * dr;
  for (int b = blk * blockDim.x + threadIdx.x; b < n; b += nblk * blockDim.x) {
    const int j = b / W, i = b % W;
    double ez;
    if (j == 0) ez = (((3.0 * phi[b]) - (4.0 * phi[b + W])) + phi[b + 2 * W]) / tdz;
    else if (j == nz) ez = (((4.0 * phi[b - W]) - (3.0 * phi[b])) - phi[b - 2 * W]) / tdz;
    else ez = (phi[b - W] - phi[b + W]) / tdz;
    const double er = (i == 0 || i == nr) ? 0.0 : (phi[b - 1] - phi[b + 1]) / tdr;
    Ez[b] = ez;
    Er[b] = er;
    if (Erf) {
      Ezf[b] = (float)ez;
      Erf[b] = (float)er;
    }
  }
}

__global__ void __launch_bounds__(256) k_field(const double* phi, int nr, int nz, double dr,
                                               double dz, double* Er, double* Ez, float* Erf,
                                               float* Ezf) {
  field_nodes(phi, nr, nz, dr, dz, Er, Ez, Erf, Ezf, blockIdx.x, gridDim.x);
}

void field(const Grid& g, FieldWork& fw, hipStream_t s) {
  const int64_t n = (int64_t)(g.nr + 1) * (g.nz + 1);
  k_field<<<grid_for(n), 256, 0, s>>>(fw.phi, g.nr, g.nz, g.dr, g.dz, fw.Er, fw.Ez, fw.Erf,
                                      fw.Ezf);
}

// ---------------------------------------------------------------------------
// wave-aggregated absorbed counters: one atomic per (boundary, species) per wave
__device__ inline void count_codes(int code, unsigned long long* ctr) {
  const int lane = threadIdx.x & 63;
  uint64_t pending = __ballot(code >= 0);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int c = __shfl(code, leader, 64);
    const uint64_t m = __ballot(code == c);
    if (lane == leader) atomicAdd(&ctr[c], (unsigned long long)__popcll(m));
    pending &= ~m;
  }
}


// ---------------------------------------------------------------------------
// this step's scheduled particles, appended after the pushed ones (the slots
// after alive + created, which the push does not touch), as extra blocks of
// the field's launch, followed by the particles the cathode emits; the
// push's first thread then rolls the step counters.  Both read the same
// counters (no launch between them changes them; the emitted counts come
// from the injection launch's first block), so they take the same decision;
// the roll leaves n_created to the next collisions, which set it.
struct InjectPlan {
  uint32_t pos, cnt, base, id0;
  uint32_t ne, nn;  // emitted electrons and atoms, after the cnt scheduled ones
  uint32_t ns;      // sputtered atoms, after those
  int64_t a;        // first schedule entry
  bool have, fits;
};

__device__ inline InjectPlan inject_plan(const DevState* st, const Schedule& sc, uint32_t cap,
                                         uint32_t ne, uint32_t nn, uint32_t ns) {
  InjectPlan ip;
  ip.pos = st->sched_pos;
  ip.have = sc.off && ip.pos < st->sched_n;
  ip.a = ip.have ? sc.off[ip.pos] : 0;
  ip.cnt = ip.have ? (uint32_t)(sc.off[ip.pos + 1] - ip.a) : 0u;
  ip.ne = ne;
  ip.nn = nn;
  ip.ns = ns;
  ip.base = st->n_alive + st->n_created;
  ip.id0 = st->next_id + st->n_created;
  const uint64_t tot = (uint64_t)ip.cnt + ne + nn + ns;
  ip.fits = (uint64_t)ip.base + tot <= cap && (uint64_t)ip.id0 + tot <= 0xFFFFFFFFull;
  if (!ip.fits) ip.cnt = ip.ne = ip.nn = ip.ns = 0;
  return ip;
}

// Cathode emission (paper Sec. 2.3): the annuli of the cathode nodes inside
// the tip, i = 0 .. nring-1 (part of [(i - 1/2) dr, (i + 1/2) dr] below
// r_tip), each with the surface field F_i = beta (-E_z(r_i, 0)) from the
// electrode's one-sided difference of phi (the field stage's expression)
// and the Fowler-Nordheim current J(F_i) a_i, J = (A F^2 / phi_w)
// exp(-B phi_w^(3/2) / F) for F > 0; cum[i] = running sum in ascending i.
constexpr double kFnA = 1.541434e-6;  // A eV V^-2
constexpr double kFnB = 6.830890e9;   // eV^(-3/2) V m^-1
constexpr double kKB = 1.380649e-23;  // J/K
constexpr int kMaxRings = 1024;

// Sputtering (paper Sec. 2.3, yield of Yamamura and Tawara): the published
// fit for Cu on Cu at normal incidence (Z1 = Z2 = 29, M1 = M2 = 63.546 u,
// so alpha* and E_th take their equal-mass values) with the Cu parameters
// U_s = 3.49 eV, Q = 1.30, W = 0.73, s = 2.5:
//   Y(E) = 0.042 (Q alpha* / U_s) S_n(E) / (1 + Gamma k_e eps^0.3)
//          (1 - sqrt(E_th / E))^s for E > E_th = 6.7 U_s, else 0, with
//   eps = 0.03255 / (Z1 Z2 sqrt(Z1^(2/3) + Z2^(2/3))) M2 / (M1 + M2) E,
//   S_n = 84.78 Z1 Z2 / sqrt(Z1^(2/3) + Z2^(2/3)) M1 / (M1 + M2) s_n(eps),
//   s_n(eps) = 0.5 ln(1 + 1.2288 eps) / (eps + 0.1728 sqrt(eps) + 0.008 eps^0.1504),
//   k_e = 0.079 (M1 + M2)^(3/2) / (M1^(3/2) M2^(1/2)) Z1^(2/3) Z2^(1/2) / (Z1^(2/3) + Z2^(2/3))^(3/4),
//   Gamma = W / (1 + (M1 / 7)^3).
constexpr double kYtUs = 3.49, kYtQ = 1.30, kYtW = 0.73, kYtS = 2.5, kYtEmax = 1000.0;
constexpr int kMaxSputRings = 4096;

__device__ inline double sputter_yield(double E) {
  const double Z = 29.0, M = 63.546;
  const double z23 = pow(Z, 2.0 / 3.0);
  const double zs = z23 + z23;
  const double eps = ((0.03255 / ((Z * Z) * sqrt(zs))) * (M / (M + M))) * E;
  const double sn = (0.5 * log(1.0 + (1.2288 * eps))) /
                    ((eps + (0.1728 * sqrt(eps))) + (0.008 * pow(eps, 0.1504)));
  const double Sn = (((84.78 * (Z * Z)) / sqrt(zs)) * (M / (M + M))) * sn;
  const double ke = ((0.079 * pow(M + M, 1.5)) / (pow(M, 1.5) * sqrt(M))) *
                    ((z23 * sqrt(Z)) / pow(zs, 0.75));
  const double gam = kYtW / (1.0 + pow(M / 7.0, 3.0));
  const double alpha = (0.249 * pow(M / M, 0.56)) + (0.0035 * pow(M / M, 1.5));
  const double Eth = 6.7 * kYtUs;
  if (!(E > Eth)) return 0.0;
  return (((0.042 * ((kYtQ * alpha) / kYtUs)) * Sn) / (1.0 + ((gam * ke) * pow(eps, 0.3)))) *
         pow(1.0 - sqrt(Eth / E), kYtS);
}

__device__ inline void ring_bounds(const Grid& g, int i, double& lo, double& hi) {
  lo = ((double)i - 0.5) * g.dr;
  hi = ((double)i + 0.5) * g.dr;
  if (lo < 0.0) lo = 0.0;
  if (hi > g.em_rtip) hi = g.em_rtip;
}

__device__ inline double emission_rings(const double* phi, const Grid& g, int nring, double* cum) {
  const int W = g.nr + 1;
  const double tdz = 2.0 * g.dz;
  double I = 0.0;
  for (int i = 0; i < nring; ++i) {
    double lo, hi;
    ring_bounds(g, i, lo, hi);
    double c = 0.0;
    if (hi > lo) {
      const double ez = (((3.0 * phi[i]) - (4.0 * phi[i + W])) + phi[i + 2 * W]) / tdz;
      const double F = (-ez) * g.em_beta;
      if (F > 0.0) {
        const double J = ((kFnA * (F * F)) / g.em_phi) *
                         exp(-((kFnB * (g.em_phi * sqrt(g.em_phi))) / F));
        c = J * (kPI * ((hi * hi) - (lo * lo)));
      }
    }
    I = I + c;
    cum[i] = I;
  }
  return I;
}

// super-particles this step: floor(I dt / (e W) + carry) electrons and
// floor(ratio I dt / (e W) + carry') atoms; the fractions carry over
__device__ inline void emission_counts(const DevState* st, const Grid& g, double I, uint32_t n[2],
                                       double acc[2]) {
  const double x[2] = {((I * g.dt) / (kQE * g.W)) + st->em_acc[0],
                       (((g.em_ratio * I) * g.dt) / (kQE * g.W)) + st->em_acc[1]};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double f = floor(x[k]);
    acc[k] = x[k] - f;
    n[k] = f < 4.0e9 ? (uint32_t)f : 0xF0000000u;  // beyond any capacity: the guard refuses it
  }
}

template <typename T, bool BND>
__device__ inline void inject_records(const PartsT<T>& P, const DevState* st, const Grid& g,
                                      const Schedule& sc, const InjectPlan& ip, const double* cum,
                                      int nring, double I, const uint32_t* spre, int nsr,
                                      uint32_t blk, uint32_t nblk) {
  const uint32_t tot = ip.cnt + ip.ne + ip.nn + ip.ns;
  const uint32_t q_sput = ip.cnt + ip.ne + ip.nn;
  for (uint32_t q = blk * blockDim.x + threadIdx.x; q < tot; q += nblk * blockDim.x) {
    const uint32_t d = ip.base + q, id = ip.id0 + q;
    T r, z;
    RecT<T> v;
    uint32_t s;
    if (BND && q >= q_sput) {
      // sputtered: the annulus whose whole atoms this is (spre: inclusive
      // running counts), radius uniform in area in it, on the cathode,
      // normal to it with a Thompson energy truncated at kYtEmax (purpose 6)
      const uint32_t k = q - q_sput;
      int lo_i = 0, hi_i = nsr - 1;  // first annulus with k < spre[i]
      while (lo_i < hi_i) {
        const int mid = (lo_i + hi_i) >> 1;
        if (k < spre[mid]) hi_i = mid;
        else lo_i = mid + 1;
      }
      uint32_t w[4];
      philox(id, 0u, st->step, 6u << 24, g.seed_lo, g.seed_hi, w);
      const double u2 = u53(w[0], w[1]), u3 = u53(w[2], w[3]);
      double lo = ((double)lo_i - 0.5) * g.dr, hi = ((double)lo_i + 0.5) * g.dr;
      if (lo < 0.0) lo = 0.0;
      if (hi > g.R) hi = g.R;
      double rr = sqrt((lo * lo) + (u2 * ((hi * hi) - (lo * lo))));
      if (!(rr < g.R)) rr = lo;
      const double Fmax = (kYtEmax / (kYtEmax + kYtUs)) * (kYtEmax / (kYtEmax + kYtUs));
      const double qq = sqrt(u3 * Fmax);
      const double E = (kYtUs * qq) / (1.0 - qq);
      r = (T)rr;
      z = (T)0.0;
      s = 1u;
      v = RecT<T>{(T)0.0, (T)0.0, (T)sqrt(((2.0 * E) * kQE) / g.em_mass), id, s};
    } else if (!BND || q < ip.cnt) {
      const int64_t src = ip.a + q;
      r = (T)sc.r[src];
      z = (T)sc.z[src];
      s = sc.sp[src];
      v = RecT<T>{(T)sc.vr[src], (T)sc.vt[src], (T)sc.vz[src], id, s};
    } else {
      // emitted: annulus by u1 I against the running sums, radius uniform in
      // area in it, on the cathode; an electron at rest, an atom with the
      // normal speed of a flux-Maxwellian at em_T (purpose 5 draws)
      const bool electron = q < ip.cnt + ip.ne;
      uint32_t w[4];
      philox(id, 0u, st->step, 5u << 24, g.seed_lo, g.seed_hi, w);
      const double u1 = u53(w[0], w[1]), u2 = u53(w[2], w[3]);
      const double target = u1 * I;
      int ring = -1;
      for (int i = 0; i < nring; ++i)
        if (target < cum[i]) {
          ring = i;
          break;
        }
      if (ring < 0)
        for (int i = nring - 1; i >= 0; --i)
          if (cum[i] > (i > 0 ? cum[i - 1] : 0.0)) {
            ring = i;
            break;
          }
      double lo, hi;
      ring_bounds(g, ring, lo, hi);
      r = (T)sqrt((lo * lo) + (u2 * ((hi * hi) - (lo * lo))));
      z = (T)0.0;
      double vz = 0.0;
      if (!electron) {
        philox(id, 0u, st->step, (5u << 24) | 1u, g.seed_lo, g.seed_hi, w);
        const double u3 = u53(w[0], w[1]);
        vz = sqrt((((2.0 * kKB) * g.em_T) / g.em_mass) * (-log(1.0 - u3)));
      }
      s = electron ? 0u : 1u;
      v = RecT<T>{(T)0.0, (T)0.0, (T)vz, id, s};
    }
    P.x[d] = PosT<T>{r, z};
    P.v[d] = v;
    if (P.mu) P.mu[d] = 1u;  // scheduled, emitted and sputtered particles stand for W
    int i, j;
    T fr, fz;
    cell_of<T>(g, r, z, i, j, fr, fz);
    P.key[d] = key_class(s) * g.C + (uint32_t)(j * g.nr + i);
  }
}

// (one thread) the arrays now hold alive + created + injected + emitted
__device__ inline void roll_counters(DevState* st, const InjectPlan& ip) {
  if (!ip.fits) atomicOr(&st->err, 1u);
  if (ip.have) st->sched_pos = ip.pos + 1;
  const uint32_t tot = ip.cnt + ip.ne + ip.nn + ip.ns;
  if (ip.fits) {
    st->em_acc[0] = st->em_acc_next[0];
    st->em_acc[1] = st->em_acc_next[1];
    st->emitted[0] += ip.ne;
    st->emitted[1] += ip.nn;
    st->sputtered += ip.ns;
  }
  st->created += st->n_created;
  st->pushed += st->n_alive + st->n_created;
  st->n_total = ip.base + tot;
  st->next_id = ip.id0 + tot;
  st->step += 1;
}

// The external circuit (paper Sec. 2.3), one thread, before this step's
// push: V <- V + (dt / C)((V0 - V) / R - I), I = -(Delta sum Z absorbed at
// the anode since the last update) e W / dt; the next Poisson solve uses V.
__device__ inline void circuit_update(DevState* st, const Grid& g, const SpeciesParams& spp) {
  long long za = 0;
  for (int s = 0; s < kNS; ++s) za += (long long)spp.Z[s] * (long long)st->absorbed[kNS + s];
  const double I = ((-(double)(za - st->circ_zanode)) * (kQE * g.W)) / g.dt;
  st->V_gap = st->V_gap + ((g.dt / g.circ_C) * (((g.circ_V0 - st->V_gap) / g.circ_R) - I));
  st->circ_zanode = za;
}

// (BND: emission or sputtering on: their annuli's sums in dynamic LDS, cum
// then spre; a separate instantiation keeps them out of the plain launch)
template <typename T, bool BND>
__global__ void __launch_bounds__(256) k_field_inject(const double* phi, int nr, int nz, double dr,
                                                      double dz, double* Er, double* Ez,
                                                      float* Erf, float* Ezf, PartsT<T> P,
                                                      DevState* st, Grid g, SpeciesParams spp,
                                                      Schedule sc, uint32_t cap, uint32_t nf,
                                                      int nring) {
  if (blockIdx.x < nf) {
    field_nodes(phi, nr, nz, dr, dz, Er, Ez, Erf, Ezf, blockIdx.x, nf);
    return;
  }
  if (!BND) {
    const InjectPlan ip = inject_plan(st, sc, cap, 0u, 0u, 0u);
    if (blockIdx.x == nf && threadIdx.x == 0) {
      st->em_now[0] = st->em_now[1] = st->em_now[2] = 0u;
      st->em_acc_next[0] = st->em_acc[0];
      st->em_acc_next[1] = st->em_acc[1];
      if (g.circ_C > 0.0) circuit_update(st, g, spp);
    }
    inject_records<T, false>(P, st, g, sc, ip, nullptr, 0, 0.0, nullptr, 0, blockIdx.x - nf,
                             gridDim.x - nf);
    return;
  }
  extern __shared__ double dyn[];
  double* cum = dyn;                                         // [nring]
  uint32_t* spre = (uint32_t*)(dyn + (nring > 0 ? nring : 1));  // [nr + 1] when sputtering
  __shared__ double Ish;
  __shared__ uint32_t wsum[4];
  uint32_t n[2] = {0u, 0u};
  double acc[2] = {0.0, 0.0};
  double I = 0.0;
  if (nring > 0) {
    if (threadIdx.x == 0) Ish = emission_rings(phi, g, nring, cum);
    __syncthreads();
    I = Ish;
    emission_counts(st, g, I, n, acc);
  }
  // sputtered atoms: the whole atoms of every annulus, inclusive running
  // counts in LDS (a block scan over chunks of 256 annuli)
  const int nsr = g.sput_on ? g.nr + 1 : 0;
  uint32_t ns = 0;
  for (int i0 = 0; i0 < nsr; i0 += 256) {
    const int i = i0 + (int)threadIdx.x;
    const uint32_t c = (i < nsr) ? (uint32_t)(g.sput[i] >> 32) : 0u;
    uint32_t tot;
    const uint32_t ex = block_scan256(c, &tot, wsum);
    if (i < nsr) spre[i] = ns + ex + c;
    ns += tot;
  }
  __syncthreads();
  const InjectPlan ip = inject_plan(st, sc, cap, n[0], n[1], ns);
  if (blockIdx.x == nf) {
    if (threadIdx.x == 0) {
      st->em_now[0] = n[0];
      st->em_now[1] = n[1];
      st->em_now[2] = ns;
      st->em_acc_next[0] = acc[0];
      st->em_acc_next[1] = acc[1];
      if (g.circ_C > 0.0) circuit_update(st, g, spp);
    }
    // the atoms taken from every annulus (the push subtracts them; none when
    // the injection does not fit)
    for (int i = (int)threadIdx.x; i < nsr; i += (int)blockDim.x)
      g.sput_take[i] = ip.fits ? spre[i] - (i > 0 ? spre[i - 1] : 0u) : 0u;
  }
  inject_records<T, true>(P, st, g, sc, ip, cum, nring, I, spre, nsr, blockIdx.x - nf,
                          gridDim.x - nf);
}

// emission annuli: those with part of their annulus inside the tip (0: off)
inline int emission_ring_count(const Grid& g) {
  if (!(g.em_beta > 0.0)) return 0;
  int n = 0;
  while (n <= g.nr && ((double)n - 0.5) * g.dr < g.em_rtip) ++n;
  return n < kMaxRings ? n : kMaxRings;
}

template <typename T>
void field_and_inject(const Grid& g, FieldWork& fw, const PartsT<T>& P, DevState* st,
                      const SpeciesParams& spp, const Schedule& sc, int64_t cap, hipStream_t s) {
  const int64_t n = (int64_t)(g.nr + 1) * (g.nz + 1);
  const int nf = grid_for(n), ni = grid_for(sc.off ? sc.max_count : 1);
  const int nring = emission_ring_count(g);
  if (nring > 0 || g.sput_on) {
    const size_t lds = sizeof(double) * (size_t)(nring > 0 ? nring : 1) +
                       (g.sput_on ? sizeof(uint32_t) * (size_t)(g.nr + 1) : 0);
    k_field_inject<T, true><<<nf + ni, 256, lds, s>>>(fw.phi, g.nr, g.nz, g.dr, g.dz, fw.Er,
                                                      fw.Ez, fw.Erf, fw.Ezf, P, st, g, spp, sc,
                                                      (uint32_t)cap, (uint32_t)nf, nring);
  } else {
    k_field_inject<T, false><<<nf + ni, 256, 0, s>>>(fw.phi, g.nr, g.nz, g.dr, g.dz, fw.Er,
                                                     fw.Ez, fw.Erf, fw.Ezf, P, st, g, spp, sc,
                                                     (uint32_t)cap, (uint32_t)nf, 0);
  }
}
template void field_and_inject<double>(const Grid&, FieldWork&, const Parts&, DevState*,
                                       const SpeciesParams&, const Schedule&, int64_t,
                                       hipStream_t);
template void field_and_inject<float>(const Grid&, FieldWork&, const PartsF&, DevState*,
                                      const SpeciesParams&, const Schedule&, int64_t,
                                      hipStream_t);

// gather (bilinear, the deposit's weights) and leapfrog push in the record's
// precision T: v += (q/m) E dt, Cartesian move, rotation back to the r-z
// plane; absorbed particles get the sentinel key, the others their new key
// The record of sorted position p comes from U[perm[p]] (live particles) or
// S[p] (created this step) and goes to S[p], the id and label with it.
// With heavy subcycling the heavy species advance only on heavy steps, with
// their own step; on the other steps their record is moved unchanged and its
// key recomputed (a collision may have changed the label).
// (SPUT: cathode sputtering on; a separate instantiation keeps the yield's
// registers out of the plain push)
template <typename T, bool SPUT>
__global__ void __launch_bounds__(256) k_push(Flow<T> f, DevState* st, Grid g, SpeciesParams spp,
                                              const T* Er, const T* Ez, Schedule sc,
                                              uint32_t cap) {
  const uint32_t n_alive = st->n_alive;
  const uint32_t n = n_alive + st->n_created;
  const bool heavy_now = st->heavy_now != 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0)
    roll_counters(st, inject_plan(st, sc, cap, st->em_now[0], st->em_now[1], st->em_now[2]));
  if (SPUT && blockIdx.x == 0)
    for (int i = (int)threadIdx.x; i <= g.nr; i += (int)blockDim.x) {
      const unsigned long long t = (unsigned long long)g.sput_take[i] << 32;
      if (t) atomicAdd(&g.sput[i], ~t + 1ull);  // minus the atoms taken this step
    }
  const int W = g.nr + 1;
  const bool sub = g.heavy_every > 1;
  const PartsT<T>& D = f.S;
  for (ChunkWalk<64> cw((n + blockDim.x - 1) / blockDim.x); cw.more(); cw.next()) {
    const uint32_t p = cw.chunk() * blockDim.x + threadIdx.x;
    int code = -1;
    if (p < n) {
      const bool old = p < n_alive;
      const uint32_t q = old ? f.perm[p] : p;
      const PartsT<T>& P = old ? f.U : f.S;
      int i, j;
      T fr, fz;
      const PosT<T> x0 = P.x[q];
      const RecT<T> v0 = P.v[q];
      const T r = x0.r, z0 = x0.z;
      cell_of<T>(g, r, z0, i, j, fr, fz);
      const int b = j * W + i;
      const T gr = (T)1 - fr, gz = (T)1 - fz;
      const T w00 = gr * gz, w10 = fr * gz, w01 = gr * fz, w11 = fr * fz;
      const T er = (((w00 * Er[b]) + (w10 * Er[b + 1])) + (w01 * Er[b + W])) + (w11 * Er[b + W + 1]);
      const T ez = (((w00 * Ez[b]) + (w10 * Ez[b + 1])) + (w01 * Ez[b + W])) + (w11 * Ez[b + W + 1]);
      const int s = (int)v0.sp;
      const bool heavy = s != 0;
      T vr = v0.vr, vz = v0.vz, vt = v0.vt;
      T rn = r, z = z0;
      if (!heavy || heavy_now) {
        const bool hs = heavy && sub;
        const T qm = (T)(hs ? spp.qmdt_heavy[s] : spp.qmdt[s]);
        const T dt = (T)(hs ? g.dt_heavy : g.dt);
        vr = vr + (qm * er);
        vz = vz + (qm * ez);
        const T x = r + (vr * dt);
        const T y = vt * dt;
        z = z0 + (vz * dt);
        rn = sqrt((x * x) + (y * y));
        if (rn > (T)0) {
          const T c = x / rn, sn = y / rn;
          const T vr2 = (c * vr) + (sn * vt);
          const T vt2 = (c * vt) - (sn * vr);
          vr = vr2;
          vt = vt2;
        }
      }
      D.x[p] = PosT<T>{rn, z};
      D.v[p] = RecT<T>{vr, vt, vz, v0.id, v0.sp};
      if (D.mu) D.mu[p] = P.mu[q];
      int bnd = -1;
      if (z < (T)0) bnd = 0;
      else if (!(z < (T)g.L)) bnd = 1;
      else if (!(rn < (T)g.R)) bnd = 2;
      if (bnd >= 0) {
        code = bnd * kNS + s;
        D.key[p] = g.sentinel;
        if (SPUT && bnd == 0 && spp.Z[s] > 0) {
          // an ion on the cathode: its yield to the annulus of its nearest node
          const double vrd = (double)vr, vtd = (double)vt, vzd = (double)vz;
          const double v2 = ((vrd * vrd) + (vtd * vtd)) + (vzd * vzd);
          const double E = ((0.5 * spp.m[s]) * v2) / kQE;
          int ring = (int)(((double)rn / g.dr) + 0.5);
          if (ring > g.nr) ring = g.nr;
          const double Y = sputter_yield(E);
          if (Y > 0.0) atomicAdd(&g.sput[ring], (unsigned long long)floor(Y * 4294967296.0));
        }
      } else {
        int i2, j2;
        T a, c;
        cell_of<T>(g, rn, z, i2, j2, a, c);
        D.key[p] = key_class((uint32_t)s) * g.C + (uint32_t)(j2 * g.nr + i2);
      }
    }
    count_codes(code, st->absorbed);
  }
}

template <>
void push<double>(const Flow<double>& f, DevState* st, const Grid& g, const SpeciesParams& sp,
                  const FieldWork& fw, const Schedule& sc, int64_t cap, hipStream_t s) {
  if (g.sput_on)
    k_push<double, true><<<grid_for(cap), 256, 0, s>>>(f, st, g, sp, fw.Er, fw.Ez, sc,
                                                       (uint32_t)cap);
  else
    k_push<double, false><<<grid_for(cap), 256, 0, s>>>(f, st, g, sp, fw.Er, fw.Ez, sc,
                                                        (uint32_t)cap);
}
template <>
void push<float>(const Flow<float>& f, DevState* st, const Grid& g, const SpeciesParams& sp,
                 const FieldWork& fw, const Schedule& sc, int64_t cap, hipStream_t s) {
  if (g.sput_on)
    k_push<float, true><<<grid_for(cap), 256, 0, s>>>(f, st, g, sp, fw.Erf, fw.Ezf, sc,
                                                      (uint32_t)cap);
  else
    k_push<float, false><<<grid_for(cap), 256, 0, s>>>(f, st, g, sp, fw.Erf, fw.Ezf, sc,
                                                       (uint32_t)cap);
}

// host-initiated append of n particles already copied to src
template <typename T>
__global__ void __launch_bounds__(256) k_append(PartsT<T> P, const DevState* st, Grid g,
                                                PartsT<T> src, uint32_t n) {
  const uint32_t base = st->n_total;
  const uint32_t id0 = st->next_id;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const uint32_t d = base + q;
    const PosT<T> x = src.x[q];
    RecT<T> v = src.v[q];
    const T r = x.r, z = x.z;
    const uint32_t s = v.sp;
    v.id = id0 + q;
    P.x[d] = x;
    P.v[d] = v;
    if (P.mu) P.mu[d] = src.mu ? src.mu[q] : (uint16_t)1u;
    int i, j;
    T fr, fz;
    cell_of<T>(g, r, z, i, j, fr, fz);
    P.key[d] = key_class(s) * g.C + (uint32_t)(j * g.nr + i);
  }
}
__global__ void k_append_end(DevState* st, uint32_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->n_total += n;
    st->next_id += n;
  }
}

template <typename T>
void append(const PartsT<T>& P, DevState* st, const Grid& g, const PartsT<T>& src, uint32_t n,
            hipStream_t s) {
  if (n == 0) return;
  k_append<T><<<grid_for(n), 256, 0, s>>>(P, st, g, src, n);
  k_append_end<<<1, 64, 0, s>>>(st, n);
}
template void append<double>(const Parts&, DevState*, const Grid&, const Parts&, uint32_t,
                             hipStream_t);
template void append<float>(const PartsF&, DevState*, const Grid&, const PartsF&, uint32_t,
                            hipStream_t);

// ---------------------------------------------------------------------------
// snapshot: counts and kinetic energy per species (per-block partials, summed
// on the host in block order), Cu2+ spectra by comparison with the edges
template <typename T>
__global__ void __launch_bounds__(256) k_diag(PartsT<T> P, const DevState* st, Grid g,
                                              SpeciesParams spp, const double* edges,
                                              unsigned long long* counts, double* ke,
                                              unsigned long long* spec,
                                              unsigned long long* real) {
  __shared__ unsigned long long sc[kNS], sm[kNS];
  __shared__ double sk[256][kNS];
  const uint32_t n = st->n_total;
  if (threadIdx.x < kNS) sc[threadIdx.x] = sm[threadIdx.x] = 0;
  double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
  __syncthreads();
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    if (P.key[p] == g.sentinel) continue;
    const RecT<T> v = P.v[p];
    const int s = (int)v.sp;
    atomicAdd(&sc[s], 1ull);
    atomicAdd(&sm[s], P.mu ? (unsigned long long)P.mu[p] : 1ull);  // real particles / W
    const double vr = v.vr, vt = v.vt, vz = v.vz;
    const double v2 = ((vr * vr) + (vt * vt)) + (vz * vz);
    acc[s] += (0.5 * spp.m[s]) * v2;
    if (s >= 3 && s <= 5) {  // the Cu2+ labels
      const double e = ((0.5 * spp.m[s]) * v2) / kQE;
      int bin;
      if (e < edges[0]) bin = 64;
      else if (!(e < edges[64])) bin = 65;
      else {
        int lo = 0, hi = 64;  // edges[lo] <= e < edges[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (e < edges[mid]) hi = mid;
          else lo = mid;
        }
        bin = lo;
      }
      atomicAdd(&spec[(s - 3) * 66 + bin], 1ull);
    }
  }
  for (int s = 0; s < kNS; ++s) sk[threadIdx.x][s] = acc[s];
  __syncthreads();
  if (threadIdx.x < kNS) {
    double t = 0.0;
    for (int q = 0; q < 256; ++q) t += sk[q][threadIdx.x];
    ke[blockIdx.x * kNS + threadIdx.x] = t;
    counts[blockIdx.x * kNS + threadIdx.x] = sc[threadIdx.x];
    real[blockIdx.x * kNS + threadIdx.x] = sm[threadIdx.x];
  }
}

template <typename T>
void diag_snapshot(const PartsT<T>& P, const DevState* st, const Grid& g, const SpeciesParams& sp,
                   const double* edges, unsigned long long* counts, double* ke,
                   unsigned long long* spec, unsigned long long* real, hipStream_t s) {
  k_diag<T><<<kDiagBlocks, 256, 0, s>>>(P, st, g, sp, edges, counts, ke, spec, real);
}
template void diag_snapshot<double>(const Parts&, const DevState*, const Grid&,
                                    const SpeciesParams&, const double*, unsigned long long*,
                                    double*, unsigned long long*, unsigned long long*,
                                    hipStream_t);
template void diag_snapshot<float>(const PartsF&, const DevState*, const Grid&,
                                   const SpeciesParams&, const double*, unsigned long long*,
                                   double*, unsigned long long*, unsigned long long*,
                                   hipStream_t);

}  // namespace pd
