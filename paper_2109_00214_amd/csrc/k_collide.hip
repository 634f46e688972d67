// k_collide.hip -- DSMC electron-impact collisions (paper Sec. 2.1-2.2).
//
// One trial per electron per step (Eq. 4 with the exact exponential over
// the summed channels).  Four launches:
//   decide  -- one lane per electron (electrons occupy sorted positions
//              [0, off[C]) because keys are species-major): counter-based
//              Philox draws keyed by particle id, one uniform Cu and one
//              Cu+ target in the electron's cell (with the step-wise chain
//              on, also one Cu2+ of any label and one Cu3+), relative speed, sigma
//              from the sqrt(E) tables, x_k = dt g n_t sigma_k, the test
//              R1 < 1 - exp(-X) and the channel; successful trials claim
//              their target with atomicMin of the sorted position;
//   resolve -- the lowest position wins each target; counts per channel
//              and the number of electrons each winner creates (0/1/2);
//   scan    -- exclusive scan of those counts in sorted order: slots and
//              ids of new electrons are therefore independent of timing;
//   apply   -- Eqs. 5-6 (binary update) with isotropic directions
//              (Eq. 7 with I = 1/(4 pi), Marsaglia's method); ionizing
//              events run the stages of Eqs. 12-15.
// All floating-point expressions are evaluated exactly as written (the
// library is compiled without contraction), so the results are identical
// to any other evaluation of the same binary64 expressions.
#include "pd_internal.h"

namespace pd {

static inline int grid_for(int64_t n, int block = 256) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (int)g;
}

__device__ inline double sigma_of(const CollideParams& cp, int k, double g) {
  const double sq = g * cp.ck[k];
  const double eps = sq * sq;
  if (eps < cp.thr[k]) return 0.0;
  const int n = cp.tabn[k];
  const double* t = cp.tab[k];
  const double x = sq / cp.dsq[k];
  if (x >= (double)(n - 1)) return t[n - 1];
  const int i = (int)x;
  return t[i] + ((x - (double)i) * (t[i + 1] - t[i]));
}

// isotropic unit vector (Marsaglia 1972); counter (id, 0, step, purpose<<24 | d)
__device__ inline void isotropic(const CollideParams& cp, uint32_t id, uint32_t step,
                                 uint32_t purpose, double n[3]) {
  for (uint32_t d = 0; d < 64; ++d) {
    uint32_t w[4];
    philox(id, 0u, step, (purpose << 24) | d, cp.seed_lo, cp.seed_hi, w);
    const double u1 = (2.0 * u53(w[0], w[1])) - 1.0;
    const double u2 = (2.0 * u53(w[2], w[3])) - 1.0;
    const double q = (u1 * u1) + (u2 * u2);
    if (q < 1.0 && q > 0.0) {
      const double t = sqrt(1.0 - q);
      n[0] = (2.0 * u1) * t;
      n[1] = (2.0 * u2) * t;
      n[2] = 1.0 - (2.0 * q);
      return;
    }
  }
  n[0] = 0.0;
  n[1] = 0.0;
  n[2] = 1.0;
}

// The literal construction of Eqs. 16-20 for the last stage of a double
// ionization: v5 = R^-1(theta, phi) R^-1(chi, psi) R(theta, phi) (cos(chi) v),
// theta and phi the polar angles of v (phi = 0 on the z axis), with the
// rotation matrix of Eq. 20; every product and sum as written, in order.
__device__ inline void rotation(double theta, double phi, double Rm[9]) {
  const double ct = cos(theta), st = sin(theta), cf = cos(phi), sf = sin(phi);
  Rm[0] = ct * cf;
  Rm[1] = ct * sf;
  Rm[2] = -st;
  Rm[3] = -sf;
  Rm[4] = cf;
  Rm[5] = 0.0;
  Rm[6] = st * cf;
  Rm[7] = st * sf;
  Rm[8] = ct;
}

__device__ inline void split_literal(const double v[3], double chi, double psi, double v5[3]) {
  const double vm = sqrt(((v[0] * v[0]) + (v[1] * v[1])) + (v[2] * v[2]));
  const double theta = (vm > 0.0) ? acos(v[2] / vm) : 0.0;
  const double vp = sqrt((v[0] * v[0]) + (v[1] * v[1]));
  const double phi = (vp > 0.0) ? atan2(v[1], v[0]) : 0.0;
  const double a = cos(chi);
  const double sv[3] = {a * v[0], a * v[1], a * v[2]};
  double Rt[9], Rc[9], t1[3], t2[3];
  rotation(theta, phi, Rt);
  rotation(chi, psi, Rc);
#pragma unroll
  for (int k = 0; k < 3; ++k)  // Eq. 17: into the local frame
    t1[k] = ((Rt[3 * k] * sv[0]) + (Rt[3 * k + 1] * sv[1])) + (Rt[3 * k + 2] * sv[2]);
#pragma unroll
  for (int k = 0; k < 3; ++k)  // Eq. 18: scatter (the inverse is the transpose)
    t2[k] = ((Rc[k] * t1[0]) + (Rc[3 + k] * t1[1])) + (Rc[6 + k] * t1[2]);
#pragma unroll
  for (int k = 0; k < 3; ++k)  // Eq. 19: back to the laboratory frame
    v5[k] = ((Rt[k] * t2[0]) + (Rt[3 + k] * t2[1])) + (Rt[6 + k] * t2[2]);
}

// binary collision, Eqs. 5-6
__device__ inline void binary(double v1[3], double v2[3], double two_dE_mr, double f1, double f2,
                              const double n[3]) {
  const double u0 = v1[0] - v2[0], u1 = v1[1] - v2[1], u2 = v1[2] - v2[2];
  const double g2 = ((u0 * u0) + (u1 * u1)) + (u2 * u2);
  double gp2 = g2 + two_dE_mr;
  if (gp2 < 0.0) gp2 = 0.0;
  const double gp = sqrt(gp2);
  const double u[3] = {u0, u1, u2};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double du = (gp * n[c]) - u[c];
    v1[c] = v1[c] + (du * f1);
    v2[c] = v2[c] - (du * f2);
  }
}

// Unequal weights (Sec. 2.2 leaves them to the rejection or the merging
// method; this is the rejection reading): an event between records of
// multiplicities mp (projectile) and mt (target) stands for min(mp, mt) real
// collisions.  The side with the smaller multiplicity always takes the
// outcome, the other with probability min/its own, from one draw of the
// projectile (purpose 7, draw 0).  The decision leaves the answer in the
// choice byte: kNoProjectile / kNoTarget mark a side that keeps its state
// (equal multiplicities draw nothing and mark nothing).  A target that takes
// an ionizing outcome is relabelled whole and its electrons carry its
// multiplicity.
constexpr uint32_t kChannelBits = 0x1Fu, kNoProjectile = 0x20u, kNoTarget = 0x40u;
__device__ inline uint32_t side_bits(const CollideParams& cp, uint32_t id, uint32_t step,
                                     uint32_t mp, uint32_t mt) {
  if (mp == mt) return 0u;
  uint32_t w[4];
  philox(id, 0u, step, 7u << 24, cp.seed_lo, cp.seed_hi, w);
  const double u = u53(w[0], w[1]);
  if (mp > mt) return (u < ((double)mt / (double)mp)) ? 0u : kNoProjectile;
  return (u < ((double)mp / (double)mt)) ? 0u : kNoTarget;
}

// electrons a resolved electron event creates, from its choice byte: none
// for no event, a lost one (bit 7) or a target that keeps its state; the
// elastic and Coulomb channels none, double ionization two, the others one
__device__ inline uint32_t created_by(uint32_t c) {
  if (!c || (c & 0x80u) || (c & kNoTarget)) return 0u;
  const int ch = (int)(c & kChannelBits) - 1;
  return (ch == 0 || ch == kCEI || ch == kCEE) ? 0u : (ch == 2 ? 2u : 1u);
}

// the heavy-projectile channels run on this step (a table is set and the
// sort marked a heavy step)
__device__ inline bool heavy_trials(const CollideParams& cp, const DevState* st) {
  return cp.heavy && st->heavy_now != 0u;
}

// (T: precision of the particle record; the collision arithmetic is FP64)
// (indices e, tc, t1 are sorted positions; the records are read in U
// through perm)
// Blocks from ndec on deposit the sorted state's charge into Q instead: the
// decisions are a chain of dependent loads with few electrons, the deposit
// a bandwidth-bound pass over the charged particles, and neither reads what
// the other writes.
template <typename T>
__global__ void __launch_bounds__(256) k_decide(Flow<T> f, const uint32_t* off, const DevState* st,
                                                Grid g, CollideParams cp, uint8_t* choice,
                                                uint32_t* target, uint32_t* claim,
                                                uint32_t* csum, SpeciesParams spp,
                                                unsigned long long* Q, uint32_t ndec) {
  if (blockIdx.x >= ndec) {
    deposit_blocks<T>(f, off, g, spp, Q, blockIdx.x - ndec, gridDim.x - ndec);
    return;
  }
  const PartsT<T>& P = f.U;
  const uint32_t C = g.C;
  const uint32_t n_e = off[C];
  const uint32_t step = st->step;
  // the resolution adds the created electrons of every chunk of 256 electrons
  // into the sum of its group of 32 chunks: clear those sums
  {
    const uint32_t ncs = ((n_e + 255) / 256 + 31) / 32;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ncs; i += ndec * blockDim.x)
      csum[i] = 0u;
  }
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n_e; e += ndec * blockDim.x) {
    const uint32_t cell = f.skey[e];
    const uint32_t pe = f.perm[e];
    const int ci = (int)(cell % (uint32_t)g.nr);
    const uint32_t b_cu = off[C + cell], n_cu = off[C + cell + 1] - b_cu;
    const uint32_t b_c1 = off[2 * C + cell], n_c1 = off[2 * C + cell + 1] - b_c1;
    const RecT<T> ev = P.v[pe];
    const uint32_t id = ev.id;
    uint32_t w[4], t[4];
    philox(id, 0u, step, 0u, cp.seed_lo, cp.seed_hi, w);
    philox(id, 0u, step, 1u << 24, cp.seed_lo, cp.seed_hi, t);
    const double R1 = u53(w[0], w[1]);
    const double R2 = u53(w[2], w[3]);
    const uint32_t tc = b_cu + __umulhi(t[0], n_cu);
    const uint32_t t1 = b_c1 + __umulhi(t[1], n_c1);
    const double evr = ev.vr, evt = ev.vt, evz = ev.vz;
    double x[kNEC] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double Vc = cp.Vcell[ci];
    // the weight the density counts per candidate: the picked target's
    auto wt = [&](uint32_t tpos) {
      return P.mu ? (double)P.mu[f.perm[tpos]] * cp.W : cp.W;
    };
    // Cu target: EL, SI, DI share the pick and the relative speed
    if (n_cu > 0) {
      const RecT<T> tv = P.v[f.perm[tc]];
      const double dvr = evr - (double)tv.vr, dvt = evt - (double)tv.vt,
                   dvz = evz - (double)tv.vz;
      const double gg = sqrt(((dvr * dvr) + (dvt * dvt)) + (dvz * dvz));
      const double dens = ((double)n_cu * wt(tc)) / Vc;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (k == 2 && !cp.enable_di) continue;
        x[k] = ((cp.dt * gg) * dens) * sigma_of(cp, k, gg);
      }
    }
    if (n_c1 > 0) {
      const RecT<T> tv = P.v[f.perm[t1]];
      const double dvr = evr - (double)tv.vr, dvt = evt - (double)tv.vt,
                   dvz = evz - (double)tv.vz;
      const double gg = sqrt(((dvr * dvr) + (dvt * dvt)) + (dvz * dvz));
      const double dens = ((double)n_c1 * wt(t1)) / Vc;
      x[3] = ((cp.dt * gg) * dens) * sigma_of(cp, 3, gg);
      // Coulomb with the same Cu+ (position 6)
      if (cp.coulomb && cp.tabn[kCEI] > 0) x[6] = ((cp.dt * gg) * dens) * sigma_of(cp, kCEI, gg);
    }
    // the step-wise chain on: a Cu2+ target of any label (the labels share
    // one key class) and a Cu3+ target, words 2 and 3 of the same draw
    uint32_t t2 = 0, t3 = 0;
    if (cp.chain) {
#pragma unroll
      for (int c = 3; c <= 4; ++c) {
        const int k = c + 1;  // SI3 on class 3, SI4 on class 4
        const uint32_t bt = off[(uint32_t)c * C + cell], nt = off[(uint32_t)c * C + cell + 1] - bt;
        const uint32_t tp = bt + __umulhi(t[c - 1], nt);
        if (c == 3) t2 = tp;
        else t3 = tp;
        if (nt > 0 && cp.tabn[k] > 0) {
          const RecT<T> tv = P.v[f.perm[tp]];
          const double dvr = evr - (double)tv.vr, dvt = evt - (double)tv.vt,
                       dvz = evz - (double)tv.vz;
          const double gg = sqrt(((dvr * dvr) + (dvt * dvt)) + (dvz * dvz));
          const double dens = ((double)nt * wt(tp)) / Vc;
          x[k] = ((cp.dt * gg) * dens) * sigma_of(cp, k, gg);
        }
      }
    }
    // electron-electron Coulomb (position 7): one of the other electrons of
    // the cell (word 0 of the draw (purpose 1, 1)), never the projectile;
    // every pair is tried from both sides, so half weight
    uint32_t te = 0;
    if (cp.cee) {
      const uint32_t b0 = off[cell], n0 = off[cell + 1] - b0 - 1u;
      if (n0 > 0 && cp.tabn[kCEE] > 0) {
        uint32_t t2w[4];
        philox(id, 0u, step, (1u << 24) | 1u, cp.seed_lo, cp.seed_hi, t2w);
        uint32_t u = __umulhi(t2w[0], n0);
        if (b0 + u >= e) u += 1u;
        te = b0 + u;
        const RecT<T> tv = P.v[f.perm[te]];
        const double dvr = evr - (double)tv.vr, dvt = evt - (double)tv.vt,
                     dvz = evz - (double)tv.vz;
        const double gg = sqrt(((dvr * dvr) + (dvt * dvt)) + (dvz * dvz));
        const double dens = ((double)n0 * wt(te)) / Vc;
        x[7] = 0.5 * (((cp.dt * gg) * dens) * sigma_of(cp, kCEE, gg));
      }
    }
    const double X = ((((((x[0] + x[1]) + x[2]) + x[3]) + x[4]) + x[5]) + x[6]) + x[7];
    const double pc = 1.0 - exp(-X);
    int q = -1;
    if (R1 < pc) {
      const double u = R2 * X;
      double c = 0.0;
#pragma unroll
      for (int k = 0; k < kNEC; ++k) {
        c = c + x[k];
        if (q < 0 && u < c) q = k;
      }
      if (q < 0) {
        for (int k = kNEC - 1; k >= 0; --k)
          if (x[k] > 0.0) {
            q = k;
            break;
          }
      }
    }
    if (q >= 0) {
      const int ch = echannel(q);
      const uint32_t tp = (ch == 3 || ch == kCEI) ? t1
                        : (ch == 4)              ? t2
                        : (ch == 5)              ? t3
                        : (ch == kCEE)           ? te
                                                 : tc;
      const uint32_t side = P.mu ? side_bits(cp, id, step, P.mu[pe], P.mu[f.perm[tp]]) : 0u;
      choice[e] = (uint8_t)((uint32_t)(ch + 1) | side);
      target[e] = tp;
      atomicMin(&claim[tp], e);
      if (cp.cee) atomicMin(&claim[e], e);
    } else {
      choice[e] = 0;
    }
  }
  // Heavy projectiles on heavy steps (Sec. 2.3's ion-neutral charge exchange
  // and neutral-neutral elastic collisions): the Cu range [off[C], off[2C])
  // tries NN against another Cu of its cell (half weight: every pair is tried
  // from both sides), the Cu+ range [off[2C], off[3C]) tries CEX against a Cu;
  // an event claims its target and its projectile.
  if (!heavy_trials(cp, st)) return;
  const uint32_t h0 = off[C], h1 = off[3 * C], h_mid = off[2 * C];
  for (uint32_t p = h0 + blockIdx.x * blockDim.x + threadIdx.x; p < h1; p += ndec * blockDim.x) {
    const bool nn = p < h_mid;
    const int k = nn ? kNN : kCEX;
    choice[p] = 0;
    if (cp.tabn[k] == 0) continue;
    const uint32_t cell = f.skey[p] - (nn ? C : 2 * C);
    const int ci = (int)(cell % (uint32_t)g.nr);
    const uint32_t b = off[C + cell], nt = off[C + cell + 1] - b;
    const uint32_t partners = nn ? nt - 1u : nt;
    if (nt == 0 || partners == 0) continue;
    const RecT<T> pv = P.v[f.perm[p]];
    uint32_t w[4], t[4];
    philox(pv.id, 0u, step, 0u, cp.seed_lo, cp.seed_hi, w);
    philox(pv.id, 0u, step, 1u << 24, cp.seed_lo, cp.seed_hi, t);
    const double R1 = u53(w[0], w[1]);
    uint32_t u = __umulhi(t[0], partners);
    if (nn && b + u >= p) u += 1u;  // never the projectile itself
    const uint32_t tp = b + u;
    const RecT<T> tv = P.v[f.perm[tp]];
    const double dvr = (double)pv.vr - (double)tv.vr, dvt = (double)pv.vt - (double)tv.vt,
                 dvz = (double)pv.vz - (double)tv.vz;
    const double gg = sqrt(((dvr * dvr) + (dvt * dvt)) + (dvz * dvz));
    const double wgt = P.mu ? (double)P.mu[f.perm[tp]] * cp.W : cp.W;
    const double dens = ((double)partners * wgt) / cp.Vcell[ci];
    double x = ((cp.dt_heavy * gg) * dens) * sigma_of(cp, k, gg);
    if (nn) x = 0.5 * x;
    const double pc = 1.0 - exp(-x);
    if (R1 < pc) {
      const uint32_t side =
          P.mu ? side_bits(cp, pv.id, step, P.mu[f.perm[p]], P.mu[f.perm[tp]]) : 0u;
      choice[p] = (uint8_t)((uint32_t)(k + 1) | side);
      target[p] = tp;
      atomicMin(&claim[tp], p);
      atomicMin(&claim[p], p);
    }
  }
}

// Claims are resolved per chunk of 256 electrons: a winner keeps its channel
// and counts the electrons it creates (0, 1 or 2); the chunk's total goes to
// bsum[chunk] and is added to csum[chunk / 32] (integer sums: the same in
// any order), from which the apply takes the created electrons before any
// chunk with one round of loads.  A wave takes one chunk, four consecutive
// electrons per lane: one 32-bit load of their choice bytes and the loads
// of their events issued together, so that a wave keeps four electrons'
// chains of dependent loads in flight; the chunk's total is the wave's sum.
__global__ void __launch_bounds__(256) k_resolve(const uint32_t* off, DevState* st, Grid g,
                                                 CollideParams cp, uint8_t* choice,
                                                 const uint32_t* target, const uint32_t* claim,
                                                 uint32_t* bsum, uint32_t* csum) {
  __shared__ uint32_t tally[1 + kNC];  // conflicts, events per channel: one atomic per block
  const uint32_t n_e = off[g.C];
  const uint32_t nb = (n_e + 255) / 256;
  const int lane = threadIdx.x & 63;
  if (threadIdx.x <= kNC) tally[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t nw = gridDim.x * (blockDim.x / 64);  // waves of the launch
  for (uint32_t b = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); b < nb; b += nw) {
    const uint32_t e0 = b * 256 + 4 * (uint32_t)lane;
    uint32_t cw = 0;
    if (e0 + 4 <= n_e) {
      cw = *(const uint32_t*)(choice + e0);  // e0 is a multiple of 4
    } else {
      for (uint32_t k = 0; k < 4; ++k)
        if (e0 + k < n_e) cw |= (uint32_t)choice[e0 + k] << (8 * k);
    }
    uint32_t cnt = 0;
    if (cw) {
      uint32_t tp[4], ct[4], cs[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) tp[k] = ((cw >> (8 * k)) & 0xFFu) ? target[e0 + k] : 0u;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool ev = ((cw >> (8 * k)) & 0xFFu) != 0u;
        ct[k] = ev ? claim[tp[k]] : 0u;
        cs[k] = (ev && cp.cee) ? claim[e0 + k] : 0u;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t c = (cw >> (8 * k)) & 0xFFu, e = e0 + k;
        if (!c) continue;
        if (ct[k] == e && (!cp.cee || cs[k] == e)) {
          atomicAdd(&tally[1 + ((int)(c & kChannelBits) - 1)], 1u);
          cnt += created_by(c);
        } else {
          atomicAdd(&tally[0], 1u);
          // with electron-electron collisions the apply resets the claims
          // of the losers too (bit 7 marks them)
          choice[e] = cp.cee ? (uint8_t)(c | 0x80u) : (uint8_t)0;
        }
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if (lane == 0) {
      bsum[b] = cnt;
      if (cnt) atomicAdd(&csum[b >> 5], cnt);
    }
  }
  // heavy events: an event happens iff it holds both of its claims; the
  // losers keep their channel with bit 7 set, so that the apply resets the
  // claims they made
  if (heavy_trials(cp, st)) {
    const uint32_t h0 = off[g.C], h1 = off[3 * g.C];
    for (uint32_t p0 = h0 + blockIdx.x * 256u; p0 < h1; p0 += gridDim.x * 256u) {
      const uint32_t p = p0 + threadIdx.x;
      int ch = -1;
      bool lost = false;
      if (p < h1) {
        const uint32_t c = choice[p];
        if (c) {
          if (claim[target[p]] == p && claim[p] == p) {
            ch = (int)(c & kChannelBits) - 1;
          } else {
            lost = true;
            choice[p] = (uint8_t)(c | 0x80u);
          }
        }
      }
      const uint64_t ml = __ballot(lost);
      if (lane == 0 && ml) atomicAdd(&tally[0], (uint32_t)__popcll(ml));
#pragma unroll
      for (int k = kCEX; k <= kNN; ++k) {
        const uint64_t m = __ballot(ch == k);
        if (lane == 0 && m) atomicAdd(&tally[1 + k], (uint32_t)__popcll(m));
      }
    }
  }
  __syncthreads();
  if (threadIdx.x <= kNC && tally[threadIdx.x]) {
    unsigned long long* dst = (threadIdx.x == 0) ? &st->conflicts : &st->events[threadIdx.x - 1];
    atomicAdd(dst, (unsigned long long)tally[threadIdx.x]);
  }
}

__device__ inline void cic_atomic(unsigned long long* Q, int b, int W, long long Z,
                                  const long long v[4]) {
  atomicAdd(&Q[b], (unsigned long long)(Z * v[0]));
  atomicAdd(&Q[b + 1], (unsigned long long)(Z * v[1]));
  atomicAdd(&Q[b + W], (unsigned long long)(Z * v[2]));
  atomicAdd(&Q[b + W + 1], (unsigned long long)(Z * v[3]));
}

// The winners' outcomes; the created slots of a chunk start at the created
// electrons of the chunks before it, in electron order inside the chunk.
// The chunks before chunk b are the whole groups of 32 before its group
// (csum) and the chunks of its group before it (bsum): one round of loads,
// taken only by a block whose electrons create some; the electrons' own
// counts come again from their choice bytes.  A thread reads the choices
// of kApplyPer electrons at once, so that one round of blocks covers them
// (rather than rounds of one chunk each, every one waiting for its loads).
constexpr int kApplyPer = 8;
static_assert(32 % kApplyPer == 0, "a block's chunks lie in one group of 32");

// the choice bytes of electrons e0 .. e0 + kApplyPer - 1 (0 past n_e)
__device__ inline void apply_choices(const uint8_t* __restrict__ choice, uint32_t e0,
                                     uint32_t n_e, uint32_t* ck) {
  static_assert(kApplyPer == 8, "one 64-bit load");
  if (e0 + kApplyPer <= n_e) {
    const uint2 cw = *(const uint2*)(choice + e0);
#pragma unroll
    for (int k = 0; k < kApplyPer; ++k) ck[k] = ((k < 4 ? cw.x : cw.y) >> (8 * (k & 3))) & 0xFFu;
  } else {
#pragma unroll
    for (int k = 0; k < kApplyPer; ++k) ck[k] = (e0 + k < n_e) ? choice[e0 + k] : 0u;
  }
}
// this thread's share of the created electrons of the chunks before chunk b
// (the whole groups of 32 before its group, then its group's chunks before
// it); the block's sum of the shares is the count
__device__ inline uint32_t created_before_part(const uint32_t* __restrict__ csum,
                                               const uint32_t* __restrict__ bsum, uint32_t b) {
  const uint32_t grp = b >> 5;
  uint32_t s = 0;
  for (uint32_t i = threadIdx.x; i < grp; i += 256) s += csum[i];
  if (threadIdx.x < (b & 31u)) s += bsum[(grp << 5) + threadIdx.x];
  return s;
}
// (LIT: the literal Eqs. 16-20 split; a separate instantiation keeps its
// trigonometric registers out of the default apply)
template <typename T, bool LIT>
__global__ void __launch_bounds__(256) k_apply(Flow<T> f, const uint32_t* off, DevState* st, Grid g,
                                               CollideParams cp, SpeciesParams spp,
                                               unsigned long long* Q, const uint8_t* choice,
                                               const uint32_t* target, const uint32_t* bsum,
                                               const uint32_t* csum, uint32_t* claim,
                                               uint32_t cap) {
  __shared__ uint32_t sh[4];
  __shared__ uint32_t lev[256 * kApplyPer], lcb[256 * kApplyPer];
  __shared__ uint8_t lch[256 * kApplyPer];
  const PartsT<T>& P = f.U;
  const PartsT<T>& S = f.S;
  const uint32_t n_e = off[g.C];
  const uint32_t nb = (n_e + 255) / 256;
  const uint32_t n_alive = st->n_alive;
  const uint32_t next_id = st->next_id;
  const uint32_t step = st->step;
  const uint32_t err0 = st->err;
  // kApplyPer consecutive electrons per thread, their choice bytes in one
  // load: block bk takes the kApplyPer chunks of 256 from chunk bk kApplyPer
  // (the grid covers the capacity).  Its choices and its share of the
  // created electrons before it are requested before the total below, so
  // that the three wait together.
  const uint32_t nbk = (n_e + 256 * kApplyPer - 1) / (256 * kApplyPer);
  const uint32_t bk = blockIdx.x;
  const uint32_t e0 = bk * (256 * kApplyPer) + threadIdx.x * kApplyPer;
  uint32_t ck[kApplyPer];
  apply_choices(choice, e0, n_e, ck);
  const uint32_t pre = bk < nbk ? created_before_part(csum, bsum, bk * kApplyPer) : 0u;
  // the created electrons of every chunk: their total must fit (capacity,
  // id space), else the step creates nothing and flags the error; every
  // block decides the same from the same sums
  const uint32_t all = block_range_sum(csum, 0, (nb + 31) / 32, sh);
  const bool fits = !err0 && (uint64_t)n_alive + all <= cap &&
                    (uint64_t)next_id + all <= 0xFFFFFFFFull;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->n_created = fits ? all : 0u;
    if (!fits) atomicOr(&st->err, 1u);
  }
  if (!fits) return;
  if (bk < nbk) {
    uint32_t mine = 0, nev = 0;
#pragma unroll
    for (int k = 0; k < kApplyPer; ++k) {
      mine += created_by(ck[k]);
      nev += ck[k] ? 1u : 0u;
    }
    uint32_t run = 0;  // created electrons before the thread's next electron
    if (__syncthreads_or(mine != 0u)) {  // the same for the whole block
      uint32_t before, tot;
      block_scan256(pre, &before, sh);
      run = before + block_scan256(mine, &tot, sh);
    }
    // the block's events listed in electron order with their first created
    // slots, then taken one per thread (a thread's own electrons would run
    // the outcome code once per electron with an event in any lane)
    uint32_t evtot;
    uint32_t ev = block_scan256(nev, &evtot, sh);
#pragma unroll
    for (int k = 0; k < kApplyPer; ++k) {
      if (ck[k]) {
        lev[ev] = e0 + k;
        lcb[ev] = run;
        lch[ev] = (uint8_t)ck[k];
        ++ev;
      }
      run += created_by(ck[k]);
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < evtot; j += 256) {
      const uint32_t e = lev[j], cbase = lcb[j], c = lch[j];
      const uint32_t tp = target[e];
      if (c & 0x80u) {  // lost, with projectile claims: reset both
        claim[tp] = 0xFFFFFFFFu;
        claim[e] = 0xFFFFFFFFu;
        continue;
      }
      if (cp.cee) claim[e] = 0xFFFFFFFFu;
      const int ch = (int)(c & kChannelBits) - 1;
      const bool up = !(c & kNoProjectile), ut = !(c & kNoTarget);  // the sides that take it
      const uint32_t pe = f.perm[e], pt = f.perm[tp];
      const RecT<T> ve = P.v[pe];
      RecT<T> vt = P.v[pt];
      const uint32_t id = ve.id;
      double e1[3] = {ve.vr, ve.vt, ve.vz};
      double A[3] = {vt.vr, vt.vt, vt.vz};
      double nh[3];
      claim[tp] = 0xFFFFFFFFu;
      // stage 1: elastic, or inelastic losing the channel threshold (Eq. 12)
      isotropic(cp, id, step, 2u, nh);
      binary(e1, A, cp.two_dE_mr[ch], cp.f1[ch], cp.f2[ch], nh);
      vt.vr = (T)A[0];
      vt.vt = (T)A[1];
      vt.vz = (T)A[2];
      if (ch == 0 || ch == kCEI || ch == kCEE) {  // elastic
        if (ut) P.v[pt] = vt;
        RecT<T> v1 = ve;
        v1.vr = (T)e1[0];
        v1.vt = (T)e1[1];
        v1.vz = (T)e1[2];
        if (up) P.v[pe] = v1;
        continue;
      }
      // stage 2 (Eq. 13): the target keeps its slot and id, changes label;
      // the new electron e2 takes the target's position and velocity
      const int sp_old = (int)vt.sp, sp_new = (int)product_of(ch, vt.sp);
      vt.sp = (uint32_t)sp_new;
      const long long mt = P.mu ? (long long)P.mu[pt] : 1ll;  // the target's multiplicity
      if (ut) P.v[pt] = vt;
      const PosT<T> xt = P.x[pt];
      if (Q && ut) {
        // the deposit counted the target with its old charge and none of
        // the new electrons: add the target's change with e2 (at the target)
        // and, for e6, one electron at the primary's place
        const long long zt = ((long long)spp.Z[sp_new] - spp.Z[sp_old] + spp.Z[0]) * mt;
        long long v[4];
        if (zt) {
          const int b = cic_fixed<T>(g, xt.r, xt.z, v);
          cic_atomic(Q, b, g.nr + 1, zt, v);
        }
        if (ch == 2) {
          const PosT<T> xe = P.x[pe];
          const int b = cic_fixed<T>(g, xe.r, xe.z, v);
          cic_atomic(Q, b, g.nr + 1, (long long)spp.Z[0] * mt, v);
        }
      }
      double e2[3] = {A[0], A[1], A[2]};
      // stage 3 (Eq. 14): e1-e2 elastic, equal masses
      isotropic(cp, id, step, 3u, nh);
      binary(e1, e2, 0.0, 0.5, 0.5, nh);
      const uint32_t slot = n_alive + cbase;
      const uint32_t nid = next_id + cbase;
      if (ut) {
        S.x[slot] = xt;
        S.v[slot] = RecT<T>{(T)e2[0], (T)e2[1], (T)e2[2], nid, 0u};
        if (S.mu) S.mu[slot] = (uint16_t)mt;
      }
      if (ch == 2) {
        // stage 4 (Eq. 15): e3 splits into the two orthogonal edges of the
        // rectangle whose diagonal is v3
        double v5[3];
        if (LIT) {
          // cos(chi) ~ U[0,1), psi ~ U[0,2 pi): purpose 4, draw 0
          uint32_t w4[4];
          philox(id, 0u, step, 4u << 24, cp.seed_lo, cp.seed_hi, w4);
          const double chi = acos(u53(w4[0], w4[1]));
          const double psi = (2.0 * kPI) * u53(w4[2], w4[3]);
          split_literal(e1, chi, psi, v5);
        } else {
          isotropic(cp, id, step, 4u, nh);
          const double d = ((e1[0] * nh[0]) + (e1[1] * nh[1])) + (e1[2] * nh[2]);
          v5[0] = d * nh[0];
          v5[1] = d * nh[1];
          v5[2] = d * nh[2];
        }
        if (ut) {
          const uint32_t s6 = slot + 1;
          S.x[s6] = P.x[pe];
          S.v[s6] = RecT<T>{(T)(e1[0] - v5[0]), (T)(e1[1] - v5[1]), (T)(e1[2] - v5[2]),
                            nid + 1, 0u};
          if (S.mu) S.mu[s6] = (uint16_t)mt;
        }
        e1[0] = v5[0];
        e1[1] = v5[1];
        e1[2] = v5[2];
      }
      RecT<T> v1 = ve;
      v1.vr = (T)e1[0];
      v1.vt = (T)e1[1];
      v1.vz = (T)e1[2];
      if (up) P.v[pe] = v1;
    }
  }
  // heavy events (disjoint from every other event); every heavy trial that
  // claimed resets its two claims, won or lost
  if (!heavy_trials(cp, st)) return;
  const uint32_t h0 = off[g.C], h1 = off[3 * g.C];
  for (uint32_t p = h0 + blockIdx.x * blockDim.x + threadIdx.x; p < h1;
       p += gridDim.x * blockDim.x) {
    const uint32_t c = choice[p];
    if (!c) continue;
    const uint32_t tp = target[p];
    if (!(c & 0x80u)) {
      const int ch = (int)(c & kChannelBits) - 1;
      const bool up = !(c & kNoProjectile), ut = !(c & kNoTarget);
      const uint32_t pp = f.perm[p], pt = f.perm[tp];
      RecT<T> a = P.v[pp], b = P.v[pt];
      if (ch == kCEX) {
        // the charge passes from the ion to the atom: the labels swap, the
        // charge moves from the projectile's place to the target's (each
        // side that takes the outcome with its own multiplicity)
        const uint32_t sa = a.sp, sb = b.sp;
        if (up) a.sp = sb;
        if (ut) b.sp = sa;
        if (Q) {
          long long v[4];
          const PosT<T> xa = P.x[pp], xb = P.x[pt];
          const long long dzp = (long long)spp.Z[sb] - spp.Z[sa];
          const long long ma = P.mu ? (long long)P.mu[pp] : 1ll;
          const long long mb = P.mu ? (long long)P.mu[pt] : 1ll;
          int bn;
          if (up) {
            bn = cic_fixed<T>(g, xa.r, xa.z, v);
            cic_atomic(Q, bn, g.nr + 1, dzp * ma, v);
          }
          if (ut) {
            bn = cic_fixed<T>(g, xb.r, xb.z, v);
            cic_atomic(Q, bn, g.nr + 1, -dzp * mb, v);
          }
        }
      } else {
        // elastic, equal masses, isotropic in the centre-of-mass frame
        double A[3] = {a.vr, a.vt, a.vz}, B[3] = {b.vr, b.vt, b.vz};
        double nh[3];
        isotropic(cp, a.id, step, 2u, nh);
        binary(A, B, 0.0, cp.f1[ch], cp.f2[ch], nh);
        a.vr = (T)A[0];
        a.vt = (T)A[1];
        a.vz = (T)A[2];
        b.vr = (T)B[0];
        b.vt = (T)B[1];
        b.vz = (T)B[2];
      }
      if (up) P.v[pp] = a;
      if (ut) P.v[pt] = b;
    }
    claim[tp] = 0xFFFFFFFFu;
    claim[p] = 0xFFFFFFFFu;
  }
}

template <typename T>
void collide(const Flow<T>& P, const uint32_t* off, DevState* st, const Grid& g,
             const CollideParams& cp, const SpeciesParams& sp, int64_t* Q, CollideWork& w,
             uint32_t* bsum, int64_t cap, hipStream_t s) {
  // grids for the electrons (a few percent of the capacity in a steady
  // state); the launches loop over whatever there is
  const int gr = grid_for(cap) < 1024 ? grid_for(cap) : 1024;
  // one block per kApplyPer chunks of the capacity (the electrons are fewer)
  const int nb = (int)((cap + 256 * kApplyPer - 1) / (256 * kApplyPer));
  // deposit blocks after the decision blocks (dispatched in order)
  int nd = 0;
  if (Q) nd = (int)((cap + 255) / 256) < 4096 ? (int)((cap + 255) / 256) : 4096;
  k_decide<T><<<gr + nd, 256, 0, s>>>(P, off, st, g, cp, w.choice, w.target, w.claim, w.csum,
                                      sp, (unsigned long long*)Q, (uint32_t)gr);
  // the resolution: one wave per chunk
  int nr = (int)((cap + 1023) / 1024);
  if (nr > 4096) nr = 4096;
  k_resolve<<<nr, 256, 0, s>>>(off, st, g, cp, w.choice, w.target, w.claim, bsum, w.csum);
  // created-electron slots: each apply block adds up the chunk sums before
  // its chunk; the guard (in every block) flags an overflow and then nothing
  // is created, so every later launch touches only [0, n_alive)
  if (cp.split_literal)
    k_apply<T, true><<<nb, 256, 0, s>>>(P, off, st, g, cp, sp, (unsigned long long*)Q, w.choice,
                                        w.target, bsum, w.csum, w.claim, (uint32_t)cap);
  else
    k_apply<T, false><<<nb, 256, 0, s>>>(P, off, st, g, cp, sp, (unsigned long long*)Q, w.choice,
                                         w.target, bsum, w.csum, w.claim, (uint32_t)cap);
}
template void collide<double>(const Flow<double>&, const uint32_t*, DevState*, const Grid&,
                              const CollideParams&, const SpeciesParams&, int64_t*, CollideWork&,
                              uint32_t*, int64_t, hipStream_t);
template void collide<float>(const Flow<float>&, const uint32_t*, DevState*, const Grid&,
                             const CollideParams&, const SpeciesParams&, int64_t*, CollideWork&,
                             uint32_t*, int64_t, hipStream_t);

}  // namespace pd
