/*
 * pd_oracle.c -- plain FP64 CPU oracle of the r-z PIC-DSMC step
 * (arXiv 2109.00214, Sections 2.1-2.3).  TEST INFRASTRUCTURE ONLY: it is
 * loaded by the tests, the smoke check and the benchmark's CPU-baseline leg,
 * never by the product path.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math).  Every
 * floating-point value is one binary64 expression evaluated left to right
 * as parenthesised; round-to-nearest-even; no fused multiply-add.
 *
 * Step order (the paper only says the PIC and DSMC parts are coupled):
 *   sort -> collide (decide, claim, apply, create) -> deposit -> Poisson ->
 *   field -> gather+push -> compact + inject -> step counter.
 *
 * Parity pins for every function are in tests/test_oracle_*.py.  Two
 * pieces are pinned only by conservation identities ("parity unpinned"
 * beyond them): the scattering law of the e-e stage of the double
 * ionization (Sec. 2.2, Eq. 14 names a Coulomb-like stage but gives no law;
 * an isotropic elastic collision of equal masses in the centre-of-mass
 * frame is used) and the energy sharing of the single-ionization events
 * (Sec. 2.2 refers to earlier work for them and states no scheme).
 */
#include "pd_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* CODATA 2018 */
#define Q_E 1.602176634e-19
#define EPS0 8.8541878128e-12
#define PI_D 3.14159265358979323846
#define K_B 1.380649e-23
/* Fowler-Nordheim constants of the elementary form J = (A F^2 / phi)
 * exp(-B phi^(3/2) / F): A in A eV V^-2, B in eV^(-3/2) V m^-1           */
#define FN_A 1.541434e-6
#define FN_B 6.830890e9

static char g_err[256];
static int fail(const char* msg) {
  snprintf(g_err, sizeof g_err, "%s", msg);
  return -1;
}
const char* or_last_error(void) { return g_err; }

struct or_sim {
  int nr, nz;
  int64_t ncell; /* nr*nz */
  double R, L, V, dt, W;
  uint64_t seed;
  int enable_di, deposit_off, collisions_off;
  int heavy_every;  /* heavy particles advance every heavy_every steps (1: every step) */
  int split_literal; /* 1: the double ionization's last stage by the literal Eqs. 16-20 */
  /* cathode emission (Sec. 2.3): off while em_beta == 0 */
  double em_beta, em_rtip, em_phi, em_ratio, em_T;
  double em_acc_e, em_acc_n; /* fractional super-particles carried to the next step */
  int64_t emitted[2];        /* cumulative: electrons, neutrals */
  /* external circuit (Sec. 2.3): off while circ_C == 0 */
  double circ_V0, circ_R, circ_C;
  int64_t circ_zanode; /* sum of Z absorbed at the anode at the last update */
  /* sputtering at the cathode (Sec. 2.3): off while sput_on == 0 */
  int sput_on;
  uint64_t* sput;      /* per cathode annulus: yields in units of 2^-32 */
  int64_t* sput_now;   /* atoms to emit this step, per annulus */
  int64_t sputtered;   /* cumulative */

  int Z[OR_NSPECIES];
  double m[OR_NSPECIES];
  int species_set;

  int xs_set[OR_NCHANNELS];
  int xs_n[OR_NCHANNELS];
  double xs_thr[OR_NCHANNELS], xs_dsq[OR_NCHANNELS];
  double* xs_tab[OR_NCHANNELS];

  /* host tables */
  double dr, dz, qunit;
  double qmdt[OR_NSPECIES];
  double *Vnode, *Vcell;  /* [nr+1], [nr] (radial factor times dz) */
  double *ra, *rb, *rc;   /* radial FV coefficients [nr+1] */
  double *S;              /* sine table [(nz+1)*(nz+1)], S[k*(nz+1)+j] */
  double *mu;             /* z eigenvalues [nz+1] */
  double mr[OR_NCHANNELS], f1[OR_NCHANNELS], f2[OR_NCHANNELS], ck[OR_NCHANNELS];
  double two_dE_mr[OR_NCHANNELS];
  double edges[65];

  /* particles */
  int64_t n, cap;
  double *r, *z, *vr, *vt, *vz;
  uint8_t* sp;
  uint16_t* mult; /* multiplicity: the super-particle stands for mult * W */
  uint32_t *id, *key;
  uint8_t* alive;
  int64_t n_sorted; /* particles present at the sort (before creation) */

  /* collide stage record (sorted positions) */
  uint8_t* choice;
  uint32_t* target;
  uint8_t* win;
  uint32_t* claim;
  int64_t coll_cap;

  /* grids: node-major, r fastest, (nz+1) rows of (nr+1) */
  int64_t* Q;
  double *phi, *Er, *Ez;
  int64_t* off; /* CSR offsets [OR_NKEYS*ncell+1] */

  /* injection schedule */
  int sched_n, sched_pos;
  int64_t* sched_off;
  double *s_r, *s_z, *s_vr, *s_vt, *s_vz;
  uint8_t* s_sp;

  int64_t step, next_id;
  int64_t events[OR_NCHANNELS], conflicts, created;
  int64_t absorbed[3][OR_NSPECIES], injected[OR_NSPECIES];
  int64_t charge_absorbed, charge_injected;
};

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
 * 32x32->64 multiplications with a Weyl-sequence key schedule.          */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* counter = (particle id, 0, step, purpose<<24 | draw); key = seed */
static void draw4(const or_sim* s, uint32_t id, uint32_t purpose, uint32_t d,
                  uint32_t w[4]) {
  uint32_t ctr[4] = {id, 0u, (uint32_t)s->step, (purpose << 24) | d};
  uint32_t key[2] = {(uint32_t)s->seed, (uint32_t)(s->seed >> 32)};
  or_philox4x32_10(ctr, key, w);
}

/* uniform double in [0,1) from two words: top 53 bits of (hi:lo) */
static double u53(uint32_t hi, uint32_t lo) {
  uint64_t b = (((uint64_t)hi << 32) | (uint64_t)lo) >> 11;
  return (double)b * 0x1p-53;
}

/* ------------------------------------------------------------------ */
static void* xalloc(size_t n) {
  void* p = calloc(n ? n : 1, 1);
  if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
  return p;
}

or_sim* or_create(int nr, int nz, double R, double L, double V, double dt,
                  double weight, uint64_t seed, int enable_di,
                  int deposit_off, int collisions_off) {
  if (nr < 2 || nz < 2 || !(R > 0) || !(L > 0) || !(dt > 0) || !(weight > 0) ||
      !isfinite(V)) {
    fail("or_create: invalid domain");
    return NULL;
  }
  or_sim* s = (or_sim*)xalloc(sizeof(or_sim));
  s->nr = nr; s->nz = nz; s->ncell = (int64_t)nr * nz;
  s->R = R; s->L = L; s->V = V; s->dt = dt; s->W = weight; s->seed = seed;
  s->enable_di = enable_di; s->deposit_off = deposit_off;
  s->collisions_off = collisions_off;
  s->heavy_every = 1;
  s->dr = R / (double)nr;
  s->dz = L / (double)nz;
  s->qunit = (Q_E * weight) * 0x1p-40;
  const double dr = s->dr, dz = s->dz;

  /* node volumes (linear weighting in r, Verboncoeur) and cell volumes */
  s->Vnode = (double*)xalloc(sizeof(double) * (nr + 1));
  s->Vcell = (double*)xalloc(sizeof(double) * nr);
  s->Vnode[0] = ((PI_D * (dr * dr)) * dz) / 3.0;
  for (int i = 1; i < nr; ++i) s->Vnode[i] = (((2.0 * PI_D) * ((double)i * dr)) * dr) * dz;
  s->Vnode[nr] = (PI_D * dz) * ((R * dr) - ((dr * dr) / 3.0));
  for (int i = 0; i < nr; ++i) {
    double ri = (double)i * dr, ri1 = (double)(i + 1) * dr;
    s->Vcell[i] = (PI_D * ((ri1 * ri1) - (ri * ri))) * dz;
  }

  /* finite-volume radial operator: control interval [r_{i-1/2}, r_{i+1/2}]
   * clipped to [0, R]; zero flux through r = 0 and r = R.               */
  s->ra = (double*)xalloc(sizeof(double) * (nr + 1));
  s->rb = (double*)xalloc(sizeof(double) * (nr + 1));
  s->rc = (double*)xalloc(sizeof(double) * (nr + 1));
  for (int i = 0; i <= nr; ++i) {
    double A;
    if (i == 0) A = (dr * dr) / 8.0;
    else if (i == nr) A = ((R * dr) / 2.0) - ((dr * dr) / 8.0);
    else A = ((double)i * dr) * dr;
    double rm = (i == 0) ? 0.0 : ((double)i - 0.5) * dr;
    double rp = (i == nr) ? 0.0 : ((double)i + 0.5) * dr;
    s->ra[i] = rm / (dr * A);
    s->rc[i] = rp / (dr * A);
    s->rb[i] = -(s->ra[i] + s->rc[i]);
  }

  /* DST-I table over the z nodes and the eigenvalues of the 3-point d2/dz2 */
  s->S = (double*)xalloc(sizeof(double) * (size_t)(nz + 1) * (nz + 1));
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= nz; ++j) {
      int64_t m = ((int64_t)k * j) % (2 * (int64_t)nz);
      int neg = 0;
      if (m >= nz) { m -= nz; neg = 1; }
      if (2 * m > nz) m = nz - m;
      double v = (m == 0) ? 0.0 : sin((PI_D * (double)m) / (double)nz);
      s->S[(size_t)k * (nz + 1) + j] = neg ? -v : v;
    }
  s->mu = (double*)xalloc(sizeof(double) * (nz + 1));
  for (int k = 0; k <= nz; ++k) {
    double h = sin((PI_D * (double)k) / (2.0 * (double)nz));
    s->mu[k] = -(4.0 * (h * h)) / (dz * dz);
  }

  for (int b = 0; b <= 64; ++b) s->edges[b] = pow(10.0, (3.0 * (double)b) / 64.0);

  int64_t nn = (int64_t)(nr + 1) * (nz + 1);
  s->Q = (int64_t*)xalloc(sizeof(int64_t) * nn);
  s->phi = (double*)xalloc(sizeof(double) * nn);
  s->Er = (double*)xalloc(sizeof(double) * nn);
  s->Ez = (double*)xalloc(sizeof(double) * nn);
  s->off = (int64_t*)xalloc(sizeof(int64_t) * (6 * s->ncell + 1));
  /* vacuum potential before the first solve */
  for (int j = 0; j <= nz; ++j)
    for (int i = 0; i <= nr; ++i)
      s->phi[(int64_t)j * (nr + 1) + i] = (-V) + (V * ((double)j / (double)nz));
  /* default charge numbers */
  const int Zd[OR_NSPECIES] = {-1, 0, 1, 2, 2, 2};
  for (int k = 0; k < OR_NSPECIES; ++k) s->Z[k] = Zd[k];
  return s;
}

void or_destroy(or_sim* s) {
  if (s) { free(s->sput); free(s->sput_now); }
  if (!s) return;
  for (int k = 0; k < OR_NCHANNELS; ++k) free(s->xs_tab[k]);
  free(s->Vnode); free(s->Vcell); free(s->ra); free(s->rb); free(s->rc);
  free(s->S); free(s->mu);
  free(s->r); free(s->z); free(s->vr); free(s->vt); free(s->vz);
  free(s->sp); free(s->mult); free(s->id); free(s->key); free(s->alive);
  free(s->choice); free(s->target); free(s->win); free(s->claim);
  free(s->Q); free(s->phi); free(s->Er); free(s->Ez); free(s->off);
  free(s->sched_off); free(s->s_r); free(s->s_z); free(s->s_vr); free(s->s_vt);
  free(s->s_vz); free(s->s_sp);
  free(s);
}

/* the species each channel's target is drawn from (any Cu2+ tag for SI3:
 * all tags have the Cu2+ mass) and the label the target takes             */
static const int TARGET_OF[OR_NCHANNELS] = {OR_CU, OR_CU, OR_CU, OR_CU1, OR_CU2_STEP, OR_CU3,
                                            OR_CU, OR_CU, OR_CU1, OR_E};
static const int PROJECTILE_OF[OR_NCHANNELS] = {OR_E, OR_E, OR_E, OR_E,   OR_E,
                                                OR_E, OR_CU1, OR_CU, OR_E, OR_E};
static const int PRODUCT_OF[OR_NCHANNELS] = {OR_CU, OR_CU1, OR_CU2_DOUBLE, OR_CU2_STEP, OR_CU3,
                                             OR_CU4, OR_CU1, OR_CU, OR_CU1, OR_E};
/* the electron channels in cumulative-sum order, and the key class their
 * target is drawn from (0: another electron)                             */
static const int ECH[OR_NELECTRON_CHANNELS] = {OR_EL, OR_SI, OR_DI, OR_SI2, OR_SI3, OR_SI4,
                                               OR_CEI, OR_CEE};
static const int ECLS[OR_NELECTRON_CHANNELS] = {1, 1, 1, 2, 3, 4, 2, 0};

static void derive_pairs(or_sim* s) {
  /* projectile PROJECTILE_OF[channel], target TARGET_OF[channel] */
  const int* tgt = TARGET_OF;
  for (int k = 0; k < OR_NCHANNELS; ++k) {
    double m1 = s->m[PROJECTILE_OF[k]], m2 = s->m[tgt[k]];
    s->mr[k] = (m1 * m2) / (m1 + m2);
    s->f1[k] = s->mr[k] / m1;
    s->f2[k] = s->mr[k] / m2;
    s->ck[k] = sqrt(s->mr[k] / (2.0 * Q_E));
    s->two_dE_mr[k] = (k == OR_EL || k >= OR_CEX) ? 0.0 : (2.0 * (-(s->xs_thr[k] * Q_E))) / s->mr[k];
  }
}

int or_set_species(or_sim* s, int n, const int* Z, const double* mass) {
  if (n != OR_NSPECIES) return fail("or_set_species: need 8 species");
  if (Z[OR_CU2_DOUBLE] != Z[OR_CU2_STEP] || Z[OR_CU2_INIT] != Z[OR_CU2_STEP] ||
      mass[OR_CU2_DOUBLE] != mass[OR_CU2_STEP] || mass[OR_CU2_INIT] != mass[OR_CU2_STEP])
    return fail("or_set_species: the Cu2+ tags must share one charge and mass");
  for (int k = 0; k < n; ++k)
    if (!(mass[k] > 0) || !isfinite(mass[k])) return fail("or_set_species: bad mass");
  for (int k = 0; k < n; ++k) { s->Z[k] = Z[k]; s->m[k] = mass[k]; }
  for (int k = 0; k < n; ++k) s->qmdt[k] = (((double)s->Z[k] * Q_E) / s->m[k]) * s->dt;
  s->species_set = 1;
  derive_pairs(s);
  return 0;
}

int or_set_cross_section(or_sim* s, int ch, double thr, int n, double dsq,
                         const double* sigma) {
  if (ch < 0 || ch >= OR_NCHANNELS) return fail("or_set_cross_section: channel");
  if (n < 2 || !(dsq > 0) || !(thr >= 0)) return fail("or_set_cross_section: table");
  int ex;
  double mant = frexp(dsq, &ex);
  if (mant != 0.5) return fail("or_set_cross_section: dsqrtE must be a power of 2");
  for (int i = 0; i < n; ++i)
    if (!(sigma[i] >= 0) || !isfinite(sigma[i])) return fail("or_set_cross_section: sigma");
  free(s->xs_tab[ch]);
  s->xs_tab[ch] = (double*)xalloc(sizeof(double) * n);
  memcpy(s->xs_tab[ch], sigma, sizeof(double) * n);
  s->xs_n[ch] = n; s->xs_thr[ch] = thr; s->xs_dsq[ch] = dsq; s->xs_set[ch] = 1;
  if (s->species_set) derive_pairs(s);
  return 0;
}

/* ------------------------------------------------------------------ */
static void reserve(or_sim* s, int64_t need) {
  if (need <= s->cap) return;
  int64_t c = s->cap ? s->cap : 1024;
  while (c < need) c *= 2;
  s->r = (double*)realloc(s->r, sizeof(double) * c);
  s->z = (double*)realloc(s->z, sizeof(double) * c);
  s->vr = (double*)realloc(s->vr, sizeof(double) * c);
  s->vt = (double*)realloc(s->vt, sizeof(double) * c);
  s->vz = (double*)realloc(s->vz, sizeof(double) * c);
  s->sp = (uint8_t*)realloc(s->sp, c);
  s->mult = (uint16_t*)realloc(s->mult, sizeof(uint16_t) * c);
  s->id = (uint32_t*)realloc(s->id, sizeof(uint32_t) * c);
  s->key = (uint32_t*)realloc(s->key, sizeof(uint32_t) * c);
  s->alive = (uint8_t*)realloc(s->alive, c);
  if (!s->r || !s->z || !s->vr || !s->vt || !s->vz || !s->sp || !s->mult || !s->id ||
      !s->key || !s->alive) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
  s->cap = c;
}

/* cell of a position: i = min((int)(r/dr), nr-1), j likewise in z */
static void cell_of(const or_sim* s, double r, double z, int* ci, int* cj,
                    double* fr, double* fz) {
  double xr = r / s->dr, xz = z / s->dz;
  int i = (int)xr, j = (int)xz;
  if (i > s->nr - 1) i = s->nr - 1;
  if (j > s->nz - 1) j = s->nz - 1;
  *ci = i; *cj = j;
  *fr = xr - (double)i;
  *fz = xz - (double)j;
}

/* sort key: key class of the species (the three Cu2+ tags share one),
 * then cell = j*nr + i                                                 */
static const int KEY_CLASS[OR_NSPECIES] = {0, 1, 2, 3, 3, 3, 4, 5};

static uint32_t key_of(const or_sim* s, double r, double z, int sp) {
  int i, j; double fr, fz;
  cell_of(s, r, z, &i, &j, &fr, &fz);
  return (uint32_t)((int64_t)KEY_CLASS[sp] * s->ncell + (int64_t)j * s->nr + i);
}

static int check_particles(const or_sim* s, int64_t n, const double* r,
                           const double* z, const double* vr, const double* vt,
                           const double* vz, const uint8_t* sp) {
  for (int64_t p = 0; p < n; ++p) {
    if (!isfinite(r[p]) || !isfinite(z[p]) || !isfinite(vr[p]) ||
        !isfinite(vt[p]) || !isfinite(vz[p]))
      return fail("inject: non-finite value");
    if (!(r[p] >= 0.0) || !(r[p] < s->R) || !(z[p] >= 0.0) || !(z[p] < s->L))
      return fail("inject: position outside the domain");
    if (sp[p] >= OR_NSPECIES) return fail("inject: species out of range");
  }
  return 0;
}

static void append(or_sim* s, int64_t n, const double* r, const double* z,
                   const double* vr, const double* vt, const double* vz,
                   const uint8_t* sp, const uint16_t* mult) {
  reserve(s, s->n + n);
  for (int64_t p = 0; p < n; ++p) {
    int64_t q = s->n + p;
    s->r[q] = r[p]; s->z[q] = z[p]; s->vr[q] = vr[p]; s->vt[q] = vt[p];
    s->vz[q] = vz[p]; s->sp[q] = sp[p];
    s->mult[q] = mult ? mult[p] : 1;
    s->id[q] = (uint32_t)(s->next_id + p);
    s->key[q] = key_of(s, r[p], z[p], sp[p]);
    s->alive[q] = 1;
    s->injected[sp[p]] += 1;
    s->charge_injected += s->Z[sp[p]];
  }
  s->n += n;
  s->next_id += n;
}

int or_inject(or_sim* s, int64_t n, const double* r, const double* z,
              const double* vr, const double* vt, const double* vz,
              const uint8_t* sp) {
  if (n < 0) return fail("inject: n < 0");
  if (s->next_id + n > (int64_t)UINT32_MAX) return fail("inject: id overflow");
  if (check_particles(s, n, r, z, vr, vt, vz, sp)) return -1;
  append(s, n, r, z, vr, vt, vz, sp, NULL);
  return 0;
}

/* injection with multiplicities (unequal weights): particle p stands for
 * mult[p] * W real particles, 1 <= mult[p] <= 65535                      */
int or_inject_weighted(or_sim* s, int64_t n, const double* r, const double* z,
                       const double* vr, const double* vt, const double* vz,
                       const uint8_t* sp, const uint16_t* mult) {
  if (n < 0) return fail("inject: n < 0");
  if (s->next_id + n > (int64_t)UINT32_MAX) return fail("inject: id overflow");
  if (check_particles(s, n, r, z, vr, vt, vz, sp)) return -1;
  for (int64_t p = 0; p < n; ++p)
    if (mult[p] < 1) return fail("inject: multiplicity below 1");
  append(s, n, r, z, vr, vt, vz, sp, mult);
  return 0;
}

int or_schedule_injection(or_sim* s, int nsteps, const int64_t* offs,
                          const double* r, const double* z, const double* vr,
                          const double* vt, const double* vz, const uint8_t* sp) {
  if (nsteps < 0 || offs[0] != 0) return fail("schedule: bad offsets");
  for (int k = 0; k < nsteps; ++k)
    if (offs[k + 1] < offs[k]) return fail("schedule: offsets decrease");
  int64_t tot = offs[nsteps];
  if (check_particles(s, tot, r, z, vr, vt, vz, sp)) return -1;
  free(s->sched_off); free(s->s_r); free(s->s_z); free(s->s_vr); free(s->s_vt);
  free(s->s_vz); free(s->s_sp);
  s->sched_off = (int64_t*)xalloc(sizeof(int64_t) * (nsteps + 1));
  memcpy(s->sched_off, offs, sizeof(int64_t) * (nsteps + 1));
  s->s_r = (double*)xalloc(sizeof(double) * tot);
  s->s_z = (double*)xalloc(sizeof(double) * tot);
  s->s_vr = (double*)xalloc(sizeof(double) * tot);
  s->s_vt = (double*)xalloc(sizeof(double) * tot);
  s->s_vz = (double*)xalloc(sizeof(double) * tot);
  s->s_sp = (uint8_t*)xalloc(tot);
  memcpy(s->s_r, r, sizeof(double) * tot); memcpy(s->s_z, z, sizeof(double) * tot);
  memcpy(s->s_vr, vr, sizeof(double) * tot); memcpy(s->s_vt, vt, sizeof(double) * tot);
  memcpy(s->s_vz, vz, sizeof(double) * tot); memcpy(s->s_sp, sp, tot);
  s->sched_n = nsteps; s->sched_pos = 0;
  return 0;
}

/* ------------------------------------------------------------------ */
/* 1. sort: stable by key (ties keep the input order)                   */
static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

void or_stage_sort(or_sim* s) {
  int64_t n = s->n;
  uint64_t* kv = (uint64_t*)xalloc(sizeof(uint64_t) * (n ? n : 1));
  for (int64_t p = 0; p < n; ++p) {
    s->key[p] = key_of(s, s->r[p], s->z[p], s->sp[p]);
    kv[p] = ((uint64_t)s->key[p] << 32) | (uint64_t)p; /* index breaks ties */
  }
  qsort(kv, (size_t)n, sizeof(uint64_t), cmp_u64);
  double* tmp = (double*)xalloc(sizeof(double) * (n ? n : 1));
  double* arrs[5] = {s->r, s->z, s->vr, s->vt, s->vz};
  for (int a = 0; a < 5; ++a) {
    for (int64_t p = 0; p < n; ++p) tmp[p] = arrs[a][kv[p] & 0xffffffffu];
    memcpy(arrs[a], tmp, sizeof(double) * n);
  }
  uint32_t* t32 = (uint32_t*)tmp;
  for (int64_t p = 0; p < n; ++p) t32[p] = s->id[kv[p] & 0xffffffffu];
  memcpy(s->id, t32, sizeof(uint32_t) * n);
  for (int64_t p = 0; p < n; ++p) t32[p] = (uint32_t)(kv[p] >> 32);
  memcpy(s->key, t32, sizeof(uint32_t) * n);
  uint8_t* t8 = (uint8_t*)tmp;
  for (int64_t p = 0; p < n; ++p) t8[p] = s->sp[kv[p] & 0xffffffffu];
  memcpy(s->sp, t8, n);
  uint16_t* t16 = (uint16_t*)tmp;
  for (int64_t p = 0; p < n; ++p) t16[p] = s->mult[kv[p] & 0xffffffffu];
  memcpy(s->mult, t16, sizeof(uint16_t) * n);
  free(tmp);
  free(kv);
  /* CSR offsets over the flattened (key class, cell) key space */
  int64_t nk = OR_NKEYS * s->ncell;
  memset(s->off, 0, sizeof(int64_t) * (nk + 1));
  for (int64_t p = 0; p < n; ++p) s->off[s->key[p] + 1] += 1;
  for (int64_t k = 0; k < nk; ++k) s->off[k + 1] += s->off[k];
  s->n_sorted = n;
}

/* ------------------------------------------------------------------ */
/* 2-5. DSMC collisions (Eqs. 4-7 and the four stages of Eqs. 12-15)   */

/* integrated cross section at relative speed g: tables are uniform in
 * sqrt(energy in eV), linear interpolation, zero below threshold,
 * clamped at the last entry                                            */
static double sigma_of(const or_sim* s, int k, double g) {
  double sq = g * s->ck[k];
  double eps = sq * sq;
  if (eps < s->xs_thr[k]) return 0.0;
  int n = s->xs_n[k];
  const double* t = s->xs_tab[k];
  double x = sq / s->xs_dsq[k];
  if (x >= (double)(n - 1)) return t[n - 1];
  int i = (int)x;
  return t[i] + ((x - (double)i) * (t[i + 1] - t[i]));
}

double or_cross_section(const or_sim* s, int channel, double g) {
  return sigma_of(s, channel, g);
}

/* isotropic unit vector by Marsaglia's (1972) rejection method; each
 * purpose has its own draw counter; the cap is never reached in practice */
void or_isotropic(const or_sim* s, uint32_t id, uint32_t purpose, double n[3]) {
  for (uint32_t d = 0; d < 64; ++d) {
    uint32_t w[4];
    draw4(s, id, purpose, d, w);
    double u1 = (2.0 * u53(w[0], w[1])) - 1.0;
    double u2 = (2.0 * u53(w[2], w[3])) - 1.0;
    double q = (u1 * u1) + (u2 * u2);
    if (q < 1.0 && q > 0.0) {
      double t = sqrt(1.0 - q);
      n[0] = (2.0 * u1) * t;
      n[1] = (2.0 * u2) * t;
      n[2] = 1.0 - (2.0 * q);
      return;
    }
  }
  n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
}

/* binary collision, Eqs. 5-6: u = v1 - v2, |u'|^2 = |u|^2 + 2 dE / m_r
 * (clamped at 0), u' = |u'| n, v1 += (u'-u) m_r/m1, v2 -= (u'-u) m_r/m2  */
static void binary(double v1[3], double v2[3], double two_dE_mr, double f1,
                   double f2, const double n[3]) {
  double u[3] = {v1[0] - v2[0], v1[1] - v2[1], v1[2] - v2[2]};
  double g2 = ((u[0] * u[0]) + (u[1] * u[1])) + (u[2] * u[2]);
  double gp2 = g2 + two_dE_mr;
  if (gp2 < 0.0) gp2 = 0.0;
  double gp = sqrt(gp2);
  for (int c = 0; c < 3; ++c) {
    double du = (gp * n[c]) - u[c];
    v1[c] = v1[c] + (du * f1);
    v2[c] = v2[c] - (du * f2);
  }
}

static void coll_reserve(or_sim* s, int64_t n) {
  if (n <= s->coll_cap) return;
  free(s->choice); free(s->target); free(s->win); free(s->claim);
  s->choice = (uint8_t*)xalloc(n);
  s->target = (uint32_t*)xalloc(sizeof(uint32_t) * n);
  s->win = (uint8_t*)xalloc(n);
  s->claim = (uint32_t*)xalloc(sizeof(uint32_t) * n);
  s->coll_cap = n;
}

/* Unequal weights (Sec. 2.2 leaves them to the rejection or the merging
 * method): an event between super-particles of multiplicities mp and mt
 * stands for min(mp, mt) real collisions.  The side with the smaller
 * multiplicity always takes the outcome, the other with probability
 * min/its own, decided by one draw (purpose 7, draw 0) per event; with
 * equal multiplicities both sides take it and nothing is drawn.  A target
 * that takes an ionizing outcome is relabelled as a whole and the electrons
 * it emits carry its multiplicity, so every ionizing event conserves
 * charge exactly; charge exchange between unequal multiplicities conserves
 * it on average only.                                                      */
static void take_sides(const or_sim* s, uint32_t id, uint32_t mp, uint32_t mt, int* up,
                       int* ut) {
  *up = 1;
  *ut = 1;
  if (mp == mt) return;
  uint32_t w[4];
  draw4(s, id, 7, 0, w);
  double u = u53(w[0], w[1]);
  if (mp > mt) *up = u < ((double)mt / (double)mp);
  else *ut = u < ((double)mp / (double)mt);
}

void or_stage_collide(or_sim* s) {
  int64_t n = s->n;
  coll_reserve(s, n ? n : 1);
  memset(s->choice, 0, n);
  memset(s->win, 0, n);
  if (s->collisions_off) return;
  const int64_t C = s->ncell;
  const int64_t n_e = s->off[C]; /* electrons occupy [0, off[C]) */

  /* decide: reads the pre-collision state only (Eq. 4).  Each electron
   * draws one target of each target class in its cell (Cu, Cu+, Cu2+ of any
   * tag, Cu3+, and with electron-electron Coulomb collisions one of the
   * other electrons): the channels of one target class share the draw and
   * the relative speed.  Channels from SI3 on take part only when their
   * tables are set.  The electron-electron channel tries every pair from
   * both sides, so its x carries a factor 1/2 and its density counts the
   * other N - 1 electrons.                                                */
  const int cee = s->xs_set[OR_CEE];
  for (int64_t p = 0; p < n_e; ++p) {
    int64_t cell = s->key[p]; /* key class 0 */
    int ci = (int)(cell % s->nr);
    int64_t b[5], nt[5], tp[5];
    uint32_t w[4], t[4];
    draw4(s, s->id[p], 0, 0, w);
    draw4(s, s->id[p], 1, 0, t);
    double R1 = u53(w[0], w[1]);
    double R2 = u53(w[2], w[3]);
    for (int c = 1; c <= 4; ++c) {
      b[c] = s->off[c * C + cell];
      nt[c] = s->off[c * C + cell + 1] - b[c];
      /* uniform pick: floor(u32 * n / 2^32), word c-1 of the second draw */
      tp[c] = b[c] + (int64_t)(((uint64_t)t[c - 1] * (uint64_t)nt[c]) >> 32);
    }
    /* another electron of the cell (word 0 of the draw (purpose 1, 1)),
     * never the projectile itself */
    b[0] = s->off[cell];
    nt[0] = s->off[cell + 1] - b[0] - 1; /* the others */
    tp[0] = 0;
    if (cee && nt[0] > 0) {
      uint32_t t2[4];
      draw4(s, s->id[p], 1, 1, t2);
      int64_t u = (int64_t)(((uint64_t)t2[0] * (uint64_t)nt[0]) >> 32);
      if (b[0] + u >= p) u += 1;
      tp[0] = b[0] + u;
    }
    double x[OR_NELECTRON_CHANNELS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int e = 0; e < OR_NELECTRON_CHANNELS; ++e) {
      int k = ECH[e], c = ECLS[e];
      if (nt[c] <= 0 || !s->xs_set[k]) continue;
      if (k == OR_DI && !s->enable_di) continue;
      double dvr = s->vr[p] - s->vr[tp[c]];
      double dvt = s->vt[p] - s->vt[tp[c]];
      double dvz = s->vz[p] - s->vz[tp[c]];
      double g = sqrt(((dvr * dvr) + (dvt * dvt)) + (dvz * dvz));
      double sig = sigma_of(s, k, g);
      /* the cell's count times the picked target's weight */
      double dens = ((double)nt[c] * ((double)s->mult[tp[c]] * s->W)) / s->Vcell[ci];
      x[e] = ((s->dt * g) * dens) * sig;
      if (k == OR_CEE) x[e] = 0.5 * x[e];
    }
    double X = ((((((x[0] + x[1]) + x[2]) + x[3]) + x[4]) + x[5]) + x[6]) + x[7];
    double pc = 1.0 - exp(-X);
    if (!(R1 < pc)) continue;
    double u = R2 * X, c = 0.0;
    int ce = -1;
    for (int e = 0; e < OR_NELECTRON_CHANNELS; ++e) {
      c = c + x[e];
      if (u < c) { ce = e; break; }
    }
    if (ce < 0)
      for (int e = OR_NELECTRON_CHANNELS - 1; e >= 0; --e)
        if (x[e] > 0.0) { ce = e; break; }
    s->choice[p] = (uint8_t)(ECH[ce] + 1);
    s->target[p] = (uint32_t)tp[ECLS[ce]];
  }

  /* heavy projectiles (Sec. 2.3 lists ion-neutral charge exchange and
   * neutral-neutral elastic collisions; their cross sections are given
   * here as tables like the others).  They collide on the steps that move
   * them, over the heavy step K dt.  Each Cu+ draws one Cu of its cell (CEX);
   * each Cu draws one other Cu of its cell (NN), and since every pair is
   * then tried from both sides, its probability carries a factor 1/2 and
   * the partner density counts the other N - 1 atoms.  One channel each:
   * the event test is R1 < 1 - exp(-x).                                   */
  const int K = s->heavy_every;
  const int heavy_now = (K <= 1) || ((s->step % K) == 0);
  const double dth = (double)K * s->dt;
  for (int hc = 0; hc < 2 && heavy_now; ++hc) {
    const int k = hc == 0 ? OR_CEX : OR_NN;
    if (!s->xs_set[k]) continue;
    const int pc_cls = hc == 0 ? 2 : 1; /* projectile key class: Cu+ or Cu */
    for (int64_t p = s->off[pc_cls * C]; p < s->off[(pc_cls + 1) * C]; ++p) {
      int64_t cell = (int64_t)s->key[p] - (int64_t)pc_cls * C;
      int ci = (int)(cell % s->nr);
      int64_t b = s->off[C + cell], nt = s->off[C + cell + 1] - b;
      int64_t partners = hc == 0 ? nt : nt - 1;
      if (partners < 1) continue;
      uint32_t w[4], t[4];
      draw4(s, s->id[p], 0, 0, w);
      draw4(s, s->id[p], 1, 0, t);
      double R1 = u53(w[0], w[1]);
      int64_t u = (int64_t)(((uint64_t)t[0] * (uint64_t)partners) >> 32);
      if (hc == 1 && b + u >= p) u += 1; /* skip the projectile itself */
      int64_t tp = b + u;
      double dvr = s->vr[p] - s->vr[tp];
      double dvt = s->vt[p] - s->vt[tp];
      double dvz = s->vz[p] - s->vz[tp];
      double g = sqrt(((dvr * dvr) + (dvt * dvt)) + (dvz * dvz));
      double dens = ((double)partners * ((double)s->mult[tp] * s->W)) / s->Vcell[ci];
      double x = ((dth * g) * dens) * sigma_of(s, k, g);
      if (hc == 1) x = 0.5 * x;
      double pc = 1.0 - exp(-x);
      if (!(R1 < pc)) continue;
      s->choice[p] = (uint8_t)(k + 1);
      s->target[p] = (uint32_t)tp;
    }
  }

  /* claim: a particle takes part in at most one event per step; the event
   * of the lowest sorted projectile position touching it wins it (an
   * electron event touches its target, a heavy event its target and its
   * projectile), and an event happens iff it wins everything it touches */
  for (int64_t p = 0; p < n; ++p) s->claim[p] = UINT32_MAX;
  /* (with electron-electron collisions an electron can be a target, so
   * every electron event then claims its projectile as well)            */
  for (int64_t p = 0; p < n; ++p) {
    if (!s->choice[p]) continue;
    uint32_t t = s->target[p];
    if (s->claim[t] == UINT32_MAX) s->claim[t] = (uint32_t)p;
    if ((p >= n_e || cee) && s->claim[p] == UINT32_MAX) s->claim[p] = (uint32_t)p;
  }
  for (int64_t p = 0; p < n; ++p)
    if (s->choice[p]) {
      int won = s->claim[s->target[p]] == (uint32_t)p;
      if (p >= n_e || cee) won = won && s->claim[p] == (uint32_t)p;
      if (won) s->win[p] = 1;
      else s->conflicts += 1;
    }

  /* apply + create, winners in sorted order; new electrons appended with
   * ids next_id++ (the stage-2 electron first, then the stage-4 one)   */
  int64_t n_new = 0;
  for (int64_t p = 0; p < n_e; ++p)
    if (s->win[p]) n_new += (s->choice[p] == OR_EL + 1 || s->choice[p] == OR_CEI + 1 ||
                        s->choice[p] == OR_CEE + 1) ? 0 : (s->choice[p] == OR_DI + 1 ? 2 : 1);
  reserve(s, n + n_new);
  for (int64_t p = 0; p < n_e; ++p) {
    if (!s->win[p]) continue;
    int ch = s->choice[p] - 1;
    uint32_t tp = s->target[p];
    const uint16_t mt = s->mult[tp];
    int up, ut;
    take_sides(s, s->id[p], s->mult[p], mt, &up, &ut);
    double e1[3] = {s->vr[p], s->vt[p], s->vz[p]};
    double A[3] = {s->vr[tp], s->vt[tp], s->vz[tp]};
    double nh[3];
    s->events[ch] += 1;
    /* stage 1: elastic (dE = 0) or inelastic with the channel threshold */
    or_isotropic(s, s->id[p], 2, nh);
    binary(e1, A, s->two_dE_mr[ch], s->f1[ch], s->f2[ch], nh);
    if (ut) { s->vr[tp] = A[0]; s->vt[tp] = A[1]; s->vz[tp] = A[2]; }
    if (ch == OR_EL || ch == OR_CEI || ch == OR_CEE) { /* elastic */
      if (up) { s->vr[p] = e1[0]; s->vt[p] = e1[1]; s->vz[p] = e1[2]; }
      continue;
    }
    /* stage 2: the excited target emits e2, which inherits its position
     * and post-stage-1 velocity; the target keeps its slot and id        */
    if (ut) s->sp[tp] = (uint8_t)PRODUCT_OF[ch];
    double e2[3] = {A[0], A[1], A[2]};
    /* stage 3: e1-e2 elastic, equal masses (m_r/m = 1/2), isotropic    */
    or_isotropic(s, s->id[p], 3, nh);
    binary(e1, e2, 0.0, 0.5, 0.5, nh);
    int64_t q = s->n;
    if (ut) {
      s->r[q] = s->r[tp]; s->z[q] = s->z[tp];
      s->vr[q] = e2[0]; s->vt[q] = e2[1]; s->vz[q] = e2[2];
      s->sp[q] = OR_E; s->mult[q] = mt;
      s->id[q] = (uint32_t)s->next_id; s->alive[q] = 1;
      s->key[q] = key_of(s, s->r[q], s->z[q], OR_E);
      s->n += 1; s->next_id += 1; s->created += 1;
    }
    if (ch == OR_DI) {
      /* stage 4: e3 splits into two orthogonal edges of the rectangle
       * whose diagonal is v3: v5 = (v3.n)n stays, v6 = v3 - v5 is new;
       * or, literally (Eqs. 16-20), v5 = cos(chi) |v3| turned by (chi, psi)
       * about v3 with cos(chi) ~ U[0,1), psi ~ U[0,2pi) (purpose 4, draw 0) */
      double v5[3];
      if (s->split_literal) {
        uint32_t w[4];
        draw4(s, s->id[p], 4, 0, w);
        double chi = acos(u53(w[0], w[1]));
        double psi = (2.0 * PI_D) * u53(w[2], w[3]);
        or_split_literal(e1, chi, psi, v5);
      } else {
        or_isotropic(s, s->id[p], 4, nh);
        double d = ((e1[0] * nh[0]) + (e1[1] * nh[1])) + (e1[2] * nh[2]);
        v5[0] = d * nh[0]; v5[1] = d * nh[1]; v5[2] = d * nh[2];
      }
      double v6[3] = {e1[0] - v5[0], e1[1] - v5[1], e1[2] - v5[2]};
      e1[0] = v5[0]; e1[1] = v5[1]; e1[2] = v5[2];
      if (ut) {
        q = s->n;
        s->r[q] = s->r[p]; s->z[q] = s->z[p];
        s->vr[q] = v6[0]; s->vt[q] = v6[1]; s->vz[q] = v6[2];
        s->sp[q] = OR_E; s->mult[q] = mt;
        s->id[q] = (uint32_t)s->next_id; s->alive[q] = 1;
        s->key[q] = key_of(s, s->r[q], s->z[q], OR_E);
        s->n += 1; s->next_id += 1; s->created += 1;
      }
    }
    if (up) { s->vr[p] = e1[0]; s->vt[p] = e1[1]; s->vz[p] = e1[2]; }
  }

  /* heavy events: charge exchange passes the charge from the ion to the
   * atom, each keeping its position and velocity (the labels swap);
   * neutral-neutral elastic scattering is Eq. 5 with dE = 0, equal masses,
   * an isotropic direction in the centre-of-mass frame                   */
  for (int64_t p = n_e; p < s->n_sorted; ++p) {
    if (!s->win[p]) continue;
    int ch = s->choice[p] - 1;
    uint32_t tp = s->target[p];
    int up, ut;
    take_sides(s, s->id[p], s->mult[p], s->mult[tp], &up, &ut);
    s->events[ch] += 1;
    if (ch == OR_CEX) {
      uint8_t a = s->sp[p], b = s->sp[tp];
      if (up) s->sp[p] = b;
      if (ut) s->sp[tp] = a;
      continue;
    }
    double A[3] = {s->vr[p], s->vt[p], s->vz[p]};
    double B[3] = {s->vr[tp], s->vt[tp], s->vz[tp]};
    double nh[3];
    or_isotropic(s, s->id[p], 2, nh);
    binary(A, B, 0.0, s->f1[ch], s->f2[ch], nh);
    if (up) { s->vr[p] = A[0]; s->vt[p] = A[1]; s->vz[p] = A[2]; }
    if (ut) { s->vr[tp] = B[0]; s->vt[tp] = B[1]; s->vz[tp] = B[2]; }
  }
}

/* ------------------------------------------------------------------ */
/* 6. deposit, Eqs. 9-10: bilinear (cloud-in-cell) weights rounded to
 *    2^-20 per dimension; complementary weights make each particle
 *    contribute exactly Z * 2^40                                         */
void or_stage_deposit(or_sim* s) {
  const int nr = s->nr;
  int64_t nn = (int64_t)(nr + 1) * (s->nz + 1);
  memset(s->Q, 0, sizeof(int64_t) * nn);
  if (s->deposit_off) return;
  for (int64_t p = 0; p < s->n; ++p) {
    int i, j; double fr, fz;
    cell_of(s, s->r[p], s->z[p], &i, &j, &fr, &fz);
    int64_t ar = (int64_t)floor((fr * 1048576.0) + 0.5), br = 1048576 - ar;
    int64_t az = (int64_t)floor((fz * 1048576.0) + 0.5), bz = 1048576 - az;
    int64_t Zp = s->Z[s->sp[p]] * (int64_t)s->mult[p]; /* W_alpha of Eq. 9 */
    int64_t b = (int64_t)j * (nr + 1) + i;
    s->Q[b] += Zp * (br * bz);
    s->Q[b + 1] += Zp * (ar * bz);
    s->Q[b + nr + 1] += Zp * (br * az);
    s->Q[b + nr + 2] += Zp * (ar * az);
  }
}

void or_set_charge(or_sim* s, const int64_t* Q) {
  memcpy(s->Q, Q, sizeof(int64_t) * (size_t)(s->nr + 1) * (s->nz + 1));
}

/* set the node potential directly (tests of the field and gather stages) */
void or_set_potential(or_sim* s, const double* phi) {
  memcpy(s->phi, phi, sizeof(double) * (size_t)(s->nr + 1) * (s->nz + 1));
}

/* ------------------------------------------------------------------ */
/* 7. Poisson, Eq. 8 read as lap(phi) = -rho/eps0 in r-z, finite volume:
 *    Dirichlet at z = 0, L; zero flux at r = 0 and r = R.
 *    phi = phi_vac + phi_p; phi_p by a sine transform in z (DST-I over
 *    the interior z nodes), a tridiagonal solve per mode in r, and the
 *    inverse transform.  The tridiagonal solve eliminates from both ends:
 *    rows 0 .. m-1 downwards from the axis and rows nr .. m+1 upwards from
 *    the wall (m = nr / 2), each pivot's reciprocal multiplying its row;
 *    row m takes both neighbours' eliminated rows, then the back
 *    substitution runs from m outwards both ways.                       */
int or_poisson_solve(const or_sim* s, const double* f, double* phi_p) {
  const int nr = s->nr, nz = s->nz, W = nr + 1;
  double* fh = (double*)xalloc(sizeof(double) * (size_t)(nz + 1) * W);
  double* g = (double*)xalloc(sizeof(double) * (size_t)(nz + 1) * W);
  double* cp = (double*)xalloc(sizeof(double) * W);
  double* dp = (double*)xalloc(sizeof(double) * W);
  double* cq = (double*)xalloc(sizeof(double) * W);
  double* dq = (double*)xalloc(sizeof(double) * W);
  for (int k = 1; k < nz; ++k)
    for (int i = 0; i <= nr; ++i) {
      double acc = 0.0;
      for (int j = 1; j < nz; ++j)
        acc = acc + (f[(size_t)j * W + i] * s->S[(size_t)k * (nz + 1) + j]);
      fh[(size_t)k * W + i] = acc;
    }
  const int m = nr / 2;
  for (int k = 1; k < nz; ++k) {
    const double* rhs = fh + (size_t)k * W;
    const double mu = s->mu[k];
    /* rows 0 .. m-1: row i less ra[i] times the eliminated row i-1 */
    for (int i = 0; i < m; ++i) {
      double den = s->rb[i] + mu, num = rhs[i];
      if (i > 0) {
        den = den - (s->ra[i] * cp[i - 1]);
        num = num - (s->ra[i] * dp[i - 1]);
      }
      const double inv = 1.0 / den;
      cp[i] = s->rc[i] * inv;
      dp[i] = num * inv;
    }
    /* rows nr .. m+1: row i less rc[i] times the eliminated row i+1 */
    for (int i = nr; i > m; --i) {
      double den = s->rb[i] + mu, num = rhs[i];
      if (i < nr) {
        den = den - (s->rc[i] * cq[i + 1]);
        num = num - (s->rc[i] * dq[i + 1]);
      }
      const double inv = 1.0 / den;
      cq[i] = s->ra[i] * inv;
      dq[i] = num * inv;
    }
    double* x = g + (size_t)k * W;
    {
      double den = s->rb[m] + mu, num = rhs[m];
      if (m > 0) {
        den = den - (s->ra[m] * cp[m - 1]);
        num = num - (s->ra[m] * dp[m - 1]);
      }
      if (m < nr) {
        den = den - (s->rc[m] * cq[m + 1]);
        num = num - (s->rc[m] * dq[m + 1]);
      }
      x[m] = num * (1.0 / den);
    }
    for (int i = m - 1; i >= 0; --i) x[i] = dp[i] - (cp[i] * x[i + 1]);
    for (int i = m + 1; i <= nr; ++i) x[i] = dq[i] - (cq[i] * x[i - 1]);
  }
  const double scale = 2.0 / (double)nz;
  for (int j = 0; j <= nz; ++j)
    for (int i = 0; i <= nr; ++i) {
      if (j == 0 || j == nz) { phi_p[(size_t)j * W + i] = 0.0; continue; }
      double acc = 0.0;
      for (int k = 1; k < nz; ++k)
        acc = acc + (g[(size_t)k * W + i] * s->S[(size_t)k * (nz + 1) + j]);
      phi_p[(size_t)j * W + i] = acc * scale;
    }
  free(fh); free(g); free(cp); free(dp); free(cq); free(dq);
  return 0;
}

/* Residual of a potential for the node charge Q.  Each node row of the
 * finite-volume equation lap(phi) = -rho/eps0 (rho = Q qunit / V_node) is
 * multiplied by the node's control volume w_i = A_i dz, A_i the integral of
 * r dr over its radial control interval.  With phi holding the electrode
 * values on rows 0 and nz, w (rho/eps0 + lap phi) is b - A phi, and b is
 * w rho/eps0 plus w phi_electrode/dz^2 on the rows next to the electrodes. */
void or_poisson_residual(const or_sim* s, const int64_t* Q, const double* phi,
                         double* rnorm, double* bnorm) {
  const int nr = s->nr, nz = s->nz, W = nr + 1;
  const double dr = s->dr, dz = s->dz, dz2 = dz * dz;
  double rr = 0.0, bb = 0.0;
  for (int j = 1; j < nz; ++j)
    for (int i = 0; i <= nr; ++i) {
      double A;
      if (i == 0) A = (dr * dr) / 8.0;
      else if (i == nr) A = ((s->R * dr) / 2.0) - ((dr * dr) / 8.0);
      else A = ((double)i * dr) * dr;
      const double w = A * dz;
      const size_t q = (size_t)j * W + i;
      const double rho = ((double)Q[q] * s->qunit) / s->Vnode[i];
      double lap = s->rb[i] * phi[q];
      if (i > 0) lap = lap + (s->ra[i] * phi[q - 1]);
      if (i < nr) lap = lap + (s->rc[i] * phi[q + 1]);
      lap = lap + (((phi[q - W] - (2.0 * phi[q])) + phi[q + W]) / dz2);
      const double r = w * ((rho / EPS0) + lap);
      double b = w * (rho / EPS0);
      if (j == 1) b = b + ((w * phi[i]) / dz2);
      if (j == nz - 1) b = b + ((w * phi[(size_t)nz * W + i]) / dz2);
      rr = rr + (r * r);
      bb = bb + (b * b);
    }
  *rnorm = sqrt(rr);
  *bnorm = sqrt(bb);
}

void or_stage_poisson(or_sim* s) {
  const int nr = s->nr, nz = s->nz, W = nr + 1;
  size_t nn = (size_t)(nz + 1) * W;
  double* f = (double*)xalloc(sizeof(double) * nn);
  double* pp = (double*)xalloc(sizeof(double) * nn);
  for (int j = 1; j < nz; ++j)
    for (int i = 0; i <= nr; ++i) {
      double rho = ((double)s->Q[(size_t)j * W + i] * s->qunit) / s->Vnode[i];
      f[(size_t)j * W + i] = -(rho / EPS0);
    }
  or_poisson_solve(s, f, pp);
  for (int j = 0; j <= nz; ++j) {
    double vac = (-s->V) + (s->V * ((double)j / (double)nz));
    for (int i = 0; i <= nr; ++i) s->phi[(size_t)j * W + i] = vac + pp[(size_t)j * W + i];
  }
  free(f); free(pp);
}

/* 8. E = -grad(phi): central differences; second-order one-sided at the
 *    electrodes; E_r = 0 on the axis and at r = R (zero-flux wall)      */
void or_stage_field(or_sim* s) {
  const int nr = s->nr, nz = s->nz, W = nr + 1;
  const double tdz = 2.0 * s->dz, tdr = 2.0 * s->dr;
  const double* P = s->phi;
  for (int j = 0; j <= nz; ++j)
    for (int i = 0; i <= nr; ++i) {
      size_t b = (size_t)j * W + i;
      double ez;
      if (j == 0) ez = (((3.0 * P[b]) - (4.0 * P[b + W])) + P[b + 2 * W]) / tdz;
      else if (j == nz) ez = (((4.0 * P[b - W]) - (3.0 * P[b])) - P[b - 2 * W]) / tdz;
      else ez = (P[b - W] - P[b + W]) / tdz;
      double er = (i == 0 || i == nr) ? 0.0 : (P[b - 1] - P[b + 1]) / tdr;
      s->Ez[b] = ez;
      s->Er[b] = er;
    }
}

/* ------------------------------------------------------------------ */
/* Heavy-particle subcycling (Sec. 2.3: the heavy particles' time step is
 * ten times the electrons'): with heavy_every = K > 1 the electrons are
 * pushed every step with dt, the heavy species only on the steps whose
 * counter is a multiple of K, with the step K dt, and they stay where they
 * are in between (collisions still change their velocity and label).      */
int or_set_split_literal(or_sim* s, int on) {
  s->split_literal = on ? 1 : 0;
  return 0;
}

int or_set_heavy_subcycle(or_sim* s, int every) {
  if (every < 1 || every > 1000) return fail("or_set_heavy_subcycle: every must be in 1..1000");
  s->heavy_every = every;
  return 0;
}

/* 9. gather (the deposit's bilinear weights, unrounded) and leapfrog push
 *    in 2D3V: v += (q/m) E dt; straight move in the particle's local
 *    Cartesian frame; rotate back to the r-z plane                        */
static void circuit_update(or_sim* s); /* boundary physics, below */
static void sputter_yield(or_sim* s, int64_t p);
static void sputter_take(or_sim* s);

void or_stage_push(or_sim* s) {
  circuit_update(s);
  sputter_take(s);
  const int nr = s->nr, W = nr + 1;
  const int K = s->heavy_every;
  const int heavy_now = (K <= 1) || ((s->step % K) == 0);
  const double dt_h = (double)K * s->dt;
  for (int64_t p = 0; p < s->n; ++p) {
    const int heavy = s->sp[p] != OR_E;
    if (heavy && !heavy_now) {
      /* not a heavy step: the particle stays; its key follows its label */
      s->alive[p] = 1;
      s->key[p] = key_of(s, s->r[p], s->z[p], s->sp[p]);
      continue;
    }
    const double dt = (heavy && K > 1) ? dt_h : s->dt;
    int i, j; double fr, fz;
    cell_of(s, s->r[p], s->z[p], &i, &j, &fr, &fz);
    size_t b = (size_t)j * W + i;
    double gr = 1.0 - fr, gz = 1.0 - fz;
    double w00 = gr * gz, w10 = fr * gz, w01 = gr * fz, w11 = fr * fz;
    double Er = (((w00 * s->Er[b]) + (w10 * s->Er[b + 1])) + (w01 * s->Er[b + W])) + (w11 * s->Er[b + W + 1]);
    double Ez = (((w00 * s->Ez[b]) + (w10 * s->Ez[b + 1])) + (w01 * s->Ez[b + W])) + (w11 * s->Ez[b + W + 1]);
    double qm = (heavy && K > 1) ? (((double)s->Z[s->sp[p]] * Q_E) / s->m[s->sp[p]]) * dt_h
                                 : s->qmdt[s->sp[p]];
    double vr = s->vr[p] + (qm * Er);
    double vz = s->vz[p] + (qm * Ez);
    double vt = s->vt[p];
    double x = s->r[p] + (vr * dt);
    double y = vt * dt;
    double z = s->z[p] + (vz * dt);
    double rn = sqrt((x * x) + (y * y));
    if (rn > 0.0) {
      double c = x / rn, sn = y / rn;
      double vr2 = (c * vr) + (sn * vt);
      double vt2 = (c * vt) - (sn * vr);
      vr = vr2; vt = vt2;
    }
    s->r[p] = rn; s->z[p] = z;
    s->vr[p] = vr; s->vt[p] = vt; s->vz[p] = vz;
    int bnd = -1;
    if (z < 0.0) bnd = OR_CATHODE;
    else if (!(z < s->L)) bnd = OR_ANODE;
    else if (!(rn < s->R)) bnd = OR_OUTER;
    if (bnd >= 0) {
      s->alive[p] = 0;
      s->absorbed[bnd][s->sp[p]] += 1;
      s->charge_absorbed += s->Z[s->sp[p]];
      if (bnd == OR_CATHODE && s->sput_on && s->Z[s->sp[p]] > 0) sputter_yield(s, p);
    } else {
      s->alive[p] = 1;
      s->key[p] = key_of(s, rn, z, s->sp[p]);
    }
  }
}

/* 10. stable compaction of the absorbed particles, then this step's
 *     injected particles in the order given                              */
/* ------------------------------------------------------------------ */
/* Boundary physics of Sec. 2.3.
 *
 * Emission: a tip of radius r_tip at the centre of the cathode with field
 * enhancement beta.  Each cathode node i with part of its annulus
 * [(i - 1/2) dr, (i + 1/2) dr] (clipped to [0, r_tip]) inside the tip sees
 * the surface field F_i = beta * (-E_z(r_i, 0)) (E_z of this step's field,
 * the one-sided difference at the electrode) and emits the Fowler-Nordheim
 * current density J_i = (A F_i^2 / phi) exp(-B phi^(3/2) / F_i) (F_i > 0)
 * over the annulus area; I = sum_i J_i a_i in ascending i.  The step emits
 * floor(I dt / (e W) + carry) electron super-particles and, with the
 * neutral flux at the ratio rho of the electron flux, floor(rho I dt / (e W)
 * + carry') Cu atoms; the fractions carry over.  Each emitted particle
 * (id = the one it receives) draws (purpose 5) its annulus by u1 I against
 * the running sums and its radius uniform in area in it; it starts on the
 * cathode (z = 0), an electron at rest, an atom with the normal speed of
 * a flux-Maxwellian at T (sqrt((2 k T / m)(-ln(1 - u3))), no tangential
 * velocity).  They are appended after this step's scheduled particles,
 * electrons first.
 *
 * Circuit: the anode sits at the gap voltage V of a capacitor C charged
 * from V0 through R and discharged by the gap current.  Before each push
 * V <- V + (dt / C)((V0 - V) / R - I), I = -(Delta sum Z absorbed at the
 * anode since the last update) e W / dt (the charge the previous push
 * delivered); the next step's Poisson solve uses the new V.            */
int or_set_emission(or_sim* s, double beta, double r_tip, double phi_w, double ratio,
                    double T) {
  if (!(beta >= 0.0) || !(r_tip >= 0.0) || !(r_tip <= s->R) || !(phi_w > 0.0) ||
      !(ratio >= 0.0) || !(T >= 0.0) || !isfinite(beta) || !isfinite(phi_w) || !isfinite(ratio) ||
      !isfinite(T))
    return fail("or_set_emission: bad parameters");
  s->em_beta = beta; s->em_rtip = r_tip; s->em_phi = phi_w; s->em_ratio = ratio; s->em_T = T;
  return 0;
}

int or_set_circuit(or_sim* s, double V0, double R, double C) {
  if (!isfinite(V0) || !(R > 0.0) || !(C >= 0.0) || !isfinite(R) || !isfinite(C))
    return fail("or_set_circuit: bad parameters");
  s->circ_V0 = V0; s->circ_R = R; s->circ_C = C;
  int64_t za = 0;
  for (int sp = 0; sp < OR_NSPECIES; ++sp) za += (int64_t)s->Z[sp] * s->absorbed[OR_ANODE][sp];
  s->circ_zanode = za;
  return 0;
}

static void circuit_update(or_sim* s) {
  if (!(s->circ_C > 0.0)) return;
  int64_t za = 0;
  for (int sp = 0; sp < OR_NSPECIES; ++sp) za += (int64_t)s->Z[sp] * s->absorbed[OR_ANODE][sp];
  double I = ((-(double)(za - s->circ_zanode)) * (Q_E * s->W)) / s->dt;
  s->V = s->V + ((s->dt / s->circ_C) * (((s->circ_V0 - s->V) / s->circ_R) - I));
  s->circ_zanode = za;
}

/* Sputtering (Sec. 2.3, yield of Yamamura and Tawara): an ion of the Cu
 * family absorbed at the cathode with kinetic energy E (eV, from its velocity
 * after the push) adds the yield Y(E) of Cu on Cu to the annulus of its
 * nearest cathode node, i = (int)(r/dr + 1/2), in fixed point (floor of
 * Y 2^32).  Before each push the whole atoms of every annulus are taken
 * (integer part of its sum) and emitted at the end of the step: radius
 * uniform in area over the annulus, on the cathode, normal to it, with an
 * energy from the Thompson distribution E / (E + U_s)^3 truncated at 1 keV
 * (purpose 6 draws).
 *
 * Y(E) = 0.042 (Q alpha* / U_s) S_n(E) / (1 + Gamma k_e eps^0.3)
 *        (1 - sqrt(E_th / E))^s,                         E > E_th, else 0,
 * the published fit with Z1 = Z2 = 29, M1 = M2 = 63.546 u (so alpha* and
 * E_th take their equal-mass values, alpha* = 0.2525, E_th = 6.7 U_s), and
 * the Cu parameters U_s = 3.49 eV, Q = 1.30, W = 0.73, s = 2.5 (stand-ins
 * for the paper's ref. 32):
 *   eps = 0.03255 / (Z1 Z2 sqrt(Z1^(2/3) + Z2^(2/3))) M2 / (M1 + M2) E,
 *   S_n = 84.78 Z1 Z2 / sqrt(Z1^(2/3) + Z2^(2/3)) M1 / (M1 + M2) s_n(eps),
 *   s_n(eps) = 0.5 ln(1 + 1.2288 eps) / (eps + 0.1728 sqrt(eps) + 0.008 eps^0.1504),
 *   k_e = 0.079 (M1 + M2)^(3/2) / (M1^(3/2) M2^(1/2))
 *         Z1^(2/3) Z2^(1/2) / (Z1^(2/3) + Z2^(2/3))^(3/4),
 *   Gamma = W / (1 + (M1 / 7)^3).                                         */
#define YT_US 3.49
#define YT_Q 1.30
#define YT_W 0.73
#define YT_S 2.5
#define YT_EMAX 1000.0

double or_sputter_yield(double E) {
  const double Z = 29.0, M = 63.546;
  const double z23 = pow(Z, 2.0 / 3.0);
  const double zs = z23 + z23;
  const double eps = ((0.03255 / ((Z * Z) * sqrt(zs))) * (M / (M + M))) * E;
  const double sn = (0.5 * log(1.0 + (1.2288 * eps))) /
                    ((eps + (0.1728 * sqrt(eps))) + (0.008 * pow(eps, 0.1504)));
  const double Sn = (((84.78 * (Z * Z)) / sqrt(zs)) * (M / (M + M))) * sn;
  const double ke = ((0.079 * pow(M + M, 1.5)) / (pow(M, 1.5) * sqrt(M))) *
                    ((z23 * sqrt(Z)) / pow(zs, 0.75));
  const double gam = YT_W / (1.0 + pow(M / 7.0, 3.0));
  const double alpha = (0.249 * pow(M / M, 0.56)) + (0.0035 * pow(M / M, 1.5));
  const double Eth = 6.7 * YT_US;
  if (!(E > Eth)) return 0.0;
  return (((0.042 * ((YT_Q * alpha) / YT_US)) * Sn) / (1.0 + ((gam * ke) * pow(eps, 0.3)))) *
         pow(1.0 - sqrt(Eth / E), YT_S);
}

static int ring_of(const or_sim* s, double r) {
  int i = (int)((r / s->dr) + 0.5);
  return i > s->nr ? s->nr : i;
}

static void sputter_yield(or_sim* s, int64_t p) {
  const int sp = s->sp[p];
  double v2 = ((s->vr[p] * s->vr[p]) + (s->vt[p] * s->vt[p])) + (s->vz[p] * s->vz[p]);
  double E = ((0.5 * s->m[sp]) * v2) / Q_E;
  double Y = or_sputter_yield(E);
  s->sput[ring_of(s, s->r[p])] += (uint64_t)floor(Y * 4294967296.0);
}

int or_set_sputtering(or_sim* s, int on) {
  if (on && !s->sput) {
    s->sput = (uint64_t*)xalloc(sizeof(uint64_t) * (s->nr + 1));
    s->sput_now = (int64_t*)xalloc(sizeof(int64_t) * (s->nr + 1));
    memset(s->sput, 0, sizeof(uint64_t) * (s->nr + 1));
    memset(s->sput_now, 0, sizeof(int64_t) * (s->nr + 1));
  }
  s->sput_on = on ? 1 : 0;
  return 0;
}

/* before each push: the whole atoms of every annulus, taken for this step */
static void sputter_take(or_sim* s) {
  if (!s->sput_on) return;
  for (int i = 0; i <= s->nr; ++i) {
    s->sput_now[i] = (int64_t)(s->sput[i] >> 32);
    s->sput[i] -= (uint64_t)s->sput_now[i] << 32;
  }
}

static void sputter_emit(or_sim* s) {
  if (!s->sput_on) return;
  int64_t tot = 0;
  for (int i = 0; i <= s->nr; ++i) tot += s->sput_now[i];
  if (tot > 0) {
    double* a = (double*)xalloc(sizeof(double) * 5 * tot);
    uint8_t* sp = (uint8_t*)xalloc(tot);
    const double Fmax = (YT_EMAX / (YT_EMAX + YT_US)) * (YT_EMAX / (YT_EMAX + YT_US));
    int64_t k = 0;
    for (int i = 0; i <= s->nr; ++i)
      for (int64_t c = 0; c < s->sput_now[i]; ++c, ++k) {
        uint32_t id = (uint32_t)(s->next_id + k);
        uint32_t w[4];
        draw4(s, id, 6, 0, w);
        double u2 = u53(w[0], w[1]), u3 = u53(w[2], w[3]);
        double lo = ((double)i - 0.5) * s->dr, hi = ((double)i + 0.5) * s->dr;
        if (lo < 0.0) lo = 0.0;
        if (hi > s->R) hi = s->R;
        double r = sqrt((lo * lo) + (u2 * ((hi * hi) - (lo * lo))));
        if (!(r < s->R)) r = lo; /* the outer annulus' rounding at the wall */
        double q = sqrt(u3 * Fmax);
        double E = (YT_US * q) / (1.0 - q);
        a[k] = r;
        a[tot + k] = 0.0;
        a[2 * tot + k] = 0.0;
        a[3 * tot + k] = 0.0;
        a[4 * tot + k] = sqrt(((2.0 * E) * Q_E) / s->m[OR_CU]);
        sp[k] = OR_CU;
      }
    append(s, tot, a, a + tot, a + 2 * tot, a + 3 * tot, a + 4 * tot, sp, NULL);
    free(a); free(sp);
  }
  s->sputtered += tot;
}

static void emit(or_sim* s) {
  if (!(s->em_beta > 0.0)) return;
  const int nr = s->nr;
  double* cum = (double*)xalloc(sizeof(double) * (nr + 1));
  double I = 0.0;
  for (int i = 0; i <= nr; ++i) {
    double lo = ((double)i - 0.5) * s->dr, hi = ((double)i + 0.5) * s->dr;
    if (lo < 0.0) lo = 0.0;
    if (hi > s->em_rtip) hi = s->em_rtip;
    double c = 0.0;
    if (hi > lo) {
      double F = (-s->Ez[i]) * s->em_beta;
      if (F > 0.0) {
        double J = ((FN_A * (F * F)) / s->em_phi) *
                   exp(-((FN_B * (s->em_phi * sqrt(s->em_phi))) / F));
        c = J * (PI_D * ((hi * hi) - (lo * lo)));
      }
    }
    I = I + c;
    cum[i] = I;
  }
  double xe = ((I * s->dt) / (Q_E * s->W)) + s->em_acc_e;
  double xn = (((s->em_ratio * I) * s->dt) / (Q_E * s->W)) + s->em_acc_n;
  double fe = floor(xe), fn = floor(xn);
  s->em_acc_e = xe - fe;
  s->em_acc_n = xn - fn;
  int64_t ne = (int64_t)fe, nn = (int64_t)fn, tot = ne + nn;
  if (tot > 0) {
    double* a = (double*)xalloc(sizeof(double) * 5 * tot);
    uint8_t* sp = (uint8_t*)xalloc(tot);
    for (int64_t k = 0; k < tot; ++k) {
      uint32_t id = (uint32_t)(s->next_id + k);
      uint32_t w[4];
      draw4(s, id, 5, 0, w);
      double u1 = u53(w[0], w[1]), u2 = u53(w[2], w[3]);
      double target = u1 * I;
      int ring = -1;
      for (int i = 0; i <= nr; ++i)
        if (target < cum[i]) { ring = i; break; }
      if (ring < 0) /* rounding at the top: the last annulus that emits */
        for (int i = nr; i >= 0; --i)
          if (cum[i] > (i > 0 ? cum[i - 1] : 0.0)) { ring = i; break; }
      double lo = ((double)ring - 0.5) * s->dr, hi = ((double)ring + 0.5) * s->dr;
      if (lo < 0.0) lo = 0.0;
      if (hi > s->em_rtip) hi = s->em_rtip;
      a[k] = sqrt((lo * lo) + (u2 * ((hi * hi) - (lo * lo))));
      a[tot + k] = 0.0;
      a[2 * tot + k] = 0.0;
      a[3 * tot + k] = 0.0;
      if (k < ne) {
        a[4 * tot + k] = 0.0;
        sp[k] = OR_E;
      } else {
        draw4(s, id, 5, 1, w);
        double u3 = u53(w[0], w[1]);
        a[4 * tot + k] = sqrt((((2.0 * K_B) * s->em_T) / s->m[OR_CU]) * (-log(1.0 - u3)));
        sp[k] = OR_CU;
      }
    }
    append(s, tot, a, a + tot, a + 2 * tot, a + 3 * tot, a + 4 * tot, sp, NULL);
    free(a); free(sp);
  }
  s->emitted[0] += ne;
  s->emitted[1] += nn;
  free(cum);
}

void or_stage_compact_inject(or_sim* s) {
  int64_t w = 0;
  for (int64_t p = 0; p < s->n; ++p) {
    if (!s->alive[p]) continue;
    s->r[w] = s->r[p]; s->z[w] = s->z[p]; s->vr[w] = s->vr[p];
    s->vt[w] = s->vt[p]; s->vz[w] = s->vz[p]; s->sp[w] = s->sp[p];
    s->mult[w] = s->mult[p];
    s->id[w] = s->id[p]; s->key[w] = s->key[p]; s->alive[w] = 1;
    ++w;
  }
  s->n = w;
  if (s->sched_pos < s->sched_n) {
    int64_t a = s->sched_off[s->sched_pos], b = s->sched_off[s->sched_pos + 1];
    append(s, b - a, s->s_r + a, s->s_z + a, s->s_vr + a, s->s_vt + a, s->s_vz + a,
           s->s_sp + a, NULL);
    s->sched_pos += 1;
  }
  emit(s);
  sputter_emit(s);
}

void or_stage_end(or_sim* s) { s->step += 1; }

int or_step(or_sim* s, int nsteps) {
  if (!s->species_set) return fail("or_step: species not set");
  if (!s->collisions_off)
    for (int k = 0; k <= OR_SI2; ++k)
      if (!s->xs_set[k]) return fail("or_step: cross section missing");
  for (int t = 0; t < nsteps; ++t) {
    if (s->next_id + 2 * s->n > (int64_t)UINT32_MAX) return fail("or_step: id overflow");
    or_stage_sort(s);
    or_stage_collide(s);
    or_stage_deposit(s);
    or_stage_poisson(s);
    or_stage_field(s);
    or_stage_push(s);
    or_stage_compact_inject(s);
    or_stage_end(s);
  }
  return 0;
}

/* ------------------------------------------------------------------ */
int64_t or_count(const or_sim* s) { return s->n; }

void or_get_particles(const or_sim* s, double* r, double* z, double* vr,
                      double* vt, double* vz, uint8_t* sp, uint32_t* id,
                      uint32_t* key) {
  int64_t n = s->n;
  memcpy(r, s->r, sizeof(double) * n); memcpy(z, s->z, sizeof(double) * n);
  memcpy(vr, s->vr, sizeof(double) * n); memcpy(vt, s->vt, sizeof(double) * n);
  memcpy(vz, s->vz, sizeof(double) * n); memcpy(sp, s->sp, n);
  memcpy(id, s->id, sizeof(uint32_t) * n); memcpy(key, s->key, sizeof(uint32_t) * n);
}

void or_get_weights(const or_sim* s, uint16_t* mult) {
  memcpy(mult, s->mult, sizeof(uint16_t) * s->n);
}

void or_set_velocities(or_sim* s, const double* vr, const double* vt, const double* vz) {
  memcpy(s->vr, vr, sizeof(double) * s->n);
  memcpy(s->vt, vt, sizeof(double) * s->n);
  memcpy(s->vz, vz, sizeof(double) * s->n);
}

void or_get_field(const or_sim* s, double* phi, double* Er, double* Ez, int64_t* Q) {
  size_t nn = (size_t)(s->nr + 1) * (s->nz + 1);
  if (phi) memcpy(phi, s->phi, sizeof(double) * nn);
  if (Er) memcpy(Er, s->Er, sizeof(double) * nn);
  if (Ez) memcpy(Ez, s->Ez, sizeof(double) * nn);
  if (Q) memcpy(Q, s->Q, sizeof(int64_t) * nn);
}

void or_get_offsets(const or_sim* s, int64_t* offsets) {
  memcpy(offsets, s->off, sizeof(int64_t) * (OR_NKEYS * s->ncell + 1));
}

void or_get_collisions(const or_sim* s, uint8_t* choice, uint32_t* target, uint8_t* winner) {
  int64_t n = s->n_sorted;
  if (s->coll_cap < n) n = s->coll_cap;
  memcpy(choice, s->choice, n);
  memcpy(target, s->target, sizeof(uint32_t) * n);
  memcpy(winner, s->win, n);
}

void or_node_volumes(const or_sim* s, double* Vnode, double* Vcell) {
  memcpy(Vnode, s->Vnode, sizeof(double) * (s->nr + 1));
  memcpy(Vcell, s->Vcell, sizeof(double) * s->nr);
}

void or_get_diag(const or_sim* s, or_diag* d) {
  memset(d, 0, sizeof *d);
  d->step = s->step; d->n_alive = s->n; d->next_id = s->next_id;
  for (int k = 0; k < OR_NCHANNELS; ++k) d->events[k] = s->events[k];
  d->conflicts = s->conflicts; d->created = s->created;
  memcpy(d->absorbed, s->absorbed, sizeof d->absorbed);
  memcpy(d->injected, s->injected, sizeof d->injected);
  d->charge_absorbed = s->charge_absorbed;
  d->charge_injected = s->charge_injected;
  for (int64_t p = 0; p < s->n; ++p) {
    int sp = s->sp[p];
    d->count[sp] += 1;
    d->real[sp] += s->mult[p];
    d->charge_alive += s->Z[sp];
    double v2 = ((s->vr[p] * s->vr[p]) + (s->vt[p] * s->vt[p])) + (s->vz[p] * s->vz[p]);
    d->ke_J[sp] += (0.5 * s->m[sp]) * v2;
    if (sp >= OR_CU2_STEP && sp <= OR_CU2_INIT) {
      double ke = ((0.5 * s->m[sp]) * v2) / Q_E;
      int bin;
      if (ke < s->edges[0]) bin = 64;
      else if (!(ke < s->edges[64])) bin = 65;
      else { bin = 0; while (!(ke < s->edges[bin + 1])) ++bin; }
      d->spectrum[sp - OR_CU2_STEP][bin] += 1;
    }
  }
  /* Eq. 21 over the charge states q = 0..4 (N_2 counts every Cu2+ tag):
   * gamma = sum_{q>=1} N_q / sum_q N_q, qbar = sum_q q N_q / sum_{q>=1} N_q;
   * the counts are summed as integers, each ratio is one division        */
  int64_t N[5] = {d->real[OR_CU], d->real[OR_CU1],
                  d->real[OR_CU2_STEP] + d->real[OR_CU2_DOUBLE] + d->real[OR_CU2_INIT],
                  d->real[OR_CU3], d->real[OR_CU4]};
  int64_t ions = N[1] + N[2] + N[3] + N[4];
  int64_t qsum = N[1] + 2 * N[2] + 3 * N[3] + 4 * N[4];
  d->gamma = (ions + N[0]) > 0 ? (double)ions / (double)(ions + N[0]) : 0.0;
  d->qbar = ions > 0 ? (double)qsum / (double)ions : 0.0;
  d->V_gap = s->V;
  d->emitted[0] = s->emitted[0];
  d->emitted[1] = s->emitted[1];
  d->sputtered = s->sputtered;
}

/* ------------------------------------------------------------------ */
/* The literal splitting construction of Eqs. 16-20, used only to check
 * the projection form against it: shorten v by cos(chi), rotate into the
 * frame where v lies on +z, scatter by (chi, psi), rotate back.         */
void or_rotation(double theta, double phi, double Rm[9]) {
  double ct = cos(theta), st = sin(theta), cf = cos(phi), sf = sin(phi);
  Rm[0] = ct * cf; Rm[1] = ct * sf; Rm[2] = -st;
  Rm[3] = -sf;     Rm[4] = cf;      Rm[5] = 0.0;
  Rm[6] = st * cf; Rm[7] = st * sf; Rm[8] = ct;
}

static void matvec(const double M[9], const double x[3], double y[3]) {
  for (int a = 0; a < 3; ++a) y[a] = ((M[3 * a] * x[0]) + (M[3 * a + 1] * x[1])) + (M[3 * a + 2] * x[2]);
}
static void matTvec(const double M[9], const double x[3], double y[3]) {
  for (int a = 0; a < 3; ++a) y[a] = ((M[a] * x[0]) + (M[3 + a] * x[1])) + (M[6 + a] * x[2]);
}

void or_split_literal(const double v[3], double chi, double psi, double v5[3]) {
  double vm = sqrt(((v[0] * v[0]) + (v[1] * v[1])) + (v[2] * v[2]));
  double theta = (vm > 0.0) ? acos(v[2] / vm) : 0.0;
  double vp = sqrt((v[0] * v[0]) + (v[1] * v[1]));
  double phi = (vp > 0.0) ? atan2(v[1], v[0]) : 0.0; /* v along z: phi = 0 */
  double a = cos(chi);
  double sv[3] = {a * v[0], a * v[1], a * v[2]};
  double Rt[9], Rc[9], t1[3], t2[3];
  or_rotation(theta, phi, Rt);
  or_rotation(chi, psi, Rc);
  matvec(Rt, sv, t1);   /* Eq. 17: into the local frame */
  matTvec(Rc, t1, t2);  /* Eq. 18: scatter (R^-1 = R^T) */
  matTvec(Rt, t2, v5);  /* Eq. 19: back to the laboratory frame */
}
