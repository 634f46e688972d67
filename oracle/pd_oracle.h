/*
 * pd_oracle.h -- plain, slow FP64 CPU oracle for one r-z electrostatic
 * PIC-DSMC step with the four electron-impact channels of Yang et al.,
 * "The role of double ionization on the generation of doubly charged ions
 * in copper vacuum arcs" (arXiv 2109.00214).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant generator with the GPU library; the two
 * agree only through the written arithmetic contract (one IEEE binary64
 * expression per quantity, evaluated left to right as parenthesised, no
 * contraction into fused multiply-add).
 *
 * All functions are single-threaded.  Errors return a negative int and set
 * a message readable with or_last_error().
 */
#ifndef PD_ORACLE_H
#define PD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* species enum (fixed order); the three Cu2+ tags are separate species; the
 * step-wise chain goes on to Cu3+ and Cu4+ (Sec. 2.3) */
enum { OR_E = 0, OR_CU = 1, OR_CU1 = 2, OR_CU2_STEP = 3, OR_CU2_DOUBLE = 4,
       OR_CU2_INIT = 5, OR_CU3 = 6, OR_CU4 = 7, OR_NSPECIES = 8 };
/* classes of the sort key: e, Cu, Cu+, Cu2+ (the three tags together), Cu3+,
 * Cu4+ */
enum { OR_NKEYS = 6 };
/* collision channels.  Electron impact, in cumulative-sum order: elastic,
 * Cu -> Cu+, Cu -> Cu2+ (double), Cu+ -> Cu2+, Cu2+ -> Cu3+, Cu3+ -> Cu4+.
 * Heavy projectiles: Cu+ + Cu charge exchange, Cu + Cu elastic.  Coulomb
 * collisions of electrons with Cu+ and with other electrons, as elastic
 * channels with a tabulated momentum-transfer cross section.  Channels from
 * SI3 on take part only when their cross sections are set. */
enum { OR_EL = 0, OR_SI = 1, OR_DI = 2, OR_SI2 = 3, OR_SI3 = 4, OR_SI4 = 5,
       OR_CEX = 6, OR_NN = 7, OR_CEI = 8, OR_CEE = 9, OR_NCHANNELS = 10 };
/* the electron-impact channels, in cumulative-sum order: the six above, then
 * the Coulomb channels electron-Cu+ and electron-electron */
enum { OR_NELECTRON_CHANNELS = 8 };
/* absorbing boundaries */
enum { OR_CATHODE = 0, OR_ANODE = 1, OR_OUTER = 2 };

typedef struct or_sim or_sim;

typedef struct {
  int64_t step, n_alive, next_id;
  int64_t count[OR_NSPECIES];
  int64_t events[OR_NCHANNELS];     /* cumulative */
  int64_t conflicts;                /* cumulative */
  int64_t created;                  /* cumulative electrons made by collisions */
  int64_t absorbed[3][OR_NSPECIES]; /* cumulative, per boundary */
  int64_t injected[OR_NSPECIES];    /* cumulative, incl. initial population */
  int64_t charge_alive, charge_absorbed, charge_injected; /* sum of Z */
  double ke_J[OR_NSPECIES];
  double gamma, qbar; /* Eq. 21 over the charge states 0..4 */
  int64_t spectrum[3][66]; /* Cu2+ tags STEP, DOUBLE, INIT: 64 bins, <1 eV, >=1000 eV */
  double V_gap;            /* the gap voltage the next Poisson solve uses */
  int64_t emitted[2];      /* cumulative super-particles emitted: electrons, atoms */
  int64_t sputtered;       /* cumulative Cu atoms sputtered from the cathode */
  int64_t real[OR_NSPECIES]; /* sum of the multiplicities (real particles / W);
                              * Eq. 21 is taken over these */
} or_diag;

or_sim* or_create(int nr, int nz, double R, double L, double V, double dt,
                  double weight, uint64_t seed, int enable_di,
                  int deposit_off, int collisions_off);
void or_destroy(or_sim* s);
const char* or_last_error(void);

int or_set_species(or_sim* s, int n, const int* Z, const double* mass);
int or_set_cross_section(or_sim* s, int channel, double threshold_eV, int n,
                         double dsqrtE, const double* sigma);
int or_inject(or_sim* s, int64_t n, const double* r, const double* z,
              const double* vr, const double* vt, const double* vz,
              const uint8_t* sp);
/* unequal weights: particle p stands for mult[p] * W real particles
 * (1 <= mult <= 65535); or_inject gives every particle multiplicity 1, as
 * do the schedule, the emission and the sputtering                        */
int or_inject_weighted(or_sim* s, int64_t n, const double* r, const double* z,
                       const double* vr, const double* vt, const double* vz,
                       const uint8_t* sp, const uint16_t* mult);
void or_get_weights(const or_sim* s, uint16_t* mult);
int or_schedule_injection(or_sim* s, int nsteps, const int64_t* offsets,
                          const double* r, const double* z, const double* vr,
                          const double* vt, const double* vz, const uint8_t* sp);
int or_step(or_sim* s, int nsteps);
/* heavy-particle subcycling: heavy species advance every `every` steps with
 * the step every*dt (1, the default: every step) */
int or_set_heavy_subcycle(or_sim* s, int every);
/* boundary physics (Sec. 2.3): Fowler-Nordheim emission from a tip of radius
 * r_tip with field enhancement beta and work function phi_w (eV), with Cu
 * atoms emitted at neutral_ratio times the electron flux at temperature T
 * (beta = 0: off); the gap voltage of an RC circuit (source V0, resistance
 * R, capacitance C; C = 0: off, the voltage stays fixed)                 */
int or_set_emission(or_sim* s, double beta, double r_tip, double phi_w, double neutral_ratio,
                    double T);
int or_set_circuit(or_sim* s, double V0, double R, double C);
/* the double ionization's last stage by the literal construction of Eqs.
 * 16-20 (cos chi ~ U[0,1), psi ~ U[0,2pi)) instead of the projection form */
int or_set_split_literal(or_sim* s, int on);
/* sputtering of the cathode by the ions that reach it (Yamamura-Tawara
 * yield of Cu on Cu), emitted the step after the impacts               */
int or_set_sputtering(or_sim* s, int on);
double or_sputter_yield(double E_eV);

/* stage-level entry points (a full step is these in this order) */
void or_stage_sort(or_sim* s);
void or_stage_collide(or_sim* s);
void or_stage_deposit(or_sim* s);
void or_stage_poisson(or_sim* s);
void or_stage_field(or_sim* s);
void or_stage_push(or_sim* s);
void or_stage_compact_inject(or_sim* s);
void or_stage_end(or_sim* s); /* step counter += 1 */

int64_t or_count(const or_sim* s);
void or_get_particles(const or_sim* s, double* r, double* z, double* vr,
                      double* vt, double* vz, uint8_t* sp, uint32_t* id,
                      uint32_t* key);
void or_set_velocities(or_sim* s, const double* vr, const double* vt,
                       const double* vz);
void or_get_field(const or_sim* s, double* phi, double* Er, double* Ez,
                  int64_t* Q);
/* set the node charge directly (tests of the Poisson stage) */
void or_set_charge(or_sim* s, const int64_t* Q);
/* set the node potential directly (tests of the field and gather stages) */
void or_set_potential(or_sim* s, const double* phi);
void or_get_offsets(const or_sim* s, int64_t* offsets); /* OR_NKEYS*nr*nz + 1 */
/* per-electron decisions of the last collide stage, in sorted order */
void or_get_collisions(const or_sim* s, uint8_t* choice, uint32_t* target,
                       uint8_t* winner);
void or_get_diag(const or_sim* s, or_diag* d);

/* pure building blocks, exposed for the pin tests */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int or_poisson_solve(const or_sim* s, const double* f, double* phi_p);
/* ||b - A phi||_2 and ||b||_2 of the Poisson system written over the
 * interior z rows with every node row multiplied by its control volume
 * (which makes A symmetric), the electrode values of phi moved into b */
void or_poisson_residual(const or_sim* s, const int64_t* Q, const double* phi,
                         double* rnorm, double* bnorm);
void or_isotropic(const or_sim* s, uint32_t id, uint32_t purpose, double n[3]);
void or_rotation(double theta, double phi, double Rm[9]);
void or_split_literal(const double v[3], double chi, double psi, double v5[3]);
void or_node_volumes(const or_sim* s, double* Vnode, double* Vcell);
double or_cross_section(const or_sim* s, int channel, double g);

#ifdef __cplusplus
}
#endif
#endif
