/*
 * pd.h -- C ABI of the MI355X (gfx950) r-z electrostatic PIC-DSMC library.
 *
 * The library advances one 2D3V axisymmetric plasma in a planar diode
 * (cathode at z = 0, anode at z = L, symmetry axis r = 0, wall at r = R)
 * with the particle-in-cell / direct-simulation-Monte-Carlo step of
 * Yang et al., arXiv 2109.00214, Sec. 2:
 *   - per-cell particle lists (stable sort by species and cell),
 *   - DSMC electron-impact collisions (Sec. 2.1, Eqs. 4-7): elastic,
 *     Cu -> Cu+, Cu+ -> Cu2+ and the paper's direct Cu -> Cu2+ double
 *     ionization done as four binary stages (Sec. 2.2, Eqs. 11-15); Cu2+
 *     super-particles carry the label of the channel that made them; the
 *     step-wise chain goes on to Cu3+ and Cu4+ (Sec. 2.3) when those two
 *     channels' cross sections are set,
 *   - cloud-in-cell charge deposit (Eqs. 9-10) in int64 fixed point,
 *   - the cylindrical Poisson equation (Eq. 8) and E = -grad(phi),
 *   - field gather and leapfrog push in 2D3V (Sec. 2.1, Newton's law),
 *   - absorption at the electrodes and the wall, and injection.
 *
 * Conventions (all entry points):
 *   - Units are SI, except thresholds and spectra in eV.
 *   - Every pointer argument is a HOST pointer.  Input arrays are owned by
 *     the caller and copied during the call; output arrays are
 *     caller-allocated.  The library owns all device memory of a context.
 *   - Node arrays are node-major with r fastest: index j*(nr+1) + i for the
 *     node at r = i*R/nr, z = j*L/nz, j = 0..nz, i = 0..nr.
 *   - Particle arrays are structure-of-arrays of length n.
 *   - A non-zero return leaves the context unchanged unless stated
 *     otherwise; pd_last_error() gives a message.  No C++ exception
 *     crosses the ABI.
 *   - Calls on one context must not overlap; separate contexts are
 *     independent.  Work runs on the context's HIP stream; entry points
 *     that return data synchronise that stream first.
 *   - Results depend only on the inputs and the seed, never on the launch
 *     geometry: in the FP64 deterministic mode every integer result and
 *     every particle and node value is bit-identical to the reference
 *     arithmetic (one IEEE binary64 expression per quantity, no fused
 *     multiply-add).
 */
#ifndef PD_H
#define PD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pd_ctx pd_ctx;

typedef enum {
  PD_OK = 0,
  PD_EINVAL = -1,     /* bad argument (NaN, out of the domain, wrong size) */
  PD_ENOMEM = -2,     /* device allocation failed */
  PD_EDEVICE = -3,    /* HIP runtime error */
  PD_ESTATE = -4,     /* call not valid in the current state */
  PD_ENOCONV = -5,    /* iterative Poisson solve did not converge */
  PD_ECAPACITY = -6   /* particle capacity or 32-bit id space exhausted */
} pd_status;

/* species (fixed order); the three Cu2+ labels are separate species (they
 * must share one charge number and one mass); particles are sorted by the
 * key classes e, Cu, Cu+, Cu2+ (the three labels together), Cu3+, Cu4+ and
 * then by cell */
enum { PD_E = 0, PD_CU = 1, PD_CU1 = 2, PD_CU2_STEP = 3, PD_CU2_DOUBLE = 4,
       PD_CU2_INIT = 5, PD_CU3 = 6, PD_CU4 = 7, PD_NSPECIES = 8 };
/* collision channels.  Electron impact, in the order their probabilities
 * are summed: elastic, Cu -> Cu+, Cu -> Cu2+ (double), Cu+ -> Cu2+ (these
 * four must be set before stepping), Cu2+ of any label -> Cu3+, Cu3+ -> Cu4+.
 * Heavy projectiles (Sec. 2.3), on heavy steps over the heavy step: Cu+ + Cu
 * charge exchange (the charge passes to the atom: the two labels swap,
 * positions and velocities stay), Cu + Cu elastic (isotropic in the
 * centre-of-mass frame; each pair is tried from both sides at half weight).
 * Coulomb collisions (Sec. 2.3) of electrons with Cu+ (PD_CEI) and with other
 * electrons (PD_CEE): elastic, isotropic, with the table holding the
 * momentum-transfer cross section 4 pi lnL b90^2 (b90 = e^2 / (8 pi eps0
 * E_rel)); they follow PD_SI4 in the electrons' cumulative sum, and the
 * electron pairs are tried from both sides at half weight.  Every channel
 * from PD_SI3 on takes part only when its table is set.  A particle takes
 * part in at most one event per step: an electron event claims its target
 * (and, when PD_CEE is set, its projectile), a heavy event its target and its
 * projectile, the lowest sorted projectile position wins a claim, and an
 * event happens iff it wins all its claims. */
enum { PD_EL = 0, PD_SI = 1, PD_DI = 2, PD_SI2 = 3, PD_SI3 = 4, PD_SI4 = 5, PD_CEX = 6,
       PD_NN = 7, PD_CEI = 8, PD_CEE = 9, PD_NCHANNELS = 10 };
/* absorbing boundaries */
enum { PD_CATHODE = 0, PD_ANODE = 1, PD_OUTER = 2 };
/* precision forms: FP64 deterministic (with PD_POISSON_DIRECT64 every result
 * bit-identical to the binary64 arithmetic of the method; with
 * PD_POISSON_SPECTRAL the potential and field equal to it to rounding, the
 * integer results identical in practice), or FP32 mixed: FP32 particle record,
 * gather and push; int64 fixed-point deposit (exact); FP64 collision
 * arithmetic and diagnostics */
enum { PD_FP64_DET = 0, PD_FP32_MIXED = 1 };
/* Poisson solvers: the direct FP64 solve (sine transform in z, tridiagonal
 * in r), every sum in a fixed order (bit-identical to the method's binary64
 * arithmetic); the same direct solve with the two transforms as FP64
 * matrix-core products and the tridiagonal recurrences as parallel scans
 * (equal to the former to rounding, about 1e-15 relative, and several times
 * faster); conjugate gradients in FP32 preconditioned by a geometric
 * multigrid V-cycle inside FP64 iterative refinement; or flexible CG in FP32
 * inside the same refinement whose first direction comes from a trained
 * U-Net (pd_set_unet) applied to the residual and the others from the
 * V-cycle.  The iterative solvers start from the previous step's
 * potential and stop at the relative residual poisson_rtol; a solve that
 * does not get there falls back to the direct solve. */
enum { PD_POISSON_DIRECT64 = 0, PD_POISSON_MGPCG = 1, PD_POISSON_LEARNED = 2,
       PD_POISSON_SPECTRAL = 3 };
/* stages timed by pd_get_timing: the sort's classification and mover radix
 * passes; payload permutation (empty: the push moves the records); the
 * stayers' places with the CSR offsets; collisions (the deposit runs in
 * their first launch when collisions are on); deposit (collisions off);
 * Poisson; field (with this step's injection); push (with the counter
 * roll); injection (empty: it runs with the field) */
enum { PD_T_RADIX = 0, PD_T_PERMUTE = 1, PD_T_OFFSETS = 2, PD_T_COLLIDE = 3,
       PD_T_DEPOSIT = 4, PD_T_POISSON = 5, PD_T_FIELD = 6, PD_T_PUSH = 7,
       PD_T_INJECT = 8, PD_NTIMERS = 9 };

typedef struct {
  int32_t nr, nz;      /* cells in r and z (nr >= 2, nz >= 2) */
  double R, L;         /* wall radius and gap length, m */
  double V_cathode;    /* phi(z = 0) = -V_cathode, phi(z = L) = 0, V */
  double dt;           /* time step, s (one step for every species) */
  double weight;       /* real particles per super-particle */
  uint64_t seed;       /* Philox4x32-10 key of the collision draws */
  int64_t capacity;    /* maximum number of particles held at once */
} pd_domain;

typedef struct {
  int32_t precision;      /* PD_FP64_DET */
  int32_t poisson;        /* PD_POISSON_DIRECT64 */
  int32_t enable_di;      /* 1: include the direct Cu -> Cu2+ channel */
  int32_t deposit_off;    /* 1: skip the deposit (vacuum field), tests */
  int32_t collisions_off; /* 1: skip the DSMC stage, tests */
  int32_t timing;         /* 1: record HIP events around every stage */
  void* stream;           /* hipStream_t to run on, or NULL for a new one */
  double poisson_rtol;    /* iterative solves: target relative residual
                           * ||b - A phi|| / ||b|| of the volume-weighted
                           * system, electrode values in b (0: 1e-8) */
} pd_opts;

typedef struct {
  int64_t step, n_alive, next_id;
  int64_t count[PD_NSPECIES];
  int64_t events[PD_NCHANNELS];  /* cumulative events per channel */
  int64_t conflicts;             /* cumulative trials that lost their target */
  int64_t created;               /* cumulative electrons made by collisions */
  int64_t absorbed[3][PD_NSPECIES];
  int64_t injected[PD_NSPECIES]; /* cumulative, initial population included */
  int64_t charge_alive, charge_absorbed, charge_injected; /* sums of Z, exact */
  double ke_J[PD_NSPECIES];      /* kinetic energy per species at v(n+1/2) */
  double gamma, qbar;            /* Eq. 21 over charge states 0..4 */
  int64_t particle_steps;        /* sum over steps of the particles pushed */
  double poisson_rel_res;        /* relative residual of the current phi (FP64) */
  int64_t poisson_solves;        /* cumulative Poisson solves */
  int64_t poisson_iters;         /* cumulative CG iterations (iterative solver) */
  int64_t poisson_refinements;   /* cumulative FP64 refinement steps */
  int64_t poisson_fallbacks;     /* solves that fell back to the direct solve */
  double poisson_seconds;        /* device time of the solves made by pd_poisson
                                  * (HIP events around each solve; the steps'
                                  * solves are timed by pd_get_timing) */
  double V_gap;                  /* gap voltage the next Poisson solve uses, V */
  int64_t emitted[2];            /* cumulative super-particles emitted by the
                                  * cathode: electrons, Cu atoms (also counted
                                  * in injected) */
  int64_t sputtered;             /* cumulative Cu atoms sputtered from the
                                  * cathode (also counted in injected) */
  int64_t real[PD_NSPECIES];     /* sums of the multiplicities per species:
                                  * real particles in units of weight (equal
                                  * to count without multiplicities); gamma
                                  * and qbar are taken over these */
} pd_diag;

/* Create a context on the current HIP device for the r-z domain of the
 * 2D3V cylindrical PIC-DSMC model (Sec. 2.1: cells of nr x nz, cathode
 * at z = 0, anode at z = L, axis at r = 0).  dom and opts are copied.
 * Device memory for dom->capacity particles is allocated here.
 * PD_POISSON_SPECTRAL needs nr <= 1023 and nz <= 4096.
 * Errors: PD_EINVAL (sizes, NaN), PD_ENOMEM, PD_EDEVICE.            */
pd_status pd_create(const pd_domain* dom, const pd_opts* opts, pd_ctx** out);

/* Charge numbers Z[n] and masses mass[n] (kg) in the species order above
 * (the tracked species of Sec. 2.3 with the three Cu2+ labels of Sec. 3);
 * n must be PD_NSPECIES.  Must be called before the first step.
 * Errors: PD_EINVAL (n, a mass not positive or a charge outside -8..8,
 * Cu2+ labels of different charge or mass).                          */
pd_status pd_set_species(pd_ctx* ctx, int n, const int32_t* Z, const double* mass);

/* Integrated cross section of one channel (Eq. 4's sigma) as a table
 * uniform in sqrt(E / eV): sigma[k] at sqrt(E) = k * dsqrtE, n >= 2,
 * dsqrtE a power of two, linear interpolation, sigma = 0 below
 * threshold_eV, clamped at the last entry.  E is the energy of relative
 * motion m_r g^2 / 2.  threshold_eV is also the energy lost in the first
 * stage of an ionizing event (Sec. 2.2, Eq. 12).                     */
pd_status pd_set_cross_section(pd_ctx* ctx, int channel, double threshold_eV, int n,
                               double dsqrtE, const double* sigma);

/* Heavy-particle subcycling (Sec. 2.3: the heavy particles' time step is ten
 * times the electrons'): with every = K > 1 the electrons are pushed every
 * step with dt, the heavy species (Cu and its ions) only on the steps whose
 * counter is a multiple of K, with the step K dt, and they keep their
 * positions in between (collisions still act on them every step).  K = 1,
 * the default, pushes every species every step.  Velocities of injected
 * heavy particles are taken at the half step K dt / 2 before their first
 * push.  Errors: PD_EINVAL (K outside 1..1000), PD_ESTATE (ensemble member).*/
pd_status pd_set_heavy_subcycle(pd_ctx* ctx, int32_t every);

/* Cathode emission (Sec. 2.3): a tip of radius r_tip (m) at the centre of the
 * cathode with field-enhancement factor beta emits electrons by the
 * Fowler-Nordheim law J = (A F^2 / phi_w) exp(-B phi_w^(3/2) / F),
 * A = 1.541434e-6 A eV V^-2, B = 6.830890e9 eV^(-3/2) V m^-1, phi_w the work
 * function in eV, F = beta * (-E_z) at each cathode node whose annulus
 * [(i - 1/2) dr, (i + 1/2) dr] reaches into the tip (E_z the field stage's
 * one-sided difference at the electrode); the step emits the current's
 * super-particles (floor of I dt / (e W) plus the carried fraction) at radii
 * uniform in area over the annuli in proportion to their current, on the
 * cathode (z = 0) and at rest, and Cu atoms at neutral_ratio times that
 * flux (the paper's 3 %) with the normal speed of a flux-Maxwellian at T (K).
 * They are appended after the step's scheduled particles with the next ids.
 * beta = 0 (the default) switches emission off.  Errors: PD_EINVAL (negative
 * or non-finite values, r_tip > R, a tip wider than 1023 radial nodes),
 * PD_ESTATE (ensemble member).                                          */
pd_status pd_set_emission(pd_ctx* ctx, double beta, double r_tip, double phi_w,
                          double neutral_ratio, double T);

/* External circuit (Sec. 2.3): the gap (cathode at -V_gap, anode at 0) is a
 * capacitor C charged from the source V0 through the resistance R and
 * discharged by the gap current.  Before each step's push
 * V_gap <- V_gap + (dt / C)((V0 - V_gap) / R - I), I = -(the sum of Z of the
 * particles the previous push absorbed at the anode) e W / dt; the next
 * step's Poisson solve (and pd_poisson) uses the new V_gap.  V_gap starts at
 * V_cathode.  C = 0 switches the updates off (V_gap stays where it is).
 * Needs a direct Poisson solve.  Errors: PD_EINVAL (R <= 0, C < 0,
 * non-finite), PD_ESTATE (iterative solver, ensemble member).          */
pd_status pd_set_circuit(pd_ctx* ctx, double V0, double R, double C);

/* The last stage of a double ionization (Sec. 2.2, Eq. 15) by the literal
 * construction of Eqs. 16-20 (on != 0): v5 = R^-1(theta, phi) R^-1(chi, psi)
 * R(theta, phi) (cos(chi) v3) with the rotation matrix of Eq. 20, theta and
 * phi the polar angles of v3, cos(chi) uniform on [0, 1) and psi on
 * [0, 2 pi); v6 = v3 - v5.  The default (on = 0) is the equivalent projection
 * form v5 = (v3 . n) n with n uniform on the sphere, which needs no
 * trigonometric function.  Errors: PD_ESTATE (ensemble member).        */
pd_status pd_set_split_literal(pd_ctx* ctx, int32_t on);

/* Cathode sputtering (Sec. 2.3, yield of Yamamura and Tawara): an ion
 * absorbed at the cathode with kinetic energy E (eV, from its velocity after
 * the push) adds Y(E), the published fit for Cu on Cu at normal incidence
 * with the Cu parameters U_s = 3.49 eV, Q = 1.30, W = 0.73, s = 2.5
 * (threshold 6.7 U_s), to the annulus of its nearest cathode node, in fixed
 * point (floor of Y 2^32, so the sums are exact and order-free); the next
 * step emits the whole atoms of every annulus at radii uniform in area over
 * it, on the cathode, moving normal to it with an energy from the Thompson
 * distribution E / (E + U_s)^3 truncated at 1 keV, after the emitted
 * particles, and carries the fractions.  on = 0 (the default) switches it
 * off.  Errors: PD_EINVAL (more than 4096 cathode annuli), PD_ESTATE
 * (ensemble member).                                                   */
pd_status pd_set_sputtering(pd_ctx* ctx, int32_t on);

/* Append n super-particles now (Sec. 2.1: each stands for weight real
 * particles): positions r, z (0 <= r < R, 0 <= z < L), velocities vr, vt,
 * vz at the half step before their first push (leapfrog), species sp[n].
 * All arrays are caller host memory of length n, read during the call.  They receive ids next_id, next_id+1, ...
 * Errors: PD_EINVAL (non-finite, outside the domain, species >= 8) and
 * PD_ECAPACITY; the context is unchanged on error.                   */
pd_status pd_inject(pd_ctx* ctx, int64_t n, const double* r, const double* z,
                    const double* vr, const double* vt, const double* vz,
                    const uint8_t* sp);

/* Unequal weights (Sec. 2.2 names the rejection and the merging method for
 * super-particles of different weights; this is the rejection reading).
 * pd_set_weighted(ctx, 1) gives every record a multiplicity mu (1 for the
 * particles present; the records then stand for mu * weight real
 * particles); it cannot be turned off.  With multiplicities:
 *   - the deposit weights each particle's charge by mu (Eq. 9's W_alpha);
 *   - Eq. 4's target density is the cell's count times the picked target's
 *     weight mu_t * weight;
 *   - an event stands for min(mu_p, mu_t) real collisions: the side with
 *     the smaller multiplicity always takes the outcome, the other with
 *     probability min/its own (one Philox draw of the projectile, purpose
 *     7, draw 0); a target that takes an ionizing outcome is relabelled
 *     whole and the electrons it emits carry its multiplicity, so ionizing
 *     events conserve charge exactly (charge exchange between unequal
 *     multiplicities conserves it on average only);
 *   - scheduled, emitted and sputtered particles have multiplicity 1;
 *   - the counters of pd_diag stay counts of records (super-particles),
 *     real[] sums the multiplicities and Eq. 21 is taken over real[].
 * FP64 record only; not with the circuit (its current counts records).
 * With every mu = 1 the results are bit-identical to a context without
 * multiplicities.  Errors: PD_EINVAL (FP32, circuit on, on = 0 after on),
 * PD_ENOMEM, PD_ESTATE (in an ensemble).                                 */
pd_status pd_set_weighted(pd_ctx* ctx, int32_t on);

/* pd_inject with multiplicities mu[n] (1 <= mu <= 65535), caller host
 * memory; needs pd_set_weighted.  Errors as pd_inject, and PD_EINVAL for a
 * multiplicity of 0, PD_ESTATE without multiplicities.                   */
pd_status pd_inject_weighted(pd_ctx* ctx, int64_t n, const double* r, const double* z,
                             const double* vr, const double* vt, const double* vz,
                             const uint8_t* sp, const uint16_t* mu);

/* The multiplicities of the alive particles, in the order of
 * pd_get_particles, into a caller host array of length >= cap (all 1
 * without multiplicities).  Errors: PD_EINVAL (NULL, cap too small).     */
pd_status pd_get_weights(pd_ctx* ctx, int64_t cap, uint16_t* mu);

/* Upload an injection schedule (the cathode spot's particle source of
 * Sec. 2.3, given as explicit records) for the next nsteps steps: step k appends
 * particles offsets[k] .. offsets[k+1]-1 (offsets[0] = 0) at the end of
 * the step, after absorption, in the order given, with fresh ids.  The
 * whole schedule is copied to device memory now.  Replaces any earlier
 * schedule; steps past its end inject nothing.                        */
pd_status pd_schedule_injection(pd_ctx* ctx, int nsteps, const int64_t* offsets,
                                const double* r, const double* z, const double* vr,
                                const double* vt, const double* vz, const uint8_t* sp);

/* Enqueue nsteps full steps on the context's stream and return.  Step n
 * (the PIC-DSMC cycle of Sec. 2.1 with the collisions of Secs. 2.2-2.3):
 * sort -> collide (Eqs. 4-7, 11-15) -> deposit (Eqs. 9-10) -> Poisson
 * (Eq. 8) -> field -> gather+push -> absorb -> inject.  Needs the species
 * and, unless collisions are off, the tables of channels PD_EL..PD_SI2
 * (PD_ESTATE otherwise).  Capacity overflow found on the device is reported
 * by the next call that synchronises (PD_ECAPACITY); the context is then
 * unusable (PD_ESTATE).                                               */
pd_status pd_step(pd_ctx* ctx, int nsteps);

/* Wait for all enqueued work; reports device-side errors.            */
pd_status pd_synchronize(pd_ctx* ctx);

/* Counts, cumulative events and the snapshot reductions, among them the
 * ionization degree and mean ion charge of Eq. 21 (Sec. 3).  out is
 * caller host memory.                                                 */
pd_status pd_get_diagnostics(pd_ctx* ctx, pd_diag* out);

/* Kinetic-energy spectrum (Sec. 3.3, Figs. 8-9) of one Cu2+ label (tag 0 = step-wise, 1 =
 * direct double ionization, 2 = initial): out[0..63] count particles
 * with 10^(3b/64) <= E/eV < 10^(3(b+1)/64); out[64] counts E < 1 eV,
 * out[65] counts E >= 1000 eV.  E = M |v|^2 / 2 at v(n+1/2).          */
pd_status pd_get_spectrum(pd_ctx* ctx, int tag, int64_t out[66]);

/* Number of particles alive.                                          */
pd_status pd_get_count(pd_ctx* ctx, int64_t* n);

/* Copy the alive particles, in the order the next sort receives them,
 * into caller host arrays of length >= cap (cap >= count, else PD_EINVAL).
 * key = c * nr * nz + j * nr + i for the particle's cell (i, j) and key
 * class c (0 electrons, 1 Cu, 2 Cu+, 3 Cu2+ of every label, 4 Cu3+,
 * 5 Cu4+): the order of the per-cell lists the pairing of Sec. 2.1 draws
 * from.  Any pointer may be NULL.                                     */
pd_status pd_get_particles(pd_ctx* ctx, int64_t cap, double* r, double* z, double* vr,
                           double* vt, double* vz, uint8_t* sp, uint32_t* id,
                           uint32_t* key);

/* Potential (Eq. 8), field E = -grad(phi) and integer node charge
 * (Eqs. 9-10) of the last step ((nr+1) * (nz+1) nodes each, node-major
 * with r fastest, caller host memory; Q in units of e * weight * 2^-40).
 * Any pointer may be NULL.                                            */
pd_status pd_get_field(pd_ctx* ctx, double* phi, double* Er, double* Ez, int64_t* Q);

/* Solve the field equation for the node charge Q ((nr+1)*(nz+1) values,
 * units of e * weight * 2^-40) with the context's Poisson solver, starting
 * from the context's current potential; the context keeps Q, phi and E as
 * if a step had deposited Q.  phi (may be NULL) receives the potential,
 * iters (may be NULL) the CG iterations of this solve (0 for the direct
 * solve), rel_res (may be NULL) the relative residual reached.
 * Errors: PD_EINVAL (NULL Q), PD_ENOCONV never (the direct solve is the
 * fallback), PD_EDEVICE.                                                */
pd_status pd_poisson(pd_ctx* ctx, const int64_t* Q, double* phi, int32_t* iters,
                     double* rel_res);

/* Checkpoint of the whole state between two steps (Sec. 2: the particle
 * records, the per-cell order and offsets the next sort starts from, the node
 * charge, potential and field, the device and host counters, the collision
 * tables and the injection schedule with its position), written to one
 * binary file at `path` (host byte order, this library version's layout).
 * pd_load reads such a file into a context created with the same domain
 * (nr, nz, R, L, V, dt, weight, seed) and the same precision and switches
 * (enable_di, deposit_off, collisions_off), with capacity for the saved
 * particles; the species and cross-section tables come from the file.  A
 * context stepped on after pd_load gives bit for bit what the saved one gives
 * (for the iterative Poisson solvers: with the same solver; a network
 * attached with pd_set_unet is not part of the file).  Timing accumulators
 * are not saved.
 * Errors: PD_EINVAL (NULL path, the file cannot be opened or written, a
 * wrong magic, version, layout, domain, switch, size or count, a truncated
 * file: pd_load then leaves the context unchanged), PD_ESTATE (a member of
 * an ensemble; species not set when saving), PD_EDEVICE.               */
pd_status pd_save(pd_ctx* ctx, const char* path);
pd_status pd_load(pd_ctx* ctx, const char* path);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * fixed-order direct solve of pd_poisson for a node charge Q already in
 * device memory ((nr+1)*(nz+1) int64 values, units of e * weight * 2^-40,
 * node-major, r fastest), writing the potential phi (same layout, device
 * memory, caller-owned) on `stream` (hipStream_t; NULL: the context's
 * stream).  It enqueues four kernels and returns without synchronising:
 * no allocation, no memset, no copy.  The context supplies the grid and its
 * tables (it must not be a PD_POISSON_SPECTRAL context); the intermediate
 * arrays live in a fixed per-GPU scratch area of the library (4 MiB, held
 * until the process ends), so the grid must satisfy
 * 3 (nz-1)(nr+1) <= 524288, and calls that overlap on one GPU (different
 * streams, threads or contexts) race on it.  The scratch needs no clearing:
 * the solve writes every word before reading it.  The context's own
 * potential, field and charge are left unchanged.
 * Errors: PD_EINVAL (NULL pointers, a PD_POISSON_SPECTRAL context, a grid
 * beyond the scratch), PD_EDEVICE (current device is not the context's, or
 * a launch failure).                                                   */
pd_status pd_poisson_noalloc(pd_ctx* ctx, const int64_t* Q, double* phi, void* stream);

/* ---- ensembles of independent replicas ----------------------------------
 * Replicas (their own domain, seed, voltage, size and precision, created and
 * set up as usual with the direct Poisson solver and timing off) advance
 * together: two steps of every replica are captured once into one HIP graph
 * (replica i on worker stream i mod nstreams, so independent replicas may
 * overlap) and the graph is replayed.  The library does not own the members:
 * destroy the ensemble before them.  Calls on members between ensemble steps
 * are ordered after the ensemble's work; while a context is in an ensemble,
 * pd_step and pd_schedule_injection on it return PD_ESTATE (the graph holds
 * its buffers and the parity of its double buffer); pd_inject is allowed. */
typedef struct pd_ensemble pd_ensemble;
/* Errors: PD_EINVAL (no members, a repeated member, an iterative Poisson
 * solver, timing on), PD_ESTATE (tables not set), PD_EDEVICE (capture).  */
pd_status pd_ensemble_create(int32_t n, pd_ctx* const* members, int32_t nstreams,
                             pd_ensemble** out);
/* nsteps (even) steps of every member; returns after enqueueing.        */
pd_status pd_ensemble_step(pd_ensemble* ens, int32_t nsteps);
/* wait for the ensemble and report device errors of any member          */
pd_status pd_ensemble_synchronize(pd_ensemble* ens);
const char* pd_ensemble_last_error(const pd_ensemble* ens);
void pd_ensemble_destroy(pd_ensemble* ens);

/* ---- learned Poisson part (Eq. 8 solved with a network's help) ----------
 * A U-Net (levels, base width; 3x3 bias-free BF16 convolutions with FP32
 * accumulation and ReLU, 2x2 average pooling, nearest upsampling with skip
 * concatenation, a 1x1 FP32 output) maps [b / rms(b), r / R] -- b the
 * right-hand side of the node equations times their control volumes, on the
 * interior rows -- to the potential's charge part over its RMS, on an image
 * of the node grid (H = nz+1, W = nr+1, zero-padded to multiples of
 * 2^(levels-1); row = z node, column = r node).  Weights travel as one FP32
 * vector, layer by layer (encoder levels, then decoder levels from the
 * bottom, then the 1x1 layer), each 3x3 layer [c_out][tap][c_in] with
 * tap = 3 (dy+1) + (dx+1) the offset of the input pixel.  The network is
 * trained on the GPU on pairs dumped from a running context.  One network
 * may serve one context at a time.                                      */
typedef struct pd_unet pd_unet;

/* Network for the node grid of nr x nz cells; batch = most images per
 * forward/backward call; dataset_capacity = most stored training pairs.
 * base must be 16, 32, 48 or 64.  Weights start at zero (set them).
 * Errors: PD_EINVAL (sizes), PD_ENOMEM.                                */
pd_status pd_unet_create(int32_t nr, int32_t nz, int32_t levels, int32_t base, int32_t batch,
                         int64_t dataset_capacity, pd_unet** out);
/* number of weights; image size H x W */
pd_status pd_unet_info(const pd_unet* net, int64_t* n_params, int32_t* H, int32_t* W);
/* copy the FP32 weights in (resets the optimiser) or out */
pd_status pd_unet_set_weights(pd_unet* net, const float* w);
pd_status pd_unet_get_weights(const pd_unet* net, float* w);
/* forward of n images x[n][2][H][W] -> out[n][H][W] (host FP32 arrays) */
pd_status pd_unet_forward(pd_unet* net, int32_t n, const float* x, float* out);
/* gradient of sum(dout * out) with respect to the weights, for the same
 * inputs as pd_unet_forward (dw: n_params values)                       */
pd_status pd_unet_gradient(pd_unet* net, int32_t n, const float* x, const float* dout, float* dw);
/* store the context's current (node charge, potential) as a training pair;
 * the context's grid must be the network's.  PD_ECAPACITY when full.    */
pd_status pd_unet_add_sample(pd_unet* net, pd_ctx* ctx);
/* Adam (beta 0.9, 0.999) on minibatches of the stored pairs, mean squared
 * error of the normalised potential over the real interior nodes; loss
 * (may be NULL) receives the last epoch's mean loss.                   */
pd_status pd_unet_train(pd_unet* net, int32_t epochs, int32_t batch, double lr, uint64_t seed,
                        double* loss);
/* attach the network to a context created with PD_POISSON_LEARNED (NULL
 * detaches; the solver then uses the direct solve)                     */
pd_status pd_set_unet(pd_ctx* ctx, pd_unet* net);
const char* pd_unet_last_error(const pd_unet* net);
void pd_unet_destroy(pd_unet* net);

/* Accumulated device time per stage (ms, PD_NTIMERS entries) and the
 * number of steps timed, since creation or the last reset (requires
 * opts.timing, or pd_set_timing, for some steps).  reset != 0 clears the
 * accumulators after reading.                                          */
pd_status pd_get_timing(pd_ctx* ctx, double* ms, int64_t* steps, int reset);

/* Switch the per-stage timing on (on != 0) or off for the steps that
 * follow, as opts.timing does at creation; what was accumulated is kept.
 * The stage events cost device time (tens of microseconds per step), so a
 * throughput measurement runs with the timing off.  PD_ESTATE for a
 * member of an ensemble.                                               */
pd_status pd_set_timing(pd_ctx* ctx, int on);

/* Message of the last failed call on this context (never NULL).      */
const char* pd_last_error(const pd_ctx* ctx);

/* Free the context and its device memory.  NULL is ignored.          */
void pd_destroy(pd_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
