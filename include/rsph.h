/*
 * rsph.h -- C-ABI of the MI355X (gfx950) Riemann-SPH multiphase surface-tension
 * library (librsph.so).
 *
 * Method: Zhang, Lourenco and Hu, "Multiphase SPH for surface tension: resolving
 * zero-surface-energy modes and achieving high Reynolds number simulations",
 * arXiv 2503.16082.  Two immiscible weakly compressible fluids k (phase 0) and
 * l (phase 1), each with a reference density rho0 and a dynamic viscosity eta,
 * a common sound speed c0 and one surface-tension coefficient gamma (section 2);
 * Riemann-SPH continuity and pressure terms (section 3.1, Eqs. 6-12); viscous
 * acceleration (Eq. 13); transport-velocity position correction (section 3.2,
 * Eqs. 14-15); surface stress and its divergence with the projected,
 * momentum-conserving penalty force (section 4, Eqs. 19-33); dual-criteria time
 * stepping (section 3.3, Eqs. 16-18); 5th-order Wendland kernel with h = 1.3 dp
 * and cut-off 2h (section 5).  Domains are periodic boxes; walls (the shear and
 * impact cases of section 5 use them; the paper gives no wall scheme) are
 * layers of wall particles (fluid id 2) inside the box, which never move and
 * act on the fluid through the one-sided Riemann wall condition of the
 * Riemann-SPH scheme the paper builds on: a wall neighbour is the mirror of the
 * fluid particle (its density, volume and pressure, the latter continued
 * hydrostatically by -rho g . r_ij, and the normal velocity reflected about the
 * wall's), with the fluid's viscosity against the wall's velocity (no slip) and
 * no colour.  Three layers of dp (more than the 2.6 dp support) behind a wall
 * face keep the fluid from seeing through it.
 *
 * Conventions used by every call:
 *  - every pointer argument named in a signature is a HOST pointer; the library
 *    copies inputs before returning and never keeps a caller pointer;
 *  - particle arrays are row-major (n, dim) float64 in the caller's particle
 *    order; the library keeps each particle's original index and returns
 *    particle data in that order;
 *  - the library owns all device memory of a system or pool and frees it in
 *    rsph_destroy_system / rsph_pool_release / rsph_pool_destroy;
 *  - a hip_stream passed in (a hipStream_t cast to void*) stays owned by the
 *    caller and must outlive the system; NULL makes the library create its own;
 *  - no call throws; every call returns an rsph_status and records a message
 *    retrievable with rsph_last_error;
 *  - a system (or a pool) may be used by one host thread at a time.
 */
#ifndef RSPH_H
#define RSPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rsph_system rsph_system; /* opaque, library-owned */
typedef struct rsph_pool rsph_pool;     /* opaque, library-owned */

typedef enum {
    RSPH_OK = 0,
    RSPH_EINVAL = -1,   /* invalid argument: nothing was changed */
    RSPH_ENOMEM = -2,   /* device allocation failed */
    RSPH_EDEVICE = -3,  /* HIP runtime error */
    RSPH_ESTATE = -4,   /* call not valid in the current state (no particles, faulted) */
    RSPH_ENUMERIC = -5, /* a health check tripped during stepping: the system is faulted */
    RSPH_EBUSY = -6     /* pool admission refused: HBM budget exhausted */
} rsph_status;

/* arithmetic form of the pair loops */
enum {
    RSPH_FP64 = 0, /* every operation in FP64: the reference form */
    RSPH_MIXED = 1 /* FP32 pair loops on split (cell index + FP32 offset) positions,
                      FP64 state, integrator, reductions and diagnostics; the
                      density summation in FP64 (in 3D on distances from 31-bit
                      fixed-point cell offsets, within about 1e-9 h) */
};

/* method switches (rsph_params.flags) */
#define RSPH_NO_PENALTY 1u             /* Eq. 26 instead of Eq. 33 */
#define RSPH_NO_SHIFT 2u               /* no transport-velocity position correction (Eq. 14) */
#define RSPH_NO_DENSITY_SUMMATION 4u   /* density by the continuity equation only */
#define RSPH_GBAR_OWN_PHASE_AVERAGE 8u /* mean colour gradient of a cross-phase pair as printed in Eq. 27,
                                          (grad C_i + grad C_j)/2 of the two own-phase fields, instead of the
                                          default one-field mean (grad C_i - grad C_j)/2 */
#define RSPH_PENALTY_R3 16u            /* alternative reading of the penalty tensor (Eq. 30) */
#define RSPH_NO_SURFACE 32u            /* no surface stress and no penalty */

typedef struct {
    int32_t dim;        /* 2 or 3 */
    int32_t precision;  /* RSPH_FP64 or RSPH_MIXED */
    double box[3];      /* periodic box lengths (box[2] unused in 2D) */
    double dp;          /* initial particle spacing */
    double h_over_dp;   /* smoothing length over dp [1.3] */
    double rho0[2];     /* reference densities of fluids k and l */
    double eta[2];      /* dynamic viscosities of fluids k and l (>= 0) */
    double c0;          /* common artificial sound speed (section 2: one c0 for both fluids); 0 selects
                           the section 2 rule c0 = 10 U_max with U_max = max(u_ref, largest initial |v|),
                           taken when the particles are set */
    double gamma;       /* surface-tension coefficient (>= 0) */
    double xi;          /* penalty coefficient; < 0: 1.3 n + 0.6 for a density ratio 10^n */
    double alpha_shift; /* position-correction coefficient alpha of Eq. 14 [0.2] */
    double cfl_ad;      /* advection time-step factor of Eq. 16 [0.1] */
    double cfl_ac;      /* acoustic time-step factor of Eq. 17 [0.6] */
    double gravity[3];  /* body force g of Eq. 2 [0] */
    uint32_t flags;     /* RSPH_NO_* switches [0] */
    uint32_t reserved;
    double u_ref;       /* anticipated largest flow speed of the c0 = 0 rule (>= 0) [0] */
} rsph_params;

/* Observables of one system, all FP64, reduced on the device in a fixed order
 * over the fluid particles (wall particles are left out). */
typedef struct {
    double t;             /* simulated time */
    int64_t n_outer;      /* advection steps taken */
    int64_t n_sub;        /* acoustic substeps taken */
    double dt_ad;         /* last advection step (Eqs. 16, 18) */
    double dt_ac;         /* last acoustic substep (Eqs. 17, 18, clipped to the advection step) */
    double momentum[3];   /* sum m v */
    double kinetic;       /* sum m |v|^2 / 2 */
    double mass[2];       /* per fluid */
    double volume[2];     /* per fluid, sum m / rho */
    double vmax[2];       /* per fluid max |v| */
    double centroid[3];   /* fluid k, mass weighted, box coordinates */
    double moment2[9];    /* fluid k, mass-weighted second moment about the centroid */
    double r_eq;          /* equivalent radius of the fluid-k volume */
    double p_in;          /* mean pressure of fluid k with |r - centroid| < r_eq - 3h */
    double p_out;         /* mean pressure of fluid l with |r - centroid| > r_eq + 3h */
    double n_in, n_out;   /* particle counts of the two means */
    uint32_t health;      /* RSPH_HEALTH_* bits */
    uint32_t displaced_steps; /* advection steps whose binning found a particle more than one cell
                                 (edge >= 2h, periodic distance) from where the previous binning put
                                 it.  A diagnostic, not a fault: the first advection step from rest is
                                 bounded by the viscous criterion of Eq. 16 alone and may carry
                                 particles that far with the geometry frozen (section 3.3). */
} rsph_observables;

#define RSPH_HEALTH_NONFINITE 1u  /* NaN or Inf in velocity, density or acceleration */
#define RSPH_HEALTH_DENSITY 2u    /* rho <= 0 */
#define RSPH_HEALTH_NEIGHBOURS 4u /* more neighbours than the list holds */
#define RSPH_HEALTH_COINCIDENT 8u /* two neighbours closer than 1e-9 h */
#define RSPH_HEALTH_DT 32u        /* acoustic step collapsed below 1e-12 of its no-flow value */

/* particle fields readable with rsph_read_particles, and their width per particle */
enum {
    RSPH_FIELD_POS = 0,    /* dim */
    RSPH_FIELD_VEL = 1,    /* dim */
    RSPH_FIELD_RHO = 2,    /* 1 */
    RSPH_FIELD_P = 3,      /* 1: c0^2 (rho - rho0) */
    RSPH_FIELD_DRHO = 4,   /* 1: last continuity rate */
    RSPH_FIELD_MASS = 5,   /* 1 */
    RSPH_FIELD_PHASE = 6,  /* 1 (0.0, 1.0, or 2.0 for a wall particle) */
    /* rates of the last rsph_eval_rates: */
    RSPH_FIELD_ACC = 7,    /* dim: a^p + a^s + a^v + g */
    RSPH_FIELD_ACC_P = 8,  /* dim: Riemann pressure acceleration (Eq. 7) */
    RSPH_FIELD_ACC_S = 9,  /* dim: surface stress divergence plus penalty (Eq. 33) */
    RSPH_FIELD_ACC_V = 10, /* dim: viscous acceleration (Eq. 13) */
    RSPH_FIELD_GRADC = 11, /* dim: colour gradient (Eq. 22) */
    RSPH_FIELD_RATE_DRHO = 12, /* 1: continuity rate (Eq. 6) */
    RSPH_FIELD_B = 13,     /* dim*dim: correction matrix (Eq. 15), row-major */
    RSPH_FIELD_DR = 14,    /* dim: position correction (Eq. 14), not applied */
    RSPH_FIELD_SIGMA = 15, /* 1: W(0) + sum_j W_ij */
    RSPH_FIELD_NNB = 16,   /* 1: neighbour count */
    RSPH_FIELD_FLAGS = 17, /* 1: 1 = has a neighbour of the other fluid, +2 = it or a neighbour has */
    RSPH_FIELD_COUNT = 18
};

/* Fills *p with the documented defaults: 2D, FP64, unit box, dp = 0.02, h = 1.3 dp
 * (section 5), alpha = 0.2 (Eq. 14), CFL factors 0.1 and 0.6 (Eqs. 16-17), xi by
 * the rule of section 4.2, c0 = 1. */
void rsph_params_default(rsph_params* p);

/* Creates an empty system (no particles yet) for the problem of section 2:
 * two immiscible weakly compressible fluids k and l (rho0, eta per fluid), one
 * sound speed c0 for both (Eq. 3) and one surface-tension coefficient gamma,
 * discretised with the Wendland kernel of section 5 (h = 1.3 dp, cut-off 2h) in
 * a periodic box.  Validates params: dim in {2,3}; dp, rho0 > 0; c0 > 0, or
 * c0 = 0 with u_ref >= 0 (the section 2 rule, applied by rsph_set_particles);
 * eta, gamma >= 0; at least 3 cells of edge >= 2h per axis and at most 512;
 * all values finite.  hip_stream: a hipStream_t owned by the caller, or NULL
 * for a stream of the library's own.  *out is owned by the caller and freed with
 * rsph_destroy_system.  EINVAL (nothing created) otherwise. */
rsph_status rsph_create_system(const rsph_params* params, void* hip_stream, rsph_system** out);

/* Sets (or resets) all particles of the two-fluid system of section 2, each a
 * Lagrangian particle with position, velocity, fluid and mass (section 3.1):
 * pos, vel (n x dim), phase (n, in {0,1}, or 2 for a wall particle, whose
 * velocity is the wall's), mass (n, NULL -> rho0[phase] / sigma0 with sigma0 the
 * lattice kernel sum, so a perfect lattice has rho = rho0; 1 / sigma0 for a
 * wall particle), rho (n, NULL -> rho0[phase], 1 for a wall particle; it sets
 * the initial pressure by Eq. 3).  Positions are
 * wrapped into the box.  With c0 = 0 in the system's params, c0 becomes
 * 10 max(u_ref, largest |vel|, walls included) here (section 2).  Resets t, counters, density
 * rates and the fault state unless opts has RSPH_KEEP_CLOCK (then t and
 * counters are kept: resume).  The arrays are host memory owned by the caller
 * and copied before the call returns.  EINVAL (nothing changed) on n < 1 or
 * n > 2^26 (the slots of one pool), NaN/Inf, a phase outside {0,1,2}, mass or
 * rho <= 0, two particles closer than 1e-3 dp, or c0 = 0 with u_ref = 0 and
 * every velocity zero.  When every particle of a fluid has the same mass (the
 * default masses do), the substep passes take that mass from the system's
 * constants: results are the same either way, to rounding.
 * The extra rho argument (beyond particles, velocities, fluids and masses) lets
 * a caller restore a state for a bitwise resume. */
#define RSPH_KEEP_CLOCK 1u
rsph_status rsph_set_particles(rsph_system* sys, int64_t n, const double* pos, const double* vel,
                               const int32_t* phase, const double* mass, const double* rho,
                               uint32_t opts);

/* Restores the continuity rates D rho / Dt of Eq. 6 (n doubles, caller order,
 * host memory copied before return) after rsph_set_particles(...,
 * RSPH_KEEP_CLOCK), for a bitwise resume: the dual-criteria scheme of section
 * 3.3 carries the rate from one acoustic substep to the next.  EINVAL if n
 * differs from the particle count, ESTATE without particles. */
rsph_status rsph_set_drho(rsph_system* sys, int64_t n, const double* drho);

/* Advances n_outer advection steps of the dual-criteria scheme (section 3.3,
 * Eqs. 16-18), each with its own data-dependent number of acoustic substeps
 * that integrate Eqs. 1-2 as discretised by Eqs. 6-15 and 21-33; returns when
 * they are done (synchronises the stream).  EINVAL on n_outer < 0; ESTATE
 * without particles or when faulted; ENUMERIC if a health check trips (the
 * system is then faulted and later steps return ESTATE until
 * rsph_set_particles resets it). */
rsph_status rsph_step(rsph_system* sys, int64_t n_outer);

/* One evaluation, at the current state and with no update, of the neighbour
 * geometry, kernel sum, viscous acceleration (Eq. 13), correction matrix
 * (Eq. 15), position correction (Eq. 14), colour gradient (Eq. 22),
 * accelerations (Eqs. 7-12 and 33) and continuity rate (Eqs. 6, 9), with the
 * density as set and the pressure of Eq. 3; read them with
 * rsph_read_particles.  ESTATE without particles. */
rsph_status rsph_eval_rates(rsph_system* sys);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * single evaluation as rsph_create_system + rsph_set_particles +
 * rsph_eval_rates + rsph_read_particles(ACC, RATE_DRHO), with every particle
 * array in DEVICE memory owned by the caller and no device allocation by the
 * library.  pos, vel (n x dim), phase (n), mass and rho (n, or NULL for the
 * defaults of rsph_set_particles) are read; acc (n x dim) and drho_rate (n)
 * are written, in the caller's particle order, on hip_stream (NULL: the null
 * stream); the call returns when they are written.  Everything else lives in
 * one fixed 64 MiB array per device that the library holds until the process
 * ends (about 65,000 particles in 2D and 40,000 in 3D): larger inputs are
 * rejected with EINVAL.  Calls on one device share that array, so calls that
 * overlap on one device (two host threads, or two streams) race.  params must
 * have c0 > 0.  EINVAL also for a fluid id outside {0,1,2}, a non-finite value, a
 * mass or density <= 0, or two particles closer than 1e-3 dp. */
rsph_status rsph_eval_rates_noalloc(const rsph_params* params, int64_t n, const double* pos,
                                    const double* vel, const int32_t* phase, const double* mass,
                                    const double* rho, double* acc, double* drho_rate, void* hip_stream);

/* Reduces the observables on the device and copies them to *out (caller
 * owned): clock and step counts (section 3.3), total momentum (conserved by
 * the antisymmetric pair terms of sections 3.1 and 4), kinetic energy, fluid
 * masses and volumes, and the fluid-k centroid, second moment and mean inner
 * and outer pressures from which the oscillation period (Eq. 35) and the
 * Young-Laplace jump (Eq. 37) are measured.  ESTATE without particles. */
rsph_status rsph_read_observables(rsph_system* sys, rsph_observables* out);

/* Copies one field (RSPH_FIELD_*) of all n particles, caller order, into out
 * (host memory, n * width doubles, caller owned): the state of section 3.1
 * (position, velocity, density, Eq. 3 pressure, mass, fluid) or a rate of the
 * last rsph_eval_rates.  EINVAL if n differs from the system's particle count
 * or the field is unknown; ESTATE for a rate field before an evaluation. */
rsph_status rsph_read_particles(rsph_system* sys, int32_t field, int64_t n, double* out);

/* Binning of the last rebuild (the cell-linked list behind the kernel's
 * compact support of section 5, cells of edge >= 2h): per particle (caller
 * order) its cell key cx + nx (cy + ny cz) and its rank in cell order (cells
 * ascending, then x ascending, then caller index ascending), into caller-owned
 * host arrays of n entries.  EINVAL if n differs from the particle count. */
rsph_status rsph_read_binning(rsph_system* sys, int64_t n, uint32_t* key, int64_t* rank);

/* Neighbour lists of the last rebuild in caller indices: every j != i with
 * |r_ij| < 2h, the support of the kernel of section 5, frozen for the
 * advection step (section 3.3).  start has n + 1 entries, idx up to cap
 * entries (caller-owned host arrays), each list in the library's stencil order.
 * EINVAL if cap is too small or n differs from the particle count. */
rsph_status rsph_read_neighbours(rsph_system* sys, int64_t n, int64_t cap, int64_t* start,
                                 int64_t* idx);

/* Kernel timing: kernel_mask selects kernels by bit (1 << RSPH_KERNEL_*; 0 turns
 * timing off).  Every launch of a selected kernel is bracketed by HIP events on
 * the system's stream; rsph_read_kernel_timing returns, per kernel, the number
 * of launches that did work and their summed duration in milliseconds since the
 * last call of rsph_set_kernel_timing (which resets the totals). */
enum {
    RSPH_KERNEL_BIN = 0,
    RSPH_KERNEL_NEIGHBOURS = 1,
    RSPH_KERNEL_ADVECTION = 2,
    RSPH_KERNEL_SHIFT = 3,
    RSPH_KERNEL_COLOUR = 4,
    RSPH_KERNEL_FORCE = 5,
    RSPH_KERNEL_CONTINUITY = 6,
    RSPH_KERNEL_EVENT_FLOOR = 7, /* an empty one-block kernel bracketed the same way,
                                    launched 32 times when timing is switched on */
    RSPH_KERNEL_COUNT = 8
};
rsph_status rsph_set_kernel_timing(rsph_system* sys, int32_t kernel_mask);
rsph_status rsph_read_kernel_timing(rsph_system* sys, int64_t* launches, double* ms);

/* Launch mode of the stepping calls (rsph_step, rsph_pool_step) of the pool
 * that holds sys.  RSPH_LAUNCH_GRAPH (the default): each launch cycle (the
 * advection-step prologue and the acoustic substeps that follow it) is
 * captured once as a HIP graph on the pool's stream and replayed; a graph is
 * kept per substep count and per pool layout, and is captured again after an
 * admission or release changes the layout.  RSPH_LAUNCH_EAGER: every kernel
 * is launched individually.  Both modes launch the same kernels with the same
 * arguments, so their results are identical bit for bit.  While kernel timing
 * is on, launches are eager.  Synchronises the stream.  RSPH_EINVAL for an
 * unknown mode. */
enum { RSPH_LAUNCH_GRAPH = 0, RSPH_LAUNCH_EAGER = 1 };
rsph_status rsph_set_launch_mode(rsph_system* sys, int32_t mode);

/* Frees the system and its device memory.  NULL is ignored. */
void rsph_destroy_system(rsph_system* sys);

const char* rsph_status_string(rsph_status s);
/* Last error message of a system (or of the library when sys is NULL). */
const char* rsph_last_error(const rsph_system* sys);

/* ---- serving: many systems packed in one device array ------------------- */

/* Serving many independent simulations of the section 2 problem at once.
 * A pool packs the particles of many systems of one dimension and one
 * precision into shared device arrays and steps them together in the same
 * launches, each system with its own parameters and its own dual-criteria time
 * steps (section 3.3).  dim and precision are fixed per pool because every
 * member shares the pool's kernels and record layout.  hbm_budget_bytes bounds
 * the device memory the pool may hold (0: no bound); a pool with a bound takes
 * all of it at its first admission, so that later admissions seldom
 * reallocate.  *out is freed with rsph_pool_destroy.  EINVAL on a bad dim or
 * precision. */
rsph_status rsph_pool_create(int32_t dim, int32_t precision, size_t hbm_budget_bytes,
                             void* hip_stream, rsph_pool** out);
/* Admits a system of the section 2 problem with its particles (as
 * rsph_create_system followed by rsph_set_particles, with params->dim and
 * params->precision equal to the pool's).  EBUSY if the budget cannot hold it
 * now; EINVAL on bad input.  The returned system is owned by the pool: read it
 * with the rsph_read_* calls, release it with rsph_pool_release. */
rsph_status rsph_pool_admit(rsph_pool* pool, const rsph_params* params, int64_t n,
                            const double* pos, const double* vel, const int32_t* phase,
                            const double* mass, rsph_system** out);
/* Advances each of the count systems by n_outer[k] advection steps of the
 * dual-criteria scheme (section 3.3), each with its own substeps; all of them
 * progress in the same launches until each has done its own count.  ENUMERIC
 * if a member's health check trips: that member is faulted (its later steps
 * return ESTATE), the others keep the steps they took and may be stepped
 * again; release the faulted one with rsph_pool_release. */
rsph_status rsph_pool_step(rsph_pool* pool, rsph_system* const* systems, const int64_t* n_outer,
                           int32_t count);
/* Bytes of device memory the pool holds now (with a budget: the budget's worth
 * once the first system is admitted). */
size_t rsph_pool_bytes(const rsph_pool* pool);
/* Counts of a system (standalone or in a pool) as of the end of its last
 * stepping call, held on the host (no device access): advection steps and
 * acoustic substeps taken, and the most substeps one of its recent advection
 * steps needed (Eqs. 16-18 set that count).  Before the system's first step
 * the last figure is an estimate for that step from the uploaded velocities;
 * after it, 0 until a later step has been seen, since a first step from rest
 * is bounded by the viscous criterion alone.  A scheduler can give systems
 * that need few substeps per advection step more advection steps per stepping
 * call.  EINVAL on a NULL argument. */
rsph_status rsph_step_counts(const rsph_system* sys, int64_t* n_outer, int64_t* n_sub,
                             int64_t* substeps_per_step);
/* Removes a system (section 2 problem) from its pool and frees its slots; the
 * systems packed after it move down.  sys is invalid afterwards.  EINVAL if
 * sys is not a member of pool. */
rsph_status rsph_pool_release(rsph_pool* pool, rsph_system* sys);
/* Frees the pool and every system still in it. */
void rsph_pool_destroy(rsph_pool* pool);

#ifdef __cplusplus
}
#endif

#endif /* RSPH_H */
