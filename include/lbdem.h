/*
 * lbdem.h -- C ABI of the MI355X (gfx950) library for one coupled lattice
 * Boltzmann / discrete element time step of the unresolved particle method
 * of Rettinger & Ruede, arXiv 1711.00336 (Alg. 1, Sec. 3.3).
 *
 * Units: lattice units throughout (Sec. 3.2.2, last paragraph): dx = dt = 1,
 * c_s^2 = 1/3, fluid density rho_f = 1. Cell (i,j,k) has its centre at
 * (i+1/2, j+1/2, k+1/2); flat cell index c = i + nx*(j + ny*k). On an axis
 * that is not periodic the domain is bounded by no-slip walls at the planes
 * 0 and n of that axis. PDFs are exchanged as deviations f_q - w_q from the
 * rest state, in the D3Q19 order 0 rest; 1..6 = +x,-x,+y,-y,+z,-z;
 * 7..18 = (1,1,0),(-1,-1,0),(1,-1,0),(-1,1,0),(1,0,1),(-1,0,-1),(1,0,-1),
 * (-1,0,1),(0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1).
 *
 * Ownership: the library owns all device memory of a domain. Host arrays
 * passed in are read (or written) synchronously during the call and stay
 * owned by the caller. A domain handle is not thread-safe; separate handles
 * may be used from separate threads and streams.
 *
 * Errors: every call returns an lbdem_status; nothing throws across the ABI.
 * lbdem_last_error() returns a message for the last failure of a handle
 * (or of the calling thread when the handle is NULL). After LBDEM_E_DEVICE
 * the handle should be destroyed.
 */
#ifndef LBDEM_H
#define LBDEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBDEM_OK = 0,
    LBDEM_E_INVALID = 1,   /* bad argument, out-of-domain particle, size mismatch */
    LBDEM_E_OOM = 2,       /* device allocation failed */
    LBDEM_E_UNSTABLE = 3,  /* explicit coupling estimated unstable (add_particles),
                              non-finite particle or fluid state, |u_bar| > 0.1,
                              eps_f <= 0, particle through a wall, or a particle
                              moved further than the search skin in one
                              interaction subcycle */
    LBDEM_E_DEVICE = 4,    /* HIP runtime error */
    LBDEM_E_BUSY = 5,      /* serving: result not ready / no capacity */
    LBDEM_E_STATE = 6      /* call not valid in the handle's current state */
} lbdem_status;

enum { LBDEM_FP64 = 0, LBDEM_FP32_DEV = 1 };   /* cell-field precision */
enum { LBDEM_MEM_HOST = 0, LBDEM_MEM_DEVICE = 1 };

/* Fields readable with lbdem_read_field (FP64 output, [ncomp][Nc]). */
enum {
    LBDEM_FIELD_DRHO = 0,   /* rho - 1 of the current post-stream state (1 comp) */
    LBDEM_FIELD_J = 1,      /* sum_q c_q f_q at the last step's start (3 comps) */
    LBDEM_FIELD_EPS_F = 2,  /* fluid volume fraction of the current positions (1) */
    LBDEM_FIELD_F_ACC = 3,  /* subcycle-mean force density of the last step (3) */
    LBDEM_FIELD_DUDT = 4,   /* Du_f/Dt of the last step (3) */
    LBDEM_FIELD_GRADP = 5,  /* grad P of the last step (3) */
    LBDEM_FIELD_UPREV = 6,  /* fluid-phase velocity kept for the next time derivative (3) */
    LBDEM_FIELD_PDF = 7,    /* f_q - w_q of the current state (19) */
    LBDEM_FIELD_CURL = 8    /* curl of u_f at the start of the last subcycle of
                               the last step (3; only with use_lift, else E_STATE) */
};

/* Problem statement (Sec. 3.1, 3.2; Sec. 4.1 and 5.1 setups). */
typedef struct lbdem_params {
    int32_t n[3];            /* cells per axis (>= 1) */
    int32_t periodic[3];     /* 1 periodic, 0 no-slip walls at 0 and n */
    double tau;              /* BGK relaxation time, > 1/2 (Eq. visc_tau) */
    double rho_f;            /* fluid density in the closures (1) */
    double gravity[3];       /* g, acting on the particles (Sec. 4.1) */
    double body_force[3];    /* fluid body-force density f_b (Eq. GNS) */
    int32_t body_force_auto; /* 1: fully periodic domains get
                                f_b = -sum_p (rho_p - rho_f) V_p g / (nx ny nz),
                                walled domains f_b = 0 (Sec. 4.1 Setup) */
    double e_n;              /* dry coefficient of restitution (Eq. damping_to_stiffness) */
    double mu_c;             /* Coulomb friction coefficient (Sec. 3.1.1) */
    double T_c;              /* collision time; <= 0 selects 20 DEM substeps (Eq. collision_time) */
    double h_c;              /* lubrication cut-off gap (Sec. 3.1.3) */
    double h_min;            /* lower gap limit, 1e-5 (Sec. 3.1.3) */
    int32_t lub_stab;        /* 1: also floor the gap at 3 pi mu <d>^2 dt_DEM / (2 m_ij),
                                where the leading squeeze term relaxes a pair's
                                relative velocity by a quarter per DEM substep:
                                the explicit update then stays stable for a sphere
                                with a full shell of near-touching partners */
    int32_t use_lub;         /* lubrication on/off */
    int32_t use_am;          /* added mass on/off */
    int32_t n_int;           /* interaction subcycles per LBM step (Alg. 1) */
    int32_t n_dem;           /* DEM substeps per interaction subcycle (Alg. 1) */
    double c_am;             /* added-mass coefficient, 0.5 (Table 1) */
    int32_t precision;       /* LBDEM_FP64 or LBDEM_FP32_DEV (PDFs and cell fields
                                as FP32 deviations from the rest weights; particle
                                integration and reductions stay FP64) */
    uint32_t flags;          /* LBDEM_FLAG_* bits, 0 by default */
    int32_t use_lift;        /* 1: shear-induced lift (Table 1, Saffman form)
                                F_l = 1.61 d^2 sqrt(mu rho_f/|w_f|) ((u_f - u_p) x w_f),
                                w_f the lattice curl of u_f (Sec. 3.2.3) interpolated
                                to the particle; evaluated with the added mass from
                                u_f at each subcycle start and spread with it
                                (Alg. 1); F_l = 0 where w_f = 0. Default 0. */
    int32_t use_eilers;      /* 1: per-cell relaxation time from the Eilers
                                suspension viscosity (Eq. visc_eilers, read with
                                the denominator 1 - eps_p/eps_cp; [mu] = 2.5,
                                eps_cp = 0.64) via Eq. visc_tau_*. Default 0. */
    int32_t use_les;         /* 1: add the Smagorinsky subgrid relaxation time
                                (Eqs. visc_turb, tau_t; C_s = 0.1) from the
                                non-equilibrium momentum flux. Default 0.
                                With either flag, tau_e replaces tau in the
                                collision and in the forcing prefactor; tau
                                stays the pure-fluid value of the closures. */
    int32_t lub_contact;     /* 1 (default): lubrication (Eq. lubrication_force) also
                                while two spheres or a sphere and a wall overlap,
                                with the gap clamped at h_min as the text of
                                Sec. 3.1.3 reads; 0: on the open gap only (h > 0),
                                the reading that reproduces the rebound of Sec. 5
                                (Table 3), where the clamped force overdamps the
                                contact at the Stokes numbers studied. */
} lbdem_params;

/* lbdem_params.flags: launch every kernel of a step directly instead of
 * replaying a captured HIP graph (same results, for debugging/profiling). */
#define LBDEM_FLAG_NO_GRAPH 1u

typedef struct lbdem_diag {
    double mass_dev;         /* sum_x (rho - 1) */
    double mom_fluid[3];     /* sum_x sum_q c_q f_q */
    double mom_part[3];      /* sum_p m_p u_p */
    double u_ps;             /* mean_p u_p,z - mean_x u_f,z (Sec. 4.1, relative settling velocity) */
    double mean_eps_f;
    double min_eps_f;
    double max_u;            /* max_x |u_bar| */
    int64_t step;
    int64_t np;
} lbdem_diag;

/* Full state as host arrays (checkpoint, parity injection). */
typedef struct lbdem_state_view {
    double *df;              /* [19][Nc] f_q - w_q, post-stream */
    double *uprev;           /* [3][Nc] fluid-phase velocity of the previous step */
    int64_t step;            /* steps taken (0: no time derivative yet) */
    int64_t np;              /* particle count (in: capacity of the arrays on get) */
    double *x, *u, *omega, *accel;  /* [np][3] */
    double *d, *rho_p;       /* [np] */
} lbdem_state_view;

typedef struct lbdem_domain *lbdem_domain_t;

/* Message of the last failure on h (NULL: of the calling thread). Never NULL. */
const char *lbdem_last_error(lbdem_domain_t h);

/* Paper defaults: rho_f=1, e_n=0.88, mu_c=0.25 (Sec. 4.1), h_min=1e-5
 * (Sec. 3.1.3), c_am=0.5 (Table 1), n_int=10 (Sec. 4.1), n_dem=1, T_c auto,
 * h_c=0.5, lubrication (also in contact) and added mass on, FP64, 32x32x32
 * periodic, tau=0.8. */
lbdem_status lbdem_params_default(lbdem_params *p);

/* Route device allocations through a caller allocator (e.g. a framework's
 * caching allocator). alloc returns device memory of `bytes`, aligned to 256
 * bytes as hipMalloc's is, or NULL (E_OOM); a misaligned block is released
 * and the call that needed it fails with E_INVALID. free releases a block.
 * Pass NULLs to restore hipMalloc/hipFree. Applies to domains created
 * afterwards. */
lbdem_status lbdem_set_allocator(void *(*alloc)(size_t bytes, void *ctx),
                                 void (*free_fn)(void *ptr, void *ctx), void *ctx);

/* Stability estimate of the explicit fluid-particle coupling (Alg. 1: the
 * fluid forces are frozen over an interaction subcycle of length
 * dt_int = 1/n_int, and the added mass of Table 1 uses the previous
 * subcycle's du_p/dt). Host-only: needs no device. For spheres of diameters
 * d[n] and densities rho_p[n] in the domain p, the slip relaxes with
 * tau_p = rho_p d^2 / (18 mu f(eps_ref)) (Table 1 drag at Re -> 0, mu from
 * tau by Eq. visc_tau, eps_ref = max(V_max/8, mean solid fraction)); the
 * subcycle map of the slip is stable while dt_int < (2 - 2a) tau_p with
 * a = c_am rho_f / rho_p (a = 0 without added mass). *dt_int_max receives
 * the smallest (2 - 2a) tau_p over the particles (HUGE_VAL for n = 0).
 * Returns OK if 1/p->n_int is below it, E_UNSTABLE if not, E_INVALID for a
 * bad argument. An estimate: the in-step checks remain the authority.
 * lbdem_add_particles applies it to the domain's whole particle set. */
lbdem_status lbdem_stability_limit(const lbdem_params *p, int64_t n, const double *d, const double *rho_p,
                                   double *dt_int_max);

/* Create a domain at rest (all f_q = w_q, no particles) on the current HIP
 * device. hip_stream is a hipStream_t (NULL: the library creates one).
 * E_INVALID if tau <= 1/2, a size < 1, n_int or n_dem < 1. The coupling
 * stability estimate needs the particles and runs in lbdem_add_particles. */
lbdem_status lbdem_create(const lbdem_params *p, void *hip_stream, lbdem_domain_t *out);

/* Free everything; NULL is a no-op. */
lbdem_status lbdem_destroy(lbdem_domain_t h);

/* Append n spheres (Sec. 3.1): host arrays x,u,omega [n][3], d,rho_p [n].
 * Copied synchronously; the fluid volume fraction (Eq. fluid_volume_fraction)
 * and an automatic f_b are recomputed. E_INVALID if a centre lies outside
 * the domain (on [0, n) of a periodic axis; between walls a sphere may
 * overlap a wall by less than d/2, i.e. its centre lies strictly inside
 * (0, n): a centre on or beyond the wall plane is rejected, as the step's
 * wall check would flag it), a value is not finite, d <= 0 or rho_p <= 0.
 * E_UNSTABLE, adding nothing, if lbdem_stability_limit rejects the
 * domain's particles after the addition (raise n_int). */
lbdem_status lbdem_add_particles(lbdem_domain_t h, int64_t n, const double *x, const double *u,
                                 const double *omega, const double *d, const double *rho_p);

/* Enqueue nsteps coupled time steps (Alg. 1) on the domain's stream.
 * Asynchronous: errors detected on the device surface at lbdem_sync. */
lbdem_status lbdem_step(lbdem_domain_t h, int64_t nsteps);

/* Wait for the stream; returns E_UNSTABLE if any step flagged instability:
 * a non-finite particle state, a particle through a wall or beyond the
 * search skin within a subcycle, eps_f <= 0, more list neighbours than the
 * capacity, a non-finite density or velocity of a cell at the collision
 * (non-finite PDFs), or |u_bar| > 0.1 in a cell (outside the low-Mach range
 * of the equilibrium of Eq. LBM_EQ). The message names the conditions.
 * The flags are sticky: once set, later steps skip the particle binning and
 * neighbour search (the state is no longer meaningful), lbdem_add_particles
 * returns E_STATE, and only lbdem_set_state / lbdem_load_state clear them. */
lbdem_status lbdem_sync(lbdem_domain_t h);

/* Copy one field (FP64, [ncomp][Nc]) to host or device memory `out`
 * (caller-owned, ncomp*Nc doubles). Synchronous. */
lbdem_status lbdem_read_field(lbdem_domain_t h, int field, int mem_kind, double *out);

/* Particle data in insertion order: x, u, omega, accel [np][3] (NULL skips). */
lbdem_status lbdem_read_particles(lbdem_domain_t h, int mem_kind, double *x, double *u,
                                  double *omega, double *accel);

/* Fluid-particle forces of the last subcycle [np][3] (NULL skips):
 * added mass, drag, pressure gradient, and their sum with gravity+buoyancy
 * (and the lift when use_lift is set). */
lbdem_status lbdem_read_particle_forces(lbdem_domain_t h, double *F_am, double *F_d,
                                        double *F_pr, double *F_const);

/* Lift force of the last subcycle (Table 1), [np][3] host doubles in
 * insertion order, caller-owned. E_STATE when the domain runs without lift. */
lbdem_status lbdem_read_particle_lift(lbdem_domain_t h, double *F_l);

/* FP64 reductions of the current state (Sec. 4.1 settling velocity). */
lbdem_status lbdem_diagnostics(lbdem_domain_t h, lbdem_diag *out);

/* The same reductions, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): no device allocation at all. The per-block partials and the
 * final values live in a static device array of 12 x 1024 + 16 doubles
 * (98.4 KB) that each device holds for the life of the process; its device
 * address is looked up once per device on the first call there. Results
 * equal lbdem_diagnostics exactly (same kernels, same summation order).
 * All calls on one device share the array: calls that overlap in time on
 * one device (different threads or streams) race and must be serialised by
 * the caller. E_INVALID if the reduction would need more than 1024 blocks
 * of partials (the launch caps it at 1024, so this does not happen),
 * E_DEVICE if the array's address cannot be found. */
lbdem_status lbdem_diagnostics_noalloc(lbdem_domain_t h, lbdem_diag *out);

int64_t lbdem_num_cells(lbdem_domain_t h);
int64_t lbdem_num_particles(lbdem_domain_t h);

/* Whole state as host arrays. get: v->np is the capacity of the particle
 * arrays and returns the count (E_INVALID if too small). set: replaces the
 * PDFs, u_prev, step and all particles. */
lbdem_status lbdem_get_state(lbdem_domain_t h, lbdem_state_view *v);
lbdem_status lbdem_set_state(lbdem_domain_t h, const lbdem_state_view *v);

/* Checkpoint as one opaque host blob. save with blob == NULL returns the
 * size in *size; otherwise *size must be >= the size. load validates the
 * blob against the domain's shape. */
lbdem_status lbdem_save_state(lbdem_domain_t h, void *blob, size_t *size);
lbdem_status lbdem_load_state(lbdem_domain_t h, const void *blob, size_t size);

/* Per-kernel device time for benchmarks. While timing is on
 * (lbdem_set_timing(h, 1); steps then launch kernel by kernel with HIP
 * events on the domain's stream instead of replaying graphs),
 * lbdem_kernel_time returns the total device time in ms and the number of
 * launches of one kernel class since timing was switched on. Classes:
 * 0 stream-collide, 1 moments, 2 cell fields (Du/Dt, grad P), 3 added-mass
 * particle pass (first subcycle; without lift the later subcycles' added
 * mass runs inside class 11), 4 drag/pressure particle pass, 5 added-mass
 * spreading, 6 drag spreading and f_acc, 7 volume fraction (+ next
 * added-mass spreading), 8 Verlet list build, 9 DEM contact/lubrication
 * forces, 10 DEM integration, 11 particle binning and reordering, 12
 * subcycle u_f and its curl (lift only). E_INVALID for a class outside
 * 0..12. */
lbdem_status lbdem_set_timing(lbdem_domain_t h, int on);
lbdem_status lbdem_kernel_time(lbdem_domain_t h, int cls, double *ms_total, int64_t *launches);

/* Pick launch shapes for this domain by timing them on its current state:
 * the gather variant (see lbdem_set_gather_variant), the processing order
 * of the DEM force pass (slot order, or block by block with one of a few
 * block shapes, so that the particles in flight on one XCD cover a compact
 * region whose neighbours stay in its L2 cache) and the residency of the
 * streaming cell passes. Results are bit-identical across choices: every
 * gather variant sums a cell's particles in the same order, each particle's
 * DEM force is the same in any processing order, and the cell passes are
 * cell-local. Optional out: the chosen gather variant. */
lbdem_status lbdem_autotune(lbdem_domain_t h, int32_t *gather_variant);

/* Launch choices of a domain (autotuned or set by hand). */
typedef struct lbdem_tuning {
    int32_t gather_variant;   /* as lbdem_set_gather_variant; -1 automatic by density */
    int32_t dem_order;        /* DEM force pass: -1 automatic (blocked from 2^20
                                 particles on), 0 slot order, 1 blocked order */
    int32_t dem_block[3];     /* block shape of the blocked order in cells, 1..256 each
                                 (default 32 x 32 x 32) */
    int32_t cell_waves;       /* workgroups of 256 threads per CU for the streaming
                                 cell passes (moments, stream-collide), capped with
                                 reserved LDS: -1 default (4 for FP32 storage, none
                                 for FP64), 0 no cap, 1..16 */
    int32_t fuse_substep;     /* FP32 storage with n_DEM >= 3: the contact and
                                 lubrication forces of a DEM substep and its
                                 integration (Sec. 3.1.1) in one pass, the packed
                                 records alternating between two buffers; -1 default
                                 (off), 0 off (separate passes), 1 on. Results are
                                 bit-identical either way; ignored where the form
                                 does not allow it (FP64 storage, fewer substeps) */
} lbdem_tuning;

/* Read the domain's launch choices. */
lbdem_status lbdem_get_tuning(lbdem_domain_t h, lbdem_tuning *out);

/* Set them (E_INVALID for values out of range). Synchronous. */
lbdem_status lbdem_set_tuning(lbdem_domain_t h, const lbdem_tuning *t);

/* Fix the gather variant (the launch shape of the particle-to-cell sums of
 * the volume fraction and the spread forces): -1 automatic by particle
 * density (the default), 0 LDS tiles of 16x4x8 cells, 1 LDS tiles of
 * 16x4x4, 2 LDS tiles of 8x4x4, 3 one thread per cell reading the particle
 * bins from global memory (and the drag pass one thread per particle),
 * 4 LDS tiles of 16x4x16. E_INVALID for other values. */
lbdem_status lbdem_set_gather_variant(lbdem_domain_t h, int32_t variant);

/* ---- Batching: many independent domains (e.g. a parameter sweep of the
 * settling problem of Sec. 4.1) advanced together. One batch step replays a
 * single captured HIP graph that runs every domain's full coupled step, the
 * domains spread over parallel branches. */
typedef struct lbdem_batch *lbdem_batch_t;

/* n domains from p[0..n-1] (each validated as in lbdem_create), sharing one
 * stream (hip_stream, NULL: created). Errors: lbdem_last_error(NULL). */
lbdem_status lbdem_batch_create(int32_t n, const lbdem_params *p, void *hip_stream, lbdem_batch_t *out);

/* Handle of domain i, owned by the batch (not to be destroyed): use it with
 * lbdem_add_particles, lbdem_read_*, lbdem_diagnostics, lbdem_get_state. */
lbdem_status lbdem_batch_domain(lbdem_batch_t b, int32_t i, lbdem_domain_t *out);
int32_t lbdem_batch_size(lbdem_batch_t b);

/* Run lbdem_autotune on every domain. */
lbdem_status lbdem_batch_autotune(lbdem_batch_t b);

/* Enqueue nsteps coupled steps of every domain (asynchronous). */
lbdem_status lbdem_batch_step(lbdem_batch_t b, int64_t nsteps);

/* Wait; E_UNSTABLE if any domain flagged instability (message names it). */
lbdem_status lbdem_batch_sync(lbdem_batch_t b);

lbdem_status lbdem_batch_destroy(lbdem_batch_t b);

/* ---- Serving: a request loop for settling solves (the problem of
 * Sec. 4.1) of different sizes and solid fractions. A background thread
 * admits queued requests first-come-first-served while their device
 * footprint fits the HBM budget and a slot is free, keeps admitted domains
 * resident, and advances all of them chunk_steps at a time on parallel
 * streams; requests arriving meanwhile join at the next chunk boundary. */
typedef struct lbdem_server *lbdem_server_t;

typedef struct lbdem_request {
    lbdem_params params;      /* the domain (as for lbdem_create) */
    int64_t np;               /* particles, host arrays copied at submit: */
    const double *x, *u, *omega;  /* [np][3] (u, omega may be NULL: at rest) */
    const double *d, *rho_p;      /* [np] */
    int64_t steps;            /* coupled steps to run (>= 1) */
    int64_t avg_from;         /* <u_pS> is averaged over chunk ends after this step */
} lbdem_request;

typedef struct lbdem_result {
    int32_t status;           /* LBDEM_OK, the failing call's status, or E_STATE if cancelled */
    int64_t steps_done;
    double u_ps;              /* mean relative settling velocity (Sec. 4.1), time-averaged */
    double mean_eps_f;        /* <eps_f> at the end */
    double mom[3];            /* total momentum at the end */
    double t_submit, t_admit, t_done;  /* seconds on the server's clock */
} lbdem_result;

/* Message of the last failed server call of this thread. */
const char *lbdem_server_last_error(void);

/* Start a server on the current device: hbm_budget bytes for resident
 * domains, at most max_slots resident at once, chunk_steps per scheduling
 * round. */
lbdem_status lbdem_server_create(size_t hbm_budget, int32_t max_slots, int32_t chunk_steps, lbdem_server_t *out);

/* Queue a request; E_INVALID if it can never fit the budget. */
lbdem_status lbdem_server_submit(lbdem_server_t s, const lbdem_request *r, uint64_t *ticket);

/* LBDEM_OK with the result once the solve has finished, else LBDEM_E_BUSY. */
lbdem_status lbdem_server_poll(lbdem_server_t s, uint64_t ticket, lbdem_result *out);

/* Cancel a queued or running request (its result reports E_STATE). */
lbdem_status lbdem_server_cancel(lbdem_server_t s, uint64_t ticket);

lbdem_status lbdem_server_stats(lbdem_server_t s, int64_t *queued, int64_t *active, size_t *bytes_in_use);

/* Stop the loop, free every resident domain. */
lbdem_status lbdem_server_destroy(lbdem_server_t s);

#ifdef __cplusplus
}
#endif
#endif /* LBDEM_H */
