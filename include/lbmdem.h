/*
 * lbmdem: MI355X (gfx950) library for the four-way coupled lattice Boltzmann /
 * discrete element method of Rettinger & Ruede, "An efficient four-way coupled
 * lattice Boltzmann - discrete element method for fully resolved simulations of
 * particle-laden flows" (arXiv:2003.01490).
 *
 * One time step is Algorithm 1 of the paper:
 *   boundary conditions on particle and wall links, Eq. (MEM_CLI), with
 *   bounce-back where CLI lacks a second fluid node (Sec. 2.2);
 *   momentum-exchange force and torque per particle, Eqs. (MEM_Fq),
 *   (interaction_force), (interaction_torque), plus 2 w_q c_q for missing links,
 *   averaged over two time steps (Sec. 4.2);
 *   D3Q19 stream + collide, Eqs. (LBM_Collide), (LBM_Stream), with the adaptive
 *   TRT+aB operator of Sec. 2.3.2 (Eqs. MRT, TRTmatrix, TRTbulkmatrix);
 *   n_sub DEM sub-cycles: velocity-Verlet (Eqs. velocity_verlet_1/2),
 *   lubrication correction (Sec. 3.1), linear spring-dashpot contacts with
 *   Coulomb friction (Sec. 4.1.2), gravity and buoyancy;
 *   re-mapping of the spheres (Sec. 2.2) and PDF reconstruction in uncovered
 *   cells, Eq. (PDF_reconstruction).
 *
 * Units and layout: lattice units (dx = dt = rho0 = 1).  Cell (i,j,k) has its
 * centre at (i+1/2, j+1/2, k+1/2); arrays are x-fastest, index
 * i + nx*(j + ny*k); PDF arrays are q-major (19 planes of N cells).  An axis
 * with walls carries one wall-cell layer at each end; the wall planes lie at 1
 * and n-1.  The D3Q19 velocity order is the one fixed by rows 2-4 of the
 * moment matrix in App. A of the paper.
 *
 * Memory: every device buffer of a domain lives inside one region of
 * lbmdem_footprint_bytes() bytes.  The caller passes it in (e.g. a PyTorch
 * tensor) and keeps ownership: it must outlive the domain and is never freed
 * by the library.  With dev_buf == NULL the library allocates and frees it.
 * All device work of a domain is enqueued on the HIP stream given at creation.
 *
 * Errors: every function returns a status code (LBMDEM_OK or a negative
 * LBMDEM_E* value); nothing throws or aborts across this interface.  After a
 * failure, lbmdem_last_error() describes it.  A domain is not thread-safe;
 * distinct domains are independent.
 */
#ifndef LBMDEM_H
#define LBMDEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBMDEM_OK = 0,
  LBMDEM_EINVAL = -1,    /* invalid argument or configuration            */
  LBMDEM_ENOMEM = -2,    /* region too small / allocation failed          */
  LBMDEM_EDEVICE = -3,   /* HIP runtime error                              */
  LBMDEM_EOVERLAP = -4,  /* sphere overlaps a wall or another sphere       */
  LBMDEM_EUNSTABLE = -5, /* non-finite particle state detected             */
  LBMDEM_ECAPACITY = -6, /* max_spheres / contact, neighbour or bin slots full */
  LBMDEM_ESTATE = -7     /* domain already failed                          */
};

enum { LBMDEM_TRT_AB = 0, LBMDEM_TRT_B = 1, LBMDEM_TRT = 2, LBMDEM_SRT = 3 };
enum { LBMDEM_BC_CLI = 0, LBMDEM_BC_BOUNCE_BACK = 1 };
enum { LBMDEM_STORE_F64 = 0, LBMDEM_STORE_F32 = 1, LBMDEM_STORE_F16 = 2 };
enum { LBMDEM_FREE = 0, LBMDEM_PRESCRIBED = 1, LBMDEM_FIXED = 2 };
enum { LBMDEM_STOP_NONE = 0, LBMDEM_STOP_REBOUND = 1 };
enum {
  LBMDEM_FIELD_RHO = 0,   /* double[N]                                      */
  LBMDEM_FIELD_VEL = 1,   /* double[3N], component-major                    */
  LBMDEM_FIELD_PDF = 2,   /* double[19N], full f (not the stored deviation) */
  LBMDEM_FIELD_FLAGS = 3, /* uint8[N]: 0 fluid, 1 fluid in TRT+aB shell,
                             2 solid, 3 wall                                */
  LBMDEM_FIELD_OWNER = 4, /* int32[N]: sphere id of solid cells, else -1   */
  LBMDEM_FIELD_PDF_RAW = 5 /* double[19N]: what every cell's slots hold, solid
                              cells included (full f: stored value + w_q); the
                              slot of direction q of a solid cell y holds the
                              boundary value, Eq. (MEM_CLI), of the particle
                              link that streams from y into the fluid cell
                              y + c_q at the next step (written by the separate
                              boundary pass; map_kernel 3 forms it in the
                              sweep instead and leaves the slot unused)      */
};

typedef struct lbmdem_config {
  int32_t nx, ny, nz;
  int32_t walls[3];         /* per axis: 0 periodic, 1 wall layers at both ends */
  double wall_u_lo[3];      /* velocity of the wall at z = 1 (fluid side only)  */
  double wall_u_hi[3];      /* velocity of the wall at z = nz-1                 */
  double nu;                /* kinematic viscosity, Eq. (Viscosity)             */
  double magic_lambda;      /* Eq. (MagicParameter); paper: 3/16                */
  double lambda_b;          /* Eq. (lambda_b) in the shell; paper: 100          */
  double delta_ab;          /* TRT+aB shell thickness; paper: 2                 */
  int32_t collision;        /* LBMDEM_TRT_AB (default), _TRT_B, _TRT, _SRT      */
  int32_t boundary;         /* LBMDEM_BC_CLI (default) or _BOUNCE_BACK          */
  int32_t storage;          /* PDF storage: LBMDEM_STORE_F64/_F32/_F16; the two
                               reduced forms store f - w_q and collide in FP32 */
  int32_t n_sub;            /* DEM sub-cycles per time step; paper: 10          */
  int32_t force_averaging;  /* 1: average F_fp, T_fp over two time steps        */
  double gravity[3];
  double e_dry;             /* dry restitution coefficient                       */
  double poisson_ratio;     /* Eq. (tangentialCollisionParameters)               */
  double friction;          /* Coulomb coefficient mu_p                          */
  double tc;                /* > 0 collision time; <= 0: 2.31 D / c_s per contact */
  double dmin;              /* >= 0 minimal lubrication gap; < 0: (0.001 + 0.00007 R) R */
  double cut_n, cut_tt, cut_tr; /* lubrication cut-offs; paper: 2/3, 1/2, 1/2   */
  int32_t lub_mask;         /* bit0 normal, bit1 tangential translation, bit2 rotation */
  int32_t max_spheres;      /* capacity, sizes the device region                 */
  double max_radius;        /* largest sphere radius that will be added, <= 1000 */
  int32_t dem_kernel;       /* DEM sub-cycle kernel: 0 automatic (one workgroup up
                               to 256 spheres, else one thread per sphere), 1 one
                               workgroup (all-pairs neighbour search), 2 one
                               thread per sphere over a chain of launches
                               (binned neighbour search);
                               results are identical                              */
  int32_t map_kernel;       /* particle-link boundary pass: 0 automatic (one
                               block per sphere from 128 spheres when it fits),
                               1 several blocks per sphere (box slabs and row
                               chunks; the mapping from claims of the new
                               positions), 2 one block per sphere (EINVAL if its
                               LDS cube does not fit: a periodic axis shorter
                               than 2 (ceil(max_radius + 3) + 1) + 1 cells; the
                               mapping updated geometrically where a sphere's
                               membership changed), 3 fused: the boundary values
                               and momentum exchange are formed inside the sweep
                               and the mapping is updated geometrically; the DEM
                               then runs after the sweep (EINVAL for max_radius
                               below 1); the force sums differ in rounding
                               order                                             */
  int32_t overlap;          /* 1 (default): inside a step, the DEM kernels and
                               the claims (or mapping bins) of the new positions
                               run on a second, library-owned stream beside the
                               sweep (they need only the previous step's
                               forces); it waits on and rejoins the domain's
                               stream within the step.  0: everything on the
                               domain's stream.  Results are identical.          */
  double body_force[3];     /* fluid body force a (force density, lattice units),
                               Guo's forcing in the collision (test scenarios of
                               Sec. 2.4 such as the Stokes-flow sphere array); it
                               does not act on the spheres.  With a force the
                               velocity read-out is sum f c - a/2 (the stored
                               state is post-collision).  Default 0.            */
} lbmdem_config;

typedef struct lbmdem_domain lbmdem_domain;

/* Fills *cfg with the paper's parameters (Lambda = 3/16, Lambda_b = 100,
 * delta_aB = 2, cut-offs 2/3, 1/2, 1/2, n_sub = 10, T_c and delta_min by the
 * paper's relations) on a 32^3 domain with z walls, FP32 storage. */
int32_t lbmdem_config_init(lbmdem_config* cfg);

/* Exact number of device bytes a domain with this configuration needs.
 * Pure; makes no device call.  Returns 0 for an invalid configuration. */
size_t lbmdem_footprint_bytes(const lbmdem_config* cfg);

/* Creates a domain (Sec. 2.1: the D3Q19 lattice with walls and periodic
 * sides; Alg. 1 starts from it): fluid at rest (rho = 1, u = 0, i.e. every
 * population at its weight w_q), no spheres.  dev_buf is a
 * device region of at least lbmdem_footprint_bytes(cfg) bytes, 256-byte
 * aligned, owned by the caller (NULL: the library allocates one).  hip_stream
 * is a hipStream_t (NULL: the null stream).  *out receives the handle. */
int32_t lbmdem_create(const lbmdem_config* cfg, void* dev_buf, size_t dev_bytes,
                      void* hip_stream, lbmdem_domain** out);

/* Releases host resources and any library-owned device region.  Null-safe. */
int32_t lbmdem_destroy(lbmdem_domain* dom);

/* Adds n spheres (Sec. 3: position, translational and angular velocity,
 * radius, density; mass and moment of inertia of a solid sphere) from host
 * arrays of 3n positions, velocities, angular velocities and n radii and
 * densities, borrowed for the call.  ids_out (may be
 * NULL) receives their ids, which are dense and stable.  Returns
 * LBMDEM_EOVERLAP if a sphere crosses a wall plane or overlaps another sphere,
 * LBMDEM_ECAPACITY beyond max_spheres, LBMDEM_EINVAL if R > max_radius.
 * The particles are mapped at once. */
int32_t lbmdem_add_spheres(lbmdem_domain* dom, int32_t n, const double* x,
                           const double* u, const double* w, const double* radius,
                           const double* rho, int32_t* ids_out);

/* Overwrites positions (mask bit 0), velocities (bit 1), angular velocities
 * (bit 2) of n spheres between steps and re-maps them (the mapping of Sec.
 * 2.2; uncovered cells are reconstructed by Eq. PDF_reconstruction).  Host
 * arrays, 3 doubles per sphere. */
int32_t lbmdem_update_spheres(lbmdem_domain* dom, int32_t n, const int32_t* ids,
                              const double* x, const double* u, const double* w,
                              int32_t mask);

/* Motion mode of a sphere: LBMDEM_FREE, LBMDEM_FIXED (state never changes),
 * or LBMDEM_PRESCRIBED: velocity u_target (1 - exp(-c_acc t / t_st)) from rest
 * (Eq. artificial_acceleration), released to free motion once the gap to the
 * wall plane it approaches (ahead along u_target; Sec. 4.4.2) falls below
 * release_gap.  Without a wall ahead it stays prescribed. */
int32_t lbmdem_set_sphere_mode(lbmdem_domain* dom, int32_t id, int32_t mode,
                               const double* u_target, double c_acc, double t_st,
                               double release_gap);

/* Enqueues nsteps coupled time steps (Alg. 1 each) on the domain's stream;
 * returns without waiting. */
int32_t lbmdem_step(lbmdem_domain* dom, int32_t nsteps);

/* Step graphs (HIP graphs instead of per-kernel launches): with use_graph
 * != 0, lbmdem_step captures the launches of one step (Alg. 1) into a graph
 * on first use and replays it once per step; it is captured again when the
 * sphere count or the presence of prescribed motion changes.  Results are
 * identical to direct launches.  Needs a domain stream other than the null
 * stream (LBMDEM_EINVAL otherwise); while kernel timing is enabled steps are
 * launched directly.  Default 0. */
int32_t lbmdem_set_graph(lbmdem_domain* dom, int32_t use_graph);

/* Waits for the domain's stream and reports device-side failures:
 * LBMDEM_EUNSTABLE for a non-finite particle state or a fluid density outside
 * (0.5, 1.5) at one of up to 65536 sampled cells (the same cells on every
 * call; checked before the wait), LBMDEM_ECAPACITY for exhausted slots.  The
 * domain then stays failed (LBMDEM_ESTATE from later calls); other domains
 * are not affected. */
int32_t lbmdem_sync(lbmdem_domain* dom);

/* Number of spheres added so far. */
int32_t lbmdem_num_spheres(const lbmdem_domain* dom);

/* Synchronising copy of the state of sphere `id` (quantities of App. B and
 * Secs. 2.2, 3.1, 4.1.2, 4.2) into out[42] (host):
 *  0 x  3 u  6 w  9 F_fp 12 T_fp (averaged resolved hydrodynamic force/torque)
 * 15 F_tot 18 T_tot (total of the last sub-step) 21 F_lub 24 T_lub 27 F_col
 * 30 T_col 33 mode 34 R 35 rho 36 F_raw 39 T_raw (resolved, not averaged). */
int32_t lbmdem_get_sphere_state(lbmdem_domain* dom, int32_t id, double* out);

/* Synchronising copy of the states of n spheres (App. B quantities; ids[s],
 * or sphere s when ids is NULL) into host arrays of 3n doubles each:
 * positions, velocities,
 * angular velocities, averaged resolved force and torque (F_fp, T_fp of
 * Sec. 4.2) and total force and torque of the last sub-cycle.  Any output
 * pointer may be NULL to skip that quantity. */
int32_t lbmdem_get_spheres(lbmdem_domain* dom, int32_t n, const int32_t* ids, double* x, double* u,
                           double* w, double* F_fp, double* T_fp, double* F_tot, double* T_tot);

/* Synchronising copy of a whole-lattice field (LBMDEM_FIELD_*: density and
 * velocity are the moments of Sec. 2.1, flags and owners the mapping of Sec.
 * 2.2) to dst (host,
 * or device when dst_is_device != 0) of `bytes` bytes; non-fluid cells read 0
 * in RHO, VEL and PDF. */
int32_t lbmdem_get_field(lbmdem_domain* dom, int32_t field, void* dst, size_t bytes,
                         int32_t dst_is_device);

/* Synchronising probe: the density at n points (host xyz[3n], lattice units;
 * cell centres at i + 1/2) by trilinear interpolation of the cell-centre
 * densities of the current state, into out[n] (host).  A point whose eight
 * surrounding cells are not all fluid, or that lies beyond a wall layer,
 * reads NaN.  At most N/4 points per call (LBMDEM_EINVAL beyond). */
int32_t lbmdem_probe_density(lbmdem_domain* dom, int32_t n, const double* xyz, double* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the density
 * probe of lbmdem_probe_density with the points and results staged in a
 * static device array of the library (at most 65536 points per call; 2 MiB
 * held on each GPU the library runs on until the process ends) instead of the
 * domain region.  xyz (3n doubles) and out (n doubles) are DEVICE arrays; the
 * copies and the probe are enqueued on the domain's stream and the call
 * returns without waiting (results are ready once that stream has reached
 * them, e.g. after lbmdem_sync).  It calls no allocating routine.  Every call
 * on a GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other domains, other threads) race.  LBMDEM_EINVAL for n > 65536
 * or NULL arrays. */
int32_t lbmdem_probe_density_static(lbmdem_domain* dom, int32_t n, const double* xyz, double* out);

/* Overwrites all PDFs (the post-collision state f~ of Eq. LBM_Collide) with
 * the full distributions f (host, double[19N],
 * q-major), rounded to the storage precision, and recomputes the boundary
 * values of the next step. */
int32_t lbmdem_set_pdf(lbmdem_domain* dom, const double* f);

/* Bitwise checkpoint of a domain (Sec. 2 state: the current PDFs with the
 * boundary values of the next step, cell flags and owners, particle state,
 * contact histories, averaging memory and step count) into a host buffer.
 * With host_blob == NULL, *bytes receives the size needed; otherwise *bytes is
 * the buffer size on entry and the size written on return (LBMDEM_EINVAL and
 * the size needed if it is too small).  Synchronises the domain's stream. */
int32_t lbmdem_save(lbmdem_domain* dom, void* host_blob, size_t* bytes);

/* Restores a checkpoint written by lbmdem_save into a domain created with an
 * equal configuration (LBMDEM_EINVAL otherwise); continuing from it gives
 * results bit for bit equal to continuing the saved domain. */
int32_t lbmdem_restore(lbmdem_domain* dom, const void* host_blob, size_t bytes);

/* Stop rule of a domain, evaluated on the device at the end of every step:
 * LBMDEM_STOP_NONE, or LBMDEM_STOP_REBOUND (sphere 0: first apex after its
 * first contact has ended, i.e. u_z turns from positive to non-positive, the
 * rebound of Sec. 4.4); and/or a step limit (max_steps <= 0: none).  A domain
 * that meets it is frozen at the start of the next step: its state stays that
 * of the step that met the rule, and further steps do nothing.  Setting a rule
 * clears a previous stop. */
int32_t lbmdem_set_stop_rule(lbmdem_domain* dom, int32_t rule, int64_t max_steps);

/* Synchronising read of the step count and whether the domain has stopped. */
int32_t lbmdem_get_progress(lbmdem_domain* dom, int64_t* steps, int32_t* stopped);

/* ---- batches: many domains advanced together (continuous batching) -------
 * Not part of the paper's method: a serving layer that steps independent
 * domains of the method (each one Alg. 1 per step) in shared launches.
 * A batch steps all its admitted domains with one launch per kernel kind
 * (fused stream-collide, DEM sub-cycles, claims, reconstruction, boundary
 * pass), replayed from a captured HIP graph.  Domains keep their state in
 * their own regions; admission checks lbmdem_footprint_bytes() against the
 * batch's pool budget; a domain that meets its stop rule freezes without
 * affecting the others and can be retired and replaced between steps.
 * Domains must be created on the batch's stream, share one storage precision,
 * and use the slab boundary pass (map_kernel 1, or automatic below 128
 * spheres); a domain in a batch is stepped only through it. */
typedef struct lbmdem_batch lbmdem_batch;

/* hip_stream: the stream all batched work is enqueued on; pool_bytes: budget
 * for the summed footprints of the admitted domains. */
int32_t lbmdem_batch_create(void* hip_stream, size_t pool_bytes, lbmdem_batch** out);
int32_t lbmdem_batch_destroy(lbmdem_batch* batch);
/* 1 (default): replay one captured step graph; 0: launch directly. */
int32_t lbmdem_batch_set_graph(lbmdem_batch* batch, int32_t use_graph);
/* Admits a domain; *slot receives its id within the batch.  LBMDEM_ENOMEM if
 * the pool budget would be exceeded (admit it later). */
int32_t lbmdem_batch_admit(lbmdem_batch* batch, lbmdem_domain* dom, int32_t* slot);
/* Removes a domain (its state is kept; it may be read or stepped alone). */
int32_t lbmdem_batch_retire(lbmdem_batch* batch, lbmdem_domain* dom);
/* Enqueues nsteps steps of every admitted domain that has not stopped. */
int32_t lbmdem_batch_step(lbmdem_batch* batch, int32_t nsteps);
/* Synchronising: slots, step counts and stop flags of the admitted domains
 * (any array may be NULL); *n is the capacity on entry, the count on return. */
int32_t lbmdem_batch_status(lbmdem_batch* batch, int32_t* slots, int64_t* steps, int32_t* stopped,
                            int32_t* n);
/* Synchronising: slots of the admitted domains that have stopped; *n is the
 * capacity of slots on entry and the count on return. */
int32_t lbmdem_batch_done(lbmdem_batch* batch, int32_t* slots, int32_t* n);
const char* lbmdem_batch_last_error(const lbmdem_batch* batch);

/* Kernel timing with HIP events on the domain's stream (for roofline
 * reports).  enable: 0 off, 1 the sweep only (each event record adds a small
 * gap to the queue, so level 1 disturbs the step least), 2 every kernel group.
 * kernel: 0 fused stream-collide sweep, 1 DEM sub-cycles + mapping claims or
 * bins, 2 reconstruction + mapping update + boundary values and force partials.
 * get returns the summed milliseconds and launch count since enabling. */
int32_t lbmdem_set_profiling(lbmdem_domain* dom, int32_t enable);
int32_t lbmdem_get_profile(lbmdem_domain* dom, int32_t kernel, double* total_ms,
                           int64_t* count);

/* Algorithmic HBM bytes one sweep launch must move (19 loads + 19 stores of
 * the stored PDF type per cell plus the cell flag byte) for this domain. */
double lbmdem_sweep_bytes(const lbmdem_domain* dom);

/* Plain device-to-device copy kernel on `hip_stream` (bandwidth calibration
 * for hardware counters). */
int32_t lbmdem_device_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

/* Human-readable description of the last failure on this domain (or of the
 * last failed create when dom is NULL); valid until the next call. */
const char* lbmdem_last_error(const lbmdem_domain* dom);

#ifdef __cplusplus
}
#endif
#endif
