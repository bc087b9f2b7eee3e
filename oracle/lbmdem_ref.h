/*
 * Oracle of the four-way coupled lattice Boltzmann / discrete element method of
 * Rettinger & Ruede, "An efficient four-way coupled lattice Boltzmann - discrete
 * element method for fully resolved simulations of particle-laden flows".
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64 CPU
 * implementation written from the paper to check the GPU library against.  Only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or helper with the GPU library.
 *
 * Conventions (lattice units: dx = dt = rho0 = 1, c_s^2 = 1/3, Sec. 2.1):
 *   - cell (i,j,k) has its centre at (i+1/2, j+1/2, k+1/2); arrays are x-fastest,
 *     index = i + nx*(j + ny*k); PDF arrays are q-major: f[q*N + index].
 *   - an axis with walls has one wall-cell layer at each end (index 0 and n-1);
 *     the wall planes lie half-way, at 1 and n-1.
 *   - canonical cell codes returned by ref_get_flags: 0 fluid, 1 fluid inside the
 *     bulk-viscosity shell, 2 solid (owner >= 0), 3 wall.
 *
 * Status codes: 0 ok, -1 invalid argument, -2 out of memory, -4 overlap at
 * insertion, -6 capacity exceeded.
 */
#ifndef LBMDEM_REF_H
#define LBMDEM_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ref_config {
  int32_t nx, ny, nz;
  int32_t walls[3];        /* per axis: 0 periodic, 1 wall layers at both ends   */
  double wall_u_lo[3];     /* velocity of the wall at z = 1 (fluid side only)    */
  double wall_u_hi[3];     /* velocity of the wall at z = nz-1                   */
  double nu;               /* kinematic viscosity, Eq. (Viscosity)               */
  double magic_lambda;     /* Lambda of Eq. (MagicParameter), 3/16               */
  double lambda_b;         /* Lambda_b of Eq. (lambda_b), 100 for TRT+aB         */
  double delta_ab;         /* shell thickness of TRT+aB, 2                        */
  int32_t collision;       /* 0 TRT+aB, 1 TRT+B (global), 2 TRT, 3 SRT           */
  int32_t boundary;        /* 0 CLI with bounce-back fallback, 1 bounce-back     */
  int32_t n_sub;           /* DEM sub-cycles per LBM step                         */
  int32_t force_averaging; /* 1: average F_fp over two time steps                 */
  double gravity[3];
  double e_dry;            /* dry coefficient of restitution                      */
  double poisson_ratio;    /* nu_p of Eq. (tangentialCollisionParameters)        */
  double friction;         /* mu_p, Coulomb friction coefficient                  */
  double tc;               /* > 0: collision time; <= 0: T_c = 2.31 D / c_s       */
  double dmin;             /* >= 0: minimal lubrication gap; < 0: Eq. (lubricationGapSize) */
  double cut_n, cut_tt, cut_tr; /* lubrication cut-offs, Eq. (lubricationCutOff)  */
  int32_t lub_mask;        /* bit0 normal, bit1 tangential translation, bit2 rotation */
  int32_t max_spheres;
  double body_force[3];    /* fluid body force (Guo forcing), test scenarios only */
} ref_config;

typedef struct ref_domain ref_domain;

/* Sphere state vector returned by ref_get_sphere (REF_SPHERE_OUT doubles):
 *  0 x[3]  3 u[3]  6 w[3]  9 F_fp[3] 12 T_fp[3] (averaged resolved hydrodynamic)
 * 15 F_tot[3] 18 T_tot[3] (last sub-step total)  21 F_lub[3] 24 T_lub[3]
 * 27 F_col[3] 30 T_col[3] 33 mode 34 R 35 rho 36 F_raw[3] 39 T_raw[3] (un-averaged) */
#define REF_SPHERE_OUT 42

/* lattice constants: c[q*3+a], w[q], opp[q] */
void ref_lattice(int32_t* c, double* w, int32_t* opp);
/* moment matrix M (row-major 19x19) as printed in App. A, and its inverse */
void ref_moment_matrix(double* M);
int ref_moment_inverse(double* Minv);
/* relaxation rates s_nu, s_nu^-, s_b from the config */
void ref_rates(const ref_config* cfg, double* s_nu, double* s_minus, double* s_b);
/* incompressible equilibrium f^eq_q(rho, u) */
void ref_equilibrium(double rho, const double* u, double* feq);
/* one MRT collision of a single cell; shell selects Lambda_b for TRT+aB;
 * force may be NULL (no body force) */
void ref_collide(const ref_config* cfg, const double* f, int32_t shell,
                 const double* force, double* out);
/* lubrication correction on sphere i from partner j (j fields ignored for walls);
 * wall = -1 for a sphere partner, else 2*axis + side (side 0: plane at 1,
 * side 1: plane at n-1).  Returns F[3], T[3]. */
void ref_lubrication(const ref_config* cfg, const double* xi, const double* ui,
                     const double* wi, double Ri, const double* xj,
                     const double* uj, const double* wj, double Rj, int32_t wall,
                     double* F, double* T);

/* Eq. (MEM_CLI): boundary value of one particle link (direction q from the
 * fluid cell x to the solid cell x + c_q; r = x - x_p; Aq = f~_q(x),
 * Aqb = f~_qbar(x), Aqm = f~_q(x - c_q) used when cli != 0); NaN for a bad q */
double ref_link_value(int32_t q, const double* r, double R, const double* u, const double* w, double Aq,
                      double Aqb, double Aqm, int32_t cli);

/* collision time for a contact of (mean) diameter D: config value or
 * Eq. (collisionTimeChoice); minimal lubrication gap for radius R: config
 * value or Eq. (lubricationGapSize) */
double ref_collision_time(const ref_config* cfg, double D);
double ref_min_gap(const ref_config* cfg, double R);

ref_domain* ref_create(const ref_config* cfg);
void ref_destroy(ref_domain* d);
/* returns the new id (>= 0) or a negative status */
int32_t ref_add_sphere(ref_domain* d, const double* x, const double* u,
                       const double* w, double R, double rho);
/* mode 0 free, 1 prescribed ramp (u = u_target (1 - exp(-c_acc t / t_st)),
 * released when the gap to the wall plane ahead along u_target drops below
 * release_gap), 2 fixed */
/* n spheres at once, mapped once (0 or the first failure code) */
int32_t ref_add_spheres(ref_domain* d, int32_t n, const double* x, const double* u,
                        const double* w, const double* R, const double* rho);
int32_t ref_set_mode(ref_domain* d, int32_t id, int32_t mode,
                     const double* u_target, double c_acc, double t_st,
                     double release_gap);
/* mask bit0 x, bit1 u, bit2 w; re-maps the particles */
int32_t ref_update_sphere(ref_domain* d, int32_t id, const double* x,
                          const double* u, const double* w, int32_t mask);
int32_t ref_step(ref_domain* d, int32_t nsteps);
/* DEM only: one time step of n_sub sub-cycles with the given resolved forces
 * (6 doubles per sphere: F, T; NULL = zero); no fluid, no mapping */
int32_t ref_dem_step(ref_domain* d, const double* fext6);
int32_t ref_get_sphere(const ref_domain* d, int32_t id, double* out);
int32_t ref_num_spheres(const ref_domain* d);
/* field 0 rho (N), 1 velocity (3N, component-major), 2 PDF (19N, q-major);
 * non-fluid cells read 0; with a body force a the velocity is sum f c - a/2
 * (the stored PDFs are post-collision) */
int32_t ref_get_field(const ref_domain* d, int32_t field, double* dst);
int32_t ref_get_flags(const ref_domain* d, uint8_t* code, int32_t* owner);
/* overwrite the PDFs of all cells (19N, q-major) */
int32_t ref_set_pdf(ref_domain* d, const double* f);
int64_t ref_step_count(const ref_domain* d);

#ifdef __cplusplus
}
#endif
#endif
