/*
 * The oracle behind the calls of the GPU library's C interface: lbmdem_ref_*
 * takes the arguments of the lbmdem_* call of the same name (the same
 * configuration layout, sphere-state vector, field codes and status codes), so
 * that one ctypes harness drives both.  TEST INFRASTRUCTURE ONLY, like the rest
 * of the oracle: it computes in FP64 on the host whatever the configuration's
 * storage field says, ignores the fields that choose GPU kernels, and wraps
 * ref_* (lbmdem_ref.h) without adding arithmetic.
 *
 * Differences from the GPU calls: device regions and streams are not used
 * (dev_buf must be NULL, hip_stream is ignored); fields are copied to host
 * memory only, and the raw PDF field (5: boundary values kept in solid cells)
 * does not exist here; lbmdem_ref_update_spheres re-maps after each sphere in
 * turn;
 * lbmdem_ref_sync has nothing to wait for.
 */
#ifndef LBMDEM_REF_ABI_H
#define LBMDEM_REF_ABI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* field for field the layout of the GPU library's configuration */
typedef struct lbmdem_ref_config {
  int32_t nx, ny, nz;
  int32_t walls[3];
  double wall_u_lo[3];
  double wall_u_hi[3];
  double nu;
  double magic_lambda;
  double lambda_b;
  double delta_ab;
  int32_t collision;
  int32_t boundary;
  int32_t storage;          /* ignored: the oracle stores FP64 */
  int32_t n_sub;
  int32_t force_averaging;
  double gravity[3];
  double e_dry;
  double poisson_ratio;
  double friction;
  double tc;
  double dmin;
  double cut_n, cut_tt, cut_tr;
  int32_t lub_mask;
  int32_t max_spheres;
  double max_radius;        /* checked at insertion, as on the GPU */
  int32_t dem_kernel;       /* ignored */
  int32_t map_kernel;       /* ignored */
  int32_t overlap;          /* ignored */
  double body_force[3];
} lbmdem_ref_config;

typedef struct lbmdem_ref_domain lbmdem_ref_domain;

size_t lbmdem_ref_config_bytes(void);
int32_t lbmdem_ref_config_init(lbmdem_ref_config* cfg);
int32_t lbmdem_ref_create(const lbmdem_ref_config* cfg, void* dev_buf, size_t dev_bytes,
                          void* hip_stream, lbmdem_ref_domain** out);
int32_t lbmdem_ref_destroy(lbmdem_ref_domain* dom);
int32_t lbmdem_ref_add_spheres(lbmdem_ref_domain* dom, int32_t n, const double* x,
                               const double* u, const double* w, const double* radius,
                               const double* rho, int32_t* ids_out);
int32_t lbmdem_ref_update_spheres(lbmdem_ref_domain* dom, int32_t n, const int32_t* ids,
                                  const double* x, const double* u, const double* w,
                                  int32_t mask);
int32_t lbmdem_ref_set_sphere_mode(lbmdem_ref_domain* dom, int32_t id, int32_t mode,
                                   const double* u_target, double c_acc, double t_st,
                                   double release_gap);
int32_t lbmdem_ref_step(lbmdem_ref_domain* dom, int32_t nsteps);
int32_t lbmdem_ref_sync(lbmdem_ref_domain* dom);
int32_t lbmdem_ref_num_spheres(const lbmdem_ref_domain* dom);
int32_t lbmdem_ref_get_sphere_state(lbmdem_ref_domain* dom, int32_t id, double* out);
int32_t lbmdem_ref_get_spheres(lbmdem_ref_domain* dom, int32_t n, const int32_t* ids,
                               double* x, double* u, double* w, double* F_fp, double* T_fp,
                               double* F_tot, double* T_tot);
int32_t lbmdem_ref_get_field(lbmdem_ref_domain* dom, int32_t field, void* dst, size_t bytes,
                             int32_t dst_is_device);
int32_t lbmdem_ref_set_pdf(lbmdem_ref_domain* dom, const double* f);
const char* lbmdem_ref_last_error(const lbmdem_ref_domain* dom);

#ifdef __cplusplus
}
#endif
#endif
