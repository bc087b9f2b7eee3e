/*
 * lbmdem_ref_*: the oracle (lbmdem_ref.c) behind the argument lists of the GPU
 * library's C interface.  TEST INFRASTRUCTURE ONLY.  Argument marshalling and
 * checks only; every number comes from ref_*.
 */
#include "lbmdem_ref_abi.h"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbmdem_ref.h"

struct lbmdem_ref_domain {
  ref_domain* d;
  size_t N;
  double max_radius;
  char err[256];
};

static char g_create_err[256];

static int32_t fail(lbmdem_ref_domain* dom, int32_t rc, const char* msg) {
  if (dom)
    snprintf(dom->err, sizeof dom->err, "%s", msg);
  else
    snprintf(g_create_err, sizeof g_create_err, "%s", msg);
  return rc;
}

size_t lbmdem_ref_config_bytes(void) { return sizeof(lbmdem_ref_config); }

/* the paper's parameters (Lambda = 3/16, Lambda_b = 100, delta_aB = 2,
 * cut-offs 2/3, 1/2, 1/2, n_sub = 10, e_dry = 0.97; T_c and delta_min by
 * their relations) on 32^3 cells with z walls */
int32_t lbmdem_ref_config_init(lbmdem_ref_config* c) {
  if (!c) return -1;
  memset(c, 0, sizeof *c);
  c->nx = c->ny = c->nz = 32;
  c->walls[2] = 1;
  c->nu = 0.01;
  c->magic_lambda = 3.0 / 16.0;
  c->lambda_b = 100.0;
  c->delta_ab = 2.0;
  c->storage = 1;
  c->n_sub = 10;
  c->force_averaging = 1;
  c->e_dry = 0.97;
  c->poisson_ratio = 0.23;
  c->friction = 0.15;
  c->tc = -1.0;
  c->dmin = -1.0;
  c->cut_n = 2.0 / 3.0;
  c->cut_tt = 0.5;
  c->cut_tr = 0.5;
  c->lub_mask = 7;
  c->max_spheres = 16;
  c->max_radius = 12.0;
  c->overlap = 1;
  return 0;
}

int32_t lbmdem_ref_create(const lbmdem_ref_config* c, void* dev_buf, size_t dev_bytes, void* hip_stream,
                          lbmdem_ref_domain** out) {
  (void)dev_bytes;
  (void)hip_stream;
  if (!c || !out) return fail(NULL, -1, "null argument");
  *out = NULL;
  if (dev_buf) return fail(NULL, -1, "the oracle keeps its state in host memory: dev_buf must be NULL");
  ref_config r;
  memset(&r, 0, sizeof r);
  r.nx = c->nx;
  r.ny = c->ny;
  r.nz = c->nz;
  for (int a = 0; a < 3; ++a) {
    r.walls[a] = c->walls[a];
    r.wall_u_lo[a] = c->wall_u_lo[a];
    r.wall_u_hi[a] = c->wall_u_hi[a];
    r.gravity[a] = c->gravity[a];
    r.body_force[a] = c->body_force[a];
  }
  r.nu = c->nu;
  r.magic_lambda = c->magic_lambda;
  r.lambda_b = c->lambda_b;
  r.delta_ab = c->delta_ab;
  r.collision = c->collision;
  r.boundary = c->boundary;
  r.n_sub = c->n_sub;
  r.force_averaging = c->force_averaging;
  r.e_dry = c->e_dry;
  r.poisson_ratio = c->poisson_ratio;
  r.friction = c->friction;
  r.tc = c->tc;
  r.dmin = c->dmin;
  r.cut_n = c->cut_n;
  r.cut_tt = c->cut_tt;
  r.cut_tr = c->cut_tr;
  r.lub_mask = c->lub_mask;
  r.max_spheres = c->max_spheres;
  ref_domain* d = ref_create(&r);
  if (!d) return fail(NULL, -1, "invalid configuration or out of memory");
  lbmdem_ref_domain* dom = (lbmdem_ref_domain*)calloc(1, sizeof *dom);
  if (!dom) {
    ref_destroy(d);
    return fail(NULL, -2, "out of memory");
  }
  dom->d = d;
  dom->N = (size_t)c->nx * (size_t)c->ny * (size_t)c->nz;
  dom->max_radius = c->max_radius;
  *out = dom;
  return 0;
}

int32_t lbmdem_ref_destroy(lbmdem_ref_domain* dom) {
  if (!dom) return 0;
  ref_destroy(dom->d);
  free(dom);
  return 0;
}

int32_t lbmdem_ref_add_spheres(lbmdem_ref_domain* dom, int32_t n, const double* x, const double* u,
                               const double* w, const double* radius, const double* rho, int32_t* ids_out) {
  if (!dom || n < 0 || (n > 0 && (!x || !radius || !rho))) return fail(dom, -1, "invalid argument");
  for (int32_t s = 0; s < n; ++s)
    if (!(radius[s] > 0.0) || radius[s] > dom->max_radius) return fail(dom, -1, "radius above max_radius");
  const int32_t first = ref_num_spheres(dom->d);
  double* zero = NULL;
  if (n > 0 && (!u || !w)) {
    zero = (double*)calloc((size_t)3 * (size_t)n, sizeof(double));
    if (!zero) return fail(dom, -2, "out of memory");
  }
  const int32_t rc = ref_add_spheres(dom->d, n, x, u ? u : zero, w ? w : zero, radius, rho);
  free(zero);
  if (rc != 0) return fail(dom, rc, rc == -4 ? "sphere overlaps a wall or another sphere" : "insertion failed");
  if (ids_out)
    for (int32_t s = 0; s < n; ++s) ids_out[s] = first + s;
  return 0;
}

int32_t lbmdem_ref_update_spheres(lbmdem_ref_domain* dom, int32_t n, const int32_t* ids, const double* x,
                                  const double* u, const double* w, int32_t mask) {
  if (!dom || n < 0 || (n > 0 && !ids)) return fail(dom, -1, "invalid argument");
  const double z3[3] = {0.0, 0.0, 0.0};
  for (int32_t s = 0; s < n; ++s) {
    const int32_t rc = ref_update_sphere(dom->d, ids[s], x ? x + 3 * s : z3, u ? u + 3 * s : z3,
                                         w ? w + 3 * s : z3, mask);
    if (rc != 0) return fail(dom, rc, "update failed");
  }
  return 0;
}

int32_t lbmdem_ref_set_sphere_mode(lbmdem_ref_domain* dom, int32_t id, int32_t mode, const double* u_target,
                                   double c_acc, double t_st, double release_gap) {
  if (!dom) return -1;
  const double z3[3] = {0.0, 0.0, 0.0};
  const int32_t rc = ref_set_mode(dom->d, id, mode, u_target ? u_target : z3, c_acc, t_st, release_gap);
  return rc ? fail(dom, rc, "invalid sphere or mode") : 0;
}

int32_t lbmdem_ref_step(lbmdem_ref_domain* dom, int32_t nsteps) {
  if (!dom || nsteps < 0) return fail(dom, -1, "invalid argument");
  const int32_t rc = ref_step(dom->d, nsteps);
  return rc ? fail(dom, rc, "step failed") : 0;
}

int32_t lbmdem_ref_sync(lbmdem_ref_domain* dom) { return dom ? 0 : -1; }

int32_t lbmdem_ref_num_spheres(const lbmdem_ref_domain* dom) { return dom ? ref_num_spheres(dom->d) : -1; }

int32_t lbmdem_ref_get_sphere_state(lbmdem_ref_domain* dom, int32_t id, double* out) {
  if (!dom || !out) return -1;
  const int32_t rc = ref_get_sphere(dom->d, id, out);
  return rc ? fail(dom, rc, "no such sphere") : 0;
}

int32_t lbmdem_ref_get_spheres(lbmdem_ref_domain* dom, int32_t n, const int32_t* ids, double* x, double* u,
                               double* w, double* F_fp, double* T_fp, double* F_tot, double* T_tot) {
  if (!dom || n < 0) return -1;
  double st[REF_SPHERE_OUT];
  double* dst[7] = {x, u, w, F_fp, T_fp, F_tot, T_tot};
  const int at[7] = {0, 3, 6, 9, 12, 15, 18};
  for (int32_t s = 0; s < n; ++s) {
    const int32_t rc = ref_get_sphere(dom->d, ids ? ids[s] : s, st);
    if (rc) return fail(dom, rc, "no such sphere");
    for (int k = 0; k < 7; ++k)
      if (dst[k])
        for (int a = 0; a < 3; ++a) dst[k][3 * s + a] = st[at[k] + a];
  }
  return 0;
}

/* field codes as on the GPU: 0 rho, 1 velocity, 2 PDF (double), 3 cell codes
 * (uint8), 4 owners (int32) */
int32_t lbmdem_ref_get_field(lbmdem_ref_domain* dom, int32_t field, void* dst, size_t bytes,
                             int32_t dst_is_device) {
  if (!dom || !dst) return fail(dom, -1, "invalid argument");
  if (dst_is_device) return fail(dom, -1, "the oracle copies fields to host memory only");
  const size_t N = dom->N;
  size_t need;
  switch (field) {
    case 0: need = 8 * N; break;
    case 1: need = 24 * N; break;
    case 2: need = 152 * N; break;
    case 3: need = N; break;
    case 4: need = 4 * N; break;
    case 5: return fail(dom, -1, "the oracle keeps no boundary values in solid cells (field 5)");
    default: return fail(dom, -1, "unknown field");
  }
  if (bytes < need) return fail(dom, -1, "destination too small");
  if (field <= 2) {
    const int32_t rc = ref_get_field(dom->d, field, (double*)dst);
    return rc ? fail(dom, rc, "field read failed") : 0;
  }
  uint8_t* code = (uint8_t*)malloc(N);
  int32_t* owner = (int32_t*)malloc(4 * N);
  if (!code || !owner) {
    free(code);
    free(owner);
    return fail(dom, -2, "out of memory");
  }
  const int32_t rc = ref_get_flags(dom->d, code, owner);
  if (rc == 0) {
    if (field == 3)
      memcpy(dst, code, N);
    else
      memcpy(dst, owner, 4 * N);
  }
  free(code);
  free(owner);
  return rc ? fail(dom, rc, "flag read failed") : 0;
}

int32_t lbmdem_ref_set_pdf(lbmdem_ref_domain* dom, const double* f) {
  if (!dom || !f) return fail(dom, -1, "invalid argument");
  const int32_t rc = ref_set_pdf(dom->d, f);
  return rc ? fail(dom, rc, "set_pdf failed") : 0;
}

const char* lbmdem_ref_last_error(const lbmdem_ref_domain* dom) { return dom ? dom->err : g_create_err; }
