/*
 * Oracle of the four-way coupled LBM-DEM scheme (Rettinger & Ruede).
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, single-threaded FP64 restatement of
 * the paper, used to check the GPU library.  Nothing in the product links it.
 *
 * Each time step follows Algorithm 1 of the paper literally:
 *   1. fluid boundary conditions, Eq. (MEM_CLI), for every fluid-solid and
 *      fluid-wall link, from the post-collision PDFs of the previous step;
 *   2. momentum-exchange force/torque, Eqs. (MEM_Fq), (interaction_force),
 *      (interaction_torque), plus the missing-link compensation of Sec. 2.2,
 *      averaged over two time steps (Sec. 4.2);
 *   3. LBM stream + collide, Eqs. (LBM_Collide), (LBM_Stream), with the MRT
 *      operator of Eq. (MRT) evaluated with the dense moment matrix of App. A;
 *   4. n_sub DEM sub-cycles: velocity-Verlet (Eqs. velocity_verlet_1/2),
 *      lubrication (Sec. 3.1), spring-dashpot contacts (Sec. 4.1.2), gravity;
 *   5. particle re-mapping (Sec. 2.2) and PDF reconstruction, Eq.
 *      (PDF_reconstruction), in cells that turned from solid to fluid.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - surface velocity is u + w x (x - x_p) (App. B prints the factors of the
 *     cross product swapped; Sec. 4.5 fixes the sign: u_t = u_p,t - R w_y);
 *   - bounce-back fallback: delta = 1/2 in the two CLI coefficients only;
 *   - missing links: solid cell y of particle i whose neighbour y - c_q is a
 *     wall or a solid cell of another particle; arm at y - c_q/2;
 *   - first averaging step uses F_prev = F;
 *   - lubrication step function on the raw gap, magnitude on the clamped gap;
 *   - contact active for a negative gap, no clamping of the normal force;
 *   - velocity-dependent forces use the velocities before the sub-step update;
 *   - reconstruction neighbours: fluid before and after the mapping update.
 *
 * Pins (tests/test_oracle_*.py) check every part against closed forms,
 * invariants, exact arithmetic or hand-derived values.  Parity unpinned (a
 * convention with nothing outside the oracle to check it against): the
 * first-step averaging, the geometry of the bounce-back fallback, and the
 * unequal-radius choices for T_c, delta_min and the contact point.
 */
#include "lbmdem_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NQ 19
#define PI 3.14159265358979323846

enum { CELL_FLUID = 0, CELL_SHELL = 1, CELL_SOLID = 2, CELL_WALL = 3 };
enum { MODE_FREE = 0, MODE_PRESCRIBED = 1, MODE_FIXED = 2 };

/* App. A: moment transformation matrix of the MRT model (Duenweg et al. 2007). */
static const int M_APPA[NQ][NQ] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 0, 0, -1, 1, 0, 0, -1, 1, -1, 1, 0, 0, -1, 1, 0, 0, -1, 1},
    {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, -1, 0, 0, 1, -1, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1},
    {-1, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {1, -2, -2, -2, -2, -2, -2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 0, 0, 2, -2, 0, 0, -1, 1, -1, 1, 0, 0, -1, 1, 0, 0, -1, 1},
    {0, -2, 2, 0, 0, 0, 0, 1, 1, -1, -1, 1, -1, 0, 0, 1, -1, 0, 0},
    {0, 0, 0, 0, 0, -2, 2, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1},
    {0, -1, -1, 2, 2, -1, -1, 1, 1, 1, 1, -2, -2, 1, 1, -2, -2, 1, 1},
    {0, 1, 1, 0, 0, -1, -1, 1, 1, 1, 1, 0, 0, -1, -1, 0, 0, -1, -1},
    {0, 0, 0, 0, 0, 0, 0, -1, 1, 1, -1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 0, 0, -1, 1, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, -1, 1, 0, 0, 1, -1},
    {0, 1, 1, -2, -2, 1, 1, 1, 1, 1, 1, -2, -2, 1, 1, -2, -2, 1, 1},
    {0, -1, -1, 0, 0, 1, 1, 1, 1, 1, 1, 0, 0, -1, -1, 0, 0, -1, -1},
    {0, 0, 0, 0, 0, 0, 0, -1, 1, -1, 1, 0, 0, 1, -1, 0, 0, 1, -1},
    {0, 0, 0, 0, 0, 0, 0, -1, -1, 1, 1, 1, -1, 0, 0, 1, -1, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, -1, -1, 1, 1, 1, 1, -1, -1}};

/* Lattice tables derived from M: rows 1-3 are the velocity components
 * (App. A), weights are the D3Q19 ones of Qian et al. (1/3, 1/18, 1/36). */
static int LC[NQ][3];
static double LW[NQ];
static int LOPP[NQ];
static double MM[NQ][NQ];
static double MINV[NQ][NQ];
static int tables_ready = 0;

static int invert19(const double A[NQ][NQ], double out[NQ][NQ]) {
  double a[NQ][2 * NQ];
  for (int r = 0; r < NQ; ++r)
    for (int c = 0; c < 2 * NQ; ++c)
      a[r][c] = c < NQ ? A[r][c] : (c - NQ == r ? 1.0 : 0.0);
  for (int col = 0; col < NQ; ++col) {
    int piv = col;
    for (int r = col + 1; r < NQ; ++r)
      if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
    if (fabs(a[piv][col]) < 1e-300) return -1;
    if (piv != col)
      for (int c = 0; c < 2 * NQ; ++c) {
        double t = a[col][c];
        a[col][c] = a[piv][c];
        a[piv][c] = t;
      }
    double p = a[col][col];
    for (int c = 0; c < 2 * NQ; ++c) a[col][c] /= p;
    for (int r = 0; r < NQ; ++r) {
      if (r == col) continue;
      double fac = a[r][col];
      if (fac == 0.0) continue;
      for (int c = 0; c < 2 * NQ; ++c) a[r][c] -= fac * a[col][c];
    }
  }
  for (int r = 0; r < NQ; ++r)
    for (int c = 0; c < NQ; ++c) out[r][c] = a[r][NQ + c];
  return 0;
}

static void init_tables(void) {
  if (tables_ready) return;
  for (int q = 0; q < NQ; ++q) {
    for (int a = 0; a < 3; ++a) LC[q][a] = M_APPA[1 + a][q];
    int c2 = LC[q][0] * LC[q][0] + LC[q][1] * LC[q][1] + LC[q][2] * LC[q][2];
    LW[q] = c2 == 0 ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  for (int q = 0; q < NQ; ++q)
    for (int p = 0; p < NQ; ++p)
      if (LC[p][0] == -LC[q][0] && LC[p][1] == -LC[q][1] && LC[p][2] == -LC[q][2])
        LOPP[q] = p;
  for (int r = 0; r < NQ; ++r)
    for (int c = 0; c < NQ; ++c) MM[r][c] = (double)M_APPA[r][c];
  invert19(MM, MINV);
  tables_ready = 1;
}

void ref_lattice(int32_t* c, double* w, int32_t* opp) {
  init_tables();
  for (int q = 0; q < NQ; ++q) {
    for (int a = 0; a < 3; ++a) c[q * 3 + a] = LC[q][a];
    w[q] = LW[q];
    opp[q] = LOPP[q];
  }
}

void ref_moment_matrix(double* M) {
  init_tables();
  for (int r = 0; r < NQ; ++r)
    for (int c = 0; c < NQ; ++c) M[r * NQ + c] = MM[r][c];
}

int ref_moment_inverse(double* Minv) {
  init_tables();
  for (int r = 0; r < NQ; ++r)
    for (int c = 0; c < NQ; ++c) Minv[r * NQ + c] = MINV[r][c];
  return 0;
}

/* Eq. (Viscosity): nu = (1/s_nu - 1/2)/3; Eq. (MagicParameter) for s_nu^-;
 * Eq. (lambda_b) for s_b. */
void ref_rates(const ref_config* cfg, double* s_nu, double* s_minus, double* s_b) {
  double snu = 1.0 / (3.0 * cfg->nu + 0.5);
  double tau_p = 1.0 / snu - 0.5;
  *s_nu = snu;
  *s_minus = 1.0 / (0.5 + cfg->magic_lambda / tau_p);
  *s_b = 1.0 / (0.5 + cfg->lambda_b * tau_p);
}

/* incompressible equilibrium (mean density rho0 = 1, Sec. 2.1) whose moments
 * M f^eq are the m^eq of App. A */
void ref_equilibrium(double rho, const double* u, double* feq) {
  init_tables();
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int q = 0; q < NQ; ++q) {
    double cu = LC[q][0] * u[0] + LC[q][1] * u[1] + LC[q][2] * u[2];
    feq[q] = LW[q] * (rho + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

/* diagonal of S: Eqs. (RelaxationRateMatrix), (SRTmatrix), (TRTmatrix),
 * (TRTbulkmatrix); TRT+aB (Sec. 2.3.2) uses the TRT+B rates only in shell cells */
static void rate_vector(const ref_config* cfg, int shell, double S[NQ]) {
  double snu, smi, sb;
  ref_rates(cfg, &snu, &smi, &sb);
  for (int a = 0; a < NQ; ++a) S[a] = 0.0;
  if (cfg->collision == 3) {
    for (int a = 4; a < NQ; ++a) S[a] = snu;
    return;
  }
  double sbulk = snu;
  if (cfg->collision == 1) sbulk = sb;
  if (cfg->collision == 0 && shell) sbulk = sb;
  S[4] = sbulk;
  S[5] = sbulk;
  S[6] = S[7] = S[8] = smi;
  for (int a = 9; a <= 15; ++a) S[a] = snu;
  S[16] = S[17] = S[18] = smi;
}

/* Eq. (LBM_Collide) with Eq. (MRT): f~ = M^-1 (m + S (m^eq - m)); a body force
 * (test scenarios) enters by Guo's scheme in moment space. */
void ref_collide(const ref_config* cfg, const double* f, int32_t shell,
                 const double* force, double* out) {
  init_tables();
  double S[NQ];
  rate_vector(cfg, shell, S);
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < NQ; ++q) {
    rho += f[q];
    for (int a = 0; a < 3; ++a) j[a] += f[q] * LC[q][a];
  }
  double u[3];
  for (int a = 0; a < 3; ++a) u[a] = j[a] + (force ? 0.5 * force[a] : 0.0);
  double m[NQ], meq[NQ], mp[NQ];
  for (int r = 0; r < NQ; ++r) {
    double s = 0.0;
    for (int q = 0; q < NQ; ++q) s += MM[r][q] * f[q];
    m[r] = s;
    meq[r] = 0.0;
  }
  meq[0] = rho;
  meq[1] = u[0];
  meq[2] = u[1];
  meq[3] = u[2];
  meq[4] = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  meq[9] = 2.0 * u[0] * u[0] - u[1] * u[1] - u[2] * u[2];
  meq[10] = u[1] * u[1] - u[2] * u[2];
  meq[11] = u[0] * u[1];
  meq[12] = u[1] * u[2];
  meq[13] = u[0] * u[2];
  for (int r = 0; r < NQ; ++r) mp[r] = m[r] + S[r] * (meq[r] - m[r]);
  if (force) {
    double Fq[NQ];
    for (int q = 0; q < NQ; ++q) {
      double cu = LC[q][0] * u[0] + LC[q][1] * u[1] + LC[q][2] * u[2];
      double ca = LC[q][0] * force[0] + LC[q][1] * force[1] + LC[q][2] * force[2];
      double ua = u[0] * force[0] + u[1] * force[1] + u[2] * force[2];
      Fq[q] = LW[q] * (3.0 * (ca - ua) + 9.0 * cu * ca);
    }
    for (int r = 0; r < NQ; ++r) {
      double s = 0.0;
      for (int q = 0; q < NQ; ++q) s += MM[r][q] * Fq[q];
      mp[r] += (1.0 - 0.5 * S[r]) * s;
    }
  }
  for (int q = 0; q < NQ; ++q) {
    double s = 0.0;
    for (int r = 0; r < NQ; ++r) s += MINV[q][r] * mp[r];
    out[q] = s;
  }
}

/* ------------------------------------------------------------------------- */

typedef struct {
  double x[3], u[3], w[3];
  double R, rho, m, I;
  int mode;
  double utgt[3], c_acc, t_st, release_gap, t_presc;
  double Fprev[3], Tprev[3];
  int prev_valid;
  double Ffp[3], Tfp[3], Fraw[3], Traw[3];
  double Fold[3], Told[3];
  int old_valid;
  double Flub[3], Tlub[3], Fcol[3], Tcol[3], Ftot[3], Ttot[3];
} sphere_t;

struct ref_domain {
  ref_config cfg;
  int n[3];
  long N;
  double* A;       /* post-collision PDFs of the current step, q-major */
  double* B;       /* next step */
  double* fb;      /* boundary PDFs of the current step (link values) */
  uint8_t* code;   /* canonical cell code */
  int32_t* owner;  /* owning particle of solid cells */
  int P;
  sphere_t* sp;
  double* hist;    /* tangential spring per ordered pair: P x (P+6) x 4 */
  int64_t steps;
};

static long cidx(const ref_domain* d, int i, int j, int k) {
  return (long)i + (long)d->n[0] * ((long)j + (long)d->n[1] * (long)k);
}

static int wrapi(int i, int n) {
  if (i < 0) return i + n;
  if (i >= n) return i - n;
  return i;
}

/* minimum-image distance component on periodic axes */
static double minimg(const ref_domain* d, int a, double v) {
  if (d->cfg.walls[a]) return v;
  double L = (double)d->n[a];
  if (v > 0.5 * L) return v - L;
  if (v < -0.5 * L) return v + L;
  return v;
}

static void cross(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static double norm3(const double* a) { return sqrt(dot3(a, a)); }

/* rigid-body velocity of particle s at offset r = x - x_p (App. B, with the
 * factors of the cross product in the order fixed by Sec. 4.5) */
static void body_velocity(const sphere_t* s, const double* r, double* U) {
  double wr[3];
  cross(s->w, r, wr);
  for (int a = 0; a < 3; ++a) U[a] = s->u[a] + wr[a];
}

static void wall_velocity(const ref_domain* d, int k, double* uw) {
  uw[0] = uw[1] = uw[2] = 0.0;
  if (!d->cfg.walls[2]) return;
  if (k == 0)
    for (int a = 0; a < 3; ++a) uw[a] = d->cfg.wall_u_lo[a];
  else if (k == d->n[2] - 1)
    for (int a = 0; a < 3; ++a) uw[a] = d->cfg.wall_u_hi[a];
}

/* Sec. 2.2: a cell is solid if its centre lies inside (or on) a particle.  The
 * squared distance is formed in a fixed order: (dx*dx + dy*dy) + dz*dz. */
static double cell_dist2(const ref_domain* d, int i, int j, int k, const double* xp) {
  double dx = minimg(d, 0, ((double)i + 0.5) - xp[0]);
  double dy = minimg(d, 1, ((double)j + 0.5) - xp[1]);
  double dz = minimg(d, 2, ((double)k + 0.5) - xp[2]);
  return (dx * dx + dy * dy) + dz * dz;
}

static int is_wall_cell(const ref_domain* d, int i, int j, int k) {
  int ijk[3] = {i, j, k};
  for (int a = 0; a < 3; ++a)
    if (d->cfg.walls[a] && (ijk[a] == 0 || ijk[a] == d->n[a] - 1)) return 1;
  return 0;
}

/* brute-force mapping over all cells and particles; lowest id owns overlaps */
static void compute_mapping(const ref_domain* d, uint8_t* code, int32_t* owner) {
  for (int k = 0; k < d->n[2]; ++k)
    for (int j = 0; j < d->n[1]; ++j)
      for (int i = 0; i < d->n[0]; ++i) {
        long c = cidx(d, i, j, k);
        owner[c] = -1;
        if (is_wall_cell(d, i, j, k)) {
          code[c] = CELL_WALL;
          continue;
        }
        int own = -1, shell = 0;
        for (int p = 0; p < d->P; ++p) {
          const sphere_t* s = &d->sp[p];
          double d2 = cell_dist2(d, i, j, k, s->x);
          double R2 = s->R * s->R;
          double rs = s->R + d->cfg.delta_ab;
          double rs2 = rs * rs;
          if (d2 <= R2 && own < 0) own = p;
          if (d2 <= rs2) shell = 1;
        }
        if (own >= 0) {
          code[c] = CELL_SOLID;
          owner[c] = own;
        } else {
          code[c] = shell ? CELL_SHELL : CELL_FLUID;
        }
      }
}

static int is_fluid_code(uint8_t c) { return c == CELL_FLUID || c == CELL_SHELL; }

ref_domain* ref_create(const ref_config* cfg) {
  init_tables();
  if (cfg->nx < 3 || cfg->ny < 3 || cfg->nz < 3 || cfg->max_spheres < 0 ||
      cfg->n_sub < 1 || !(cfg->nu > 0.0))
    return NULL;
  ref_domain* d = (ref_domain*)calloc(1, sizeof(ref_domain));
  if (!d) return NULL;
  d->cfg = *cfg;
  d->n[0] = cfg->nx;
  d->n[1] = cfg->ny;
  d->n[2] = cfg->nz;
  d->N = (long)cfg->nx * cfg->ny * cfg->nz;
  d->A = (double*)malloc(sizeof(double) * NQ * d->N);
  d->B = (double*)malloc(sizeof(double) * NQ * d->N);
  d->fb = (double*)malloc(sizeof(double) * NQ * d->N);
  d->code = (uint8_t*)malloc(d->N);
  d->owner = (int32_t*)malloc(sizeof(int32_t) * d->N);
  int P = cfg->max_spheres > 0 ? cfg->max_spheres : 1;
  d->sp = (sphere_t*)calloc((size_t)P, sizeof(sphere_t));
  d->hist = (double*)calloc((size_t)P * (P + 6) * 4, sizeof(double));
  if (!d->A || !d->B || !d->fb || !d->code || !d->owner || !d->sp || !d->hist) {
    ref_destroy(d);
    return NULL;
  }
  /* fluid at rest with rho = 1: f = w_q */
  for (int q = 0; q < NQ; ++q)
    for (long c = 0; c < d->N; ++c) {
      d->A[q * d->N + c] = LW[q];
      d->B[q * d->N + c] = LW[q];
    }
  compute_mapping(d, d->code, d->owner);
  return d;
}

void ref_destroy(ref_domain* d) {
  if (!d) return;
  free(d->A);
  free(d->B);
  free(d->fb);
  free(d->code);
  free(d->owner);
  free(d->sp);
  free(d->hist);
  free(d);
}

/* signed surface gap to the nearest wall plane (App. B); large if none */
static double min_wall_gap(const ref_domain* d, const sphere_t* s) {
  double g = 1e300;
  for (int a = 0; a < 3; ++a) {
    if (!d->cfg.walls[a]) continue;
    double lo = (s->x[a] - 1.0) - s->R;
    double hi = (((double)d->n[a] - 1.0) - s->x[a]) - s->R;
    if (lo < g) g = lo;
    if (hi < g) g = hi;
  }
  return g;
}

/* Sec. 4.4.2: the artificial acceleration is switched off once the sphere is
 * closer than the release gap to the wall it approaches, i.e. the wall plane
 * ahead of it along the prescribed velocity (only walled axes with a nonzero
 * target component count); large if no wall lies ahead. */
static double gap_ahead(const ref_domain* d, const sphere_t* s) {
  double g = 1e300;
  for (int a = 0; a < 3; ++a) {
    if (!d->cfg.walls[a] || s->utgt[a] == 0.0) continue;
    double v = s->utgt[a] < 0.0 ? (s->x[a] - 1.0) - s->R : (((double)d->n[a] - 1.0) - s->x[a]) - s->R;
    if (v < g) g = v;
  }
  return g;
}

static void remap(ref_domain* d, int reconstruct);

/* inserts one sphere (checks of Sec. 2 set-up: inside the lattice, clear of
 * the walls and of the other spheres) without re-mapping */
static int32_t insert_sphere(ref_domain* d, const double* x, const double* u,
                             const double* w, double R, double rho) {
  if (!d || !(R > 0.0) || !(rho > 0.0)) return -1;
  if (d->P >= d->cfg.max_spheres) return -6;
  for (int a = 0; a < 3; ++a)
    if (!(x[a] >= 0.0 && x[a] < (double)d->n[a])) return -1;
  sphere_t s;
  memset(&s, 0, sizeof(s));
  for (int a = 0; a < 3; ++a) {
    s.x[a] = x[a];
    s.u[a] = u ? u[a] : 0.0;
    s.w[a] = w ? w[a] : 0.0;
  }
  s.R = R;
  s.rho = rho;
  s.m = rho * (4.0 / 3.0) * PI * R * R * R;
  s.I = 0.4 * s.m * R * R;
  s.mode = MODE_FREE;
  if (min_wall_gap(d, &s) < 0.0) return -4;
  for (int p = 0; p < d->P; ++p) {
    double dd[3];
    for (int a = 0; a < 3; ++a) dd[a] = minimg(d, a, s.x[a] - d->sp[p].x[a]);
    if (norm3(dd) - (s.R + d->sp[p].R) < 0.0) return -4;
  }
  int id = d->P;
  d->sp[id] = s;
  d->P += 1;
  return id;
}

int32_t ref_add_sphere(ref_domain* d, const double* x, const double* u,
                       const double* w, double R, double rho) {
  int32_t id = insert_sphere(d, x, u, w, R, rho);
  if (id >= 0) remap(d, 0);
  return id;
}

/* the same for n spheres (3n positions, velocities, angular velocities; NULL
 * velocities read as zero), mapped once; the spheres before a failing one stay */
int32_t ref_add_spheres(ref_domain* d, int32_t n, const double* x, const double* u,
                        const double* w, const double* R, const double* rho) {
  int32_t rc = 0;
  for (int32_t k = 0; k < n && rc >= 0; ++k)
    rc = insert_sphere(d, x + 3 * k, u ? u + 3 * k : NULL, w ? w + 3 * k : NULL, R[k], rho[k]);
  remap(d, 0);
  return rc < 0 ? rc : 0;
}

int32_t ref_set_mode(ref_domain* d, int32_t id, int32_t mode, const double* u_target,
                     double c_acc, double t_st, double release_gap) {
  if (!d || id < 0 || id >= d->P || mode < 0 || mode > 2) return -1;
  sphere_t* s = &d->sp[id];
  s->mode = mode;
  s->old_valid = 0;
  if (mode == MODE_PRESCRIBED) {
    for (int a = 0; a < 3; ++a) {
      s->utgt[a] = u_target[a];
      s->u[a] = 0.0;
      s->w[a] = 0.0;
    }
    s->c_acc = c_acc;
    s->t_st = t_st;
    s->release_gap = release_gap;
    s->t_presc = 0.0;
  }
  return 0;
}

int32_t ref_update_sphere(ref_domain* d, int32_t id, const double* x, const double* u,
                          const double* w, int32_t mask) {
  if (!d || id < 0 || id >= d->P) return -1;
  sphere_t* s = &d->sp[id];
  if (mask & 1)
    for (int a = 0; a < 3; ++a) s->x[a] = x[a];
  if (mask & 2)
    for (int a = 0; a < 3; ++a) s->u[a] = u[a];
  if (mask & 4)
    for (int a = 0; a < 3; ++a) s->w[a] = w[a];
  s->old_valid = 0;
  remap(d, 1);
  return 0;
}

/* ---------------------------- step 1 + 2 --------------------------------- */

/* smallest root in [0,1] of |r + delta c|^2 = R^2, r = x - x_p (Eq. MEM_CLI:
 * x_b = x + delta_q c_q) */
static double link_delta(const double* r, const int* c, double R) {
  double cc = (double)(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  double b = r[0] * c[0] + r[1] * c[1] + r[2] * c[2];
  double e = (r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) - R * R;
  double disc = b * b - cc * e;
  if (disc < 0.0) disc = 0.0;
  double dl = (-b - sqrt(disc)) / cc;
  if (dl < 0.0) dl = 0.0;
  if (dl > 1.0) dl = 1.0;
  return dl;
}

/* Eq. (MEM_CLI) for one particle link: the value that streams back into the
 * fluid cell x from the solid cell x + c_q, from f~_q(x) (Aq), f~_qbar(x)
 * (Aqb) and, with CLI (cli != 0), f~_q(x - c_q) (Aqm); r = x - x_p (nearest
 * image) and R, u, w of the sphere.  rb and ub receive the wall point's offset
 * r + delta c_q and its velocity, for the force of Eq. (MEM_Fq). */
static double link_value(int q, const double* r, double R, const double* u, const double* w, double Aq,
                         double Aqb, double Aqm, int cli, double* rb, double* ub) {
  double cq[3] = {LC[q][0], LC[q][1], LC[q][2]};
  double dl = link_delta(r, LC[q], R);
  for (int a = 0; a < 3; ++a) rb[a] = r[a] + dl * cq[a];
  double wr[3];
  cross(w, rb, wr);
  for (int a = 0; a < 3; ++a) ub[a] = u[a] + wr[a];
  double dd = cli ? dl : 0.5;
  double val = Aq;
  if (cli)
    val += (1.0 - 2.0 * dd) / (1.0 + 2.0 * dd) * (Aqm - Aqb);
  val -= 4.0 / (1.0 + 2.0 * dd) * LW[q] * 3.0 * dot3(ub, cq);
  return val;
}

double ref_link_value(int32_t q, const double* r, double R, const double* u, const double* w, double Aq,
                      double Aqb, double Aqm, int32_t cli) {
  double rb[3], ub[3];
  if (q < 1 || q >= NQ) return NAN;
  return link_value(q, r, R, u, w, Aq, Aqb, Aqm, cli, rb, ub);
}

static void boundary_and_forces(ref_domain* d, double* F) {
  const long N = d->N;
  const double* A = d->A;
  for (int p = 0; p < 6 * d->P; ++p) F[p] = 0.0;
  for (int k = 0; k < d->n[2]; ++k)
    for (int j = 0; j < d->n[1]; ++j)
      for (int i = 0; i < d->n[0]; ++i) {
        long x = cidx(d, i, j, k);
        if (!is_fluid_code(d->code[x])) continue;
        for (int q = 1; q < NQ; ++q) {
          int yi = wrapi(i + LC[q][0], d->n[0]);
          int yj = wrapi(j + LC[q][1], d->n[1]);
          int yk = wrapi(k + LC[q][2], d->n[2]);
          long y = cidx(d, yi, yj, yk);
          int qb = LOPP[q];
          double cq[3] = {LC[q][0], LC[q][1], LC[q][2]};
          if (d->code[y] == CELL_WALL) {
            /* Eq. (MEM_CLI) with delta = 1/2: moving-wall bounce-back */
            double uw[3];
            wall_velocity(d, yk, uw);
            d->fb[qb * N + x] = A[q * N + x] - 6.0 * LW[q] * dot3(uw, cq);
          } else if (d->code[y] == CELL_SOLID) {
            int pid = d->owner[y];
            const sphere_t* s = &d->sp[pid];
            double r[3];
            r[0] = minimg(d, 0, ((double)i + 0.5) - s->x[0]);
            r[1] = minimg(d, 1, ((double)j + 0.5) - s->x[1]);
            r[2] = minimg(d, 2, ((double)k + 0.5) - s->x[2]);
            int mi = wrapi(i - LC[q][0], d->n[0]);
            int mj = wrapi(j - LC[q][1], d->n[1]);
            int mk = wrapi(k - LC[q][2], d->n[2]);
            long xm = cidx(d, mi, mj, mk);
            int cli = d->cfg.boundary == 0 && is_fluid_code(d->code[xm]);
            double rb[3], ub[3];
            double val = link_value(q, r, s->R, s->u, s->w, A[q * N + x], A[qb * N + x], cli ? A[q * N + xm] : 0.0,
                                    cli, rb, ub);
            d->fb[qb * N + x] = val;
            /* Eq. (MEM_Fq) */
            double Fq[3], Tq[3];
            for (int a = 0; a < 3; ++a)
              Fq[a] = (cq[a] - ub[a]) * A[q * N + x] - (-cq[a] - ub[a]) * val;
            cross(rb, Fq, Tq);
            for (int a = 0; a < 3; ++a) {
              F[6 * pid + a] += Fq[a];
              F[6 * pid + 3 + a] += Tq[a];
            }
          }
        }
      }
  /* missing links (Sec. 2.2): F_q = 2 w_q c_q */
  for (int k = 0; k < d->n[2]; ++k)
    for (int j = 0; j < d->n[1]; ++j)
      for (int i = 0; i < d->n[0]; ++i) {
        long y = cidx(d, i, j, k);
        if (d->code[y] != CELL_SOLID) continue;
        int pid = d->owner[y];
        const sphere_t* s = &d->sp[pid];
        for (int q = 1; q < NQ; ++q) {
          int zi = wrapi(i - LC[q][0], d->n[0]);
          int zj = wrapi(j - LC[q][1], d->n[1]);
          int zk = wrapi(k - LC[q][2], d->n[2]);
          long z = cidx(d, zi, zj, zk);
          int missing = d->code[z] == CELL_WALL ||
                        (d->code[z] == CELL_SOLID && d->owner[z] != pid);
          if (!missing) continue;
          double Fq[3], arm[3], Tq[3];
          for (int a = 0; a < 3; ++a) Fq[a] = 2.0 * LW[q] * LC[q][a];
          arm[0] = minimg(d, 0, ((double)i + 0.5) - s->x[0]) - 0.5 * LC[q][0];
          arm[1] = minimg(d, 1, ((double)j + 0.5) - s->x[1]) - 0.5 * LC[q][1];
          arm[2] = minimg(d, 2, ((double)k + 0.5) - s->x[2]) - 0.5 * LC[q][2];
          cross(arm, Fq, Tq);
          for (int a = 0; a < 3; ++a) {
            F[6 * pid + a] += Fq[a];
            F[6 * pid + 3 + a] += Tq[a];
          }
        }
      }
}

/* ------------------------------- step 3 ---------------------------------- */

static void lbm_step(ref_domain* d) {
  const long N = d->N;
  const double* force = NULL;
  double bf[3] = {d->cfg.body_force[0], d->cfg.body_force[1], d->cfg.body_force[2]};
  if (bf[0] != 0.0 || bf[1] != 0.0 || bf[2] != 0.0) force = bf;
  double f[NQ], out[NQ];
  for (int k = 0; k < d->n[2]; ++k)
    for (int j = 0; j < d->n[1]; ++j)
      for (int i = 0; i < d->n[0]; ++i) {
        long x = cidx(d, i, j, k);
        if (!is_fluid_code(d->code[x])) continue;
        for (int q = 0; q < NQ; ++q) {
          int si = wrapi(i - LC[q][0], d->n[0]);
          int sj = wrapi(j - LC[q][1], d->n[1]);
          int sk = wrapi(k - LC[q][2], d->n[2]);
          long src = cidx(d, si, sj, sk);
          /* Eq. (LBM_Stream); links into solids/walls take the boundary value */
          if (q == 0 || is_fluid_code(d->code[src]))
            f[q] = d->A[q * N + src];
          else
            f[q] = d->fb[q * N + x];
        }
        ref_collide(&d->cfg, f, d->code[x] == CELL_SHELL, force, out);
        for (int q = 0; q < NQ; ++q) d->B[q * N + x] = out[q];
      }
}

/* ------------------------------- step 4 ---------------------------------- */

typedef struct {
  int is_wall;
  int j;           /* partner sphere or -1 */
  int slot;        /* history slot */
  double n[3];     /* unit normal from partner to i */
  double delta;    /* signed surface gap */
  double xcp[3];   /* contact point */
  double rj[3];    /* xcp - x_j (sphere partner) */
} partner_t;

static double collision_time(const ref_domain* d, double D) {
  if (d->cfg.tc > 0.0) return d->cfg.tc;
  return 2.31 * D * sqrt(3.0); /* Eq. (collisionTimeChoice), c_s = 1/sqrt(3) */
}

static double min_lub_gap(const ref_domain* d, double R) {
  if (d->cfg.dmin >= 0.0) return d->cfg.dmin;
  return (0.001 + 0.00007 * R) * R; /* Eq. (lubricationGapSize) */
}

double ref_collision_time(const ref_config* cfg, double D) {
  ref_domain tmp;
  tmp.cfg = *cfg;
  return collision_time(&tmp, D);
}

double ref_min_gap(const ref_config* cfg, double R) {
  ref_domain tmp;
  tmp.cfg = *cfg;
  return min_lub_gap(&tmp, R);
}

/* Sec. 3.1, Eqs. (lubrication_correction_*); sphere-wall forms are the limit
 * kappa_r -> infinity.  Step function on the raw gap, magnitude on
 * max(delta, delta_min). */
static void lubrication_terms(const ref_config* cfg, double dmin, const double* n,
                              double delta, const double* ui, const double* wi,
                              double Ri, const double* uj, const double* wj,
                              double Rj, int wall, double* F, double* T) {
  double mu = cfg->nu; /* rho_f = 1 */
  double dl = delta > dmin ? delta : dmin;
  double uij[3], un[3], ut[3];
  for (int a = 0; a < 3; ++a) uij[a] = ui[a] - (wall ? 0.0 : uj[a]);
  double uijn = dot3(uij, n);
  for (int a = 0; a < 3; ++a) {
    un[a] = uijn * n[a];
    ut[a] = uij[a] - un[a];
  }
  double k = wall ? 0.0 : Rj / Ri;
  if ((cfg->lub_mask & 1) && delta > 0.0 && delta < cfg->cut_n) {
    double coef = wall ? 1.0 : (k * k) / ((1.0 + k) * (1.0 + k));
    double mag = -6.0 * PI * mu * Ri * Ri * coef * (1.0 / dl - 1.0 / cfg->cut_n);
    for (int a = 0; a < 3; ++a) F[a] += mag * un[a];
  }
  if ((cfg->lub_mask & 2) && delta > 0.0 && delta < cfg->cut_tt) {
    double L = log(dl / cfg->cut_tt);
    double cf = wall ? 8.0 / 15.0
                     : 4.0 * k * (2.0 + k + 2.0 * k * k) / (15.0 * (1.0 + k) * (1.0 + k) * (1.0 + k));
    double ct = wall ? 0.1 : k * (4.0 + k) / (10.0 * (1.0 + k) * (1.0 + k));
    double fm = 6.0 * PI * mu * Ri * cf * L;
    double tm = 8.0 * PI * mu * Ri * Ri * ct * L;
    double uxn[3];
    cross(uij, n, uxn);
    for (int a = 0; a < 3; ++a) {
      F[a] += fm * ut[a];
      T[a] += tm * uxn[a];
    }
  }
  if ((cfg->lub_mask & 4) && delta > 0.0 && delta < cfg->cut_tr) {
    double L = log(dl / cfg->cut_tr);
    double cf = wall ? 2.0 / 15.0 : 2.0 * k * k / (15.0 * (1.0 + k) * (1.0 + k));
    double ct = wall ? 0.4 : 2.0 * k / (5.0 * (1.0 + k));
    double wv[3], av[3], wxn[3];
    for (int a = 0; a < 3; ++a) {
      wv[a] = wall ? wi[a] : (wi[a] + wj[a]) + (4.0 / k) * wi[a] + 4.0 * k * wj[a];
      av[a] = wall ? wi[a] : wi[a] + 0.25 * k * wj[a];
    }
    cross(wv, n, wxn);
    double an = dot3(av, n);
    double fm = -6.0 * PI * mu * Ri * Ri * cf * L;
    double tm = 8.0 * PI * mu * Ri * Ri * Ri * ct * L;
    for (int a = 0; a < 3; ++a) {
      F[a] += fm * wxn[a];
      T[a] += tm * (av[a] - an * n[a]);
    }
  }
}

void ref_lubrication(const ref_config* cfg, const double* xi, const double* ui,
                     const double* wi, double Ri, const double* xj, const double* uj,
                     const double* wj, double Rj, int32_t wall, double* F, double* T) {
  double n[3], delta;
  for (int a = 0; a < 3; ++a) F[a] = T[a] = 0.0;
  double dmin;
  if (wall < 0) {
    double dd[3];
    for (int a = 0; a < 3; ++a) dd[a] = xi[a] - xj[a];
    double dist = norm3(dd);
    for (int a = 0; a < 3; ++a) n[a] = dd[a] / dist;
    delta = dist - (Ri + Rj);
    double Rh = 2.0 * Ri * Rj / (Ri + Rj);
    dmin = cfg->dmin >= 0.0 ? cfg->dmin : (0.001 + 0.00007 * Rh) * Rh;
  } else {
    int ax = wall / 2, side = wall % 2;
    int nn[3] = {cfg->nx, cfg->ny, cfg->nz};
    n[0] = n[1] = n[2] = 0.0;
    n[ax] = side ? -1.0 : 1.0;
    delta = side ? ((((double)nn[ax]) - 1.0) - xi[ax]) - Ri : (xi[ax] - 1.0) - Ri;
    dmin = cfg->dmin >= 0.0 ? cfg->dmin : (0.001 + 0.00007 * Ri) * Ri;
  }
  lubrication_terms(cfg, dmin, n, delta, ui, wi, Ri, uj, wj, Rj, wall >= 0, F, T);
}

/* history slots per sphere: one per possible partner sphere, then 6 walls */
static int hist_stride(const ref_domain* d) {
  return (d->cfg.max_spheres > 0 ? d->cfg.max_spheres : 1) + 6;
}

/* enumerate partners of sphere i: other spheres, then wall planes */
static int build_partners(const ref_domain* d, int i, partner_t* out) {
  const sphere_t* s = &d->sp[i];
  int np = 0;
  for (int j = 0; j < d->P; ++j) {
    if (j == i) continue;
    const sphere_t* t = &d->sp[j];
    partner_t pt;
    double dd[3];
    for (int a = 0; a < 3; ++a) dd[a] = minimg(d, a, s->x[a] - t->x[a]);
    double dist = norm3(dd);
    pt.is_wall = 0;
    pt.j = j;
    pt.slot = j;
    for (int a = 0; a < 3; ++a) pt.n[a] = dd[a] / dist;
    pt.delta = dist - (s->R + t->R);
    for (int a = 0; a < 3; ++a) {
      pt.xcp[a] = s->x[a] - 0.5 * dd[a];   /* midway between the centres */
      pt.rj[a] = 0.5 * dd[a];              /* x_cp - x_j in the same image */
    }
    out[np++] = pt;
  }
  for (int a = 0; a < 3; ++a) {
    if (!d->cfg.walls[a]) continue;
    for (int side = 0; side < 2; ++side) {
      partner_t pt;
      pt.is_wall = 1;
      pt.j = -1;
      pt.slot = hist_stride(d) - 6 + 2 * a + side;
      pt.n[0] = pt.n[1] = pt.n[2] = 0.0;
      pt.n[a] = side ? -1.0 : 1.0;
      pt.delta = side ? ((((double)d->n[a]) - 1.0) - s->x[a]) - s->R : (s->x[a] - 1.0) - s->R;
      for (int b = 0; b < 3; ++b) pt.xcp[b] = s->x[b] - (s->R + 0.5 * pt.delta) * pt.n[b];
      pt.rj[0] = pt.rj[1] = pt.rj[2] = 0.0;
      out[np++] = pt;
    }
  }
  return np;
}

/* forces on sphere i at the current state.  contact: evaluate Sec. 4.1.2;
 * upd: write the tangential spring history (G7 order). */
static void eval_forces(ref_domain* d, int i, int contact, int upd, double dtp,
                        double* Fout, double* Tout) {
  sphere_t* s = &d->sp[i];
  const ref_config* cfg = &d->cfg;
  double Flub[3] = {0, 0, 0}, Tlub[3] = {0, 0, 0}, Fcol[3] = {0, 0, 0}, Tcol[3] = {0, 0, 0};
  partner_t* pts = (partner_t*)malloc(sizeof(partner_t) * (size_t)(d->P + 6));
  int np = build_partners(d, i, pts);
  double maxcut = cfg->cut_n;
  if (cfg->cut_tt > maxcut) maxcut = cfg->cut_tt;
  if (cfg->cut_tr > maxcut) maxcut = cfg->cut_tr;
  const int stride = hist_stride(d);
  for (int pi = 0; pi < np; ++pi) {
    partner_t* pt = &pts[pi];
    const sphere_t* t = pt->is_wall ? NULL : &d->sp[pt->j];
    double zero[3] = {0, 0, 0};
    const double* uj = t ? t->u : zero;
    const double* wj = t ? t->w : zero;
    double Rj = t ? t->R : 0.0;
    double* h = &d->hist[((size_t)i * stride + pt->slot) * 4];
    if (contact && pt->delta < 0.0) {
      double uij[3], un[3], Ui[3], Uj[3], ucp[3], ut[3], ri[3];
      for (int a = 0; a < 3; ++a) {
        uij[a] = s->u[a] - uj[a];
        ri[a] = pt->xcp[a] - s->x[a];
      }
      double uijn = dot3(uij, pt->n);
      for (int a = 0; a < 3; ++a) un[a] = uijn * pt->n[a];
      body_velocity(s, ri, Ui);
      if (t) {
        body_velocity(t, pt->rj, Uj);
      } else {
        Uj[0] = Uj[1] = Uj[2] = 0.0;
      }
      for (int a = 0; a < 3; ++a) {
        ucp[a] = Ui[a] - Uj[a];
        ut[a] = ucp[a] - un[a]; /* u^cp_n = u_n (App. B) */
      }
      double meff = t ? s->m * t->m / (s->m + t->m) : s->m;
      double D = t ? s->R + t->R : 2.0 * s->R;
      double Tc = collision_time(d, D);
      double le = log(cfg->e_dry);
      double kn = meff * (PI * PI + le * le) / (Tc * Tc); /* Eq. (normalDEMparameters) */
      double dn = -2.0 * meff * le / Tc;
      double kp = 2.0 * (1.0 - cfg->poisson_ratio) / (2.0 - cfg->poisson_ratio);
      double kt = kp * kn; /* Eq. (tangentialCollisionParameters) */
      double dt = sqrt(kp) * dn;
      double Fn[3];
      for (int a = 0; a < 3; ++a) Fn[a] = -kn * pt->delta * pt->n[a] - dn * un[a];
      /* tangential spring: project into the current contact plane, rescale */
      double hv[3] = {0, 0, 0};
      if (h[0] != 0.0) {
        hv[0] = h[1];
        hv[1] = h[2];
        hv[2] = h[3];
      }
      double hn = dot3(hv, pt->n);
      double ht[3];
      for (int a = 0; a < 3; ++a) ht[a] = hv[a] - hn * pt->n[a];
      double lh = norm3(hv), lht = norm3(ht);
      if (lht > 0.0)
        for (int a = 0; a < 3; ++a) hv[a] = (lh / lht) * ht[a];
      else
        for (int a = 0; a < 3; ++a) hv[a] = ht[a];
      double Fsd[3];
      for (int a = 0; a < 3; ++a) Fsd[a] = -kt * hv[a] - dt * ut[a];
      double fsd = norm3(Fsd);
      double fmax = cfg->friction * norm3(Fn);
      double Ft[3], hnew[3];
      if (fsd < fmax || fsd == 0.0) {
        for (int a = 0; a < 3; ++a) {
          Ft[a] = Fsd[a];
          hnew[a] = hv[a] + dtp * ut[a];
        }
      } else {
        for (int a = 0; a < 3; ++a) {
          double tv = Fsd[a] / fsd;
          Ft[a] = fmax * tv;
          hnew[a] = -(fmax * tv + dt * ut[a]) / kt;
        }
      }
      double Tt[3];
      cross(ri, Ft, Tt);
      for (int a = 0; a < 3; ++a) {
        Fcol[a] += Fn[a] + Ft[a];
        Tcol[a] += Tt[a];
      }
      if (upd) {
        h[0] = 1.0;
        h[1] = hnew[0];
        h[2] = hnew[1];
        h[3] = hnew[2];
      }
    } else if (upd) {
      h[0] = h[1] = h[2] = h[3] = 0.0;
    }
    if (pt->delta > 0.0 && pt->delta < maxcut) {
      double Rh = t ? 2.0 * s->R * t->R / (s->R + t->R) : s->R;
      lubrication_terms(cfg, min_lub_gap(d, Rh), pt->n, pt->delta, s->u, s->w, s->R, uj,
                        wj, Rj, pt->is_wall, Flub, Tlub);
    }
  }
  free(pts);
  double V = (4.0 / 3.0) * PI * s->R * s->R * s->R;
  for (int a = 0; a < 3; ++a) {
    double Fext = V * (s->rho - 1.0) * cfg->gravity[a];
    Fout[a] = ((s->Ffp[a] + Flub[a]) + Fcol[a]) + Fext;
    Tout[a] = (s->Tfp[a] + Tlub[a]) + Tcol[a];
    s->Flub[a] = Flub[a];
    s->Tlub[a] = Tlub[a];
    s->Fcol[a] = Fcol[a];
    s->Tcol[a] = Tcol[a];
  }
}

static void wrap_position(const ref_domain* d, double* x) {
  for (int a = 0; a < 3; ++a) {
    if (d->cfg.walls[a]) continue;
    double L = (double)d->n[a];
    if (x[a] < 0.0)
      x[a] += L;
    else if (x[a] >= L)
      x[a] -= L;
  }
}

/* Alg. 1, DEM sub-cycles with dt_p = 1/n_sub; F_fp held constant */
static void dem_substeps(ref_domain* d) {
  const int P = d->P;
  const double dtp = 1.0 / (double)d->cfg.n_sub;
  double* Fn = (double*)malloc(sizeof(double) * 6 * (size_t)(P > 0 ? P : 1));
  for (int sub = 0; sub < d->cfg.n_sub; ++sub) {
    for (int i = 0; i < P; ++i) {
      sphere_t* s = &d->sp[i];
      if (s->mode == MODE_PRESCRIBED && gap_ahead(d, s) < s->release_gap) {
        s->mode = MODE_FREE;
        s->old_valid = 0;
      }
    }
    for (int i = 0; i < P; ++i) {
      sphere_t* s = &d->sp[i];
      if (s->mode == MODE_FREE && !s->old_valid) {
        eval_forces(d, i, 0, 0, dtp, s->Fold, s->Told);
        s->old_valid = 1;
      }
    }
    /* Eq. (velocity_verlet_1) */
    for (int i = 0; i < P; ++i) {
      sphere_t* s = &d->sp[i];
      if (s->mode == MODE_FREE) {
        double c2 = dtp * dtp / (2.0 * s->m);
        for (int a = 0; a < 3; ++a) s->x[a] = (s->x[a] + dtp * s->u[a]) + c2 * s->Fold[a];
      } else if (s->mode == MODE_PRESCRIBED) {
        for (int a = 0; a < 3; ++a) s->x[a] = s->x[a] + dtp * s->u[a];
      }
      wrap_position(d, s->x);
    }
    /* lubrication, contacts and external forces at the new positions */
    for (int i = 0; i < P; ++i) eval_forces(d, i, 1, 1, dtp, &Fn[6 * i], &Fn[6 * i + 3]);
    /* Eq. (velocity_verlet_2) and its rotational analogue */
    for (int i = 0; i < P; ++i) {
      sphere_t* s = &d->sp[i];
      for (int a = 0; a < 3; ++a) {
        s->Ftot[a] = Fn[6 * i + a];
        s->Ttot[a] = Fn[6 * i + 3 + a];
      }
      if (s->mode == MODE_FREE) {
        double cu = dtp / (2.0 * s->m), cw = dtp / (2.0 * s->I);
        for (int a = 0; a < 3; ++a) {
          s->u[a] = s->u[a] + cu * (s->Fold[a] + Fn[6 * i + a]);
          s->w[a] = s->w[a] + cw * (s->Told[a] + Fn[6 * i + 3 + a]);
          s->Fold[a] = Fn[6 * i + a];
          s->Told[a] = Fn[6 * i + 3 + a];
        }
      } else if (s->mode == MODE_PRESCRIBED) {
        /* Eq. (artificial_acceleration) */
        s->t_presc += dtp;
        double ramp = 1.0 - exp(-s->c_acc * s->t_presc / s->t_st);
        for (int a = 0; a < 3; ++a) {
          s->u[a] = s->utgt[a] * ramp;
          s->w[a] = 0.0;
        }
      }
    }
  }
  free(Fn);
}

/* ------------------------------- step 5 ---------------------------------- */

/* Eq. (PDF_reconstruction) into the current post-collision buffer */
static void reconstruct_cell(ref_domain* d, double* buf, const uint8_t* oldc,
                             const uint8_t* newc, int i, int j, int k, int pid) {
  const long N = d->N;
  const sphere_t* s = &d->sp[pid];
  long x = cidx(d, i, j, k);
  double snu, smi, sb;
  ref_rates(&d->cfg, &snu, &smi, &sb);
  (void)smi;
  (void)sb;
  double rsum = 0.0;
  int nvalid = 0;
  for (int q = 1; q < NQ; ++q) {
    long y = cidx(d, wrapi(i + LC[q][0], d->n[0]), wrapi(j + LC[q][1], d->n[1]),
                  wrapi(k + LC[q][2], d->n[2]));
    if (!is_fluid_code(oldc[y]) || !is_fluid_code(newc[y])) continue;
    double r = 0.0;
    for (int p = 0; p < NQ; ++p) r += buf[p * N + y];
    rsum += r;
    nvalid += 1;
  }
  double rb = nvalid > 0 ? rsum / (double)nvalid : 1.0;
  double rel[3], ut[3];
  rel[0] = minimg(d, 0, ((double)i + 0.5) - s->x[0]);
  rel[1] = minimg(d, 1, ((double)j + 0.5) - s->x[1]);
  rel[2] = minimg(d, 2, ((double)k + 0.5) - s->x[2]);
  body_velocity(s, rel, ut);
  /* du[a][b] = d u_a / d x_b */
  double du[3][3];
  for (int b = 0; b < 3; ++b) {
    int off[3] = {0, 0, 0};
    off[b] = 1;
    long yp = cidx(d, wrapi(i + off[0], d->n[0]), wrapi(j + off[1], d->n[1]),
                   wrapi(k + off[2], d->n[2]));
    long ym = cidx(d, wrapi(i - off[0], d->n[0]), wrapi(j - off[1], d->n[1]),
                   wrapi(k - off[2], d->n[2]));
    int vp = is_fluid_code(oldc[yp]) && is_fluid_code(newc[yp]);
    int vm = is_fluid_code(oldc[ym]) && is_fluid_code(newc[ym]);
    double up[3] = {0, 0, 0}, um[3] = {0, 0, 0};
    for (int p = 0; p < NQ; ++p)
      for (int a = 0; a < 3; ++a) {
        up[a] += buf[p * N + yp] * LC[p][a];
        um[a] += buf[p * N + ym] * LC[p][a];
      }
    for (int a = 0; a < 3; ++a) {
      if (vp && vm)
        du[a][b] = 0.5 * (up[a] - um[a]);
      else if (vp)
        du[a][b] = up[a] - ut[a];
      else if (vm)
        du[a][b] = ut[a] - um[a];
      else
        du[a][b] = 0.0;
    }
  }
  for (int q = 0; q < NQ; ++q) {
    double cu = LC[q][0] * ut[0] + LC[q][1] * ut[1] + LC[q][2] * ut[2];
    double second = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double Pab = rb * ut[a] * ut[b] - rb / (3.0 * snu) * (du[a][b] + du[b][a]);
        double Hab = (double)(LC[q][a] * LC[q][b]) - (a == b ? 1.0 / 3.0 : 0.0);
        second += Pab * Hab;
      }
    buf[q * N + x] = LW[q] * (rb + 3.0 * rb * cu + 4.5 * second);
  }
}

/* Sec. 2.2: re-map all particles; cells that turned from solid to fluid get
 * their PDFs reconstructed in the current buffer A */
static void remap(ref_domain* d, int reconstruct) {
  uint8_t* nc = (uint8_t*)malloc(d->N);
  int32_t* no = (int32_t*)malloc(sizeof(int32_t) * d->N);
  compute_mapping(d, nc, no);
  if (reconstruct) {
    for (int k = 0; k < d->n[2]; ++k)
      for (int j = 0; j < d->n[1]; ++j)
        for (int i = 0; i < d->n[0]; ++i) {
          long c = cidx(d, i, j, k);
          if (d->code[c] == CELL_SOLID && is_fluid_code(nc[c]))
            reconstruct_cell(d, d->A, d->code, nc, i, j, k, d->owner[c]);
        }
  }
  memcpy(d->code, nc, d->N);
  memcpy(d->owner, no, sizeof(int32_t) * d->N);
  free(nc);
  free(no);
}

int32_t ref_dem_step(ref_domain* d, const double* fext6) {
  if (!d) return -1;
  for (int i = 0; i < d->P; ++i)
    for (int a = 0; a < 3; ++a) {
      d->sp[i].Ffp[a] = fext6 ? fext6[6 * i + a] : 0.0;
      d->sp[i].Tfp[a] = fext6 ? fext6[6 * i + 3 + a] : 0.0;
    }
  dem_substeps(d);
  return 0;
}

int32_t ref_step(ref_domain* d, int32_t nsteps) {
  if (!d || nsteps < 0) return -1;
  double* F = (double*)malloc(sizeof(double) * 6 * (size_t)(d->P > 0 ? d->P : 1));
  for (int st = 0; st < nsteps; ++st) {
    /* Alg. 1: boundary conditions and fluid-particle interaction */
    boundary_and_forces(d, F);
    for (int i = 0; i < d->P; ++i) {
      sphere_t* s = &d->sp[i];
      for (int a = 0; a < 3; ++a) {
        s->Fraw[a] = F[6 * i + a];
        s->Traw[a] = F[6 * i + 3 + a];
      }
      if (d->cfg.force_averaging) {
        if (!s->prev_valid)
          for (int a = 0; a < 3; ++a) {
            s->Fprev[a] = s->Fraw[a];
            s->Tprev[a] = s->Traw[a];
          }
        for (int a = 0; a < 3; ++a) {
          s->Ffp[a] = 0.5 * (s->Fraw[a] + s->Fprev[a]);
          s->Tfp[a] = 0.5 * (s->Traw[a] + s->Tprev[a]);
          s->Fprev[a] = s->Fraw[a];
          s->Tprev[a] = s->Traw[a];
        }
        s->prev_valid = 1;
      } else {
        for (int a = 0; a < 3; ++a) {
          s->Ffp[a] = s->Fraw[a];
          s->Tfp[a] = s->Traw[a];
        }
      }
    }
    /* LBM step into B */
    lbm_step(d);
    double* t = d->A;
    d->A = d->B;
    d->B = t;
    /* DEM sub-cycles */
    dem_substeps(d);
    /* mapping update with reconstruction (into the new current buffer) */
    remap(d, 1);
    d->steps += 1;
  }
  free(F);
  return 0;
}

int32_t ref_get_sphere(const ref_domain* d, int32_t id, double* out) {
  if (!d || id < 0 || id >= d->P) return -1;
  const sphere_t* s = &d->sp[id];
  for (int a = 0; a < 3; ++a) {
    out[0 + a] = s->x[a];
    out[3 + a] = s->u[a];
    out[6 + a] = s->w[a];
    out[9 + a] = s->Ffp[a];
    out[12 + a] = s->Tfp[a];
    out[15 + a] = s->Ftot[a];
    out[18 + a] = s->Ttot[a];
    out[21 + a] = s->Flub[a];
    out[24 + a] = s->Tlub[a];
    out[27 + a] = s->Fcol[a];
    out[30 + a] = s->Tcol[a];
    out[36 + a] = s->Fraw[a];
    out[39 + a] = s->Traw[a];
  }
  out[33] = (double)s->mode;
  out[34] = s->R;
  out[35] = s->rho;
  return 0;
}

int32_t ref_num_spheres(const ref_domain* d) { return d ? d->P : -1; }

int32_t ref_get_field(const ref_domain* d, int32_t field, double* dst) {
  if (!d) return -1;
  const long N = d->N;
  for (long c = 0; c < N; ++c) {
    int fl = is_fluid_code(d->code[c]);
    if (field == 0) {
      double r = 0.0;
      if (fl)
        for (int q = 0; q < NQ; ++q) r += d->A[q * N + c];
      dst[c] = r;
    } else if (field == 1) {
      double u[3] = {0, 0, 0};
      if (fl) {
        for (int q = 0; q < NQ; ++q)
          for (int a = 0; a < 3; ++a) u[a] += d->A[q * N + c] * LC[q][a];
        /* the stored state is post-collision, whose momentum already holds the
         * full body-force impulse; the physical velocity is half-way */
        for (int a = 0; a < 3; ++a) u[a] -= 0.5 * d->cfg.body_force[a];
      }
      for (int a = 0; a < 3; ++a) dst[a * N + c] = u[a];
    } else if (field == 2) {
      for (int q = 0; q < NQ; ++q) dst[q * N + c] = fl ? d->A[q * N + c] : 0.0;
    } else {
      return -1;
    }
  }
  return 0;
}

int32_t ref_get_flags(const ref_domain* d, uint8_t* code, int32_t* owner) {
  if (!d) return -1;
  if (code) memcpy(code, d->code, d->N);
  if (owner) memcpy(owner, d->owner, sizeof(int32_t) * d->N);
  return 0;
}

int32_t ref_set_pdf(ref_domain* d, const double* f) {
  if (!d) return -1;
  memcpy(d->A, f, sizeof(double) * NQ * d->N);
  return 0;
}

int64_t ref_step_count(const ref_domain* d) { return d ? d->steps : -1; }
