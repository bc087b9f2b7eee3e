// Discrete element part of one time step (Alg. 1, DEM sub-cycles), FP64.
//
// Prologue: per-sphere sum of the momentum-exchange partials written by the
// boundary kernel (fixed order), averaging with the previous step (Sec. 4.2;
// the first step averages with itself), copy of the positions the mapping
// starts from, and a neighbour list per sphere (candidates whose gap is below
// the largest lubrication cut-off plus a skin, ascending ids).  Then n_sub
// sub-cycles with dt_p = 1/n_sub and F_fp held constant:
//   release of prescribed spheres below their gap; velocity-Verlet start force
//   for newly free spheres; Eq. (velocity_verlet_1); lubrication (Sec. 3.1,
//   step function on the raw gap, magnitude on max(gap, delta_min)), contacts
//   (Eqs. normalCollisionForce, tangentialCollisionForce with the spring
//   projected, rescaled and reset as in Sec. 4.1.2), external force
//   V (rho_p - rho_f) g; Eq. (velocity_verlet_2) and its rotational analogue.
// Forces are gathered per sphere (each sphere sums over its own partners), so
// nothing is scattered and the pair terms come out antisymmetric exactly.
//
// Two kernels.  Few spheres: one workgroup, sub-cycles separated by workgroup
// barriers (with state, histories and lists in LDS up to DEM_LDS_MAX spheres).
// Many spheres: one thread per sphere over a chain of launches; neighbours
// are found through uniform bins, and x, u, w alternate between two buffers
// every sub-cycle (positions are advanced into the other buffer, then forces
// read the new positions and the old velocities and write the new velocities
// into the other buffer), so each sub-cycle needs only two launches.
#include "internal.hpp"

#include <climits>

namespace lbmdem {

constexpr double PI_D = 3.14159265358979323846;

struct Partner {
  int code;        // sphere id >= 0, wall -1 - (2 axis + side)
  int j;           // sphere id or -1
  double n[3];     // unit normal from partner to i
  double delta;    // signed gap
  double xcp[3];   // contact point
  double rj[3];    // xcp - x_j
};

__device__ inline void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ inline double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
__device__ inline double norm3(const double* a) { return sqrt(dot3(a, a)); }

// rigid-body surface velocity u + w x r (r = point - centre)
__device__ inline void body_vel(const double* u, const double* w, const double* r, double* U) {
  double wr[3];
  cross3(w, r, wr);
  U[0] = u[0] + wr[0];
  U[1] = u[1] + wr[1];
  U[2] = u[2] + wr[2];
}

__device__ __forceinline__ void make_sphere_partner(const DevDomain& d, const DevParticles& p, int i, int j,
                                                    Partner& pt) {
  double dd[3];
  const int n[3] = {d.nx, d.ny, d.nz};
  for (int a = 0; a < 3; ++a) dd[a] = min_image(p.x[3 * i + a] - p.x[3 * j + a], n[a], d.walls[a]);
  const double dist = norm3(dd);
  pt.code = j;
  pt.j = j;
  for (int a = 0; a < 3; ++a) pt.n[a] = dd[a] / dist;
  pt.delta = dist - (p.R[i] + p.R[j]);
  for (int a = 0; a < 3; ++a) {
    pt.xcp[a] = p.x[3 * i + a] - 0.5 * dd[a];
    pt.rj[a] = 0.5 * dd[a];
  }
}

__device__ __forceinline__ void make_wall_partner(const DevDomain& d, const DevParticles& p, int i, int a,
                                                  int side, Partner& pt) {
  // selects instead of indexing local arrays with the runtime axis, so that
  // nothing spills to scratch memory
  const double s = side ? -1.0 : 1.0;
  pt.code = -1 - (2 * a + side);
  pt.j = -1;
  pt.n[0] = a == 0 ? s : 0.0;
  pt.n[1] = a == 1 ? s : 0.0;
  pt.n[2] = a == 2 ? s : 0.0;
  const double R = p.R[i];
  const double x0 = p.x[3 * i], x1 = p.x[3 * i + 1], x2 = p.x[3 * i + 2];
  const double xa = a == 0 ? x0 : (a == 1 ? x1 : x2);
  const int na = a == 0 ? d.nx : (a == 1 ? d.ny : d.nz);
  pt.delta = side ? (((double)na - 1.0) - xa) - R : (xa - 1.0) - R;
  const double h = R + 0.5 * pt.delta;
  pt.xcp[0] = x0 - h * pt.n[0];
  pt.xcp[1] = x1 - h * pt.n[1];
  pt.xcp[2] = x2 - h * pt.n[2];
  pt.rj[0] = pt.rj[1] = pt.rj[2] = 0.0;
}

__device__ inline double collision_time(const DevDomain& d, double D) {
  return d.tc > 0.0 ? d.tc : 2.31 * D * sqrt(3.0);  // Eq. (collisionTimeChoice)
}
__device__ inline double min_lub_gap(const DevDomain& d, double R) {
  return d.dmin >= 0.0 ? d.dmin : (0.001 + 0.00007 * R) * R;  // Eq. (lubricationGapSize)
}

__device__ __forceinline__ void lubrication(const DevDomain& d, double dmin, const double* n, double delta,
                            const double* ui, const double* wi, double Ri, const double* uj,
                            const double* wj, double Rj, bool wall, double* F, double* T) {
  const double mu = d.nu;
  const double dl = delta > dmin ? delta : dmin;
  double uij[3], un[3], ut[3];
  for (int a = 0; a < 3; ++a) uij[a] = ui[a] - (wall ? 0.0 : uj[a]);
  const double uijn = dot3(uij, n);
  for (int a = 0; a < 3; ++a) {
    un[a] = uijn * n[a];
    ut[a] = uij[a] - un[a];
  }
  const double k = wall ? 0.0 : Rj / Ri;
  if ((d.lub_mask & 1) && delta > 0.0 && delta < d.cut_n) {
    const double coef = wall ? 1.0 : (k * k) / ((1.0 + k) * (1.0 + k));
    const double mag = -6.0 * PI_D * mu * Ri * Ri * coef * (1.0 / dl - 1.0 / d.cut_n);
    for (int a = 0; a < 3; ++a) F[a] += mag * un[a];
  }
  if ((d.lub_mask & 2) && delta > 0.0 && delta < d.cut_tt) {
    const double L = log(dl / d.cut_tt);
    const double cf = wall ? 8.0 / 15.0
                           : 4.0 * k * (2.0 + k + 2.0 * k * k) / (15.0 * (1.0 + k) * (1.0 + k) * (1.0 + k));
    const double ct = wall ? 0.1 : k * (4.0 + k) / (10.0 * (1.0 + k) * (1.0 + k));
    const double fm = 6.0 * PI_D * mu * Ri * cf * L;
    const double tm = 8.0 * PI_D * mu * Ri * Ri * ct * L;
    double uxn[3];
    cross3(uij, n, uxn);
    for (int a = 0; a < 3; ++a) {
      F[a] += fm * ut[a];
      T[a] += tm * uxn[a];
    }
  }
  if ((d.lub_mask & 4) && delta > 0.0 && delta < d.cut_tr) {
    const double L = log(dl / d.cut_tr);
    const double cf = wall ? 2.0 / 15.0 : 2.0 * k * k / (15.0 * (1.0 + k) * (1.0 + k));
    const double ct = wall ? 0.4 : 2.0 * k / (5.0 * (1.0 + k));
    double wv[3], av[3], wxn[3];
    for (int a = 0; a < 3; ++a) {
      wv[a] = wall ? wi[a] : (wi[a] + wj[a]) + (4.0 / k) * wi[a] + 4.0 * k * wj[a];
      av[a] = wall ? wi[a] : wi[a] + 0.25 * k * wj[a];
    }
    cross3(wv, n, wxn);
    const double an = dot3(av, n);
    const double fm = -6.0 * PI_D * mu * Ri * Ri * cf * L;
    const double tm = 8.0 * PI_D * mu * Ri * Ri * Ri * ct * L;
    for (int a = 0; a < 3; ++a) {
      F[a] += fm * wxn[a];
      T[a] += tm * (av[a] - an * n[a]);
    }
  }
}

// forces on sphere i at the current state; contact: evaluate contacts;
// upd: write the tangential-spring history
__device__ __forceinline__ void eval_forces(const DevDomain& d, const DevParticles& p, int i, bool contact,
                                            bool upd, double dtp, double* Fout, double* Tout) {
  double Flub[3] = {0, 0, 0}, Tlub[3] = {0, 0, 0}, Fcol[3] = {0, 0, 0}, Tcol[3] = {0, 0, 0};
  const double maxcut = fmax(d.cut_n, fmax(d.cut_tt, d.cut_tr));
  const double* xi = p.x + 3 * i;
  const double* ui = p.u + 3 * i;
  const double* wi = p.w + 3 * i;
  const double Ri = p.R[i];
  int* hid = p.hist_id + (size_t)i * HIST_SLOTS;
  double* hd = p.hist_d + (size_t)i * HIST_SLOTS * 3;
  const int nn = p.nbr_n[i];
  const int nwalls = 2 * (d.walls[0] + d.walls[1] + d.walls[2]);
  const double zero[3] = {0, 0, 0};
  for (int pi = 0; pi < nn + nwalls; ++pi) {
    Partner pt;
    if (pi < nn) {
      make_sphere_partner(d, p, i, p.nbr[(size_t)i * NBR_MAX + pi], pt);
    } else {
      int wk = pi - nn, a = 0;
      for (a = 0; a < 3; ++a) {
        if (!d.walls[a]) continue;
        if (wk < 2) break;
        wk -= 2;
      }
      make_wall_partner(d, p, i, a, wk, pt);
    }
    const bool is_wall = pt.j < 0;
    const double* uj = is_wall ? zero : p.u + 3 * pt.j;
    const double* wj = is_wall ? zero : p.w + 3 * pt.j;
    const double Rj = is_wall ? 0.0 : p.R[pt.j];
    int slot = -1;
    for (int s = 0; s < HIST_SLOTS; ++s)
      if (hid[s] == pt.code) slot = s;
    if (contact && pt.delta < 0.0) {
      double uij[3], un[3], Ui[3], Uj[3], ut[3], ri[3];
      for (int a = 0; a < 3; ++a) {
        uij[a] = ui[a] - uj[a];
        ri[a] = pt.xcp[a] - xi[a];
      }
      const double uijn = dot3(uij, pt.n);
      for (int a = 0; a < 3; ++a) un[a] = uijn * pt.n[a];
      body_vel(ui, wi, ri, Ui);
      if (is_wall) {
        Uj[0] = Uj[1] = Uj[2] = 0.0;
      } else {
        body_vel(uj, wj, pt.rj, Uj);
      }
      for (int a = 0; a < 3; ++a) ut[a] = (Ui[a] - Uj[a]) - un[a];
      const double mi = p.m[i];
      const double meff = is_wall ? mi : mi * p.m[pt.j] / (mi + p.m[pt.j]);
      const double D = is_wall ? 2.0 * Ri : Ri + Rj;
      const double Tc = collision_time(d, D);
      const double le = log(d.e_dry);
      const double kn = meff * (PI_D * PI_D + le * le) / (Tc * Tc);  // Eq. (normalDEMparameters)
      const double dn = -2.0 * meff * le / Tc;
      const double kp = 2.0 * (1.0 - d.poisson_ratio) / (2.0 - d.poisson_ratio);
      const double kt = kp * kn;  // Eq. (tangentialCollisionParameters)
      const double dt = sqrt(kp) * dn;
      double Fn[3];
      for (int a = 0; a < 3; ++a) Fn[a] = -kn * pt.delta * pt.n[a] - dn * un[a];
      double hv[3] = {0, 0, 0};
      if (slot >= 0)
        for (int a = 0; a < 3; ++a) hv[a] = hd[slot * 3 + a];
      const double hn = dot3(hv, pt.n);
      double ht[3];
      for (int a = 0; a < 3; ++a) ht[a] = hv[a] - hn * pt.n[a];
      const double lh = norm3(hv), lht = norm3(ht);
      if (lht > 0.0)
        for (int a = 0; a < 3; ++a) hv[a] = (lh / lht) * ht[a];
      else
        for (int a = 0; a < 3; ++a) hv[a] = ht[a];
      double Fsd[3];
      for (int a = 0; a < 3; ++a) Fsd[a] = -kt * hv[a] - dt * ut[a];
      const double fsd = norm3(Fsd);
      const double fmax = d.friction * norm3(Fn);
      double Ft[3], hnew[3];
      if (fsd < fmax || fsd == 0.0) {
        for (int a = 0; a < 3; ++a) {
          Ft[a] = Fsd[a];
          hnew[a] = hv[a] + dtp * ut[a];
        }
      } else {
        for (int a = 0; a < 3; ++a) {
          const double tv = Fsd[a] / fsd;
          Ft[a] = fmax * tv;
          hnew[a] = -(fmax * tv + dt * ut[a]) / kt;
        }
      }
      double Tt[3];
      cross3(ri, Ft, Tt);
      for (int a = 0; a < 3; ++a) {
        Fcol[a] += Fn[a] + Ft[a];
        Tcol[a] += Tt[a];
      }
      if (upd) {
        if (slot < 0)
          for (int s = 0; s < HIST_SLOTS && slot < 0; ++s)
            if (hid[s] == INT_MIN) slot = s;
        if (slot < 0) {
          atomicOr(d.status, ST_HIST_FULL);
        } else {
          hid[slot] = pt.code;
          for (int a = 0; a < 3; ++a) hd[slot * 3 + a] = hnew[a];
        }
      }
    } else if (upd && slot >= 0) {
      hid[slot] = INT_MIN;
    }
    if (pt.delta > 0.0 && pt.delta < maxcut) {
      const double Rh = is_wall ? Ri : 2.0 * Ri * Rj / (Ri + Rj);
      lubrication(d, min_lub_gap(d, Rh), pt.n, pt.delta, ui, wi, Ri, uj, wj, Rj, is_wall, Flub, Tlub);
    }
  }
  const double V = (4.0 / 3.0) * PI_D * Ri * Ri * Ri;
  const double* Ffp = p.Ffp + 6 * i;
  double* dg = p.diag + 18 * i;
  for (int a = 0; a < 3; ++a) {
    const double Fext = V * (p.rho[i] - 1.0) * d.gravity[a];
    Fout[a] = ((Ffp[a] + Flub[a]) + Fcol[a]) + Fext;
    Tout[a] = (Ffp[3 + a] + Tlub[a]) + Tcol[a];
    dg[6 + a] = Flub[a];
    dg[9 + a] = Tlub[a];
    dg[12 + a] = Fcol[a];
    dg[15 + a] = Tcol[a];
  }
}

// Momentum-exchange sum of sphere i by one wavefront: lane l adds the
// partials l, l + 64, ... in order, then a fixed shuffle tree combines the
// lanes, so the result does not depend on scheduling.  Lane 0 then averages
// with the previous step and pins the positions the mapping starts from.
__device__ __forceinline__ void resolved_force(const DevDomain& d, const DevParticles& p, int i, int lane) {
  const int nb = d.ZB * d.RB;
  double F[6] = {0, 0, 0, 0, 0, 0};
  for (int b = lane; b < nb; b += 64)
    for (int k = 0; k < 6; ++k) F[k] += d.partial[((size_t)i * nb + b) * 6 + k];
  for (int k = 0; k < 6; ++k) {
    double v = F[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    F[k] = v;
  }
  if (lane != 0) return;
  for (int k = 0; k < 6; ++k) p.Fraw[6 * i + k] = F[k];
  if (d.force_averaging) {
    if (!p.prev_valid[i])
      for (int k = 0; k < 6; ++k) p.Fprev[6 * i + k] = F[k];
    for (int k = 0; k < 6; ++k) {
      p.Ffp[6 * i + k] = 0.5 * (F[k] + p.Fprev[6 * i + k]);
      p.Fprev[6 * i + k] = F[k];
    }
    p.prev_valid[i] = 1;
  } else {
    for (int k = 0; k < 6; ++k) p.Ffp[6 * i + k] = F[k];
  }
  for (int a = 0; a < 3; ++a) p.xmap[3 * i + a] = p.x[3 * i + a];
}

// gap between spheres i and j (minimum image); the neighbour test of both
// kernels, so that they list the same partners
__device__ __forceinline__ double pair_gap(const DevDomain& d, const DevParticles& p, int i, int j) {
  const int n[3] = {d.nx, d.ny, d.nz};
  double dd[3];
  for (int a = 0; a < 3; ++a) dd[a] = min_image(p.x[3 * i + a] - p.x[3 * j + a], n[a], d.walls[a]);
  return norm3(dd) - (p.R[i] + p.R[j]);
}

__device__ __forceinline__ double list_range(const DevDomain& d) {
  return fmax(d.cut_n, fmax(d.cut_tt, d.cut_tr)) + d.skin;
}

// Gap of a prescribed sphere to the wall plane it approaches: the plane ahead
// along its target velocity on every walled axis where that is nonzero
// (Sec. 4.4.2 switches the acceleration off near the wall the sphere moves
// to); large if there is none.
__device__ inline double gap_ahead(const DevDomain& d, const DevParticles& p, int i) {
  double g = 1e300;
  const int n[3] = {d.nx, d.ny, d.nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double ut = p.presc[6 * i + a];
    if (!d.walls[a] || ut == 0.0) continue;
    const double v = ut < 0.0 ? (p.x[3 * i + a] - 1.0) - p.R[i] : (((double)n[a] - 1.0) - p.x[3 * i + a]) - p.R[i];
    g = fmin(g, v);
  }
  return g;
}

// release of a prescribed sphere below its gap; start force of a newly free one
__device__ __forceinline__ void release_and_start(const DevDomain& d, const DevParticles& p, int i, double dtp) {
  if (p.mode[i] == MODE_PRESCRIBED && gap_ahead(d, p, i) < p.presc[6 * i + 5]) {
    p.mode[i] = MODE_FREE;
    p.old_valid[i] = 0;
  }
  if (p.mode[i] == MODE_FREE && !p.old_valid[i]) {
    eval_forces(d, p, i, false, false, dtp, p.Fold + 6 * i, p.Fold + 6 * i + 3);
    p.old_valid[i] = 1;
  }
}

// Eq. (velocity_verlet_1) (free), x + dt_p u (prescribed), unchanged (fixed);
// periodic axes wrap.  xo may alias p.x + 3 i.
__device__ __forceinline__ void advance_position(const DevDomain& d, const DevParticles& p, int i, double dtp,
                                                 double* xo) {
  const int n[3] = {d.nx, d.ny, d.nz};
  const double* x = p.x + 3 * i;
  if (p.mode[i] == MODE_FREE) {
    const double c2 = dtp * dtp / (2.0 * p.m[i]);
    for (int a = 0; a < 3; ++a) xo[a] = (x[a] + dtp * p.u[3 * i + a]) + c2 * p.Fold[6 * i + a];
  } else if (p.mode[i] == MODE_PRESCRIBED) {
    for (int a = 0; a < 3; ++a) xo[a] = x[a] + dtp * p.u[3 * i + a];
  } else {
    for (int a = 0; a < 3; ++a) xo[a] = x[a];
  }
  for (int a = 0; a < 3; ++a) {
    if (d.walls[a]) continue;
    const double L = (double)n[a];
    if (xo[a] < 0.0)
      xo[a] += L;
    else if (xo[a] >= L)
      xo[a] -= L;
  }
}

// Eq. (velocity_verlet_2) and its rotational analogue from F_old and the new
// force in p.Fnew; the ramp of Eq. (artificial_acceleration) for prescribed
// spheres.  uo, wo may alias p.u + 3 i, p.w + 3 i.
__device__ __forceinline__ void advance_velocity(const DevDomain& d, const DevParticles& p, int i, double dtp,
                                                 double* uo, double* wo) {
  const double* Fn = p.Fnew + 6 * i;
  double* dg = p.diag + 18 * i;
  for (int k = 0; k < 6; ++k) dg[k] = Fn[k];
  if (p.mode[i] == MODE_FREE) {
    const double cu = dtp / (2.0 * p.m[i]), cw = dtp / (2.0 * p.I[i]);
    for (int a = 0; a < 3; ++a) {
      uo[a] = p.u[3 * i + a] + cu * (p.Fold[6 * i + a] + Fn[a]);
      wo[a] = p.w[3 * i + a] + cw * (p.Fold[6 * i + 3 + a] + Fn[3 + a]);
      p.Fold[6 * i + a] = Fn[a];
      p.Fold[6 * i + 3 + a] = Fn[3 + a];
    }
  } else if (p.mode[i] == MODE_PRESCRIBED) {
    p.tpresc[i] += dtp;
    const double ramp = 1.0 - exp(-p.presc[6 * i + 3] * p.tpresc[i] / p.presc[6 * i + 4]);
    for (int a = 0; a < 3; ++a) {
      uo[a] = p.presc[6 * i + a] * ramp;
      wo[a] = 0.0;
    }
  } else {
    for (int a = 0; a < 3; ++a) {
      uo[a] = p.u[3 * i + a];
      wo[a] = p.w[3 * i + a];
    }
  }
}

__device__ __forceinline__ void health_check(const DevDomain& d, const DevParticles& p, int i) {
  bool ok = true;
  for (int a = 0; a < 3; ++a)
    ok = ok && isfinite(p.x[3 * i + a]) && isfinite(p.u[3 * i + a]) && isfinite(p.w[3 * i + a]);
  if (!ok) atomicOr(d.status, ST_NONFINITE);
}

__device__ __forceinline__ void dem_body(const DevDomain& d, const DevParticles& p) {
  const int P = d.P;
  {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    for (int i = wave; i < P; i += nwave) resolved_force(d, p, i, lane);
  }
  __syncthreads();
  // neighbour list for this step by all pairs, partners ascending
  const double range = list_range(d);
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    int cnt = 0;
    for (int j = 0; j < P; ++j) {
      if (j == i || !(pair_gap(d, p, i, j) < range)) continue;
      if (cnt < NBR_MAX)
        p.nbr[(size_t)i * NBR_MAX + cnt] = j;
      else
        atomicOr(d.status, ST_NBR_FULL);
      cnt++;
    }
    p.nbr_n[i] = cnt < NBR_MAX ? cnt : NBR_MAX;
  }
  __syncthreads();
  const double dtp = 1.0 / (double)d.n_sub;
  for (int sub = 0; sub < d.n_sub; ++sub) {
    for (int i = threadIdx.x; i < P; i += blockDim.x) release_and_start(d, p, i, dtp);
    __syncthreads();
    for (int i = threadIdx.x; i < P; i += blockDim.x) advance_position(d, p, i, dtp, p.x + 3 * i);
    __syncthreads();
    for (int i = threadIdx.x; i < P; i += blockDim.x)
      eval_forces(d, p, i, true, true, dtp, p.Fnew + 6 * i, p.Fnew + 6 * i + 3);
    __syncthreads();
    for (int i = threadIdx.x; i < P; i += blockDim.x) advance_velocity(d, p, i, dtp, p.u + 3 * i, p.w + 3 * i);
    __syncthreads();
  }
  for (int i = threadIdx.x; i < P; i += blockDim.x) health_check(d, p, i);
}

// ---- step control -----------------------------------------------------------

// At the start of the step's DEM kernel: true if the domain does not step (it
// is frozen, or the stop rule was met at the end of the last step; the step
// control kernel then freezes it).
__device__ __forceinline__ bool dem_stopped(const DevDomain& d) { return !step_live(d.ctl); }

__global__ void k_advance(DevDomain d) { step_control(d); }

__global__ void k_advance_batch(const DevDomain* __restrict__ tab, int ndom) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < ndom) step_control(tab[k]);
}

// one workgroup, state in global memory
__device__ __forceinline__ void dem_global_run(const DevDomain& d) {
  dem_body(d, d.p);
}

__global__ __launch_bounds__(256) void k_dem(DevDomain d) {
  __builtin_amdgcn_s_setprio(3);
  if (dem_stopped(d)) return;
  dem_global_run(d);
}

// Few spheres: their state, contact histories and neighbour lists live in LDS
// for the whole step, so the sub-cycles (separated by workgroup barriers) do
// not wait on memory round trips.
constexpr int DEM_LDS_MAX = 32;

__device__ __forceinline__ void dem_lds_run(const DevDomain& d) {
  constexpr int PS = DEM_LDS_MAX;
  __shared__ double sx[3 * PS], su[3 * PS], sw[3 * PS], sR[PS], sm[PS], sI[PS], srho[PS], stp[PS];
  __shared__ double spresc[6 * PS], sFfp[6 * PS], sFold[6 * PS], sdiag[18 * PS], sFnew[6 * PS];
  __shared__ double shd[3 * HIST_SLOTS * PS];
  __shared__ int smode[PS], sold[PS], shid[HIST_SLOTS * PS], snbr[NBR_MAX * PS], snn[PS];
  const int P = d.P;
  const DevParticles& g = d.p;
  for (int t = threadIdx.x; t < P; t += blockDim.x) {
    for (int a = 0; a < 3; ++a) {
      sx[3 * t + a] = g.x[3 * t + a];
      su[3 * t + a] = g.u[3 * t + a];
      sw[3 * t + a] = g.w[3 * t + a];
    }
    sR[t] = g.R[t];
    sm[t] = g.m[t];
    sI[t] = g.I[t];
    srho[t] = g.rho[t];
    stp[t] = g.tpresc[t];
    smode[t] = g.mode[t];
    sold[t] = g.old_valid[t];
    for (int k = 0; k < 6; ++k) {
      spresc[6 * t + k] = g.presc[6 * t + k];
      sFold[6 * t + k] = g.Fold[6 * t + k];
    }
    for (int k = 0; k < HIST_SLOTS; ++k) {
      shid[HIST_SLOTS * t + k] = g.hist_id[(size_t)HIST_SLOTS * t + k];
      for (int a = 0; a < 3; ++a) shd[3 * (HIST_SLOTS * t + k) + a] = g.hist_d[3 * ((size_t)HIST_SLOTS * t + k) + a];
    }
  }
  __syncthreads();
  DevParticles l = g;
  l.x = sx;
  l.u = su;
  l.w = sw;
  l.R = sR;
  l.m = sm;
  l.I = sI;
  l.rho = srho;
  l.presc = spresc;
  l.tpresc = stp;
  l.Ffp = sFfp;
  l.Fold = sFold;
  l.diag = sdiag;
  l.Fnew = sFnew;
  l.mode = smode;
  l.old_valid = sold;
  l.hist_id = shid;
  l.hist_d = shd;
  l.nbr = snbr;
  l.nbr_n = snn;
  dem_body(d, l);
  __syncthreads();
  for (int t = threadIdx.x; t < P; t += blockDim.x) {
    for (int a = 0; a < 3; ++a) {
      g.x[3 * t + a] = sx[3 * t + a];
      g.u[3 * t + a] = su[3 * t + a];
      g.w[3 * t + a] = sw[3 * t + a];
    }
    g.tpresc[t] = stp[t];
    g.mode[t] = smode[t];
    g.old_valid[t] = sold[t];
    for (int k = 0; k < 6; ++k) {
      g.Ffp[6 * t + k] = sFfp[6 * t + k];
      g.Fold[6 * t + k] = sFold[6 * t + k];
    }
    for (int k = 0; k < 18; ++k) g.diag[18 * t + k] = sdiag[18 * t + k];
    for (int k = 0; k < HIST_SLOTS; ++k) {
      g.hist_id[(size_t)HIST_SLOTS * t + k] = shid[HIST_SLOTS * t + k];
      for (int a = 0; a < 3; ++a) g.hist_d[3 * ((size_t)HIST_SLOTS * t + k) + a] = shd[3 * (HIST_SLOTS * t + k) + a];
    }
  }
}

// The one-workgroup kernels run beside the sweep in an overlapped step: they
// are a chain of dependent FP64 work, so their waves take the highest issue
// priority on the CUs they share with the sweep's waves.
__global__ __launch_bounds__(256) void k_dem_lds(DevDomain d) {
  __builtin_amdgcn_s_setprio(3);
  if (dem_stopped(d)) return;
  dem_lds_run(d);
}

// many domains, one workgroup each (the few-sphere kernels above)
__global__ __launch_bounds__(256) void k_dem_batch(const DevDomain* __restrict__ tab, int ndom) {
  const DevDomain& d = tab[blockIdx.x];
  if (dem_stopped(d)) return;
  if (d.P <= DEM_LDS_MAX)
    dem_lds_run(d);
  else
    dem_global_run(d);
}

void launch_dem_batch(const BatchTables& b, hipStream_t s) {
  if (b.ndom > 0) hipLaunchKernelGGL(k_dem_batch, dim3(b.ndom), dim3(256), 0, s, b.tab, b.ndom);
}

void launch_advance(const DevDomain& d, hipStream_t s) { hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, s, d); }

void launch_advance_batch(const BatchTables& b, hipStream_t s) {
  if (b.ndom > 0) hipLaunchKernelGGL(k_advance_batch, dim3((b.ndom + 63) / 64), dim3(64), 0, s, b.tab, b.ndom);
}

// ---------------------------------------------------------------------------
// Grid-wide kernel for many spheres.

__device__ __forceinline__ int bin_index(const DevDomain& d, const double* x, int* b) {
  const int n[3] = {d.nx, d.ny, d.nz};
  for (int a = 0; a < 3; ++a) {
    const int nb = d.bins.n[a];
    int k = (int)floor(x[a] * (double)nb / (double)n[a]);
    b[a] = k < 0 ? 0 : (k >= nb ? nb - 1 : k);
  }
  return b[0] + d.bins.n[0] * (b[1] + d.bins.n[1] * b[2]);
}

__device__ __forceinline__ void bin_insert(const DevDomain& d, const DevParticles& p, int i) {
  const double* x = p.x + 3 * i;
  if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]))) {
    atomicOr(d.status, ST_NONFINITE);
    return;
  }
  int b[3];
  int* c = d.bins.cell + (size_t)bin_index(d, x, b) * (1 + BIN_CAP);
  const int k = atomicAdd(c, 1);
  if (k < BIN_CAP)
    c[1 + k] = i;
  else
    atomicOr(d.status, ST_NBR_FULL);
}

// the neighbour test of dem_body over the candidates of the surrounding bins,
// kept sorted by id, so both kernels produce the same list
__device__ __forceinline__ void binned_neighbours(const DevDomain& d, const DevParticles& p, int i) {
  const double* x = p.x + 3 * i;
  if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]))) {
    p.nbr_n[i] = 0;
    return;
  }
  const double range = list_range(d);
  int b[3];
  bin_index(d, x, b);
  const int n0 = d.bins.n[0], n1 = d.bins.n[1], n2 = d.bins.n[2];
  int* out = p.nbr + (size_t)i * NBR_MAX;
  int cnt = 0;
  for (int ez = 0; ez < axis_count(n2); ++ez) {
    int kz;
    if (!axis_bin(b[2], n2, d.walls[2], ez, &kz)) continue;
    for (int ey = 0; ey < axis_count(n1); ++ey) {
      int ky;
      if (!axis_bin(b[1], n1, d.walls[1], ey, &ky)) continue;
      for (int ex = 0; ex < axis_count(n0); ++ex) {
        int kx;
        if (!axis_bin(b[0], n0, d.walls[0], ex, &kx)) continue;
        const int* c = d.bins.cell + (size_t)(kx + n0 * (ky + n1 * kz)) * (1 + BIN_CAP);
        const int m = min(c[0], BIN_CAP);
        for (int e = 0; e < m; ++e) {
          const int j = c[1 + e];
          if (j == i || !(pair_gap(d, p, i, j) < range)) continue;
          if (cnt < NBR_MAX) {
            int pos = cnt;
            while (pos > 0 && out[pos - 1] > j) {
              out[pos] = out[pos - 1];
              --pos;
            }
            out[pos] = j;
          } else {
            atomicOr(d.status, ST_NBR_FULL);
          }
          cnt++;
        }
      }
    }
  }
  p.nbr_n[i] = cnt < NBR_MAX ? cnt : NBR_MAX;
}

// Many spheres: one thread per sphere, the sub-cycles as a chain of ordinary
// launches (a kernel boundary wherever every sphere must see the others'
// state): the momentum-exchange sums and the bins, the neighbour lists, then
// per sub-cycle the positions (into the other buffer) and the forces and
// velocities (into the other buffer).  Ordinary launches can run beside the
// sweep on a second stream, where a cooperative grid could not be sure of
// having all its blocks resident.  Per sphere the arithmetic and its order are
// those of the one-workgroup kernels (identical bits).
__global__ __launch_bounds__(DEM_GRID_THREADS) void k_demg_prologue(DevDomain d) {
  if (dem_stopped(d)) return;
  const int lane = threadIdx.x & 63;
  const int i = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (i >= d.P) return;
  resolved_force(d, d.p, i, lane);
  if (lane == 0) bin_insert(d, d.p, i);
}

__global__ __launch_bounds__(DEM_GRID_THREADS) void k_demg_neighbours(DevDomain d) {
  if (dem_stopped(d)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.P) binned_neighbours(d, d.p, i);
}

// state of sub-cycle `sub` (even: the first buffers), and the other buffer
__device__ __forceinline__ void subcycle_buffers(const DevParticles& p, int sub, DevParticles& a, double** x1,
                                                 double** u1, double** w1) {
  const bool odd = sub & 1;
  a = p;
  a.x = odd ? p.x2 : p.x;
  a.u = odd ? p.u2 : p.u;
  a.w = odd ? p.w2 : p.w;
  *x1 = odd ? p.x : p.x2;
  *u1 = odd ? p.u : p.u2;
  *w1 = odd ? p.w : p.w2;
}

__global__ __launch_bounds__(DEM_GRID_THREADS) void k_demg_position(DevDomain d, int sub) {
  if (dem_stopped(d)) return;
  const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
  if (sub == 0) {  // the lists are built: clear the bins for the next step
    const int nbins = d.bins.n[0] * d.bins.n[1] * d.bins.n[2];
    for (int k = gtid; k < nbins; k += gridDim.x * blockDim.x) d.bins.cell[(size_t)k * (1 + BIN_CAP)] = 0;
  }
  if (gtid >= d.P) return;
  DevParticles a;
  double *x1, *u1, *w1;
  subcycle_buffers(d.p, sub, a, &x1, &u1, &w1);
  const double dtp = 1.0 / (double)d.n_sub;
  release_and_start(d, a, gtid, dtp);
  advance_position(d, a, gtid, dtp, x1 + 3 * gtid);
}

// forces at the new positions with the old velocities, new velocities into
// the other buffer; after the last sub-cycle the state is copied back if it
// ended in the second buffers (odd n_sub, a kernel of its own) and checked.
// With `fuse` the thread then advances its own sphere's position of the next
// sub-cycle: nothing in this launch reads the buffer that goes into, and that
// step reads only the sphere's own state -- valid when no sphere can be
// released from a prescribed motion (a release evaluates forces on every
// partner's state, which needs the sub-cycle's launch boundary).
__global__ __launch_bounds__(DEM_GRID_THREADS) void k_demg_velocity(DevDomain d, int sub, int fuse) {
  if (dem_stopped(d)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.P) return;
  DevParticles a;
  double *x1, *u1, *w1;
  subcycle_buffers(d.p, sub, a, &x1, &u1, &w1);
  DevParticles b = a;
  b.x = x1;
  const double dtp = 1.0 / (double)d.n_sub;
  eval_forces(d, b, i, true, true, dtp, d.p.Fnew + 6 * i, d.p.Fnew + 6 * i + 3);
  advance_velocity(d, b, i, dtp, u1 + 3 * i, w1 + 3 * i);
  if (sub == d.n_sub - 1 && !(d.n_sub & 1)) health_check(d, d.p, i);
  if (fuse) {
    DevParticles n;
    double *xn, *un, *wn;
    subcycle_buffers(d.p, sub + 1, n, &xn, &un, &wn);
    advance_position(d, n, i, dtp, xn + 3 * i);
  }
}

__global__ __launch_bounds__(DEM_GRID_THREADS) void k_demg_epilogue(DevDomain d) {
  if (dem_stopped(d)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.P) return;
  const DevParticles& p = d.p;
  for (int a = 0; a < 3; ++a) {
    p.x[3 * i + a] = p.x2[3 * i + a];
    p.u[3 * i + a] = p.u2[3 * i + a];
    p.w[3 * i + a] = p.w2[3 * i + a];
  }
  health_check(d, p, i);
}

bool dem_many(const DevDomain& d, int kernel) { return kernel == 2 || (kernel == 0 && d.P > DEM_GRID_MIN); }

hipError_t launch_dem(const DevDomain& d, int kernel, bool no_release, hipStream_t s) {
  if (d.P <= 0) return hipSuccess;
  if (!dem_many(d, kernel)) {
    // up to 64 spheres one wavefront (its barriers cost nothing; 1 sphere
    // beside an FP64 sweep: 250 against 260 us), else four
    const unsigned T1 = d.P <= 64 ? 64u : 256u;
    if (d.P <= DEM_LDS_MAX)
      hipLaunchKernelGGL(k_dem_lds, dim3(1), dim3(T1), 0, s, d);
    else
      hipLaunchKernelGGL(k_dem, dim3(1), dim3(T1), 0, s, d);
    return hipGetLastError();
  }
  const unsigned T = DEM_GRID_THREADS;
  const unsigned blocks = (unsigned)((d.P + T - 1) / T);
  hipLaunchKernelGGL(k_demg_prologue, dim3((unsigned)(((long long)d.P * 64 + T - 1) / T)), dim3(T), 0, s, d);
  hipLaunchKernelGGL(k_demg_neighbours, dim3(blocks), dim3(T), 0, s, d);
  hipLaunchKernelGGL(k_demg_position, dim3(blocks), dim3(T), 0, s, d, 0);
  for (int sub = 0; sub < d.n_sub; ++sub) {
    const int fuse = no_release && sub + 1 < d.n_sub ? 1 : 0;
    hipLaunchKernelGGL(k_demg_velocity, dim3(blocks), dim3(T), 0, s, d, sub, fuse);
    if (!fuse && sub + 1 < d.n_sub) hipLaunchKernelGGL(k_demg_position, dim3(blocks), dim3(T), 0, s, d, sub + 1);
  }
  if (d.n_sub & 1) hipLaunchKernelGGL(k_demg_epilogue, dim3(blocks), dim3(T), 0, s, d);
  return hipGetLastError();
}

}  // namespace lbmdem
