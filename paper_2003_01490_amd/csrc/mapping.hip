// Particle mapping (Sec. 2.2), PDF reconstruction (Eq. PDF_reconstruction),
// fluid boundary conditions (Eq. MEM_CLI) and momentum exchange (Eqs. MEM_Fq,
// interaction_force, interaction_torque, missing-link compensation).
//
// Work is sphere-centric: blocks (sphere i, slab b) walk the cells of the box
// around the sphere's old and new positions, so the cost scales with the
// particles, not with the lattice.  Three kernels per mapping update:
//   claim    - cells whose centre lies in the closed ball of radius R get an
//              atomic max-claim (stamp << 32 | ~id): the lowest id wins ties of
//              overlapping spheres; cells within R + delta_aB get the stamp of
//              the TRT+aB shell;
//   recon    - cells that were solid of sphere i and are now fluid get
//              Eq. (PDF_reconstruction) from neighbours that are fluid before
//              and after (old flags are still in place);
//   commit   - flags/owner are rewritten from the claims (idempotent), and for
//              each solid cell y of sphere i and each direction q whose cell
//              x = y - c_q is fluid, the boundary value f_qbar(x, t+1) of
//              Eq. (MEM_CLI) is stored in slot qbar of y, where the next sweep
//              pulls it; its momentum-exchange force (Galilean form, Eq. MEM_Fq)
//              and torque arm x_b - x_p are summed in FP64 per thread and
//              reduced per block in a fixed order (no atomics) into
//              partial[i][b].  Links from y to a wall or to another sphere's
//              solid are missing links: F_q = 2 w_q c_q with arm y - c_q/2.
//              Extra blocks write the moving-wall bounce-back values into the
//              wall-cell slots.
// The squared distances are formed as (dx*dx + dy*dy) + dz*dz in FP64 without
// contraction, so that the flags are a deterministic function of the FP64
// positions.
#include "internal.hpp"

namespace lbmdem {

enum { S_FLUID = 0, S_SHELL = 1, S_SOLID = 2, S_WALL = 3 };

struct Box {
  int lo[3];
  int ext[3];
};

__device__ inline void sphere_box(const DevDomain& d, int i, bool with_old, Box& b) {
  const double rr = d.p.R[i] + d.delta_ab;
  const int n[3] = {d.nx, d.ny, d.nz};
  bool finite = true;
  for (int a = 0; a < 3; ++a)
    finite = finite && isfinite(d.p.x[3 * i + a]) && (!with_old || isfinite(d.p.xmap[3 * i + a]));
  if (!finite) {
    for (int a = 0; a < 3; ++a) b.lo[a] = b.ext[a] = 0;
    return;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double cn = d.p.x[3 * i + a];
    int lo = (int)floor(cn - rr) - 1;
    int hi = (int)floor(cn + rr) + 1;
    if (with_old) {
      const double co = cn + min_image(d.p.xmap[3 * i + a] - cn, n[a], d.walls[a]);
      lo = min(lo, (int)floor(co - rr) - 1);
      hi = max(hi, (int)floor(co + rr) + 1);
    }
    if (d.walls[a]) {
      lo = max(lo, 0);
      hi = min(hi, n[a] - 1);
    }
    int e = hi - lo + 1;
    if (!d.walls[a] && e >= n[a]) {
      lo = 0;
      e = n[a];
    }
    b.lo[a] = lo;
    b.ext[a] = max(e, 0);
  }
}

__device__ inline double cell_d2(const DevDomain& d, int i, int j, int k, const double* xp) {
#pragma clang fp contract(off)
  const double dx = min_image(((double)i + 0.5) - xp[0], d.nx, d.walls[0]);
  const double dy = min_image(((double)j + 0.5) - xp[1], d.ny, d.walls[1]);
  const double dz = min_image(((double)k + 0.5) - xp[2], d.nz, d.walls[2]);
  return (dx * dx + dy * dy) + dz * dz;
}

// state of a cell after the current mapping update (claims of this stamp)
__device__ inline int new_state(const DevDomain& d, long long c, uint32_t stamp, int* own) {
  if (d.flags[c] & F_WALL) return S_WALL;
  const unsigned long long k = d.claim[c];
  if ((uint32_t)(k >> 32) == stamp) {
    *own = (int)(0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull));
    return S_SOLID;
  }
  return d.shellstamp[c] == stamp ? S_SHELL : S_FLUID;
}

__device__ inline bool is_fluid_state(int s) { return s == S_FLUID || s == S_SHELL; }

template <typename T>
__device__ inline double ldv(const T* p);
template <>
__device__ inline double ldv<double>(const double* p) { return *p; }
template <>
__device__ inline double ldv<float>(const float* p) { return (double)*p; }
template <>
__device__ inline double ldv<__half>(const __half* p) { return (double)__half2float(*p); }

template <typename T>
__device__ inline void stv(T* p, double v);
template <>
__device__ inline void stv<double>(double* p, double v) { *p = v; }
template <>
__device__ inline void stv<float>(float* p, double v) { *p = (float)v; }
template <>
__device__ inline void stv<__half>(__half* p, double v) { *p = __float2half_rn((float)v); }

// iterate the cells of a box: slabs of sphere-block b, threads over x-y
#define FOR_BOX_CELLS(d, bx, b, ZB, ...)                                             \
  for (int sl = (b); sl < (bx).ext[2]; sl += (ZB)) {                                 \
    const int kk = (d).walls[2] ? (bx).lo[2] + sl : wrapmod((bx).lo[2] + sl, (d).nz); \
    const int nxy_ = (bx).ext[0] * (bx).ext[1];                                      \
    for (int t = threadIdx.x; t < nxy_; t += blockDim.x) {                           \
      const int tx = t % (bx).ext[0], ty = t / (bx).ext[0];                          \
      const int ii = (d).walls[0] ? (bx).lo[0] + tx : wrapmod((bx).lo[0] + tx, (d).nx); \
      const int jj = (d).walls[1] ? (bx).lo[1] + ty : wrapmod((bx).lo[1] + ty, (d).ny); \
      __VA_ARGS__                                                                    \
    }                                                                                \
  }

__global__ __launch_bounds__(256) void k_claim(DevDomain d, uint32_t stamp) {
  const int i = blockIdx.x / d.ZB, b = blockIdx.x % d.ZB;
  if (i >= d.P) return;
  Box bx;
  sphere_box(d, i, false, bx);
  const double xp[3] = {d.p.x[3 * i], d.p.x[3 * i + 1], d.p.x[3 * i + 2]};
  double R2, rs2;
  {
#pragma clang fp contract(off)
    const double R = d.p.R[i];
    const double rs = R + d.delta_ab;
    R2 = R * R;
    rs2 = rs * rs;
  }
  const unsigned long long key =
      ((unsigned long long)stamp << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)i);
  FOR_BOX_CELLS(d, bx, b, d.ZB, {
    const long long c = cidx(d, ii, jj, kk);
    if (!(d.flags[c] & F_WALL)) {
      const double d2 = cell_d2(d, ii, jj, kk, xp);
      if (d2 <= R2) atomicMax(&d.claim[c], key);
      if (d2 <= rs2) d.shellstamp[c] = stamp;
    }
  })
}

// Eq. (PDF_reconstruction) for cell (ii,jj,kk) formerly covered by sphere i
template <typename T>
__device__ void reconstruct(const DevDomain& d, T* buf, uint32_t stamp, int ii, int jj, int kk,
                            int i) {
  const size_t N = (size_t)d.N;
  const long long c = cidx(d, ii, jj, kk);
  double rsum = 0.0;
  int nvalid = 0;
  for (int q = 1; q < Q; ++q) {
    const long long y = cidx(d, wrapi(ii + CX[q], d.nx), wrapi(jj + CY[q], d.ny), wrapi(kk + CZ[q], d.nz));
    int o;
    if ((d.flags[y] & (F_SOLID | F_WALL)) || !is_fluid_state(new_state(d, y, stamp, &o))) continue;
    double r = 0.0;
    for (int p = 0; p < Q; ++p) r += ldv<T>(buf + (size_t)p * N + y) + WQ[p];
    rsum += r;
    nvalid += 1;
  }
  const double rb = nvalid > 0 ? rsum / (double)nvalid : 1.0;
  double rel[3], ut[3];
  rel[0] = min_image(((double)ii + 0.5) - d.p.x[3 * i], d.nx, d.walls[0]);
  rel[1] = min_image(((double)jj + 0.5) - d.p.x[3 * i + 1], d.ny, d.walls[1]);
  rel[2] = min_image(((double)kk + 0.5) - d.p.x[3 * i + 2], d.nz, d.walls[2]);
  {
    const double* wv = d.p.w + 3 * i;
    const double* uv = d.p.u + 3 * i;
    ut[0] = uv[0] + (wv[1] * rel[2] - wv[2] * rel[1]);
    ut[1] = uv[1] + (wv[2] * rel[0] - wv[0] * rel[2]);
    ut[2] = uv[2] + (wv[0] * rel[1] - wv[1] * rel[0]);
  }
  double du[3][3];  // du[a][b] = d u_a / d x_b
  const int axp[3] = {4, 1, 5}, axm[3] = {3, 2, 6};
  for (int bb = 0; bb < 3; ++bb) {
    const int qp = axp[bb], qm = axm[bb];
    const long long yp = cidx(d, wrapi(ii + CX[qp], d.nx), wrapi(jj + CY[qp], d.ny), wrapi(kk + CZ[qp], d.nz));
    const long long ym = cidx(d, wrapi(ii + CX[qm], d.nx), wrapi(jj + CY[qm], d.ny), wrapi(kk + CZ[qm], d.nz));
    int o;
    const bool vp = !(d.flags[yp] & (F_SOLID | F_WALL)) && is_fluid_state(new_state(d, yp, stamp, &o));
    const bool vm = !(d.flags[ym] & (F_SOLID | F_WALL)) && is_fluid_state(new_state(d, ym, stamp, &o));
    double up[3] = {0, 0, 0}, um[3] = {0, 0, 0};
    for (int p = 0; p < Q; ++p) {
      const double fp = ldv<T>(buf + (size_t)p * N + yp) + WQ[p];
      const double fm = ldv<T>(buf + (size_t)p * N + ym) + WQ[p];
      up[0] += fp * CX[p];
      up[1] += fp * CY[p];
      up[2] += fp * CZ[p];
      um[0] += fm * CX[p];
      um[1] += fm * CY[p];
      um[2] += fm * CZ[p];
    }
    for (int a = 0; a < 3; ++a) {
      if (vp && vm)
        du[a][bb] = 0.5 * (up[a] - um[a]);
      else if (vp)
        du[a][bb] = up[a] - ut[a];
      else if (vm)
        du[a][bb] = ut[a] - um[a];
      else
        du[a][bb] = 0.0;
    }
  }
  const double inv3s = rb / (3.0 * d.s_nu);
  for (int q = 0; q < Q; ++q) {
    const int cq[3] = {CX[q], CY[q], CZ[q]};
    const double cu = cq[0] * ut[0] + cq[1] * ut[1] + cq[2] * ut[2];
    double second = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int bb = 0; bb < 3; ++bb) {
        const double Pab = rb * ut[a] * ut[bb] - inv3s * (du[a][bb] + du[bb][a]);
        const double Hab = (double)(cq[a] * cq[bb]) - (a == bb ? 1.0 / 3.0 : 0.0);
        second += Pab * Hab;
      }
    const double f = WQ[q] * (rb + 3.0 * rb * cu + 4.5 * second);
    stv<T>(buf + (size_t)q * N + c, f - WQ[q]);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_recon(DevDomain d, int cur, uint32_t stamp) {
  const int i = blockIdx.x / d.ZB, b = blockIdx.x % d.ZB;
  if (i >= d.P) return;
  Box bx;
  sphere_box(d, i, true, bx);
  T* buf = (T*)d.pdf[cur];
  FOR_BOX_CELLS(d, bx, b, d.ZB, {
    const long long c = cidx(d, ii, jj, kk);
    if ((d.flags[c] & F_SOLID) && d.owner[c] == i) {
      int o;
      if (new_state(d, c, stamp, &o) != S_SOLID) reconstruct<T>(d, buf, stamp, ii, jj, kk, i);
    }
  })
}

// smallest root in [0,1] of |r + delta c|^2 = R^2 (x_b = x + delta_q c_q)
__device__ inline double link_delta(const double* r, const int* c, double R) {
  const double cc = (double)(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  const double b = r[0] * c[0] + r[1] * c[1] + r[2] * c[2];
  const double e = (r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) - R * R;
  double disc = b * b - cc * e;
  if (disc < 0.0) disc = 0.0;
  double dl = (-b - sqrt(disc)) / cc;
  return dl < 0.0 ? 0.0 : (dl > 1.0 ? 1.0 : dl);
}

template <typename T>
__global__ __launch_bounds__(256) void k_commit(DevDomain d, int cur, uint32_t stamp, int nwall) {
  const int nsb = d.P * d.ZB;
  T* buf = (T*)d.pdf[cur];
  const size_t N = (size_t)d.N;
  if ((int)blockIdx.x >= nsb) {
    // moving-wall bounce-back into wall-cell slots: slot (y, q) receives
    // f~_qbar(x) + 6 w_q (u_w . c_q) for the fluid cell x = y + c_q
    const int t = (blockIdx.x - nsb) * blockDim.x + threadIdx.x;
    if (t >= nwall) return;
    int rem = t, ii = 0, jj = 0, kk = 0;
    const int wz = d.walls[2], wy = d.walls[1];
    const int nyi = d.ny - 2 * wy, nzi = d.nz - 2 * wz;
    if (wz && rem < 2 * d.nx * d.ny) {
      kk = rem < d.nx * d.ny ? 0 : d.nz - 1;
      rem %= d.nx * d.ny;
      ii = rem % d.nx;
      jj = rem / d.nx;
    } else {
      if (wz) rem -= 2 * d.nx * d.ny;
      if (wy && rem < 2 * d.nx * nzi) {
        jj = rem < d.nx * nzi ? 0 : d.ny - 1;
        rem %= d.nx * nzi;
        ii = rem % d.nx;
        kk = rem / d.nx + wz;
      } else {
        if (wy) rem -= 2 * d.nx * nzi;
        ii = rem < nyi * nzi ? 0 : d.nx - 1;
        rem %= nyi * nzi;
        jj = rem % nyi + wy;
        kk = rem / nyi + wz;
      }
    }
    double uw[3] = {0, 0, 0};
    if (wz && kk == 0) {
      uw[0] = d.wall_u_lo[0];
      uw[1] = d.wall_u_lo[1];
      uw[2] = d.wall_u_lo[2];
    } else if (wz && kk == d.nz - 1) {
      uw[0] = d.wall_u_hi[0];
      uw[1] = d.wall_u_hi[1];
      uw[2] = d.wall_u_hi[2];
    }
    const long long y = cidx(d, ii, jj, kk);
    for (int q = 1; q < Q; ++q) {
      int xi = ii + CX[q], xj = jj + CY[q], xk = kk + CZ[q];
      if (d.walls[0] ? (xi < 0 || xi >= d.nx) : false) continue;
      if (d.walls[1] ? (xj < 0 || xj >= d.ny) : false) continue;
      if (d.walls[2] ? (xk < 0 || xk >= d.nz) : false) continue;
      xi = wrapi(xi, d.nx);
      xj = wrapi(xj, d.ny);
      xk = wrapi(xk, d.nz);
      const long long x = cidx(d, xi, xj, xk);
      int o;
      if (!is_fluid_state(new_state(d, x, stamp, &o))) continue;
      const double v = ldv<T>(buf + (size_t)OPP[q] * N + x) +
                       6.0 * WQ[q] * (uw[0] * CX[q] + uw[1] * CY[q] + uw[2] * CZ[q]);
      stv<T>(buf + (size_t)q * N + y, v);
    }
    return;
  }
  const int i = blockIdx.x / d.ZB, b = blockIdx.x % d.ZB;
  Box bx;
  sphere_box(d, i, true, bx);
  const double xp[3] = {d.p.x[3 * i], d.p.x[3 * i + 1], d.p.x[3 * i + 2]};
  const double up[3] = {d.p.u[3 * i], d.p.u[3 * i + 1], d.p.u[3 * i + 2]};
  const double wp[3] = {d.p.w[3 * i], d.p.w[3 * i + 1], d.p.w[3 * i + 2]};
  const double R = d.p.R[i];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  FOR_BOX_CELLS(d, bx, b, d.ZB, {
    const long long yc = cidx(d, ii, jj, kk);
    int own = -1;
    const int ns = new_state(d, yc, stamp, &own);
    if (ns != S_WALL) {
      d.flags[yc] = ns == S_SOLID ? F_SOLID : (ns == S_SHELL ? F_SHELL : (uint8_t)0);
      if (ns == S_SOLID) d.owner[yc] = own;
      if (ns == S_SOLID && own == i) {
        for (int q = 1; q < Q; ++q) {
          const int cq[3] = {CX[q], CY[q], CZ[q]};
          // wall layers shield every non-wall cell, so y - c_q stays in range
          const int xi = wrapi(ii - cq[0], d.nx), xj = wrapi(jj - cq[1], d.ny),
                    xk = wrapi(kk - cq[2], d.nz);
          const long long x = cidx(d, xi, xj, xk);
          int zo = -1;
          const int zs = new_state(d, x, stamp, &zo);
          double Fq[3], arm[3];
          if (is_fluid_state(zs)) {
            double r[3];
            r[0] = min_image(((double)xi + 0.5) - xp[0], d.nx, d.walls[0]);
            r[1] = min_image(((double)xj + 0.5) - xp[1], d.ny, d.walls[1]);
            r[2] = min_image(((double)xk + 0.5) - xp[2], d.nz, d.walls[2]);
            const double dl = link_delta(r, cq, R);
            for (int a = 0; a < 3; ++a) arm[a] = r[a] + dl * cq[a];
            double ub[3];
            ub[0] = up[0] + (wp[1] * arm[2] - wp[2] * arm[1]);
            ub[1] = up[1] + (wp[2] * arm[0] - wp[0] * arm[2]);
            ub[2] = up[2] + (wp[0] * arm[1] - wp[1] * arm[0]);
            const int qb = OPP[q];
            const double gq = ldv<T>(buf + (size_t)q * N + x);
            const double gqb = ldv<T>(buf + (size_t)qb * N + x);
            bool cli = false;
            long long xm = 0;
            if (d.boundary == 0) {
              const int mi = wrapi(xi - cq[0], d.nx), mj = wrapi(xj - cq[1], d.ny),
                        mk = wrapi(xk - cq[2], d.nz);
              xm = cidx(d, mi, mj, mk);
              int mo;
              cli = is_fluid_state(new_state(d, xm, stamp, &mo));
            }
            const double dd = cli ? dl : 0.5;
            double val = gq;
            if (cli) val += (1.0 - 2.0 * dd) / (1.0 + 2.0 * dd) * (ldv<T>(buf + (size_t)q * N + xm) - gqb);
            val -= 4.0 / (1.0 + 2.0 * dd) * WQ[q] * 3.0 * (ub[0] * cq[0] + ub[1] * cq[1] + ub[2] * cq[2]);
            stv<T>(buf + (size_t)qb * N + yc, val);
            const double fq = gq + WQ[q], fb = val + WQ[q];
            for (int a = 0; a < 3; ++a) Fq[a] = (cq[a] - ub[a]) * fq - (-cq[a] - ub[a]) * fb;
          } else if (zs == S_WALL || (zs == S_SOLID && zo != i)) {
            for (int a = 0; a < 3; ++a) Fq[a] = 2.0 * WQ[q] * cq[a];
            arm[0] = min_image(((double)ii + 0.5) - xp[0], d.nx, d.walls[0]) - 0.5 * cq[0];
            arm[1] = min_image(((double)jj + 0.5) - xp[1], d.ny, d.walls[1]) - 0.5 * cq[1];
            arm[2] = min_image(((double)kk + 0.5) - xp[2], d.nz, d.walls[2]) - 0.5 * cq[2];
          } else {
            continue;
          }
          acc[0] += Fq[0];
          acc[1] += Fq[1];
          acc[2] += Fq[2];
          acc[3] += arm[1] * Fq[2] - arm[2] * Fq[1];
          acc[4] += arm[2] * Fq[0] - arm[0] * Fq[2];
          acc[5] += arm[0] * Fq[1] - arm[1] * Fq[0];
        }
      }
    }
  })
  // fixed-order block reduction: wavefront shuffles, then across wavefronts
  __shared__ double red[6][8];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < 6; ++k) {
    double v = acc[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[k][wid] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double v = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int w8 = 0; w8 < nw; ++w8) v += red[threadIdx.x][w8];
    d.partial[((size_t)i * d.ZB + b) * 6 + threadIdx.x] = v;
  }
}

static int wall_cell_count(const DevDomain& d) {
  int n = 0;
  const int nzi = d.nz - 2 * d.walls[2], nyi = d.ny - 2 * d.walls[1];
  if (d.walls[2]) n += 2 * d.nx * d.ny;
  if (d.walls[1]) n += 2 * d.nx * nzi;
  if (d.walls[0]) n += 2 * nyi * nzi;
  return n;
}

template <typename T>
static void launch_mapping_t(const DevDomain& d, int cur, uint32_t stamp, bool reconstruct,
                             hipStream_t s) {
  const int nsb = d.P * d.ZB;
  if (nsb > 0) {
    hipLaunchKernelGGL(k_claim, dim3(nsb), dim3(256), 0, s, d, stamp);
    if (reconstruct) hipLaunchKernelGGL(k_recon<T>, dim3(nsb), dim3(256), 0, s, d, cur, stamp);
  }
  const int nwall = wall_cell_count(d);
  const int wblocks = (nwall + 255) / 256;
  if (nsb + wblocks > 0)
    hipLaunchKernelGGL(k_commit<T>, dim3(nsb + wblocks), dim3(256), 0, s, d, cur, stamp, nwall);
}

void launch_mapping(const DevDomain& d, int cur, uint32_t stamp, bool reconstruct, hipStream_t s) {
  if (d.storage == 0)
    launch_mapping_t<double>(d, cur, stamp, reconstruct, s);
  else if (d.storage == 1)
    launch_mapping_t<float>(d, cur, stamp, reconstruct, s);
  else
    launch_mapping_t<__half>(d, cur, stamp, reconstruct, s);
}

}  // namespace lbmdem
