// Particle mapping (Sec. 2.2), PDF reconstruction (Eq. PDF_reconstruction),
// fluid boundary conditions (Eq. MEM_CLI) and momentum exchange (Eqs. MEM_Fq,
// interaction_force, interaction_torque, missing-link compensation).
//
// Work is sphere-centric: blocks walk the cells of the box around a sphere's
// old and new positions, so the cost scales with the particles, not with the
// lattice.  Two forms of the mapping update:
// - slab pass (few spheres; blocks (sphere i, slab b)):
//   claim    - cells whose centre lies in the closed ball of radius R get an
//              atomic max-claim (stamp << 32 | ~id): the lowest id wins ties of
//              overlapping spheres; cells within R + delta_aB get the stamp of
//              the TRT+aB shell;
//   recon    - cells that were solid of sphere i and are now fluid get
//              Eq. (PDF_reconstruction) from neighbours that are fluid before
//              and after (old flags are still in place);
//   commit   - flags/owner are rewritten from the claims (idempotent) and the
//              links are formed (below);
// - ball pass (many spheres; one block per sphere) and fused step: the
//   spheres are filed in mapping bins, and each cell whose membership in a
//   sphere's ball or shell changed gets the state of the new positions from
//   the spheres of its 27 bins (k_recon_geo reconstructs, k_remap_geo
//   rewrites flags, owners and cell words); only the cells near the ends of
//   the balls' row chords are tested.  The ball pass then forms the links
//   from the cell words.
// Links: for each solid cell y of sphere i and each direction q whose cell
// x = y - c_q is fluid, the boundary value f_qbar(x, t+1) of Eq. (MEM_CLI) is
// stored in slot qbar of y, where the next sweep pulls it; its
// momentum-exchange force (Galilean form, Eq. MEM_Fq) and torque arm
// x_b - x_p are summed in FP64 per thread and reduced per block in a fixed
// order (no atomics) into partial[i][b].  Links from y to a wall or to another
// sphere's solid are missing links: F_q = 2 w_q c_q with arm y - c_q/2.
// Inside a step these kernels run after the sweep and the DEM (the claims or
// bins beside the sweep), before the step control advances the domain: they
// use the next mapping stamp and work on the buffer the sweep has just
// written (the next current one).  A mapping update outside the step (new or
// moved spheres) works on the current buffer, then takes the new stamp.
// (Moving-wall bounce-back is done by the sweep itself.)
// The squared distances are formed as (dx*dx + dy*dy) + dz*dz in FP64 without
// contraction, so that the flags are a deterministic function of the FP64
// positions.
#include "internal.hpp"

namespace lbmdem {

enum { S_FLUID = 0, S_SHELL = 1, S_SOLID = 2, S_WALL = 3 };
// staged neighbour codes relative to the sphere a block works for
enum { L_FLUID = 0, L_SHELL = 1, L_OWN = 2, L_OTHER = 3, L_WALL = 4 };
constexpr int STAGE_BYTES = 32768;

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
#pragma unroll
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

// cells whose centre can lie within R of the mapped centre of sphere i
// (the cells a mapping update can uncover)
__device__ inline void mapped_ball_box(const DevDomain& d, int i, Box& b) {
  const double R = d.p.R[i];
  const int n[3] = {d.nx, d.ny, d.nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double co = d.p.xmap[3 * i + a];
    if (!isfinite(co)) {
      for (int e = 0; e < 3; ++e) b.lo[e] = b.ext[e] = 0;
      return;
    }
    int lo = (int)floor(co - R) - 1;
    int hi = (int)floor(co + R) + 1;
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

// state of a cell after the current mapping update (claims of this stamp);
// the three loads are independent so that they are in flight together
__device__ inline int new_state(const DevDomain& d, long long c, uint32_t stamp, int* own) {
  const uint8_t fl = d.flags[c];
  const unsigned long long k = d.claim[c];
  const uint32_t ss = d.shellstamp[c];
  if (fl & F_WALL) return S_WALL;
  if ((uint32_t)(k >> 32) == stamp) {
    *own = (int)(0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull));
    return S_SOLID;
  }
  return ss == stamp ? S_SHELL : S_FLUID;
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
    const int kk = (d).walls[2] ? (bx).lo[2] + sl : wrap_near((bx).lo[2] + sl, (d).nz); \
    const int nxy_ = (bx).ext[0] * (bx).ext[1];                                      \
    for (int t = threadIdx.x; t < nxy_; t += blockDim.x) {                           \
      const int tx = t % (bx).ext[0], ty = t / (bx).ext[0];                          \
      const int ii = (d).walls[0] ? (bx).lo[0] + tx : wrap_near((bx).lo[0] + tx, (d).nx); \
      const int jj = (d).walls[1] ? (bx).lo[1] + ty : wrap_near((bx).lo[1] + ty, (d).ny); \
      __VA_ARGS__                                                                    \
    }                                                                                \
  }

// Claims of sphere i's solid cells with a stamped key; the largest key (this
// stamp, lowest id) wins a cell inside several spheres.  With `lists` (the
// neighbour lists of this step are valid: the many-sphere DEM built them from
// the positions at the start of the step with a skin, so they hold every
// sphere that can touch i now), a sphere whose ball meets no other claims its
// cells with plain stores: no other sphere claims them, and every older key
// is smaller.
__device__ __forceinline__ bool claims_exclusive(const DevDomain& d, int i) {
  const int nn = d.p.nbr_n[i];
  if (nn >= NBR_MAX) return false;  // a list that overflowed may miss a neighbour
  const int n[3] = {d.nx, d.ny, d.nz};
  for (int k = 0; k < nn; ++k) {
    const int j = d.p.nbr[(size_t)i * NBR_MAX + k];
    double s2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double v = min_image(d.p.x[3 * i + a] - d.p.x[3 * j + a], n[a], d.walls[a]);
      s2 += v * v;
    }
    // balls that are 1e-6 apart share no cell centre, whatever the rounding
    if (!(sqrt(s2) - (d.p.R[i] + d.p.R[j]) >= 1e-6)) return false;
  }
  return true;
}

constexpr int CLAIM_ROWS = 1024;  // row chords a claim block keeps in LDS

__device__ __forceinline__ void claim_block(const DevDomain& d, int blk, uint32_t stamp, bool lists) {
  const int i = blk / d.ZB, b = blk % d.ZB;
  if (i >= d.P) return;
  const bool excl = lists && claims_exclusive(d, i);
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
  // x-chords of the box's rows: the cells whose centres can lie within
  // R + delta_aB of the centre have x index in [s, e] (packed s | e << 16;
  // s > e: none), from the row's exact y and z offsets widened by 1e-3, far
  // more than rounding moves a chord's end; the exact tests run on those
  // cells only.  A box that nearly spans a periodic x axis keeps every cell.
  __shared__ uint32_t chord[CLAIM_ROWS];
  const int n[3] = {d.nx, d.ny, d.nz};
  const bool chorded = bx.ext[1] * bx.ext[2] <= CLAIM_ROWS && (d.walls[0] || bx.ext[0] + 2 <= n[0]);
  if (chorded) {
    constexpr double EPS = 1e-3;
    for (int r = threadIdx.x; r < bx.ext[1] * bx.ext[2]; r += blockDim.x) {
      const int gy = bx.lo[1] + r % bx.ext[1], gz = bx.lo[2] + r / bx.ext[1];
      const int jj = d.walls[1] ? gy : wrap_near(gy, n[1]), kk = d.walls[2] ? gz : wrap_near(gz, n[2]);
      const double dy = min_image(((double)jj + 0.5) - xp[1], n[1], d.walls[1]);
      const double dz = min_image(((double)kk + 0.5) - xp[2], n[2], d.walls[2]);
      const double rho = rs2 - (dy * dy + dz * dz);
      const double a = sqrt(fmax(rho, 0.0)) + EPS;
      int s0 = max(0, (int)ceil(xp[0] - a - 0.5) - bx.lo[0]);
      int e0 = min(bx.ext[0] - 1, (int)floor(xp[0] + a - 0.5) - bx.lo[0]);
      if (rho < -EPS || e0 < s0) s0 = 1, e0 = 0;
      chord[r] = (uint32_t)s0 | ((uint32_t)e0 << 16);
    }
    __syncthreads();
  }
  // wall layers (the first and last layer of a walled axis) are never
  // claimed; they are known from the coordinates, so no flag is read
  const int nxy = bx.ext[0] * bx.ext[1];
  for (int sl = b; sl < bx.ext[2]; sl += d.ZB) {
    const int kk = d.walls[2] ? bx.lo[2] + sl : wrap_near(bx.lo[2] + sl, d.nz);
    for (int t = threadIdx.x; t < nxy; t += blockDim.x) {
      const int tx = t % bx.ext[0], ty = t / bx.ext[0];
      if (chorded) {
        const uint32_t ch = chord[ty + bx.ext[1] * sl];
        if (tx < (int)(ch & 0xFFFFu) || tx > (int)(ch >> 16)) continue;
      }
      const int ii = d.walls[0] ? bx.lo[0] + tx : wrap_near(bx.lo[0] + tx, d.nx);
      const int jj = d.walls[1] ? bx.lo[1] + ty : wrap_near(bx.lo[1] + ty, d.ny);
      const long long c = cidx(d, ii, jj, kk);
      const bool wall = (d.walls[0] && (ii == 0 || ii == d.nx - 1)) || (d.walls[1] && (jj == 0 || jj == d.ny - 1)) ||
                        (d.walls[2] && (kk == 0 || kk == d.nz - 1));
      if (!wall) {
        const double d2 = cell_d2(d, ii, jj, kk, xp);
        if (d2 <= R2) {
          if (excl)
            d.claim[c] = key;
          else
            atomicMax(&d.claim[c], key);
        }
        if (d2 <= rs2) d.shellstamp[c] = stamp;
      }
    }
  }
}

// Whether a mapping kernel runs, which buffer it works on and its stamp:
// inside a step (in_step = 1) the domain must be live and the buffer is the
// one the sweep wrote; outside, only a frozen domain is skipped.  The claims
// always carry the next stamp.
__device__ __forceinline__ bool map_live(const DevCtl* c, int in_step) {
  return in_step ? step_live(c) : !c->frozen;
}
__device__ __forceinline__ int map_buffer(const DevCtl* c, int in_step) { return c->cur ^ (in_step ? 1 : 0); }
__device__ __forceinline__ uint32_t map_stamp(const DevCtl* c) { return c->stamp + 1u; }

__global__ __launch_bounds__(256) void k_claim(DevDomain d, int in_step, int lists) {
  __builtin_amdgcn_s_setprio(3);  // runs beside the sweep in an overlapped step
  if (!map_live(d.ctl, in_step)) return;
  claim_block(d, blockIdx.x, map_stamp(d.ctl), lists != 0);
}

// the new stamp after a mapping update outside the step
__global__ void k_new_stamp(DevCtl* ctl) { ctl->stamp += 1; }

// Eq. (PDF_reconstruction) for cell (ii,jj,kk) formerly covered by sphere i
// (one thread; `usable(y, i, j, k)` says whether neighbour y at (i, j, k) is
// fluid before and after the mapping update)
template <typename T, typename V>
__device__ void reconstruct_with(const DevDomain& d, T* buf, int ii, int jj, int kk, int i, V usable) {
  const size_t N = (size_t)d.N;
  const long long c = cidx(d, ii, jj, kk);
  double rsum = 0.0;
  int nvalid = 0;
  for (int q = 1; q < Q; ++q) {
    const int yi = wrapi(ii + CX[q], d.nx), yj = wrapi(jj + CY[q], d.ny), yk = wrapi(kk + CZ[q], d.nz);
    const long long y = cidx(d, yi, yj, yk);
    if (!usable(y, yi, yj, yk)) continue;
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
    const int pi = wrapi(ii + CX[qp], d.nx), pj = wrapi(jj + CY[qp], d.ny), pk = wrapi(kk + CZ[qp], d.nz);
    const int mi = wrapi(ii + CX[qm], d.nx), mj = wrapi(jj + CY[qm], d.ny), mk = wrapi(kk + CZ[qm], d.nz);
    const long long yp = cidx(d, pi, pj, pk);
    const long long ym = cidx(d, mi, mj, mk);
    const bool vp = usable(yp, pi, pj, pk);
    const bool vm = usable(ym, mi, mj, mk);
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
__device__ void reconstruct(const DevDomain& d, T* buf, uint32_t stamp, int ii, int jj, int kk, int i) {
  reconstruct_with<T>(d, buf, ii, jj, kk, i, [&](long long y, int, int, int) {
    int o;
    return !(d.flags[y] & (F_SOLID | F_WALL)) && is_fluid_state(new_state(d, y, stamp, &o));
  });
}

// Eq. (PDF_reconstruction) for cell c formerly covered by sphere i, computed
// by one wavefront: lane q (1..18) checks neighbour x + c_q and forms its
// density and velocity from 19 independent loads; the lanes' values are then
// combined in q order (the same order as a serial loop) and lane q writes f_q.
// The same for any rule `usable(y, i, j, k)` that says whether neighbour y
// (at (i, j, k)) is fluid before and after the mapping update.
template <typename T, typename V>
__device__ void reconstruct_wave_with(const DevDomain& d, T* buf, long long c, int i, int lane, V usable) {
  const size_t N = (size_t)d.N;
  const int ii = (int)(c % d.nx), jj = (int)((c / d.nx) % d.ny), kk = (int)(c / ((long long)d.nx * d.ny));
  bool valid = false;
  double rn = 0.0, un[3] = {0.0, 0.0, 0.0};
  if (lane >= 1 && lane < Q) {
    const int yi = wrapi(ii + CX[lane], d.nx), yj = wrapi(jj + CY[lane], d.ny), yk = wrapi(kk + CZ[lane], d.nz);
    const long long y = cidx(d, yi, yj, yk);
    valid = usable(y, yi, yj, yk);
    if (valid) {
      double f[Q];
#pragma unroll
      for (int p = 0; p < Q; ++p) f[p] = ldv<T>(buf + (size_t)p * N + y) + WQ[p];
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        rn += f[p];
        un[0] += f[p] * CX[p];
        un[1] += f[p] * CY[p];
        un[2] += f[p] * CZ[p];
      }
    }
  }
  double rsum = 0.0;
  int nvalid = 0;
  for (int q = 1; q < Q; ++q) {
    const int v = __shfl((int)valid, q, 64);
    const double r = __shfl(rn, q, 64);
    if (v) {
      rsum += r;
      nvalid += 1;
    }
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
#pragma unroll
  for (int bb = 0; bb < 3; ++bb) {
    const bool vp = __shfl((int)valid, axp[bb], 64) != 0;
    const bool vm = __shfl((int)valid, axm[bb], 64) != 0;
    double up[3], um[3];
    for (int a = 0; a < 3; ++a) {
      up[a] = __shfl(un[a], axp[bb], 64);
      um[a] = __shfl(un[a], axm[bb], 64);
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
  if (lane < Q) {
    const int q = lane;
    const int cq[3] = {CX[q], CY[q], CZ[q]};
    const double inv3s = rb / (3.0 * d.s_nu);
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
__device__ void reconstruct_wave(const DevDomain& d, T* buf, uint32_t stamp, long long c, int i, int lane) {
  reconstruct_wave_with<T>(d, buf, c, i, lane, [&](long long y, int, int, int) {
    int o;
    return !(d.flags[y] & (F_SOLID | F_WALL)) && is_fluid_state(new_state(d, y, stamp, &o));
  });
}

// Cells of a box whose membership in a ball of squared radius r2[m] (m <
// NR, increasing) can differ between an old and a new centre, row by row
// (one thread per x-row): from each row's exact y and z offsets, the x-chord
// of each ball widened by 1e-3 and its sure inside narrowed by 1e-3 (rounding
// moves a chord's end by far less); per radius the cells of the union of the
// two chords outside the common sure inside are visited, where visit(ii, jj,
// kk) applies the exact test (a cell near the chords of two radii is visited
// twice).  The box (ext rows of slab sl = b, b + ZB, ...) is in coordinates
// unwrapped around its centre, in which the old and new centres have x =
// cx[0] and cx[1]; a box that nearly spans a periodic x axis has each of its
// cells visited once.
template <int NR, typename F>
__device__ __forceinline__ void chord_changes(const DevDomain& d, const Box& bx, int b, int ZB, const double* xo,
                                              const double* xn, const double* cx, const double* r2, F visit) {
  constexpr double EPS = 1e-3;
  const int nsl = b < bx.ext[2] ? (bx.ext[2] - 1 - b) / ZB + 1 : 0;
  const int nrows = bx.ext[1] * nsl;
  const bool whole_x = !d.walls[0] && bx.ext[0] + 2 > d.nx;
  for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
    const int ty = r % bx.ext[1], sl = b + ZB * (r / bx.ext[1]);
    const int jj = d.walls[1] ? bx.lo[1] + ty : wrap_near(bx.lo[1] + ty, d.ny);
    const int kk = d.walls[2] ? bx.lo[2] + sl : wrap_near(bx.lo[2] + sl, d.nz);
    // up to two segments [sa, ea] of box x indices per radius
    int sa[2 * NR], ea[2 * NR];
#pragma unroll
    for (int k = 0; k < 2 * NR; ++k) sa[k] = 1, ea[k] = 0;
    if (whole_x) {
      sa[0] = 0;
      ea[0] = bx.ext[0] - 1;
    } else {
      double yz[2];  // squared y-z offsets of the row from the two centres
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const double* c = k ? xn : xo;
        const double dy = min_image(((double)jj + 0.5) - c[1], d.ny, d.walls[1]);
        const double dz = min_image(((double)kk + 0.5) - c[2], d.nz, d.walls[2]);
        yz[k] = dy * dy + dz * dz;
      }
#pragma unroll
      for (int m = 0; m < NR; ++m) {
        int us = bx.ext[0], ue = -1, is = 0, ie = bx.ext[0] - 1;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const double rho = r2[m] - yz[k];
          if (rho >= -EPS) {
            const double a = sqrt(fmax(rho, 0.0)) + EPS;
            us = min(us, (int)ceil(cx[k] - a - 0.5) - bx.lo[0]);
            ue = max(ue, (int)floor(cx[k] + a - 0.5) - bx.lo[0]);
          }
          // sure inside: |g + 0.5 - cx| < a_in, i.e. g in
          // [floor(cx - a_in - 0.5) + 1, ceil(cx + a_in - 0.5) - 1]
          const double ain = rho > 0.0 ? sqrt(rho) - EPS : -1.0;
          if (ain > 0.0) {
            is = max(is, (int)floor(cx[k] - ain - 0.5) + 1 - bx.lo[0]);
            ie = min(ie, (int)ceil(cx[k] + ain - 0.5) - 1 - bx.lo[0]);
          } else {
            is = 1, ie = 0;
          }
        }
        const int s0 = max(us, 0), e0 = min(ue, bx.ext[0] - 1);
        sa[2 * m] = s0;
        ea[2 * m] = is <= ie ? min(e0, is - 1) : e0;  // both balls surely hold [is, ie]
        sa[2 * m + 1] = is <= ie ? max(s0, ie + 1) : 1;
        ea[2 * m + 1] = is <= ie ? e0 : 0;
      }
    }
    // one loop over the cells of all segments, so that visit is inlined once
    int tot = 0;
#pragma unroll
    for (int k = 0; k < 2 * NR; ++k) tot += max(ea[k] - sa[k] + 1, 0);
    for (int q = 0; q < tot; ++q) {
      int g = 0, rem = q;
#pragma unroll
      for (int k = 0; k < 2 * NR; ++k) {
        const int len = max(ea[k] - sa[k] + 1, 0);
        if (rem >= 0 && rem < len) g = sa[k] + rem;
        rem -= len;
      }
      visit(d.walls[0] ? bx.lo[0] + g : wrap_near(bx.lo[0] + g, d.nx), jj, kk);
    }
  }
}

constexpr int RECON_LIST = 1024;

template <typename T>
__device__ __forceinline__ void recon_block(const DevDomain& d, int blk, int cur, uint32_t stamp) {
  const int i = blk / d.ZB, b = blk % d.ZB;
  if (i >= d.P) return;
  __shared__ long long cand[RECON_LIST];
  __shared__ int ncand;
  if (threadIdx.x == 0) ncand = 0;
  __syncthreads();
  Box bx;
  mapped_ball_box(d, i, bx);
  T* buf = (T*)d.pdf[cur];
  const double xo[3] = {d.p.xmap[3 * i], d.p.xmap[3 * i + 1], d.p.xmap[3 * i + 2]};
  const double xn[3] = {d.p.x[3 * i], d.p.x[3 * i + 1], d.p.x[3 * i + 2]};
  double R2;
  {
#pragma clang fp contract(off)
    const double R = d.p.R[i];
    R2 = R * R;
  }
  // A cell leaves sphere i only if its centre was inside the old ball and is
  // outside the new one: the same FP64 test both mappings made, applied to
  // the cells near the ends of the balls' row chords, so only this thin shell
  // of cells touches memory.  Cells to rebuild are listed in LDS and then
  // rebuilt one wavefront each.
  auto visit = [&](int ii, int jj, int kk) {
    if (cell_d2(d, ii, jj, kk, xo) <= R2 && !(cell_d2(d, ii, jj, kk, xn) <= R2)) {
      const long long c = cidx(d, ii, jj, kk);
      if ((d.flags[c] & F_SOLID) && d.owner[c] == i) {
        int o;
        if (new_state(d, c, stamp, &o) != S_SOLID) {
          const int k = atomicAdd(&ncand, 1);
          if (k < RECON_LIST)
            cand[k] = c;
          else
            reconstruct<T>(d, buf, stamp, ii, jj, kk, i);  // list full: rebuild here
        }
      }
    }
  };
  // the box is unwrapped around the old centre
  const double cx[2] = {xo[0], xo[0] + min_image(xn[0] - xo[0], d.nx, d.walls[0])};
  chord_changes<1>(d, bx, b, d.ZB, xo, xn, cx, &R2, visit);
  __syncthreads();
  const int n = min(ncand, RECON_LIST);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  for (int e = wave; e < n; e += nwave) reconstruct_wave<T>(d, buf, stamp, cand[e], i, lane);
}

template <typename T>
__global__ __launch_bounds__(256) void k_recon(DevDomain d, int in_step) {
  if (!map_live(d.ctl, in_step)) return;
  recon_block<T>(d, blockIdx.x, map_buffer(d.ctl, in_step), map_stamp(d.ctl));
}

template <typename T>
__device__ __forceinline__ double raw_to_d(T v);
template <>
__device__ __forceinline__ double raw_to_d<double>(double v) { return v; }
template <>
__device__ __forceinline__ double raw_to_d<float>(float v) { return (double)v; }
template <>
__device__ __forceinline__ double raw_to_d<__half>(__half v) { return (double)__half2float(v); }

// A link of the boundary passes, packed: index t of the solid cell y in the
// block's cell set (bits 0-15), q (16-20), qbar (21-25) and c_q + 1 per axis
// (26-31).
__device__ __forceinline__ uint32_t link_entry(int t, int q) {
  return (uint32_t)t | ((uint32_t)q << 16) | ((uint32_t)OPP[q] << 21) | ((uint32_t)(CX[q] + 1) << 26) |
         ((uint32_t)(CY[q] + 1) << 28) | ((uint32_t)(CZ[q] + 1) << 30);
}

constexpr int LINK_UNROLL = 2;       // links in flight per thread, slab pass
constexpr int BALL_LINK_UNROLL = 1;  // ball pass: fewer registers, five waves per SIMD

// State code of the cell z = y - m c_q seen from sphere i: from the staged
// slab (index cidx0 of y, staged row pitch HX, HY) or from the global arrays.
__device__ __forceinline__ int slab_code(const DevDomain& d, const uint8_t* st, bool stg, int cidx0, int HX,
                                         int HY, const int* c, int m, long long zg, uint32_t stamp, int i) {
  if (stg) return st[cidx0 - m * (c[0] + HX * (c[1] + HY * c[2]))];
  int zo = -1;
  const int zs = new_state(d, zg, stamp, &zo);
  return zs == S_WALL ? L_WALL : (zs == S_SOLID ? (zo == i ? L_OWN : L_OTHER) : (zs == S_SHELL ? L_SHELL : L_FLUID));
}

// Links k0, k0 + blockDim.x, ... (at most U below tot) of one row chunk of
// a slab block, all loads issued before any is used: the cell is entry bits
// 0-15 = tx + EX ty of the chunk (plane kk, rows from jy0, columns from ix0).
// y - c_q fluid: boundary value of Eq. (MEM_CLI) into slot qbar of y (delta =
// 1/2 in the coefficients where y - 2 c_q is not fluid), force of Eq.
// (MEM_Fq) and its torque; y - c_q a wall or another sphere's solid: the
// missing-link force 2 w_q c_q with the arm to the mid-point of the link.
// The same arithmetic as ball_links.
template <typename T, int U>
__device__ __forceinline__ void slab_links(const DevDomain& d, T* buf, size_t N, const uint8_t* st, bool stg,
                                           const uint32_t* lk, int k0, int tot, int EX, int HX, int HY, int ix0,
                                           int jy0, int kk, int i, uint32_t stamp, const double* xp,
                                           const double* up, const double* wp, double R, double* acc) {
  bool ok[U], cli[U];
  int code[U], q[U], qb[U], cq[U][3], y[U][2];
  long long xg[U], yc[U];
  T gq[U], gqb[U], gm[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = k0 + u * (int)blockDim.x;
    ok[u] = k < tot;
    const uint32_t e = ok[u] ? lk[k] : 0u;
    const int t = (int)(e & 0xFFFFu);
    q[u] = (int)((e >> 16) & 31u);
    qb[u] = (int)((e >> 21) & 31u);
    cq[u][0] = (int)((e >> 26) & 3u) - 1;
    cq[u][1] = (int)((e >> 28) & 3u) - 1;
    cq[u][2] = (int)((e >> 30) & 3u) - 1;
    const int tx = t % EX, ty = t / EX;
    y[u][0] = d.walls[0] ? ix0 + tx : wrap_near(ix0 + tx, d.nx);
    y[u][1] = d.walls[1] ? jy0 + ty : wrap_near(jy0 + ty, d.ny);
    yc[u] = cidx(d, y[u][0], y[u][1], kk);
    const int cidx0 = (tx + 2) + HX * ((ty + 2) + HY * 2);
    // wall layers shield every non-wall cell, so y - c_q stays in range
    const int xi = wrapi(y[u][0] - cq[u][0], d.nx), xj = wrapi(y[u][1] - cq[u][1], d.ny),
              xk = wrapi(kk - cq[u][2], d.nz);
    xg[u] = cidx(d, xi, xj, xk);
    code[u] = ok[u] ? slab_code(d, st, stg, cidx0, HX, HY, cq[u], 1, xg[u], stamp, i) : L_OWN;
    cli[u] = false;
    gq[u] = gqb[u] = gm[u] = (T)0.0f;
    if (code[u] <= L_SHELL) {
      long long xmg = 0;
      if (d.boundary == 0) {
        xmg = cidx(d, wrapi(xi - cq[u][0], d.nx), wrapi(xj - cq[u][1], d.ny), wrapi(xk - cq[u][2], d.nz));
        cli[u] = slab_code(d, st, stg, cidx0, HX, HY, cq[u], 2, xmg, stamp, i) <= L_SHELL;
      }
      gq[u] = buf[(size_t)q[u] * N + xg[u]];
      gqb[u] = buf[(size_t)qb[u] * N + xg[u]];
      if (cli[u]) gm[u] = buf[(size_t)q[u] * N + xmg];
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (!ok[u]) continue;
    const int* c = cq[u];
    const double wq = c[0] * c[0] + c[1] * c[1] + c[2] * c[2] == 1 ? 1.0 / 18 : 1.0 / 36;
    double Fq[3], arm[3];
    if (code[u] <= L_SHELL) {
      const int xi = wrapi(y[u][0] - c[0], d.nx), xj = wrapi(y[u][1] - c[1], d.ny), xk = wrapi(kk - c[2], d.nz);
      double r[3];
      r[0] = min_image(((double)xi + 0.5) - xp[0], d.nx, d.walls[0]);
      r[1] = min_image(((double)xj + 0.5) - xp[1], d.ny, d.walls[1]);
      r[2] = min_image(((double)xk + 0.5) - xp[2], d.nz, d.walls[2]);
      const double dl = link_delta(r, c, R);
      for (int a = 0; a < 3; ++a) arm[a] = r[a] + dl * c[a];
      double ub[3];
      ub[0] = up[0] + (wp[1] * arm[2] - wp[2] * arm[1]);
      ub[1] = up[1] + (wp[2] * arm[0] - wp[0] * arm[2]);
      ub[2] = up[2] + (wp[0] * arm[1] - wp[1] * arm[0]);
      const double dd = cli[u] ? dl : 0.5;
      const double vq = raw_to_d<T>(gq[u]);
      double val = vq;
      if (cli[u]) val += (1.0 - 2.0 * dd) / (1.0 + 2.0 * dd) * (raw_to_d<T>(gm[u]) - raw_to_d<T>(gqb[u]));
      val -= 4.0 / (1.0 + 2.0 * dd) * wq * 3.0 * (ub[0] * c[0] + ub[1] * c[1] + ub[2] * c[2]);
      stv<T>(buf + (size_t)qb[u] * N + yc[u], val);
      const double fq = vq + wq, fb = val + wq;
      for (int a = 0; a < 3; ++a) Fq[a] = (c[a] - ub[a]) * fq - (-c[a] - ub[a]) * fb;
    } else {
      for (int a = 0; a < 3; ++a) Fq[a] = 2.0 * wq * c[a];
      arm[0] = min_image(((double)y[u][0] + 0.5) - xp[0], d.nx, d.walls[0]) - 0.5 * c[0];
      arm[1] = min_image(((double)y[u][1] + 0.5) - xp[1], d.ny, d.walls[1]) - 0.5 * c[1];
      arm[2] = min_image(((double)kk + 0.5) - xp[2], d.nz, d.walls[2]) - 0.5 * c[2];
    }
    acc[0] += Fq[0];
    acc[1] += Fq[1];
    acc[2] += Fq[2];
    acc[3] += arm[1] * Fq[2] - arm[2] * Fq[1];
    acc[4] += arm[2] * Fq[0] - arm[0] * Fq[2];
    acc[5] += arm[0] * Fq[1] - arm[1] * Fq[0];
  }
}

template <typename T>
__device__ __forceinline__ void commit_block(const DevDomain& d, int blk, int cur, uint32_t stamp) {
  T* buf = (T*)d.pdf[cur];
  const size_t N = (size_t)d.N;
  const int nbs = d.ZB * d.RB;
  const int i = blk / nbs, b = blk % nbs;
  const int bz = b / d.RB, brow = b % d.RB;
  Box bx;
  sphere_box(d, i, true, bx);
  const double xp[3] = {d.p.x[3 * i], d.p.x[3 * i + 1], d.p.x[3 * i + 2]};
  const double xo[3] = {d.p.xmap[3 * i], d.p.xmap[3 * i + 1], d.p.xmap[3 * i + 2]};
  const double up[3] = {d.p.u[3 * i], d.p.u[3 * i + 1], d.p.u[3 * i + 2]};
  const double wp[3] = {d.p.w[3 * i], d.p.w[3 * i + 1], d.p.w[3 * i + 2]};
  const double R = d.p.R[i];
  double R2, rs2;
  {
#pragma clang fp contract(off)
    const double rs = R + d.delta_ab;
    R2 = R * R;
    rs2 = rs * rs;
  }
  // States of the slab's cells and of a 2-cell halo (the CLI needs x - c_q of
  // the fluid cell x = y - c_q) are staged in LDS, so link detection needs no
  // dependent global loads; boxes too large for LDS take the global path.
  // A block works on row chunks of COMMIT_ROWS rows of the box slabs
  // (slab bz, bz + ZB, ...; chunk brow, brow + RB, ...).
  const int EX = bx.ext[0], EY = bx.ext[1], HX = EX + 4, HY = COMMIT_ROWS + 4;
  const bool staged = HX * HY * 5 <= STAGE_BYTES;
  __shared__ uint8_t st[STAGE_BYTES];
  __shared__ uint32_t lk[(Q - 1) * 256];  // one chunk's links (at most 18 per cell)
  __shared__ int wsum[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int sl = bz; sl < bx.ext[2]; sl += d.ZB) {
    const int kz = bx.lo[2] + sl;
    const int kk = d.walls[2] ? kz : wrap_near(kz, d.nz);
    // does this plane cut the new solid ball of sphere i?
    const double dzc = min_image(((double)kk + 0.5) - xp[2], d.nz, d.walls[2]);
    const bool cuts = dzc * dzc <= R2;
    for (int ry0 = brow * COMMIT_ROWS; ry0 < EY; ry0 += d.RB * COMMIT_ROWS) {
      const int nrow = min(COMMIT_ROWS, EY - ry0);
      if (staged && cuts) {
        __syncthreads();
        // eight entries per thread and pass (one pass for boxes up to ~40
        // cells wide), all loads issued before any use
        const int NS = HX * HY * 5;
        for (int t0 = threadIdx.x; t0 < NS; t0 += 8 * blockDim.x) {
          bool in[8];
          uint8_t fl[8];
          unsigned long long kc[8];
          uint32_t ss[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int t = t0 + u * blockDim.x;
            const int hx = t % HX, r = t / HX, hy = r % HY, hz = r / HY;
            const int gx = bx.lo[0] - 2 + hx, gy = bx.lo[1] + ry0 - 2 + hy, gz = kz - 2 + hz;
            in[u] = t < NS && (!d.walls[0] || (gx >= 0 && gx < d.nx)) &&
                    (!d.walls[1] || (gy >= 0 && gy < d.ny)) && (!d.walls[2] || (gz >= 0 && gz < d.nz));
            if (in[u]) {
              const long long c = cidx(d, wrap_near(gx, d.nx), wrap_near(gy, d.ny), wrap_near(gz, d.nz));
              fl[u] = d.flags[c];
              kc[u] = d.claim[c];
              ss[u] = d.shellstamp[c];
            }
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int t = t0 + u * blockDim.x;
            if (t >= NS) continue;
            uint8_t code = L_WALL;
            if (in[u] && !(fl[u] & F_WALL)) {
              if ((uint32_t)(kc[u] >> 32) == stamp) {
                const int o = (int)(0xFFFFFFFFu - (uint32_t)(kc[u] & 0xFFFFFFFFull));
                code = o == i ? L_OWN : L_OTHER;
              } else {
                code = ss[u] == stamp ? L_SHELL : L_FLUID;
              }
            }
            st[t] = code;
          }
        }
        __syncthreads();
      }
      const int ncell = EX * nrow;
      // the cell's state: staged when its plane cuts the solid ball (then
      // only another sphere's solid needs the claim for its owner)
      const bool stg = staged && cuts;
      for (int t0 = 0; t0 < ncell; t0 += blockDim.x) {
        const int t = t0 + threadIdx.x;
        uint32_t mask = 0u;
        if (t < ncell) {
          const int tx = t % EX, ty = t / EX;
          const int ii = d.walls[0] ? bx.lo[0] + tx : wrap_near(bx.lo[0] + tx, d.nx);
          const int jj = d.walls[1] ? bx.lo[1] + ry0 + ty : wrap_near(bx.lo[1] + ry0 + ty, d.ny);
          // only cells within the old or new shell ball of i can change through i
          if (cell_d2(d, ii, jj, kk, xp) <= rs2 || cell_d2(d, ii, jj, kk, xo) <= rs2) {
            const long long yc = cidx(d, ii, jj, kk);
            const int cidx0 = (tx + 2) + HX * ((ty + 2) + HY * 2);
            const int sc = stg ? (int)st[cidx0] : -1;
            int own = -1, ns;
            if (sc == L_OWN) {
              ns = S_SOLID;
              own = i;
            } else if (sc == L_SHELL || sc == L_FLUID) {
              ns = sc == L_SHELL ? S_SHELL : S_FLUID;
            } else if (sc == L_WALL) {
              ns = S_WALL;
            } else {
              ns = new_state(d, yc, stamp, &own);
            }
            if (ns != S_WALL) {
              d.flags[yc] = ns == S_SOLID ? F_SOLID : (ns == S_SHELL ? F_SHELL : (uint8_t)0);
              if (ns == S_SOLID) d.owner[yc] = own;
            }
            if (ns == S_SOLID && own == i) {
              // the links of y: directions whose y - c_q is not this sphere's solid
#pragma unroll
              for (int q = 1; q < Q; ++q) {
                const int c[3] = {CX[q], CY[q], CZ[q]};
                const long long xg = stg ? 0 : cidx(d, wrapi(ii - c[0], d.nx), wrapi(jj - c[1], d.ny), wrapi(kk - c[2], d.nz));
                if (slab_code(d, st, stg, cidx0, HX, HY, c, 1, xg, stamp, i) != L_OWN) mask |= 1u << q;
              }
            }
          }
        }
        // ordered compaction of the chunk's links (cell order, then direction)
        const int cnt = __popc(mask);
        int v = cnt;
        for (int o = 1; o < 64; o <<= 1) {
          const int w = __shfl_up(v, o, 64);
          if (lane >= o) v += w;
        }
        if (lane == 63) wsum[wid] = v;
        __syncthreads();
        int off = v - cnt, tot = 0;
        for (int w = 0; w < nw; ++w) {
          if (w < wid) off += wsum[w];
          tot += wsum[w];
        }
#pragma unroll
        for (int q = 1; q < Q; ++q)
          if (mask & (1u << q)) lk[off++] = link_entry(t, q);
        __syncthreads();
        for (int k0 = threadIdx.x; k0 < tot; k0 += LINK_UNROLL * blockDim.x)
          slab_links<T, LINK_UNROLL>(d, buf, N, st, stg, lk, k0, tot, EX, HX, HY, bx.lo[0], bx.lo[1] + ry0, kk, i,
                                     stamp, xp, up, wp, R, acc);
        __syncthreads();  // the list, the wave sums and the staged states are reused
      }
    }
  }
  // fixed-order block reduction: wavefront shuffles, then across wavefronts
  __shared__ double red[6][8];
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
    d.partial[((size_t)i * nbs + b) * 6 + threadIdx.x] = v;
  }
}

constexpr int FOLD_ADVANCE_MAX_BLOCKS = 512;

// With `advance`, the last block of the launch to finish runs the step
// control (saving a launch at the end of the step): every block has read the
// step state by the time it counts itself done, so none can see it change.
__device__ __forceinline__ void last_block_advance(const DevDomain& d) {
  __shared__ int last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(&d.ctl->done_blocks, 1u) == gridDim.x - 1u;
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __threadfence();
    d.ctl->done_blocks = 0u;
    step_control(d);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_commit(DevDomain d, int in_step, int advance) {
  if (map_live(d.ctl, in_step)) commit_block<T>(d, blockIdx.x, map_buffer(d.ctl, in_step), map_stamp(d.ctl));
  if (advance) last_block_advance(d);
}

// Many spheres: one block per sphere.  The states of all cells within R + 3 of
// the new centre (every cell a link of the sphere or its CLI neighbour can
// touch) are staged in LDS in one pass with many loads in flight; then the
// flags of the cells in the old and new shell balls are committed, the
// sphere's solid cells that have a non-own neighbour are listed, and their
// links are formed as in k_commit.  Dynamic LDS: edge^3 state bytes plus the
// surface list.
// threads per block of the in-step geometric kernels (one block per sphere)
constexpr int GEO_THREADS = 64;

// mapping bin of a position
__device__ __forceinline__ int mbin_index(const DevDomain& d, const double* x, int* b) {
  const int n[3] = {d.nx, d.ny, d.nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int nb = d.mbins.n[a];
    const int k = (int)floor(x[a] * (double)nb / (double)n[a]);
    b[a] = k < 0 ? 0 : (k >= nb ? nb - 1 : k);
  }
  return b[0] + d.mbins.n[0] * (b[1] + d.mbins.n[1] * b[2]);
}

constexpr uint8_t L_UNSET = 5;  // cell outside the staged ball



// Links k0, k0 + blockDim.x, ... (at most U of them below tot) of sphere i,
// all loads issued before any is used.  y - c_q fluid: boundary value of
// Eq. (MEM_CLI) into slot qbar of y (delta = 1/2 in the coefficients where
// y - 2 c_q is not fluid), force of Eq. (MEM_Fq) and its torque about the
// centre; y - c_q a wall or another sphere's solid: the missing-link force
// 2 w_q c_q with the arm to the mid-point of the link.
template <typename T, int U>
__device__ __forceinline__ void ball_links(const DevDomain& d, T* buf, size_t N, const uint8_t* st,
                                           const uint32_t* lk, int k0, int tot, int he, const int* lo,
                                           const double* xp, const double* up, const double* wp, double R,
                                           double* acc) {
  bool ok[U], cli[U];
  int code[U], q[U], qb[U], cq[U][3], y[U][3], xg[U], xmg[U];
  T gq[U], gqb[U], gm[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = k0 + u * (int)blockDim.x;
    ok[u] = k < tot;
    const uint32_t e = ok[u] ? lk[k] : 0u;
    const int t = (int)(e & 0xFFFFu);
    q[u] = (int)((e >> 16) & 31u);
    qb[u] = (int)((e >> 21) & 31u);
    cq[u][0] = (int)((e >> 26) & 3u) - 1;
    cq[u][1] = (int)((e >> 28) & 3u) - 1;
    cq[u][2] = (int)((e >> 30) & 3u) - 1;
    const int h[3] = {t % he, (t / he) % he, t / (he * he)};
    y[u][0] = d.walls[0] ? lo[0] + h[0] : wrap_near(lo[0] + h[0], d.nx);
    y[u][1] = d.walls[1] ? lo[1] + h[1] : wrap_near(lo[1] + h[1], d.ny);
    y[u][2] = d.walls[2] ? lo[2] + h[2] : wrap_near(lo[2] + h[2], d.nz);
    const int off = cq[u][0] + he * (cq[u][1] + he * cq[u][2]);
    code[u] = ok[u] ? (int)st[t - off] : L_OWN;
    cli[u] = false;
    xg[u] = xmg[u] = 0;
    gq[u] = gqb[u] = gm[u] = (T)0.0f;
    if (code[u] <= L_SHELL) {
      // wall layers shield every non-wall cell, so y - c_q stays in range
      const int xi = wrapi(y[u][0] - cq[u][0], d.nx), xj = wrapi(y[u][1] - cq[u][1], d.ny),
                xk = wrapi(y[u][2] - cq[u][2], d.nz);
      xg[u] = (int)cidx(d, xi, xj, xk);
      if (d.boundary == 0 && st[t - 2 * off] <= L_SHELL) {
        cli[u] = true;
        xmg[u] = (int)cidx(d, wrapi(xi - cq[u][0], d.nx), wrapi(xj - cq[u][1], d.ny), wrapi(xk - cq[u][2], d.nz));
      }
      gq[u] = buf[(size_t)q[u] * N + xg[u]];
      gqb[u] = buf[(size_t)qb[u] * N + xg[u]];
      if (cli[u]) gm[u] = buf[(size_t)q[u] * N + xmg[u]];
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (!ok[u]) continue;
    const int* c = cq[u];
    const double wq = c[0] * c[0] + c[1] * c[1] + c[2] * c[2] == 1 ? 1.0 / 18 : 1.0 / 36;
    double Fq[3], arm[3];
    if (code[u] <= L_SHELL) {
      const int xi = wrapi(y[u][0] - c[0], d.nx), xj = wrapi(y[u][1] - c[1], d.ny), xk = wrapi(y[u][2] - c[2], d.nz);
      double r[3];
      r[0] = min_image(((double)xi + 0.5) - xp[0], d.nx, d.walls[0]);
      r[1] = min_image(((double)xj + 0.5) - xp[1], d.ny, d.walls[1]);
      r[2] = min_image(((double)xk + 0.5) - xp[2], d.nz, d.walls[2]);
      const double dl = link_delta(r, c, R);
      for (int a = 0; a < 3; ++a) arm[a] = r[a] + dl * c[a];
      double ub[3];
      ub[0] = up[0] + (wp[1] * arm[2] - wp[2] * arm[1]);
      ub[1] = up[1] + (wp[2] * arm[0] - wp[0] * arm[2]);
      ub[2] = up[2] + (wp[0] * arm[1] - wp[1] * arm[0]);
      const double dd = cli[u] ? dl : 0.5;
      const double vq = raw_to_d<T>(gq[u]);
      double val = vq;
      if (cli[u]) val += (1.0 - 2.0 * dd) / (1.0 + 2.0 * dd) * (raw_to_d<T>(gm[u]) - raw_to_d<T>(gqb[u]));
      val -= 4.0 / (1.0 + 2.0 * dd) * wq * 3.0 * (ub[0] * c[0] + ub[1] * c[1] + ub[2] * c[2]);
      stv<T>(buf + (size_t)qb[u] * N + cidx(d, y[u][0], y[u][1], y[u][2]), val);
      const double fq = vq + wq, fb = val + wq;
      for (int a = 0; a < 3; ++a) Fq[a] = (c[a] - ub[a]) * fq - (-c[a] - ub[a]) * fb;
    } else {
      for (int a = 0; a < 3; ++a) Fq[a] = 2.0 * wq * c[a];
      arm[0] = min_image(((double)y[u][0] + 0.5) - xp[0], d.nx, d.walls[0]) - 0.5 * c[0];
      arm[1] = min_image(((double)y[u][1] + 0.5) - xp[1], d.ny, d.walls[1]) - 0.5 * c[1];
      arm[2] = min_image(((double)y[u][2] + 0.5) - xp[2], d.nz, d.walls[2]) - 0.5 * c[2];
    }
    acc[0] += Fq[0];
    acc[1] += Fq[1];
    acc[2] += Fq[2];
    acc[3] += arm[1] * Fq[2] - arm[2] * Fq[1];
    acc[4] += arm[2] * Fq[0] - arm[0] * Fq[2];
    acc[5] += arm[0] * Fq[1] - arm[1] * Fq[0];
  }
}

template <typename T>
__device__ __forceinline__ void commit_ball(const DevDomain& d, int in_step, int i) {
  const int cur = map_buffer(d.ctl, in_step);
  T* buf = (T*)d.pdf[cur];
  const size_t N = (size_t)d.N;
  extern __shared__ uint8_t smem[];
  const int he = d.stage_edge, H = he / 2;
  const int NS = he * he * he;
  uint8_t* st = smem;
  uint16_t* list = reinterpret_cast<uint16_t*>(smem + ((NS + 15) & ~15));
  uint32_t* lk = reinterpret_cast<uint32_t*>(smem + ((NS + 15) & ~15) + ((2 * d.list_cap + 15) & ~15));
  __shared__ double red[6][4];
  const double xp[3] = {d.p.x[3 * i], d.p.x[3 * i + 1], d.p.x[3 * i + 2]};
  const double up[3] = {d.p.u[3 * i], d.p.u[3 * i + 1], d.p.u[3 * i + 2]};
  const double wp[3] = {d.p.w[3 * i], d.p.w[3 * i + 1], d.p.w[3 * i + 2]};
  const double R = d.p.R[i];
  double rl2;
  {
#pragma clang fp contract(off)
    const double rl = R + 3.0;
    rl2 = rl * rl;
  }
  const int n[3] = {d.nx, d.ny, d.nz};
  bool finite = isfinite(xp[0]) && isfinite(xp[1]) && isfinite(xp[2]);
  int lo[3];
  for (int a = 0; a < 3; ++a) lo[a] = finite ? (int)floor(xp[a]) - H : 0;
  // the mapping bins were last read by the mapping update before this launch:
  // emptied here for the next step
  if (in_step && finite && threadIdx.x == 0) {
    int b[3];
    d.mbins.cell[(size_t)mbin_index(d, xp, b) * (1 + BIN_CAP)] = 0;
  }

  // Row chords, kept in the link list's LDS (unused until step 3): of each
  // x-row of the staged cube, the cells whose centres can lie within R + 3 of
  // the centre are those with x index in [s, e] (packed s | e << 16; s > e:
  // none), from the row's exact y and z offsets, widened by 1e-3.  Rows of a
  // cube that nearly spans a periodic x axis keep every cell.
  constexpr double EPS = 1e-3;
  constexpr int CH = (Q - 1) * BALL_THREADS;
  uint32_t* chord = lk;
  const bool chorded = he * he <= CH && (d.walls[0] || he + 2 <= n[0]);
  if (chorded) {
    for (int r = threadIdx.x; r < he * he; r += blockDim.x) {
      const int gy = lo[1] + r % he, gz = lo[2] + r / he;
      const int jj = d.walls[1] ? gy : wrap_near(gy, n[1]), kk = d.walls[2] ? gz : wrap_near(gz, n[2]);
      const double dy = min_image(((double)jj + 0.5) - xp[1], n[1], d.walls[1]);
      const double dz = min_image(((double)kk + 0.5) - xp[2], n[2], d.walls[2]);
      const double rho = rl2 - (dy * dy + dz * dz);
      const double a = sqrt(fmax(rho, 0.0)) + EPS;
      int s0 = max(0, (int)ceil(xp[0] - a - 0.5) - lo[0]), e0 = min(he - 1, (int)floor(xp[0] + a - 0.5) - lo[0]);
      if (rho < -EPS || e0 < s0) s0 = 1, e0 = 0;
      chord[r] = (uint32_t)s0 | ((uint32_t)e0 << 16);
    }
    __syncthreads();
  }

  // 1. stage the states of the cells within R + 3 of the centre (every
  // link's y - c_q and y - 2 c_q lies within R + 2 sqrt(2)), from the cell
  // words (flags | (owner + 1) << 8) the mapping update has just written;
  // eight cells per thread and pass, all loads issued before use
  for (int t0 = threadIdx.x; t0 < NS; t0 += 8 * blockDim.x) {
    long long cc[8];
    uint8_t code[8];
    uint32_t cw[8];
    bool ld[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + u * blockDim.x;
      ld[u] = false;
      code[u] = L_UNSET;
      if (t < NS && finite) {
        const int g[3] = {lo[0] + t % he, lo[1] + (t / he) % he, lo[2] + t / (he * he)};
        bool out = false;
        int ijk[3];
        for (int a = 0; a < 3; ++a) {
          if (d.walls[a]) {
            out = out || g[a] < 0 || g[a] >= n[a];
            ijk[a] = g[a];
          } else {
            ijk[a] = wrap_near(g[a], n[a]);
          }
        }
        if (out) {
          code[u] = L_WALL;
        } else {
          const int hx = t % he;
          const uint32_t ch = chorded ? chord[t / he] : 0xFFFF0000u;
          if (hx >= (int)(ch & 0xFFFFu) && hx <= (int)(ch >> 16)) {
            cc[u] = cidx(d, ijk[0], ijk[1], ijk[2]);
            ld[u] = true;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (ld[u]) cw[u] = d.cellw[cc[u]];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + u * blockDim.x;
      if (t >= NS) continue;
      if (ld[u]) {
        if (cw[u] & F_WALL)
          code[u] = L_WALL;
        else if (cw[u] & F_SOLID)
          code[u] = (int)(cw[u] >> 8) - 1 == i ? L_OWN : L_OTHER;
        else
          code[u] = L_FLUID;  // fluid, in a TRT+aB shell or not
      }
      st[t] = code[u];
    }
  }
  __syncthreads();

  // 2. solid cells of this sphere with a neighbour that is not, listed in
  // cube order (ordered compaction: wavefront ballots and per-wave offsets),
  // so that every cell is summed by the same thread on every run.  Only the
  // central box of edge 2 ceil(R) + 3 can hold cells of this sphere (their
  // centres lie within R of x_p); its x-fastest order is the cube's.  The
  // wave counts alternate between two slots, so one barrier per pass does.
  __shared__ int wcount[2][4];
  int base = 0;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int rc = (int)ceil(R) + 1, E = 2 * rc + 1, h0 = H - rc;
  const int NE = finite ? E * E * E : 0;
  for (int t0 = 0, pass = 0; t0 < NE; t0 += blockDim.x, pass ^= 1) {
    const int u = t0 + threadIdx.x;
    const int t = h0 + u % E + he * (h0 + (u / E) % E + he * (h0 + u / (E * E)));
    bool surf = false;
    if (u < NE && st[t] == L_OWN) {
#pragma unroll
      for (int q = 1; q < Q; ++q) surf = surf || st[t + CX[q] + he * (CY[q] + he * CZ[q])] != L_OWN;
    }
    const unsigned long long m = __ballot(surf);
    if (lane == 0) wcount[pass][wid] = __popcll(m);
    __syncthreads();
    int off = base, tot = 0;
    for (int w = 0; w < nw; ++w) {
      if (w < wid) off += wcount[pass][w];
      tot += wcount[pass][w];
    }
    if (surf) list[off + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)t;
    base += tot;
  }
  __syncthreads();

  // 3. links: the listed cells in chunks of one cell per thread; a chunk's
  // links (y, q) with y - c_q not this sphere's solid are listed direction by
  // direction, cells in order within a direction (ordered compaction), then
  // shared out over all threads: a wavefront's loads then walk neighbouring
  // cells of one PDF plane, so the uses of a line come close together
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int nl = base;  // the same in every thread
  __shared__ int qcnt[Q][4];
  for (int c0 = 0; c0 < nl; c0 += blockDim.x) {
    const int e = c0 + threadIdx.x;
    uint32_t mask = 0u;
    int t = 0;
    if (e < nl) {
      t = list[e];
#pragma unroll
      for (int q = 1; q < Q; ++q)
        if (st[t - CX[q] - he * (CY[q] + he * CZ[q])] != L_OWN) mask |= 1u << q;
    }
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long bq[Q];
#pragma unroll
    for (int q = 1; q < Q; ++q) {
      bq[q] = __ballot((mask >> q) & 1u);
      if (lane == 0) qcnt[q][wid] = __popcll(bq[q]);
    }
    __syncthreads();
    int tot = 0;
#pragma unroll
    for (int q = 1; q < Q; ++q) {
      int pre = 0, all = 0;
      for (int w = 0; w < nw; ++w) {
        if (w < wid) pre += qcnt[q][w];
        all += qcnt[q][w];
      }
      if (mask & (1u << q)) lk[tot + pre + __popcll(bq[q] & below)] = link_entry(t, q);
      tot += all;
    }
    __syncthreads();
    for (int k0 = threadIdx.x; k0 < tot; k0 += BALL_LINK_UNROLL * blockDim.x)
      ball_links<T, BALL_LINK_UNROLL>(d, buf, N, st, lk, k0, tot, he, lo, xp, up, wp, R, acc);
    __syncthreads();  // the next chunk reuses the list and the wave sums
  }
  // 4. fixed-order block reduction
  for (int k = 0; k < 6; ++k) {
    double v = acc[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[k][wid] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double v = 0.0;
    for (int w4 = 0; w4 < (int)(blockDim.x >> 6); ++w4) v += red[threadIdx.x][w4];
    d.partial[(size_t)i * 6 + threadIdx.x] = v;
  }
}

// one block per sphere, taken in the space-filling-curve order and spread over
// the XCDs in contiguous runs, so that neighbouring spheres, whose staging
// balls and links share cache lines, are served by the same L2.  At least
// five waves per SIMD (at most 96 VGPRs, one link in flight per thread):
// 1.66 ms at 10,000 spheres, against 1.78 ms with four waves and two links
// and ~1.9 ms with the three waves the unconstrained allocation allows
template <typename T>
__global__ __launch_bounds__(BALL_THREADS) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_commit_ball(DevDomain d,
                                                                                             int in_step,
                                                                                             int advance) {
  const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  if (map_live(d.ctl, in_step) && t < d.P) commit_ball<T>(d, in_step, d.p.order[t]);
  if (advance) last_block_advance(d);
}


static void launch_claim(const DevDomain& d, int in_step, bool lists, hipStream_t s) {
  const int nsb = d.P * d.ZB;
  if (nsb > 0) hipLaunchKernelGGL(k_claim, dim3(nsb), dim3(256), 0, s, d, in_step, (in_step && lists) ? 1 : 0);
}

// ---- geometric mapping of the fused step ------------------------------------
// With the particle links formed in the sweep, the mapping update needs the
// flags and owners of the new positions and the reconstruction of uncovered
// cells only.  Both follow from the positions alone: the state of a cell is
// solid of the lowest id whose closed ball holds its centre, else shell within
// R + delta_aB of some sphere, else fluid (walls never change) -- evaluated
// from the spheres listed in the 27 mapping bins around the cell (every sphere
// whose shell ball can hold the centre is among them, the bin edge being at
// least R_max + delta_aB + 1).  Inside a step each sphere visits the cells of
// its old and new shell boxes and rewrites only those where its own solid or
// shell membership changed: a cell whose state changes has some sphere whose
// membership changed, and every sphere that rewrites a cell writes the same
// value.  Outside a step (new, moved or restored spheres) every cell is
// evaluated.


// insert (clear = 0) or remove (clear = 1: zero the count of its bin) every
// sphere by its current position
__global__ void k_mbins(DevDomain d, int in_step, int clear) {
  if (in_step ? !step_live(d.ctl) : d.ctl->frozen) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.P) return;
  const double* x = d.p.x + 3 * i;
  if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]))) {
    atomicOr(d.status, ST_NONFINITE);
    return;
  }
  int b[3];
  int* c = d.mbins.cell + (size_t)mbin_index(d, x, b) * (1 + BIN_CAP);
  if (clear) {
    c[0] = 0;
    return;
  }
  const int k = atomicAdd(c, 1);
  if (k < BIN_CAP)
    c[1 + k] = i;
  else
    atomicOr(d.status, ST_NBR_FULL);
}

// state of non-wall cell (i, j, k) at the current positions (S_FLUID,
// S_SHELL or S_SOLID with *own the lowest id)
__device__ inline int geo_state(const DevDomain& d, int i, int j, int k, int* own) {
  const double xc[3] = {(double)i + 0.5, (double)j + 0.5, (double)k + 0.5};
  int b[3];
  mbin_index(d, xc, b);
  const int n0 = d.mbins.n[0], n1 = d.mbins.n[1], n2 = d.mbins.n[2];
  int best = 0x7FFFFFFF;
  bool shell = false;
  for (int ez = 0; ez < axis_count(n2); ++ez) {
    int kz;
    if (!axis_bin(b[2], n2, d.walls[2], ez, &kz)) continue;
    for (int ey = 0; ey < axis_count(n1); ++ey) {
      int ky;
      if (!axis_bin(b[1], n1, d.walls[1], ey, &ky)) continue;
      for (int ex = 0; ex < axis_count(n0); ++ex) {
        int kx;
        if (!axis_bin(b[0], n0, d.walls[0], ex, &kx)) continue;
        const int* c = d.mbins.cell + (size_t)(kx + n0 * (ky + n1 * kz)) * (1 + BIN_CAP);
        const int m = min(c[0], BIN_CAP);
        for (int e = 0; e < m; ++e) {
          const int s = c[1 + e];
          double R2, rs2;
          {
#pragma clang fp contract(off)
            const double R = d.p.R[s];
            const double rs = R + d.delta_ab;
            R2 = R * R;
            rs2 = rs * rs;
          }
          const double d2 = cell_d2(d, i, j, k, d.p.x + 3 * s);
          if (d2 <= R2 && s < best) best = s;
          if (d2 <= rs2) shell = true;
        }
      }
    }
  }
  *own = best;
  return best != 0x7FFFFFFF ? S_SOLID : (shell ? S_SHELL : S_FLUID);
}

__device__ __forceinline__ bool wall_cell(const DevDomain& d, int i, int j, int k) {
  return (d.walls[0] && (i == 0 || i == d.nx - 1)) || (d.walls[1] && (j == 0 || j == d.ny - 1)) ||
         (d.walls[2] && (k == 0 || k == d.nz - 1));
}

// Reconstruction inside a step (one block per sphere i): cells of i's solid
// at the mapped positions (flags and owners in place) that are not solid at
// the new positions, from neighbours fluid before (flags) and after
// (geo_state); written into the buffer the sweep has just filled.
template <typename T>
__global__ __launch_bounds__(256) void k_recon_geo(DevDomain d) {
  if (!step_live(d.ctl)) return;
  const int i = blockIdx.x;
  if (i >= d.P) return;
  T* buf = (T*)d.pdf[map_buffer(d.ctl, 1)];
  __shared__ long long cand[RECON_LIST];
  __shared__ int ncand;
  if (threadIdx.x == 0) ncand = 0;
  __syncthreads();
  Box bx;
  mapped_ball_box(d, i, bx);
  const double xo[3] = {d.p.xmap[3 * i], d.p.xmap[3 * i + 1], d.p.xmap[3 * i + 2]};
  const double xn[3] = {d.p.x[3 * i], d.p.x[3 * i + 1], d.p.x[3 * i + 2]};
  double R2;
  {
#pragma clang fp contract(off)
    const double R = d.p.R[i];
    R2 = R * R;
  }
  auto usable = [&](long long y, int yi, int yj, int yk) {
    int o;
    return !(d.flags[y] & (F_SOLID | F_WALL)) && geo_state(d, yi, yj, yk, &o) != S_SOLID;
  };
  auto visit = [&](int ii, int jj, int kk) {
    if (cell_d2(d, ii, jj, kk, xo) <= R2 && !(cell_d2(d, ii, jj, kk, xn) <= R2)) {
      const long long c = cidx(d, ii, jj, kk);
      int o;
      if ((d.flags[c] & F_SOLID) && d.owner[c] == i && geo_state(d, ii, jj, kk, &o) != S_SOLID) {
        const int k = atomicAdd(&ncand, 1);
        if (k < RECON_LIST)
          cand[k] = c;
        else
          reconstruct_with<T>(d, buf, ii, jj, kk, i, usable);  // list full: rebuild here
      }
    }
  };
  // the box is unwrapped around the old centre
  const double cx[2] = {xo[0], xo[0] + min_image(xn[0] - xo[0], d.nx, d.walls[0])};
  chord_changes<1>(d, bx, 0, 1, xo, xn, cx, &R2, visit);
  __syncthreads();
  const int n = min(ncand, RECON_LIST);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  for (int e = wave; e < n; e += nwave) reconstruct_wave_with<T>(d, buf, cand[e], i, lane, usable);
}

// Flags and owners inside a step (one block per sphere i): the cells of the
// old and new shell boxes where i's solid or shell membership changed get the
// state of the new positions.
__global__ __launch_bounds__(256) void k_remap_geo(DevDomain d) {
  if (!step_live(d.ctl)) return;
  const int i = blockIdx.x;
  if (i >= d.P) return;
  Box bx;
  sphere_box(d, i, true, bx);
  const double xo[3] = {d.p.xmap[3 * i], d.p.xmap[3 * i + 1], d.p.xmap[3 * i + 2]};
  const double xn[3] = {d.p.x[3 * i], d.p.x[3 * i + 1], d.p.x[3 * i + 2]};
  double R2, rs2;
  {
#pragma clang fp contract(off)
    const double R = d.p.R[i];
    const double rs = R + d.delta_ab;
    R2 = R * R;
    rs2 = rs * rs;
  }
  // the cells where i's solid or shell membership changed lie near the ends
  // of the row chords of its old and new balls of radius R and R + delta_aB
  auto visit = [&](int ii, int jj, int kk) {
    if (wall_cell(d, ii, jj, kk)) return;
    const double d2o = cell_d2(d, ii, jj, kk, xo), d2n = cell_d2(d, ii, jj, kk, xn);
    if ((d2o <= R2) != (d2n <= R2) || (d2o <= rs2) != (d2n <= rs2)) {
      int own;
      const int st = geo_state(d, ii, jj, kk, &own);
      const long long c = cidx(d, ii, jj, kk);
      const uint8_t fl = st == S_SOLID ? F_SOLID : (st == S_SHELL ? F_SHELL : (uint8_t)0);
      d.flags[c] = fl;
      if (st == S_SOLID) d.owner[c] = own;
      if (d.cellw) d.cellw[c] = (uint32_t)fl | (st == S_SOLID ? (uint32_t)(own + 1) << 8 : 0u);
    }
  };
  // the box is unwrapped around the new centre
  const double cx[2] = {xn[0] + min_image(xo[0] - xn[0], d.nx, d.walls[0]), xn[0]};
  const double r2[2] = {R2, rs2};
  chord_changes<2>(d, bx, 0, 1, xo, xn, cx, r2, visit);
}

// End of a fused step: the mapping bins are emptied (by the positions they
// were filled with) and one thread runs the step control.
__global__ void k_advance_fused(DevDomain d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.P) {
    const double* x = d.p.x + 3 * i;
    if (isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2])) {
      int b[3];
      d.mbins.cell[(size_t)mbin_index(d, x, b) * (1 + BIN_CAP)] = 0;
    }
  }
  if (i == 0) step_control(d);
}

// Outside a step: the state of every cell at the current positions into the
// stage (2 bits of state, owner + 1 above them), reconstruction of cells that
// leave a solid, then the commit.
__global__ void k_geo_stage(DevDomain d) {
  if (d.ctl->frozen) return;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < (size_t)d.N;
       c += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % d.nx), j = (int)((c / d.nx) % d.ny), k = (int)(c / ((size_t)d.nx * d.ny));
    if (wall_cell(d, i, j, k)) {
      d.stage32[c] = (uint32_t)S_WALL;
      continue;
    }
    int own;
    const int st = geo_state(d, i, j, k, &own);
    d.stage32[c] = (uint32_t)st | (st == S_SOLID ? ((uint32_t)(own + 1) << 2) : 0u);
  }
}

template <typename T>
__global__ void k_recon_full(DevDomain d) {
  if (d.ctl->frozen) return;
  T* buf = (T*)d.pdf[map_buffer(d.ctl, 0)];
  auto usable = [&](long long y, int, int, int) {
    return !(d.flags[y] & (F_SOLID | F_WALL)) && (d.stage32[y] & 3u) <= (uint32_t)S_SHELL;
  };
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < (size_t)d.N;
       c += (size_t)gridDim.x * blockDim.x) {
    if (!(d.flags[c] & F_SOLID) || (d.stage32[c] & 3u) > (uint32_t)S_SHELL) continue;
    const int i = (int)(c % d.nx), j = (int)((c / d.nx) % d.ny), k = (int)(c / ((size_t)d.nx * d.ny));
    reconstruct_with<T>(d, buf, i, j, k, d.owner[c], usable);
  }
}

__global__ void k_commit_full(DevDomain d) {
  if (d.ctl->frozen) return;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < (size_t)d.N;
       c += (size_t)gridDim.x * blockDim.x) {
    const uint32_t v = d.stage32[c];
    const int st = (int)(v & 3u);
    if (st == S_WALL) continue;
    const uint8_t fl = st == S_SOLID ? F_SOLID : (st == S_SHELL ? F_SHELL : (uint8_t)0);
    d.flags[c] = fl;
    if (st == S_SOLID) d.owner[c] = (int)(v >> 2) - 1;
    if (d.cellw) d.cellw[c] = (uint32_t)fl | (st == S_SOLID ? (v >> 2) << 8 : 0u);
  }
}

static dim3 cells_grid(long long N) {
  long long b = (N + 255) / 256;
  return dim3((unsigned)(b > 65536 ? 65536 : (b < 1 ? 1 : b)));
}

void launch_mapping_geo(const DevDomain& d, bool reconstruct, hipStream_t s) {
  const dim3 gp((unsigned)((d.P + 255) / 256 > 0 ? (d.P + 255) / 256 : 1));
  if (d.P > 0) hipLaunchKernelGGL(k_mbins, gp, dim3(256), 0, s, d, 0, 0);
  hipLaunchKernelGGL(k_geo_stage, cells_grid(d.N), dim3(256), 0, s, d);
  if (reconstruct) {
    if (d.storage == 0)
      hipLaunchKernelGGL(k_recon_full<double>, cells_grid(d.N), dim3(256), 0, s, d);
    else if (d.storage == 1)
      hipLaunchKernelGGL(k_recon_full<float>, cells_grid(d.N), dim3(256), 0, s, d);
    else
      hipLaunchKernelGGL(k_recon_full<__half>, cells_grid(d.N), dim3(256), 0, s, d);
  }
  hipLaunchKernelGGL(k_commit_full, cells_grid(d.N), dim3(256), 0, s, d);
  if (d.P > 0) hipLaunchKernelGGL(k_mbins, gp, dim3(256), 0, s, d, 0, 1);
}

void launch_update_fused(const DevDomain& d, hipStream_t s) {
  const unsigned gp = (unsigned)((d.P + 255) / 256 > 0 ? (d.P + 255) / 256 : 1);
  if (d.P > 0) {
    hipLaunchKernelGGL(k_mbins, dim3(gp), dim3(256), 0, s, d, 1, 0);
    if (d.storage == 0)
      hipLaunchKernelGGL(k_recon_geo<double>, dim3((unsigned)d.P), dim3(GEO_THREADS), 0, s, d);
    else if (d.storage == 1)
      hipLaunchKernelGGL(k_recon_geo<float>, dim3((unsigned)d.P), dim3(GEO_THREADS), 0, s, d);
    else
      hipLaunchKernelGGL(k_recon_geo<__half>, dim3((unsigned)d.P), dim3(GEO_THREADS), 0, s, d);
    hipLaunchKernelGGL(k_remap_geo, dim3((unsigned)d.P), dim3(GEO_THREADS), 0, s, d);
  }
  hipLaunchKernelGGL(k_advance_fused, dim3(gp), dim3(256), 0, s, d);
}

// ---- mapping update and boundary values ------------------------------------
// Slab pass (few spheres): claims, then reconstruction and the commit with
// the boundary values from the claims.  Ball pass (many spheres): the
// geometric update of flags and owners (the kernels above, from the mapping
// bins), then the boundary values from the flags and owners.

void launch_map_prepare(const DevDomain& d, bool lists, hipStream_t s) {
  if (!d.map_ball) {
    launch_claim(d, 1, lists, s);
    return;
  }
  const unsigned gp = (unsigned)((d.P + 255) / 256 > 0 ? (d.P + 255) / 256 : 1);
  if (d.P > 0) hipLaunchKernelGGL(k_mbins, dim3(gp), dim3(256), 0, s, d, 1, 0);
}

template <typename T>
static void launch_update_t(const DevDomain& d, bool reconstruct, int in_step, int advance, hipStream_t s) {
  const int nsb = d.P * d.ZB;
  if (nsb <= 0) {
    if (advance) launch_advance(d, s);
    return;
  }
  if (d.map_ball) {
    // inside a step: reconstruction and the flags and owners of the new
    // positions (outside, launch_mapping has updated them)
    if (in_step) {
      if (reconstruct) hipLaunchKernelGGL(k_recon_geo<T>, dim3((unsigned)d.P), dim3(GEO_THREADS), 0, s, d);
      hipLaunchKernelGGL(k_remap_geo, dim3((unsigned)d.P), dim3(GEO_THREADS), 0, s, d);
    }
  } else if (reconstruct) {
    hipLaunchKernelGGL(k_recon<T>, dim3(nsb), dim3(256), 0, s, d, in_step);
  }
  // The step control rides on the last block only where the launch has few
  // blocks: the count of finished blocks is one device-wide atomic per block,
  // which costs more than the saved launch once there are thousands.
  const int blocks = d.map_ball ? xcd_grid(d.P) : nsb * d.RB;
  const int fold = advance && blocks <= FOLD_ADVANCE_MAX_BLOCKS;
  if (d.map_ball) {
    hipLaunchKernelGGL(k_commit_ball<T>, dim3(blocks), dim3(BALL_THREADS), ball_lds_bytes(d.stage_edge, d.list_cap), s, d,
                       in_step, fold);
  } else {
    hipLaunchKernelGGL(k_commit<T>, dim3(blocks), dim3(256), 0, s, d, in_step, fold);
  }
  if (advance && !fold) launch_advance(d, s);
}

static void launch_update_any(const DevDomain& d, bool reconstruct, int in_step, int advance, hipStream_t s) {
  if (d.storage == 0)
    launch_update_t<double>(d, reconstruct, in_step, advance, s);
  else if (d.storage == 1)
    launch_update_t<float>(d, reconstruct, in_step, advance, s);
  else
    launch_update_t<__half>(d, reconstruct, in_step, advance, s);
}

void launch_update_and_advance(const DevDomain& d, hipStream_t s) { launch_update_any(d, true, 1, 1, s); }

void launch_mapping(const DevDomain& d, bool reconstruct, hipStream_t s) {
  if (d.map_ball) {
    launch_mapping_geo(d, reconstruct, s);
    launch_update_any(d, false, 0, 0, s);
  } else {
    launch_claim(d, 0, false, s);
    launch_update_any(d, reconstruct, 0, 0, s);
  }
  hipLaunchKernelGGL(k_new_stamp, dim3(1), dim3(1), 0, s, d.ctl);
}

// ---- batched mapping update (slab blocks; one launch per kernel for all domains)

__global__ __launch_bounds__(256) void k_claim_batch(const DevDomain* __restrict__ tab, const int* __restrict__ start,
                                                     int ndom) {
  const int k = batch_domain(start, ndom, (int)blockIdx.x);
  const DevDomain& d = tab[k];
  if (!step_live(d.ctl)) return;
  claim_block(d, (int)blockIdx.x - start[k], map_stamp(d.ctl), false);
}

template <typename T>
__global__ __launch_bounds__(256) void k_recon_batch(const DevDomain* __restrict__ tab, const int* __restrict__ start,
                                                     int ndom) {
  const int k = batch_domain(start, ndom, (int)blockIdx.x);
  const DevDomain& d = tab[k];
  if (!step_live(d.ctl)) return;
  recon_block<T>(d, (int)blockIdx.x - start[k], map_buffer(d.ctl, 1), map_stamp(d.ctl));
}

template <typename T>
__global__ __launch_bounds__(256) void k_commit_batch(const DevDomain* __restrict__ tab, const int* __restrict__ start,
                                                      int ndom) {
  const int k = batch_domain(start, ndom, (int)blockIdx.x);
  const DevDomain& d = tab[k];
  if (!step_live(d.ctl)) return;
  commit_block<T>(d, (int)blockIdx.x - start[k], map_buffer(d.ctl, 1), map_stamp(d.ctl));
}

void launch_claim_batch(const BatchTables& b, hipStream_t s) {
  if (b.claim_blocks > 0)
    hipLaunchKernelGGL(k_claim_batch, dim3(b.claim_blocks), dim3(256), 0, s, b.tab, b.claim_start, b.ndom);
}

template <typename T>
static void launch_update_batch_t(const BatchTables& b, hipStream_t s) {
  if (b.claim_blocks > 0)
    hipLaunchKernelGGL(k_recon_batch<T>, dim3(b.claim_blocks), dim3(256), 0, s, b.tab, b.claim_start, b.ndom);
  if (b.commit_blocks > 0)
    hipLaunchKernelGGL(k_commit_batch<T>, dim3(b.commit_blocks), dim3(256), 0, s, b.tab, b.commit_start, b.ndom);
}

void launch_update_batch(const BatchTables& b, hipStream_t s) {
  if (b.storage == 0)
    launch_update_batch_t<double>(b, s);
  else if (b.storage == 1)
    launch_update_batch_t<float>(b, s);
  else
    launch_update_batch_t<__half>(b, s);
}

}  // namespace lbmdem
