// Fused sweep of many-sphere domains: the particle-link boundary conditions
// (Eq. MEM_CLI, with bounce-back where the second fluid node is missing, Sec.
// 2.2) and the momentum exchange (Eqs. MEM_Fq, interaction_force,
// interaction_torque, plus 2 w_q c_q for missing links) are formed inside the
// stream-collide sweep of Alg. 1, from the post-collision values the sweep
// reads anyway, instead of by a separate pass over the spheres' surfaces.
//
// One block per tile of fbx x fby cells in one z plane:
//   1. the cell words (flag byte and owner) of the tile and a one-cell halo
//      are staged in LDS, row by row;
//   2. every fluid cell lists its links (directions q whose cell x + c_q is
//      solid) and every solid cell its missing links (y - c_q a wall or another
//      sphere's solid); the spheres they belong to form the tile's table;
//   3. the links are numbered by ordered compaction (cell order, then q) and
//      processed in rounds of FT_ROUND, one link per thread, with all loads of
//      a round in flight together: the boundary value f_qbar(x, t+1) of Eq.
//      (MEM_CLI) from f~_q(x), f~_qbar(x) and f~_q(x - c_q), its force and the
//      torque about the sphere centre, all in FP64 with the arithmetic of the
//      sphere-centric boundary pass;
//   4. the forces and torques of the tile are summed per sphere exactly (an
//      order-independent fixed-point sum, see fx_add) and stored, stamped with
//      the step, in the sphere's slot for this tile; k_force_reduce sums a
//      sphere's slots in slot order;
//   5. each cell replaces the values it pulled from solid cells by its
//      boundary values (rounded to the storage type, as if stored and
//      reloaded) and collides as in the plain sweep.
// The values pulled from solid cells are never used, so solid cells' slots
// need no boundary values, and nothing but this kernel reads the links.
#include "collide.hpp"

namespace lbmdem {

constexpr int FT_THREADS = 256;                 // cells per tile (fbx * fby)
constexpr int FT_HALO_MAX = (256 + 2) * 3 * 3;  // staged cells of the widest tile
constexpr int FT_TABLE = 48;                    // spheres one tile can meet
constexpr int FT_HASH = 128;                    // open-addressing table of their ids
constexpr int FT_ROUND = 128;                   // links per round

// compile-time copies of the velocity set (unrolled loops index registers)
constexpr int KCX[Q] = {0, 0, 0, -1, 1, 0, 0, -1, 1, -1, 1, 0, 0, -1, 1, 0, 0, -1, 1};
constexpr int KCY[Q] = {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, -1, 0, 0, 1, -1, 0, 0};
constexpr int KCZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1};
constexpr int KOPP[Q] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 16, 15, 18, 17, 12, 11, 14, 13};

// the velocity set packed into constants (no memory access for a per-lane q):
// c_q + 1 in two bits per axis, the opposite direction in five bits
constexpr unsigned long long pack_c(const int* c) {
  unsigned long long v = 0;
  for (int q = 0; q < Q; ++q) v |= (unsigned long long)(c[q] + 1) << (2 * q);
  return v;
}
constexpr unsigned long long PCX = pack_c(KCX), PCY = pack_c(KCY), PCZ = pack_c(KCZ);
constexpr unsigned long long pack_opp(int lo) {
  unsigned long long v = 0;
  for (int q = lo; q < lo + 12 && q < Q; ++q) v |= (unsigned long long)KOPP[q] << (5 * (q - lo));
  return v;
}
constexpr unsigned long long POPP0 = pack_opp(0), POPP1 = pack_opp(12);
__device__ __forceinline__ int cq_of(unsigned long long pk, int q) { return (int)((pk >> (2 * q)) & 3ull) - 1; }
__device__ __forceinline__ int opp_of(int q) {
  return q < 12 ? (int)((POPP0 >> (5 * q)) & 31ull) : (int)((POPP1 >> (5 * (q - 12))) & 31ull);
}

// the value the plain sweep would pull after the boundary pass stored v
template <typename T>
__device__ __forceinline__ typename Store<T>::C stored_value(double v);
template <>
__device__ __forceinline__ double stored_value<double>(double v) { return v; }
template <>
__device__ __forceinline__ float stored_value<float>(double v) { return (float)v; }
template <>
__device__ __forceinline__ float stored_value<__half>(double v) { return __half2float(__float2half_rn((float)v)); }

template <typename T>
__device__ __forceinline__ double load_d(const T* p);
template <>
__device__ __forceinline__ double load_d<double>(const double* p) { return *p; }
template <>
__device__ __forceinline__ double load_d<float>(const float* p) { return (double)*p; }
template <>
__device__ __forceinline__ double load_d<__half>(const __half* p) { return (double)__half2float(*p); }

// table slot of sphere o (inserted before)
__device__ __forceinline__ int tile_slot(const int* hkey, const int* hslot, int o) {
  for (int k = 0; k < FT_HASH; ++k) {
    const int h = (o + k) & (FT_HASH - 1);
    if (hkey[h] == o) return hslot[h];
    if (hkey[h] < 0) break;
  }
  return -1;
}

__device__ __forceinline__ void tile_insert(int* hkey, int o, int* err) {
  for (int k = 0; k < FT_HASH; ++k) {
    const int h = (o + k) & (FT_HASH - 1);
    const int prev = atomicCAS(&hkey[h], -1, o);
    if (prev == -1 || prev == o) return;
  }
  *err = 1;
}

// position of the tile (tile indices bx, by, plane z) in the link box of a
// sphere centred at xs with radius R (box origin floor(x - R - 2.5) per axis,
// not below the first layer on an axis with walls), or -1 if it lies outside
__device__ __forceinline__ int slot_index(const DevDomain& d, const double* xs, double R, int bx, int by, int z) {
  int rel[3];
  const int t[3] = {bx, by, z};
  const int tiles[3] = {d.fgx, d.fgy, d.nz};
  const int edge[3] = {d.fbx, d.fby, 1};
  const int cap[3] = {d.sl_nx, d.sl_ny, d.sl_nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int lo = (int)floor(xs[a] - R - 2.5);
    if (d.walls[a] && lo < 0) lo = 0;
    const int tl = lo >= 0 ? lo / edge[a] : -((-lo + edge[a] - 1) / edge[a]);
    int r = t[a] - tl;
    if (!d.walls[a]) r = wrapmod(r, tiles[a]);
    if (r < 0 || r >= cap[a]) return -1;
    rel[a] = r;
  }
  return (rel[2] * d.sl_ny + rel[1]) * d.sl_nx + rel[0];
}

// Tile partials are accumulated exactly, in any order: each value v is split
// into h = rint(v 2^30) and l = rint((v - h 2^-30) 2^80) (the subtraction is
// exact), and the two integer parts are summed with 64-bit LDS atomics.  The
// partial is the exact sum of the values rounded to 2^-81, rounded once to
// FP64: deterministic, and at least as accurate as a sequential FP64 sum.
__device__ __forceinline__ void fx_add(unsigned long long* hi, unsigned long long* lo, double v) {
  const double h = rint(v * 0x1p30);
  const double l = rint((v - h * 0x1p-30) * 0x1p80);
  atomicAdd(hi, (unsigned long long)(long long)h);
  atomicAdd(lo, (unsigned long long)(long long)l);
}
__device__ __forceinline__ double fx_value(unsigned long long hi, unsigned long long lo) {
  return (double)(long long)hi * 0x1p-30 + (double)(long long)lo * 0x1p-80;
}

// cell word of the fused step: flag byte | (owner + 1) << 8
constexpr uint32_t CW_WALL = F_WALL;
__device__ __forceinline__ int cw_owner(uint32_t w) { return (int)(w >> 8) - 1; }

// (at most 128 VGPRs: four waves per SIMD)
template <typename T, bool FORCED>
__global__ __launch_bounds__(FT_THREADS) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_sweep_fused(DevDomain d) {
  using C = typename Store<T>::C;
  __shared__ uint32_t swd[FT_HALO_MAX];
  __shared__ int hkey[FT_HASH], hslot[FT_HASH];
  __shared__ int tab_id[FT_TABLE];
  __shared__ double tab[FT_TABLE][10];  // x (3), R, u (3), w (3)
  __shared__ unsigned long long fxh[FT_TABLE][6], fxl[FT_TABLE][6];
  __shared__ uint32_t lk[FT_ROUND];
  __shared__ double lval[FT_ROUND];
  __shared__ double lres[6][FT_ROUND];
  __shared__ int lslot[FT_ROUND];
  __shared__ int wsum[FT_THREADS / 64];
  __shared__ int s_ntab, s_err;

  if (!step_live(d.ctl)) return;  // uniform over the grid
  const int BX = (int)blockDim.x, BY = (int)blockDim.y, nthr = BX * BY;
  const int tx = (int)threadIdx.x, ty = (int)threadIdx.y;
  const int tid = tx + BX * ty;
  const int lane = tid & 63, wid = tid >> 6, nw = (nthr + 63) >> 6;
  const int tl = (int)blockIdx.x;
  const int bx = tl % d.fgx, rr = tl / d.fgx, by = rr % d.fgy, z = rr / d.fgy;
  const int x0 = bx * BX, y0 = by * BY;
  const int x = x0 + tx, y = y0 + ty;
  const bool in = x < d.nx && y < d.ny;
  const int HX = BX + 2, HY = BY + 2;
  const int cur = d.ctl->cur;
  const uint32_t stamp = d.ctl->stamp;
  const T* src = (const T*)(cur ? d.pdf[1] : d.pdf[0]);
  T* dst = (T*)(cur ? d.pdf[0] : d.pdf[1]);
  const size_t N = (size_t)d.N;
  const unsigned int idx = in ? (unsigned int)cidx(d, x, y, z) : 0u;

  // the cell's own pulls (walls replaced), in flight while the links are formed
  C g[Q];
  if (in) pull_cell<T, false>(d, src, x, y, z, idx, g);

  for (int h = tid; h < FT_HASH; h += nthr) hkey[h] = -1;
  for (int k = tid; k < FT_TABLE * 6; k += nthr) {
    (&fxh[0][0])[k] = 0ull;
    (&fxl[0][0])[k] = 0ull;
  }
  if (tid == 0) {
    s_ntab = 0;
    s_err = 0;
  }

  // 1. cell words of the tile and a one-cell halo, row by row (cells beyond a
  // wall layer count as wall; periodic axes wrap)
  {
    const int xi = x0 + tx;  // interior column of this thread
    const bool xin = xi < d.nx;
    const int xe = tx == 0 ? x0 - 1 : x0 + BX;  // edge columns (threads 0 and 1)
    int xew = xe;
    bool xeo = false;
    if (xe < 0 || xe >= d.nx) {
      if (d.walls[0]) xeo = true;
      else xew = wrapmod(xe, d.nx);
    }
    int xiw = xi;
    bool xio = false;
    if (!xin) {
      if (d.walls[0]) xio = true;
      else xiw = wrapmod(xi, d.nx);
    }
    // row r = hy + HY hz of the halo: thread row ty takes r = ty, ty + BY, ...
    int hy = ty, hz = 0;
    while (hy >= HY) {
      hy -= HY;
      ++hz;
    }
    for (; hz < 3;) {
      int gy = y0 - 1 + hy, gz = z - 1 + hz;
      const bool rowout = (d.walls[1] && (gy < 0 || gy >= d.ny)) || (d.walls[2] && (gz < 0 || gz >= d.nz));
      if (gy < 0) gy += d.ny;
      else if (gy >= d.ny) gy = gy - d.ny < d.ny ? gy - d.ny : wrapmod(gy, d.ny);
      gz = wrapi(gz, d.nz);
      const size_t rb = ((size_t)gz * d.ny + gy) * d.nx;
      const int hb = HX * (hy + HY * hz);
      swd[hb + tx + 1] = (rowout || xio) ? CW_WALL : d.cellw[rb + xiw];
      if (tx < 2) swd[hb + (tx == 0 ? 0 : BX + 1)] = (rowout || xeo) ? CW_WALL : d.cellw[rb + xew];
      hy += BY;
      while (hy >= HY) {
        hy -= HY;
        ++hz;
      }
    }
  }
  __syncthreads();

  // 2. the cell's links: fluid cell -> directions q with x + c_q solid;
  // solid cell -> missing links (y - c_q a wall or another sphere's solid)
  const int hc = (tx + 1) + HX * ((ty + 1) + HY);
  const uint32_t wc = in ? swd[hc] : CW_WALL;
  uint32_t mask = 0u;
  const bool fluid = in && !(wc & (F_SOLID | F_WALL));
  if (fluid) {
    int last = -1;
#pragma unroll
    for (int q = 1; q < Q; ++q) {
      const uint32_t wy = swd[hc + KCX[q] + HX * (KCY[q] + HY * KCZ[q])];
      if (wy & F_SOLID) {
        mask |= 1u << q;
        const int o = cw_owner(wy);
        if (o != last && o >= 0 && o < d.P) tile_insert(hkey, o, &s_err);
        last = o;
      }
    }
  } else if (in && (wc & F_SOLID)) {
    const int own = cw_owner(wc);
#pragma unroll
    for (int q = 1; q < Q; ++q) {
      const uint32_t wz = swd[hc - (KCX[q] + HX * (KCY[q] + HY * KCZ[q]))];
      if ((wz & F_WALL) || ((wz & F_SOLID) && cw_owner(wz) != own)) mask |= 1u << q;
    }
    if (mask && own >= 0 && own < d.P) tile_insert(hkey, own, &s_err);
  }
  __syncthreads();

  // the tile's table of spheres (compaction of the hash by one wavefront)
  if (wid == 0) {
    int count = 0;
    for (int base = 0; base < FT_HASH; base += 64) {
      const int h = base + lane;
      const bool v = hkey[h] >= 0;
      const unsigned long long m = __ballot(v);
      if (v) {
        const int s = count + __popcll(m & ((1ull << lane) - 1ull));
        hslot[h] = s < FT_TABLE ? s : -1;
        if (s < FT_TABLE) tab_id[s] = hkey[h];
      }
      count += __popcll(m);
    }
    if (lane == 0) {
      s_ntab = count < FT_TABLE ? count : FT_TABLE;
      if (count > FT_TABLE) s_err = 1;
    }
  }
  // ordered numbering of the links: wavefront scan, then across wavefronts
  const int cnt = __popc(mask);
  int v = cnt;
  for (int o = 1; o < 64; o <<= 1) {
    const int w = __shfl_up(v, o, 64);
    if (lane >= o) v += w;
  }
  if (lane == 63 || tid == nthr - 1) wsum[wid] = v;
  __syncthreads();
  int off = v - cnt, total = 0;
  for (int w = 0; w < nw; ++w) {
    if (w < wid) off += wsum[w];
    total += wsum[w];
  }
  const int ntab = s_ntab;
  if (s_err) {
    if (tid == 0) atomicOr(d.status, ST_TILE_FULL);
    total = 0;  // uniform: the results of this step are void (reported at sync)
  }
  for (int k = tid; k < ntab * 10; k += nthr) {
    const int s = k / 10, c = k % 10, i = tab_id[s];
    tab[s][c] = c < 3 ? d.p.x[3 * i + c] : (c == 3 ? d.p.R[i] : (c < 7 ? d.p.u[3 * i + c - 4] : d.p.w[3 * i + c - 7]));
  }

  // 3./4. link rounds
  const bool solid_cell = !fluid;
  for (int r0 = 0; r0 < total; r0 += FT_ROUND) {
    __syncthreads();  // previous round's buffers are free; the table is loaded
    if (cnt && off < r0 + FT_ROUND && off + cnt > r0) {
      int e = off;
#pragma unroll
      for (int q = 1; q < Q; ++q)
        if (mask & (1u << q)) {
          if (e >= r0 && e < r0 + FT_ROUND)
            lk[e - r0] = (uint32_t)tx | ((uint32_t)ty << 9) | ((uint32_t)q << 18) | (solid_cell ? (1u << 23) : 0u);
          ++e;
        }
    }
    __syncthreads();
    const int nr = min(FT_ROUND, total - r0);
    if (tid < nr) {
      const uint32_t e = lk[tid];
      const int ctx = (int)(e & 511u), cty = (int)((e >> 9) & 511u), q = (int)((e >> 18) & 31u);
      const bool missing = (e >> 23) & 1u;
      const int cxx = x0 + ctx, cyy = y0 + cty;
      const int hcc = (ctx + 1) + HX * ((cty + 1) + HY);
      const int c[3] = {cq_of(PCX, q), cq_of(PCY, q), cq_of(PCZ, q)};
      const int offq = c[0] + HX * (c[1] + HY * c[2]);
      const double wq = c[0] * c[0] + c[1] * c[1] + c[2] * c[2] == 1 ? 1.0 / 18 : 1.0 / 36;
      const int s = tile_slot(hkey, hslot, cw_owner(missing ? swd[hcc] : swd[hcc + offq]));
      lslot[tid] = s;
      if (s >= 0) {
        const double xp[3] = {tab[s][0], tab[s][1], tab[s][2]};
        double Fq[3], arm[3];
        if (!missing) {
          const double R = tab[s][3];
          const double up[3] = {tab[s][4], tab[s][5], tab[s][6]}, wp[3] = {tab[s][7], tab[s][8], tab[s][9]};
          const size_t cc = (size_t)cidx(d, cxx, cyy, z);
          const int qb = opp_of(q);
          const bool cli = d.boundary == 0 && !(swd[hcc - offq] & (F_SOLID | F_WALL));
          const T gq = src[(size_t)q * N + cc];
          const T gqb = src[(size_t)qb * N + cc];
          T gm = (T)0.0f;
          if (cli) {
            // x - c_q is fluid, so it is no wall cell and lies in range
            const size_t cm =
                (size_t)cidx(d, wrapi(cxx - c[0], d.nx), wrapi(cyy - c[1], d.ny), wrapi(z - c[2], d.nz));
            gm = src[(size_t)q * N + cm];
          }
          double r[3];
          r[0] = min_image(((double)cxx + 0.5) - xp[0], d.nx, d.walls[0]);
          r[1] = min_image(((double)cyy + 0.5) - xp[1], d.ny, d.walls[1]);
          r[2] = min_image(((double)z + 0.5) - xp[2], d.nz, d.walls[2]);
          const double dl = link_delta(r, c, R);
          for (int a = 0; a < 3; ++a) arm[a] = r[a] + dl * c[a];
          double ub[3];
          ub[0] = up[0] + (wp[1] * arm[2] - wp[2] * arm[1]);
          ub[1] = up[1] + (wp[2] * arm[0] - wp[0] * arm[2]);
          ub[2] = up[2] + (wp[0] * arm[1] - wp[1] * arm[0]);
          const double dd = cli ? dl : 0.5;
          const double vq = load_d<T>(&gq);
          double val = vq;
          if (cli) val += (1.0 - 2.0 * dd) / (1.0 + 2.0 * dd) * (load_d<T>(&gm) - load_d<T>(&gqb));
          val -= 4.0 / (1.0 + 2.0 * dd) * wq * 3.0 * (ub[0] * c[0] + ub[1] * c[1] + ub[2] * c[2]);
          lval[tid] = val;
          const double fq = vq + wq, fb = val + wq;
          for (int a = 0; a < 3; ++a) Fq[a] = (c[a] - ub[a]) * fq - (-c[a] - ub[a]) * fb;
        } else {
          for (int a = 0; a < 3; ++a) Fq[a] = 2.0 * wq * c[a];
          arm[0] = min_image(((double)cxx + 0.5) - xp[0], d.nx, d.walls[0]) - 0.5 * c[0];
          arm[1] = min_image(((double)cyy + 0.5) - xp[1], d.ny, d.walls[1]) - 0.5 * c[1];
          arm[2] = min_image(((double)z + 0.5) - xp[2], d.nz, d.walls[2]) - 0.5 * c[2];
        }
        lres[0][tid] = Fq[0];
        lres[1][tid] = Fq[1];
        lres[2][tid] = Fq[2];
        lres[3][tid] = arm[1] * Fq[2] - arm[2] * Fq[1];
        lres[4][tid] = arm[2] * Fq[0] - arm[0] * Fq[2];
        lres[5][tid] = arm[0] * Fq[1] - arm[1] * Fq[0];
      }
    }
    __syncthreads();
    // each cell sums its own links of the round (usually all of one sphere)
    // and adds the sums to the tile accumulators (exact, so any grouping
    // gives the same bits)
    if (cnt && off < r0 + nr && off + cnt > r0) {
      const int e0 = max(off, r0) - r0, e1 = min(off + cnt, r0 + nr) - r0;
      int sa = -1;
      double a[6] = {0, 0, 0, 0, 0, 0};
      for (int e = e0; e < e1; ++e) {
        const int se = lslot[e];
        if (se < 0) continue;
        if (se != sa) {
          if (sa >= 0)
            for (int k = 0; k < 6; ++k) fx_add(&fxh[sa][k], &fxl[sa][k], a[k]);
          sa = se;
          for (int k = 0; k < 6; ++k) a[k] = 0.0;
        }
        for (int k = 0; k < 6; ++k) a[k] += lres[k][e];
      }
      if (sa >= 0)
        for (int k = 0; k < 6; ++k) fx_add(&fxh[sa][k], &fxl[sa][k], a[k]);
    }
    // the cell's boundary values of this round replace its pulls from solids
    if (fluid && off < r0 + FT_ROUND && off + cnt > r0) {
      int e = off;
#pragma unroll
      for (int q = 1; q < Q; ++q)
        if (mask & (1u << q)) {
          if (e >= r0 && e < r0 + nr) g[KOPP[q]] = stored_value<T>(lval[e - r0]);
          ++e;
        }
    }
  }

  // the tile's partial of each sphere into that sphere's slot for this tile
  // (after every cell's sums have reached the accumulators)
  __syncthreads();
  for (int j = tid; j < 6 * ntab && total > 0; j += nthr) {
    const int s = j / 6, comp = j % 6, i = tab_id[s];
    const double xs[3] = {tab[s][0], tab[s][1], tab[s][2]};
    const int sl = slot_index(d, xs, tab[s][3], bx, by, z);
    if (sl < 0) {
      atomicOr(d.status, ST_TILE_FULL);
      continue;
    }
    d.slot[((size_t)i * d.sl_per + sl) * 6 + comp] = fx_value(fxh[s][comp], fxl[s][comp]);
    if (comp == 0) d.slot_stamp[(size_t)i * d.sl_per + sl] = stamp;
  }

  // 5. collide and store (every cell, so that wavefronts write whole lines)
  if (in)
    collide_store<T, FORCED>(d, dst, idx, (uint8_t)(wc & 0xFFu), g, (C)d.s_plus, (C)d.s_minus,
                             (C)(d.s_bulk_shell - d.s_plus), (C)(d.s_bulk_other - d.s_plus));
}

// Resolved force and torque of each sphere: its tile partials of this step,
// summed in slot order (one wavefront per sphere, fixed-order shuffle tree).
__global__ __launch_bounds__(256) void k_force_reduce(DevDomain d) {
  if (!step_live(d.ctl)) return;
  const int lane = threadIdx.x & 63;
  const int i = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (i >= d.P) return;
  const uint32_t stamp = d.ctl->stamp;
  double F[6] = {0, 0, 0, 0, 0, 0};
  const size_t base = (size_t)i * d.sl_per;
  for (int s = lane; s < d.sl_per; s += 64)
    if (d.slot_stamp[base + s] == stamp)
      for (int k = 0; k < 6; ++k) F[k] += d.slot[(base + s) * 6 + k];
  for (int k = 0; k < 6; ++k) {
    double v = F[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    F[k] = v;
  }
  if (lane == 0)
    for (int k = 0; k < 6; ++k) d.partial[(size_t)i * 6 + k] = F[k];
}

template <typename T>
static void launch_fused_t(const DevDomain& d, hipStream_t s) {
  const dim3 block((unsigned)d.fbx, (unsigned)d.fby);
  const dim3 grid((unsigned)(d.fgx * d.fgy * d.nz));
  if (d.forced)
    hipLaunchKernelGGL((k_sweep_fused<T, true>), grid, block, 0, s, d);
  else
    hipLaunchKernelGGL((k_sweep_fused<T, false>), grid, block, 0, s, d);
}

void launch_sweep_fused(const DevDomain& d, hipStream_t s) {
  if (d.storage == 0)
    launch_fused_t<double>(d, s);
  else if (d.storage == 1)
    launch_fused_t<float>(d, s);
  else
    launch_fused_t<__half>(d, s);
}

void launch_force_reduce(const DevDomain& d, hipStream_t s) {
  if (d.P > 0) hipLaunchKernelGGL(k_force_reduce, dim3((unsigned)((d.P * 64 + 255) / 256)), dim3(256), 0, s, d);
}

}  // namespace lbmdem
