// Fused D3Q19 pull stream + TRT+aB collide (Eqs. LBM_Stream, LBM_Collide, MRT
// with the rates of Eqs. TRTmatrix / TRTbulkmatrix, adaptive shell of Sec. 2.3.2).
//
// One thread per cell, one block per whole x-row group where rows are at most
// 256 cells (512 at FP16), so that the +-1 x-shifted loads of a row stay
// inside the block and every source value is fetched from HBM once (wider
// rows are split into pieces; the x-shifted loads then fetch one shared line
// per piece twice).  The PDF slots of solid cells carry the boundary
// values of the particle links that stream out of them (written by the
// boundary kernel), so a fluid cell pulls 19 values without branching.  Wall
// layers are fixed, so the sweep knows from the cell's coordinates which
// values come from a wall: a cell next to a wall layer replaces them by the
// moving-wall bounce-back value f~_qbar(x) + 6 w_q (u_w . c_q) of Sec. 2.2
// (half-way walls), formed from its own post-collision values.  For z walls
// that is a branch uniform over a block (a block lies in one z plane).
// Solid and wall cells are updated like fluid cells: their results are never
// read (the boundary kernel rewrites every slot a fluid cell pulls from a
// solid cell), and letting every lane load and store keeps each wavefront's
// accesses whole cache lines (lanes that skipped their cell made partial-line
// writes, which cost a quarter of the bandwidth in a 16 % solid suspension).
//
// Collision in deviation variables g = f - w_q:
//   TRT in velocity space: g~_q = g_q - s+ (g+_q - e+_q) - s- (g-_q - e-_q),
//   which equals M^-1 S_TRT (m^eq - M f) because the moment rows of App. A are
//   each even or odd under q -> q-bar; plus, for rows 5 and 6 of M (kinetic
//   energy and its square), the rank-2 correction
//   w_q (s_b - s+) [M_4q (m4eq - m4)/N_4 + M_5q (m5eq - m5)/N_5]
//   with N_4 = 2/3, N_5 = 2 (M^-1 = W M^T diag(1/N)).  s_b is the TRT+B rate
//   in shell cells (TRT+aB), everywhere (TRT+B), or s+ (TRT, SRT).
#include "collide.hpp"

namespace lbmdem {

// one domain: tiles of whole x-rows, or of row pieces on wide lattices (see
// launch_sweep_t), gx x gy tiles per z plane, x fastest; with `chunk` each
// XCD takes a contiguous run of tiles; the current buffer is read from the
// domain's step state
constexpr int SWEEP_MAX_THREADS = 512;

template <typename T, bool FORCED, bool NTLOAD>
__global__ __launch_bounds__(SWEEP_MAX_THREADS) void k_sweep(DevDomain d, int gx, int gy, int chunk) {
  using C = typename Store<T>::C;
  if (!step_live(d.ctl)) return;
  const int t = chunk ? xcd_tile((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  const int bx = t % gx, r = t / gx, by = r % gy, z = r / gy;
  if (z >= d.nz) return;
  const int cur = d.ctl->cur;
  const int x = bx * blockDim.x + threadIdx.x;
  const int y = by * blockDim.y + threadIdx.y;
  if (x >= d.nx || y >= d.ny) return;
  // (selects, not an index: a run-time index into the by-value argument would
  // place the whole descriptor in scratch memory)
  const T* src = (const T*)(cur ? d.pdf[1] : d.pdf[0]);
  T* dst = (T*)(cur ? d.pdf[0] : d.pdf[1]);
  sweep_cell<T, FORCED, NTLOAD>(d, src, dst, x, y, z, (C)d.s_plus, (C)d.s_minus,
                        (C)(d.s_bulk_shell - d.s_plus), (C)(d.s_bulk_other - d.s_plus));
}

// many domains in one launch: block b belongs to the domain k with
// start[k] <= b < start[k+1] and covers 256 consecutive cells of it
template <typename T>
__global__ __launch_bounds__(256) void k_sweep_batch(const DevDomain* __restrict__ tab,
                                                     const int* __restrict__ start, int ndom) {
  using C = typename Store<T>::C;
  const int k = batch_domain(start, ndom, (int)blockIdx.x);
  const DevDomain& d = tab[k];
  if (!step_live(d.ctl)) return;
  const long long c = (long long)(blockIdx.x - start[k]) * 256 + threadIdx.x;
  if (c >= d.N) return;
  const int x = (int)(c % d.nx), y = (int)((c / d.nx) % d.ny), z = (int)(c / ((long long)d.nx * d.ny));
  const int cur = d.ctl->cur;
  const T* src = (const T*)d.pdf[cur];
  T* dst = (T*)d.pdf[cur ^ 1];
  if (d.forced)  // uniform over the block (one domain)
    sweep_cell<T, true>(d, src, dst, x, y, z, (C)d.s_plus, (C)d.s_minus, (C)(d.s_bulk_shell - d.s_plus),
                        (C)(d.s_bulk_other - d.s_plus));
  else
    sweep_cell<T, false>(d, src, dst, x, y, z, (C)d.s_plus, (C)d.s_minus, (C)(d.s_bulk_shell - d.s_plus),
                         (C)(d.s_bulk_other - d.s_plus));
}

template <typename T>
static void launch_sweep_t(const DevDomain& d, hipStream_t s) {
  dim3 block, grid;
  if (d.nx <= 256 || (d.nx <= SWEEP_MAX_THREADS && d.nx * sizeof(T) <= 1024)) {
    // whole rows per block: the periodic x-wrap stays inside the block (a
    // 512-wide FP16 row in one block: 1.92 against 2.06 ms in 128 x 2 pieces
    // at 512^3; 384- and 512-wide FP32 rows were slower whole)
    block.x = d.nx;
    block.y = d.nx <= 256 ? 256 / d.nx : 1;
  } else {
    // the widest piece of 256 or 128 cells that divides the row: 256 x 1 at
    // 512^3 FP32 (3.80 against 3.99 ms alone with 128 x 2 and 4.00 ms with
    // whole 512-cell rows), 128 x 2 for 384-wide rows (1.55 ms; whole rows
    // 1.63 ms)
    const int cand[4] = {256, 128, 192, 64};
    block.x = 256;
    for (int c : cand)
      if (d.nx % c == 0) {
        block.x = c;
        break;
      }
    block.y = 256 / block.x;
  }
  block.z = 1;
  const int gx = (d.nx + block.x - 1) / block.x, gy = (d.ny + block.y - 1) / block.y;
  // Tile order, measured: rows of up to 256 cells, contiguous runs of tiles
  // per XCD (122.5 against 125.6 us at 128x128x256); wider rows, plain order
  // (1.56 against 1.63 ms at 384^3 FP32, 1.92 against 1.98 ms at 512^3 FP16)
  const int chunk = d.nx <= 256 ? 1 : 0;
  const int tiles = gx * gy * d.nz;
  grid = dim3(chunk ? xcd_grid(tiles) : tiles);
  // Each source value is read once, and for rows of up to 256 cells
  // non-temporal loads keep the streamed PDFs from displacing other data in
  // the caches (128x128x256: 156.3 against 160.3 us per coupled step at FP32,
  // 111.3 against 116.4 at FP16).  Wider rows share lines between blocks (rows
  // in pieces) or between the waves of a row (512-cell FP16 rows), and the
  // second read needs the line still cached (non-temporal: 1.66 against
  // 1.56 ms at 384^3 FP32, 1.97 against 1.91 ms at 512^3 FP16).
  const bool nt = d.nx <= 256;
  if (d.forced) {
    if (nt)
      hipLaunchKernelGGL((k_sweep<T, true, true>), grid, block, 0, s, d, gx, gy, chunk);
    else
      hipLaunchKernelGGL((k_sweep<T, true, false>), grid, block, 0, s, d, gx, gy, chunk);
  } else {
    if (nt)
      hipLaunchKernelGGL((k_sweep<T, false, true>), grid, block, 0, s, d, gx, gy, chunk);
    else
      hipLaunchKernelGGL((k_sweep<T, false, false>), grid, block, 0, s, d, gx, gy, chunk);
  }
}

void launch_sweep(const DevDomain& d, hipStream_t s) {
  if (d.storage == 0)
    launch_sweep_t<double>(d, s);
  else if (d.storage == 1)
    launch_sweep_t<float>(d, s);
  else
    launch_sweep_t<__half>(d, s);
}

void launch_sweep_batch(const BatchTables& b, hipStream_t s) {
  if (b.sweep_blocks <= 0) return;
  if (b.storage == 0)
    hipLaunchKernelGGL(k_sweep_batch<double>, dim3(b.sweep_blocks), dim3(256), 0, s, b.tab, b.sweep_start, b.ndom);
  else if (b.storage == 1)
    hipLaunchKernelGGL(k_sweep_batch<float>, dim3(b.sweep_blocks), dim3(256), 0, s, b.tab, b.sweep_start, b.ndom);
  else
    hipLaunchKernelGGL(k_sweep_batch<__half>, dim3(b.sweep_blocks), dim3(256), 0, s, b.tab, b.sweep_start, b.ndom);
}

}  // namespace lbmdem
