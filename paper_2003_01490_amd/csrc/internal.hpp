// Internal definitions shared by the kernels and the host API of lbmdem.
//
// Device data of one domain (all inside one caller-owned region):
//   pdf[2]      two PDF buffers, q-major planes of N cells, storing f - w_q in
//               the storage type (double / float / half); buffer `cur` holds
//               the post-collision state of the current step.  Slots of solid
//               and wall cells carry the boundary value of the link that
//               streams out of them ("ghost" values written by the boundary
//               kernel), so the sweep pulls all 19 directions unconditionally.
//   flags       uint8 per cell (SOLID / WALL / SHELL bits)
//   owner       int32 per cell, sphere id of solid cells
//   claim       uint64 per cell, (stamp << 32 | ~id) max-claim of the mapping
//   shellstamp  uint32 per cell, stamp of the last mapping that put the cell
//               inside some sphere's TRT+aB shell (both for the slab pass
//               only; null where the mapping bins serve: ball pass, fused
//               step)
//   particle SoA in FP64, per-(sphere, box-slab) force partials, contact
//   history slots, neighbour lists and a device status word.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace lbmdem {

constexpr int Q = 19;
constexpr uint8_t F_SOLID = 1;
constexpr uint8_t F_WALL = 2;
constexpr uint8_t F_SHELL = 4;

constexpr int COMMIT_ROWS = 8;   // y-rows of a box slab per boundary block
constexpr int HIST_SLOTS = 24;   // contact-history slots per sphere
constexpr int NBR_MAX = 48;      // neighbour-list capacity per sphere

constexpr int MODE_FREE = 0;
constexpr int MODE_PRESCRIBED = 1;
constexpr int MODE_FIXED = 2;

// device status bits
constexpr int ST_NONFINITE = 1;
constexpr int ST_HIST_FULL = 2;
constexpr int ST_NBR_FULL = 4;
constexpr int ST_TILE_FULL = 8;   // a fused-sweep tile met more spheres than its table holds
constexpr int ST_DENSITY = 16;    // a sampled fluid density lies outside (0.5, 1.5) or is not finite

constexpr int BIN_CAP = 15;      // sphere ids per neighbour-search bin (+1 count)

// D3Q19 velocities in the order fixed by rows 2-4 of the MRT moment matrix
// (App. A of the paper), weights 1/3, 1/18, 1/36 and opposite directions.
static __constant__ const int CX[Q] = {0, 0, 0, -1, 1, 0, 0, -1, 1, -1, 1, 0, 0, -1, 1, 0, 0, -1, 1};
static __constant__ const int CY[Q] = {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, -1, 0, 0, 1, -1, 0, 0};
static __constant__ const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1};
static __constant__ const int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 16, 15, 18, 17, 12, 11, 14, 13};
static __constant__ const double WQ[Q] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                       1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                       1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                       1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// Step state of a domain, resident on the device so that a step needs no
// per-step kernel arguments (graph replay, batched launches) and a domain can
// stop on the device.  The DEM kernel (run every step, also without spheres)
// advances it after the sweep: cur flips, stamp and steps increase, and the
// stop rule is evaluated; a stop freezes the domain at the start of the next
// step, before its mapping could change (that step's sweep output goes to the
// spare buffer and is dropped).
struct DevCtl {
  uint32_t stamp;     // claims and shell stamps of the current mapping
  int32_t cur;        // PDF buffer holding the current post-collision state
  int32_t frozen;     // 1: every kernel of this domain returns at once
  int32_t stop_req;   // the stop rule was met at the end of the last step
  int64_t steps;      // coupled steps done
  int64_t max_steps;  // stop after this many steps (<= 0: never)
  int32_t stop_rule;  // 0 none, 1 rebound of sphere 0 (first apex after its first wall contact)
  int32_t rb_phase;   // rebound tracking: 0 approach, 1 contact, 2 after contact, 3 rising
  uint32_t done_blocks;  // blocks of the step's last kernel that have finished (see k_commit)
};

// A step's kernels do nothing for a domain that is frozen or whose stop rule
// was met at the end of the last step.
__device__ __forceinline__ bool step_live(const DevCtl* c) { return !c->frozen && !c->stop_req; }

constexpr int STOP_NONE = 0;
constexpr int STOP_REBOUND = 1;

struct DevParticles {
  double* x;      // [P][3] position
  double* u;      // [P][3]
  double* w;      // [P][3]
  double* xmap;   // [P][3] position at the last mapping
  double* R;      // [P]
  double* rho;    // [P]
  double* m;      // [P]
  double* I;      // [P]
  int* mode;      // [P]
  double* presc;  // [P][6]: u_target[3], c_acc, t_st, release_gap
  double* tpresc; // [P] time since the ramp started
  double* Fprev;  // [P][6] previous un-averaged resolved F, T
  int* prev_valid;
  double* Ffp;    // [P][6] averaged resolved F, T of the current step
  double* Fraw;   // [P][6]
  double* Fold;   // [P][6] velocity-Verlet force/torque at time t
  int* old_valid;
  double* diag;   // [P][18] F_tot T_tot F_lub T_lub F_col T_col of the last sub-step
  double* Fnew;   // [P][6] scratch of the current sub-step
  int* hist_id;   // [P][HIST_SLOTS] partner code (sphere id >= 0, wall -1-face), INT_MIN free
  double* hist_d; // [P][HIST_SLOTS][3] tangential spring
  int* nbr;       // [P][NBR_MAX] candidate partners (ascending)
  int* nbr_n;     // [P]
  double* x2;     // [P][3] second buffers of x, u, w: the many-sphere DEM
  double* u2;     //        kernel alternates between the two every sub-cycle
  double* w2;
  int* order;     // [P] sphere ids in space-filling-curve order of their centres
};

// uniform bins of the many-sphere neighbour search: edge >= the largest centre
// distance at which two spheres can be neighbours
struct DevBins {
  int n[3];       // bins per axis
  int* cell;      // [n0 n1 n2][1 + BIN_CAP]: count, then ids
};

struct DevDomain {
  int nx, ny, nz;
  long long N;
  int walls[3];
  double wall_u_lo[3], wall_u_hi[3];
  double force[3];  // fluid body force (Guo forcing)
  int forced;       // force != 0
  int storage;     // 0 f64, 1 f32, 2 f16
  int boundary;    // 0 CLI, 1 BB
  double s_plus, s_minus, s_bulk_shell, s_bulk_other;
  double s_nu;     // shear rate (reconstruction)
  double delta_ab;
  void* pdf[2];
  uint8_t* flags;
  int32_t* owner;
  unsigned long long* claim;
  uint32_t* shellstamp;
  uint32_t* cellw;   // fused step: flag byte | (owner + 1) << 8 per cell (NULL otherwise)
  DevParticles p;
  int P;           // spheres present
  int ZB;          // mapping blocks per sphere along z (slabs)
  int RB;          // row blocks per slab in the boundary kernel
  double* partial; // [P][ZB * RB][6]
  int map_ball;    // boundary pass: 1 one block per sphere (k_commit_ball), 0 slab blocks
  int stage_edge;  // edge of the LDS-staged cube of k_commit_ball (odd)
  int list_cap;    // surface-cell list capacity of k_commit_ball
  int* status;
  DevCtl* ctl;
  // DEM parameters
  int n_sub;
  int force_averaging;
  double gravity[3];
  double e_dry, poisson_ratio, friction, tc, dmin, cut_n, cut_tt, cut_tr;
  int lub_mask;
  double nu;
  double skin;     // neighbour-list skin
  DevBins bins;
  // Fused step: the particle links are formed inside the sweep (tiles of
  // fbx x fby cells, fgx x fgy tiles per plane); each tile leaves one
  // momentum-exchange partial per sphere it touches in that sphere's slot
  // array (slots indexed by the tile's position in the sphere's link box of
  // sl_E cells per axis: sl_nx x sl_ny x sl_nz tiles), stamped with the step.
  // Mapping updates find the spheres around a cell through the mapping bins
  // (edge >= R_max + max(delta_aB, 1) + 1).
  int fused;
  int fbx, fby, fgx, fgy;
  int sl_E, sl_nx, sl_ny, sl_nz, sl_per;
  double* slot;          // [P][sl_per][6]
  uint32_t* slot_stamp;  // [P][sl_per]
  DevBins mbins;
  uint32_t* stage32;     // [N] cell states of a full mapping update (in the stage buffer)
};

__host__ __device__ inline long long cidx(const DevDomain& d, int i, int j, int k) {
  return (long long)i + (long long)d.nx * ((long long)j + (long long)d.ny * (long long)k);
}

__device__ inline int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
// full modulo for indices that may lie more than one period away
__device__ inline int wrapmod(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

// minimum image of a distance component on periodic axes
__device__ inline double min_image(double v, int n, int wall) {
  if (wall) return v;
  double L = (double)n;
  if (v > 0.5 * L) return v - L;
  if (v < -0.5 * L) return v + L;
  return v;
}

// i mod n for i that is almost always within one period of [0, n): one
// conditional wrap, the full modulo only when that does not land in range
__device__ __forceinline__ int wrap_near(int i, int n) {
  if (i < 0)
    i += n;
  else if (i >= n)
    i -= n;
  return (unsigned)i < (unsigned)n ? i : wrapmod(i, n);
}

__device__ inline double cell_d2(const DevDomain& d, int i, int j, int k, const double* xp) {
#pragma clang fp contract(off)
  const double dx = min_image(((double)i + 0.5) - xp[0], d.nx, d.walls[0]);
  const double dy = min_image(((double)j + 0.5) - xp[1], d.ny, d.walls[1]);
  const double dz = min_image(((double)k + 0.5) - xp[2], d.nz, d.walls[2]);
  return (dx * dx + dy * dy) + dz * dz;
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

// Bins along one axis that can hold partners of a sphere in bin b: the three
// around it (wrapped on periodic axes), or every bin when there are fewer than
// three.  Entry e of axis_count(nb) entries; false if it lies beyond a wall.
__device__ __forceinline__ int axis_count(int nb) { return nb < 3 ? nb : 3; }
__device__ __forceinline__ bool axis_bin(int b, int nb, bool wall, int e, int* k) {
  if (nb < 3) {
    *k = e;
    return true;
  }
  int v = b + e - 1;
  if (v < 0 || v >= nb) {
    if (wall) return false;
    v = v < 0 ? v + nb : v - nb;
  }
  *k = v;
  return true;
}

// Device tables of a batch of domains (one launch per kernel for all of them):
// descriptors, and for each kernel the first block of every domain (ndom + 1
// entries, the last one the total).
struct BatchTables {
  const DevDomain* tab;
  const int* sweep_start;
  const int* claim_start;   // P * ZB blocks per domain (claims, reconstruction)
  const int* commit_start;  // P * ZB * RB sphere blocks per domain
  int ndom;
  int sweep_blocks, claim_blocks, commit_blocks;
  int storage;
};

// The hardware hands workgroups to the eight XCDs round-robin by id.  Block
// w of a grid of G blocks (G a multiple of 8) takes tile (w mod 8) G/8 + w/8:
// each XCD works through one contiguous eighth of the tiles, in order, so
// tiles that share cache lines (neighbouring row pieces, spheres that are
// close in the order) are served by the same L2.
constexpr int XCDS = 8;
__device__ __forceinline__ int xcd_tile(int w, int G) { return (w & (XCDS - 1)) * (G / XCDS) + w / XCDS; }
inline int xcd_grid(int tiles) { return (tiles + XCDS - 1) / XCDS * XCDS; }

// LDS of a k_commit_ball block: the staged cube of cell codes (he^3 bytes),
// the surface-cell list (16-bit cube indices) and one chunk's link list (up
// to 18 links for each of BALL_THREADS cells, 32 bits each)
constexpr int BALL_THREADS = 256;
inline size_t ball_lds_bytes(int he, int list_cap) {
  return (((size_t)he * he * he + 15) & ~(size_t)15) + ((2 * (size_t)list_cap + 15) & ~(size_t)15) +
         4 * (size_t)(Q - 1) * BALL_THREADS;
}

// domain of block b: the k with start[k] <= b < start[k+1] (binary search)
__device__ __forceinline__ int batch_domain(const int* start, int ndom, int b) {
  int lo = 0, hi = ndom - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// At the end of the step, by one thread, after the sweep, the DEM and the
// mapping update: count the step, flip the current PDF buffer (the sweep has
// written the other one, the mapping update completed it), move the mapping
// stamp to the claims of the new positions, and evaluate the stop rule.  The
// rebound rule follows sphere 0: approach, wall or sphere contact (collision
// force of the last sub-cycle non-zero), contact over, rising (u_z > 0), apex
// (u_z <= 0 again).
__device__ inline void advance_step(const DevDomain& d, const DevParticles& p) {
  DevCtl* c = d.ctl;
  c->steps += 1;
  c->cur ^= 1;
  c->stamp += 1;
  bool stop = c->max_steps > 0 && c->steps >= c->max_steps;
  if (c->stop_rule == STOP_REBOUND && d.P > 0) {
    const bool contact = p.diag[12] != 0.0 || p.diag[13] != 0.0 || p.diag[14] != 0.0;
    const double uz = p.u[2];
    int ph = c->rb_phase;
    if (ph == 0 && contact)
      ph = 1;
    else if (ph == 1 && !contact)
      ph = 2;
    else if (ph == 2 && uz > 0.0)
      ph = 3;
    else if (ph == 3 && uz <= 0.0)
      stop = true;
    c->rb_phase = ph;
  }
  if (stop) c->stop_req = 1;
}

// Step control, one thread: a domain whose stop rule was met at the end of
// the last step (and which therefore skipped this step) freezes; otherwise
// the step is completed.
__device__ inline void step_control(const DevDomain& d) {
  DevCtl* c = d.ctl;
  if (c->frozen) return;
  if (c->stop_req) {
    c->frozen = 1;
    return;
  }
  advance_step(d, d.p);
}

// host-side launchers (implemented in the .hip files)
void launch_sweep(const DevDomain& d, hipStream_t s);
// mapping update outside the step: the flags and owners of the current
// positions (claims, or the geometric update of the ball pass), the
// (reconstruction), the boundary values on the current buffer, then the new
// stamp, in order on one stream
void launch_mapping(const DevDomain& d, bool reconstruct, hipStream_t s);
// inside a step, the part of the mapping update that needs only the new
// positions (after the DEM, beside or after the sweep): the claims of the slab
// pass (lists: the step's many-sphere neighbour lists are valid, so spheres
// that meet no other claim without atomics), or the mapping bins of the ball
// pass
void launch_map_prepare(const DevDomain& d, bool lists, hipStream_t s);
// the rest inside a step (after the sweep): reconstruction, flags and owners,
// boundary values, ending with the step control (folded into the last block
// of the boundary pass, or its own kernel when there is none)
void launch_update_and_advance(const DevDomain& d, hipStream_t s);
// step control (last kernel of a step): freeze, or count the step, flip the
// buffers, move the stamp and evaluate the stop rule
void launch_advance(const DevDomain& d, hipStream_t s);
void launch_advance_batch(const BatchTables& b, hipStream_t s);
// DEM sub-cycles.  kernel: 0 automatic, 1 single workgroup, 2 one thread per
// sphere over a chain of launches (binned neighbour search).  no_release: no
// sphere is in (or can leave) prescribed motion, which lets the chain merge
// each sub-cycle's position update into the previous velocity launch.
hipError_t launch_dem(const DevDomain& d, int kernel, bool no_release, hipStream_t s);
// whether launch_dem takes the many-sphere chain
bool dem_many(const DevDomain& d, int kernel);
constexpr int DEM_GRID_THREADS = 128;
// automatic DEM kernel choice: above this many spheres the many-sphere chain
constexpr int DEM_GRID_MIN = 256;
void launch_fields(const DevDomain& d, int field, double* dst, hipStream_t s);
void launch_set_pdf(const DevDomain& d, int q, const double* src, hipStream_t s);
// densities at n points: io holds 3n coordinates, then receives n results
void launch_probe_density(const DevDomain& d, double* io, int n, hipStream_t s);
void launch_fill_claims(const DevDomain& d, hipStream_t s);
// batched step kernels over the domains of a batch
void launch_sweep_batch(const BatchTables& b, hipStream_t s);
void launch_dem_batch(const BatchTables& b, hipStream_t s);
void launch_claim_batch(const BatchTables& b, hipStream_t s);
void launch_update_batch(const BatchTables& b, hipStream_t s);
void launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// fused step: the sweep with the particle links and momentum exchange, and
// the per-sphere sums of its tile partials (into partial[i][6])
void launch_sweep_fused(const DevDomain& d, hipStream_t s);
void launch_density_check(const DevDomain& d, hipStream_t s);
void launch_force_reduce(const DevDomain& d, hipStream_t s);
// fused step after the DEM: mapping bins of the new positions, reconstruction,
// flags and owners of the cells that change, step control
void launch_update_fused(const DevDomain& d, hipStream_t s);
// flags, owners and (reconstruction) of the current positions outside a
// step, every cell evaluated from the mapping bins (fused step, ball pass)
void launch_mapping_geo(const DevDomain& d, bool reconstruct, hipStream_t s);

}  // namespace lbmdem
