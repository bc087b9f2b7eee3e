// Host side of the lbmdem C-ABI: configuration checks, the layout of the
// caller-owned device region, sphere management, step orchestration on the
// domain's stream, read-out and profiling.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "lbmdem.h"

using namespace lbmdem;

namespace {

constexpr double PI_H = 3.14159265358979323846;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

size_t storage_size(int storage) { return storage == 0 ? 8 : (storage == 1 ? 4 : 2); }

// nominal box extent of a sphere (shell radius, one cell of motion, margins)
int box_extent(const lbmdem_config& c) { return 2 * (int)std::ceil(c.max_radius + c.delta_ab) + 6; }

// Mapping blocks per sphere: slabs (z) times row chunks (y).  Few spheres get
// many blocks each so that the launch fills the chip; with many spheres one
// block per sphere already does, and fewer partials keep the DEM prologue short.
constexpr int MAP_BLOCKS_TARGET = 2048;

// one-block-per-sphere boundary pass: staged cube edge (covers R + 3 around
// the centre), surface-list capacity (cells of a ball of radius R + 1), and
// whether it applies (auto from 128 spheres; LDS within 64 KiB; no periodic
// axis shorter than the cube, which would stage a cell twice)
constexpr int BALL_MIN_SPHERES = 128;
constexpr size_t BALL_LDS_MAX = 60000;

int stage_edge(const lbmdem_config& c) { return 2 * ((int)std::ceil(c.max_radius + 3.0) + 1) + 1; }

int list_cap(const lbmdem_config& c) {
  const double r = c.max_radius + 1.0;
  return (int)std::ceil(4.0 / 3.0 * PI_H * r * r * r) + 64;
}

bool ball_possible(const lbmdem_config& c) {
  const int he = stage_edge(c);
  const size_t lds = ball_lds_bytes(he, list_cap(c));
  if (lds > BALL_LDS_MAX || (size_t)he * he * he > 65535) return false;
  const int n[3] = {c.nx, c.ny, c.nz};
  for (int a = 0; a < 3; ++a)
    if (!c.walls[a] && n[a] < he) return false;
  return true;
}

// Fused step (map_kernel 3): tiles of the sweep, link boxes of the spheres
// (2 ceil(R_max) + 6 cells per axis) and the slot arrays they index.
struct FusedGeom {
  int bx, by, gx, gy;
  int E, snx, sny, snz;
  bool ok;
};

FusedGeom fused_geom(const lbmdem_config& c) {
  FusedGeom g{};
  if (c.nx <= 256) {
    g.bx = c.nx;
    g.by = std::max(1, 256 / c.nx);
  } else {
    const int cand[4] = {128, 256, 192, 64};
    g.bx = 256;
    for (int v : cand)
      if (c.nx % v == 0) {
        g.bx = v;
        break;
      }
    g.by = 256 / g.bx;
  }
  g.gx = (c.nx + g.bx - 1) / g.bx;
  g.gy = (c.ny + g.by - 1) / g.by;
  g.E = 2 * (int)std::ceil(std::max(c.max_radius, 0.0)) + 6;
  g.ok = c.max_spheres > 0 && c.max_radius >= 1.0 && c.max_radius <= 1000.0;
  // tiles a link box can meet along one axis (one more on a periodic axis,
  // where the wrap may pass a shorter last tile); distinct tiles take
  // distinct slots since a tile's slot is its index relative to the box's
  // first tile modulo the tile count, and a slot beyond these is reported
  auto axis = [&](int n, int b, int tiles, int wall) {
    (void)n;
    return std::min((g.E + b - 1) / b + (wall ? 1 : 2), tiles);
  };
  g.snx = axis(c.nx, g.bx, g.gx, c.walls[0]);
  g.sny = axis(c.ny, g.by, g.gy, c.walls[1]);
  g.snz = axis(c.nz, 1, c.nz, c.walls[2]);
  return g;
}

// bins of the geometric mapping: edge >= R_max + max(delta_aB, 1) + 1
void mbin_dims(const lbmdem_config& c, int* nb) {
  const int n[3] = {c.nx, c.ny, c.nz};
  double h = c.max_radius + std::max(c.delta_ab, 1.0) + 1.0;
  for (;;) {
    double tot = 1.0;
    for (int a = 0; a < 3; ++a) {
      nb[a] = std::max(1, (int)std::floor((double)n[a] / h));
      tot *= nb[a];
    }
    if (tot <= 4.0e6) return;
    h *= 1.25;
  }
}

// the fused step is chosen explicitly (map_kernel 3)
bool use_fused(const lbmdem_config& c) { return c.map_kernel == 3; }

bool use_ball(const lbmdem_config& c) {
  if (c.map_kernel == 1 || use_fused(c)) return false;
  if (c.map_kernel == 2) return true;
  return c.max_spheres >= BALL_MIN_SPHERES && ball_possible(c);
}

int zblocks(const lbmdem_config& c) {
  if (use_ball(c) || use_fused(c)) return 1;
  const int per = (MAP_BLOCKS_TARGET + std::max(c.max_spheres, 1) - 1) / std::max(c.max_spheres, 1);
  return std::max(1, std::min(std::min(c.nz, box_extent(c)), per));
}

int rowblocks(const lbmdem_config& c) {
  if (use_ball(c) || use_fused(c)) return 1;
  const int e = std::min(c.ny, box_extent(c));
  const int full = std::max(1, (e + COMMIT_ROWS - 1) / COMMIT_ROWS);
  const long long have = (long long)std::max(c.max_spheres, 1) * zblocks(c);
  const int per = (int)std::max(1LL, (MAP_BLOCKS_TARGET + have - 1) / have);
  return std::min(full, per);
}

// uniform bins of the many-sphere neighbour search: edge at least the largest
// centre distance of two listed neighbours (2 R_max + cut-off + skin), grown
// if the count would exceed a few per sphere
constexpr double NBR_SKIN = 1.0;

void bin_dims(const lbmdem_config& c, int* nb) {
  const int n[3] = {c.nx, c.ny, c.nz};
  double h = 2.0 * c.max_radius + std::max(c.cut_n, std::max(c.cut_tt, c.cut_tr)) + NBR_SKIN;
  const double limit = std::max(4096.0, 4.0 * (double)std::max(c.max_spheres, 1));
  for (;;) {
    double tot = 1.0;
    for (int a = 0; a < 3; ++a) {
      nb[a] = std::max(1, (int)std::floor((double)n[a] / h));
      tot *= nb[a];
    }
    if (tot <= limit) return;
    h *= 1.25;
  }
}

struct Layout {
  size_t pdf0, pdf1, flags, owner, claim, shellstamp, cellw, stage, slot, slot_stamp, mbins;
  size_t x, u, w, xmap, R, rho, m, I, mode, presc, tpresc, Fprev, prev_valid, Ffp, Fraw, Fold,
      old_valid, diag, Fnew, hist_id, hist_d, nbr, nbr_n, x2, u2, w2, order, bins, ctl, partial, status;
  size_t total;
};

Layout make_layout(const lbmdem_config& c) {
  Layout L;
  const size_t N = (size_t)c.nx * c.ny * c.nz;
  const size_t P = (size_t)std::max(c.max_spheres, 1);
  const size_t sz = storage_size(c.storage);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.pdf0 = take((size_t)Q * N * sz);
  L.pdf1 = take((size_t)Q * N * sz);
  L.flags = take(N);
  L.owner = take(4 * N);
  // claim words and shell stamps: the slab pass only (the ball pass and the
  // fused step update flags and owners from the positions)
  const bool claims = !use_ball(c) && !use_fused(c);
  L.claim = take(claims ? 8 * N : 0);
  L.shellstamp = take(claims ? 4 * N : 0);
  // flags | (owner + 1) << 8 in one word, read by the fused sweep and the ball
  // pass's staging
  L.cellw = take(use_fused(c) || use_ball(c) ? 4 * N : 0);
  L.stage = take(8 * N);
  // fused step (tile slots) and geometric mapping (bins of the fused step and
  // the ball pass) only; transient, so not part of a checkpoint
  {
    const bool f = use_fused(c), geo = f || use_ball(c);
    const FusedGeom g = fused_geom(c);
    const size_t per = f ? (size_t)g.snx * g.sny * g.snz : 0;
    int mb[3] = {1, 1, 1};
    if (geo) mbin_dims(c, mb);
    L.slot = take(48 * P * per);
    L.slot_stamp = take(4 * P * per);
    L.mbins = take(geo ? 4 * (size_t)mb[0] * mb[1] * mb[2] * (1 + BIN_CAP) : 0);
  }
  L.x = take(24 * P);
  L.u = take(24 * P);
  L.w = take(24 * P);
  L.xmap = take(24 * P);
  L.R = take(8 * P);
  L.rho = take(8 * P);
  L.m = take(8 * P);
  L.I = take(8 * P);
  L.mode = take(4 * P);
  L.presc = take(48 * P);
  L.tpresc = take(8 * P);
  L.Fprev = take(48 * P);
  L.prev_valid = take(4 * P);
  L.Ffp = take(48 * P);
  L.Fraw = take(48 * P);
  L.Fold = take(48 * P);
  L.old_valid = take(4 * P);
  L.diag = take(144 * P);
  L.Fnew = take(48 * P);
  L.hist_id = take(4 * P * HIST_SLOTS);
  L.hist_d = take(24 * P * HIST_SLOTS);
  L.nbr = take(4 * P * NBR_MAX);
  L.nbr_n = take(4 * P);
  L.x2 = take(24 * P);
  L.u2 = take(24 * P);
  L.w2 = take(24 * P);
  L.order = take(4 * P);
  int nb[3];
  bin_dims(c, nb);
  L.bins = take(4 * (size_t)nb[0] * nb[1] * nb[2] * (1 + BIN_CAP));
  L.ctl = take(sizeof(DevCtl));
  L.partial = take(48 * P * (size_t)zblocks(c) * (size_t)rowblocks(c));
  L.status = take(256);
  L.total = o;
  return L;
}

const char* check_config(const lbmdem_config* c) {
  if (!c) return "config is NULL";
  if (c->nx < 4 || c->ny < 4 || c->nz < 4) return "lattice must be at least 4 cells per axis";
  if ((double)c->nx * c->ny * c->nz >= 2147483647.0) return "lattice exceeds 2^31 cells";
  for (int a = 0; a < 3; ++a)
    if (c->walls[a] != 0 && c->walls[a] != 1) return "walls[] must be 0 or 1";
  if (!(c->nu > 0.0)) return "nu must be positive";
  if (!(c->magic_lambda > 0.0) || !(c->lambda_b > 0.0)) return "Lambda and Lambda_b must be positive";
  if (!(c->delta_ab >= 0.0)) return "delta_ab must be non-negative";
  if (c->collision < 0 || c->collision > 3) return "collision must be 0..3";
  if (c->boundary < 0 || c->boundary > 1) return "boundary must be 0 or 1";
  if (c->storage < 0 || c->storage > 2) return "storage must be 0..2";
  if (c->n_sub < 1) return "n_sub must be >= 1";
  if (c->max_spheres < 0) return "max_spheres must be >= 0";
  if (c->max_spheres > 0 && !(c->max_radius > 0.0)) return "max_radius must be positive";
  // the boundary passes index a block's cells with 16 bits
  if (c->max_spheres > 0 && !(c->max_radius <= 1000.0)) return "max_radius must be at most 1000";
  if (!(c->e_dry > 0.0 && c->e_dry <= 1.0)) return "e_dry must lie in (0, 1]";
  if (!(c->poisson_ratio >= 0.0 && c->poisson_ratio < 1.0)) return "poisson_ratio must lie in [0, 1)";
  if (!(c->friction >= 0.0)) return "friction must be non-negative";
  if (!(c->cut_n > 0.0 && c->cut_tt > 0.0 && c->cut_tr > 0.0)) return "cut-offs must be positive";
  if (c->dem_kernel < 0 || c->dem_kernel > 2) return "dem_kernel must be 0..2";
  if (c->map_kernel < 0 || c->map_kernel > 3) return "map_kernel must be 0..3";
  if (c->overlap != 0 && c->overlap != 1) return "overlap must be 0 or 1";
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(c->body_force[a])) return "body_force must be finite";
  if (c->map_kernel == 3 && !fused_geom(*c).ok)
    return "map_kernel 3 needs a sphere radius of at least 1";
  if (c->map_kernel == 2 && !ball_possible(*c))
    return "map_kernel 2 needs the staged cube (R_max + 4 cells each side) within 60000 bytes of LDS and "
           "within every periodic extent";
  return nullptr;
}

thread_local std::string g_create_error;

}  // namespace

struct lbmdem_batch;

struct lbmdem_domain {
  lbmdem_config cfg;
  DevDomain d;
  Layout L;
  hipStream_t stream = nullptr;
  void* region = nullptr;
  bool owns = false;
  int failed = 0;
  std::string err;
  std::vector<double> hx, hR;  // host shadow for insertion checks
  int prof = 0;  // 1: time the sweep only, 2: every kernel group
  struct Ev {
    hipEvent_t a, b;
    int kind;
  };
  std::vector<Ev> pending;
  std::vector<hipEvent_t> spare;
  double ms[3] = {0, 0, 0};
  int64_t cnt[3] = {0, 0, 0};
  int device = 0;                     // HIP device current at creation
  lbmdem_batch* batch = nullptr;      // batch the domain is admitted to
  bool may_prescribe = false;         // a sphere was given prescribed motion (or state restored)
  // second stream of an overlapped step (created on first use) and the events
  // that fork it from and join it to the domain's stream
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // one captured step, replayed per step (lbmdem_set_graph); re-captured
  // when the launches it holds change (sphere count, prescribed motion)
  int use_graph = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int g_P = -1, g_presc = -1;
};

static int32_t fail(lbmdem_domain* dom, int32_t code, const std::string& msg) {
  if (dom) dom->err = msg;
  else g_create_error = msg;
  return code;
}

#define HIPCHK(dom, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(dom, LBMDEM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

static hipEvent_t get_event(lbmdem_domain* dom) {
  if (!dom->spare.empty()) {
    hipEvent_t e = dom->spare.back();
    dom->spare.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

static void harvest(lbmdem_domain* dom) {
  for (auto& e : dom->pending) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, e.a, e.b) == hipSuccess) {
      dom->ms[e.kind] += t;
      dom->cnt[e.kind] += 1;
    }
    dom->spare.push_back(e.a);
    dom->spare.push_back(e.b);
  }
  dom->pending.clear();
}

// Brackets a launch with HIP events on stream s when profiling is on.  Each
// event record costs the queue a few microseconds, so level 1 brackets only
// the sweep (kind 0) and level 2 every kernel group.
template <typename F>
static void timed(lbmdem_domain* dom, int kind, hipStream_t s, F&& launch) {
  if (dom->prof == 0 || (dom->prof == 1 && kind != 0)) {
    launch();
    return;
  }
  if (dom->pending.size() > 4096) {
    (void)hipStreamSynchronize(dom->stream);
    harvest(dom);
  }
  lbmdem_domain::Ev ev{get_event(dom), get_event(dom), kind};
  if (ev.a) (void)hipEventRecord(ev.a, s);
  launch();
  if (ev.b) (void)hipEventRecord(ev.b, s);
  if (ev.a && ev.b) dom->pending.push_back(ev);
}

static int32_t refresh_host_positions(lbmdem_domain* dom);

static uint64_t spread21(uint64_t v) {
  v &= 0x1FFFFF;
  v = (v | v << 32) & 0x1F00000000FFFFull;
  v = (v | v << 16) & 0x1F0000FF0000FFull;
  v = (v | v << 8) & 0x100F00F00F00F00Full;
  v = (v | v << 4) & 0x10C30C30C30C30C3ull;
  v = (v | v << 2) & 0x1249249249249249ull;
  return v;
}

// Order in which the sphere-centric boundary pass takes the spheres: by the
// Morton (Z-order) code of the cell holding the centre, so that spheres close
// in the order are close in space.  It only affects speed: every order gives
// the same results.  Refreshed whenever the mapping is rebuilt from the host.
static int32_t refresh_order(lbmdem_domain* dom) {
  const size_t P = dom->hR.size();
  if (!P) return LBMDEM_OK;
  if (int32_t rc = refresh_host_positions(dom)) return rc;
  const int n[3] = {dom->cfg.nx, dom->cfg.ny, dom->cfg.nz};
  std::vector<std::pair<uint64_t, int>> key(P);
  for (size_t i = 0; i < P; ++i) {
    uint64_t code = 0;
    for (int a = 0; a < 3; ++a) {
      const double v = dom->hx[3 * i + a];
      const int c = std::isfinite(v) ? std::min(std::max((int)std::floor(v), 0), n[a] - 1) : 0;
      code |= spread21((uint64_t)c) << a;
    }
    key[i] = {code, (int)i};
  }
  std::sort(key.begin(), key.end());
  std::vector<int> ord(P);
  for (size_t i = 0; i < P; ++i) ord[i] = key[i].second;
  HIPCHK(dom, hipMemcpyAsync(dom->d.p.order, ord.data(), 4 * P, hipMemcpyHostToDevice, dom->stream));
  HIPCHK(dom, hipStreamSynchronize(dom->stream));
  return LBMDEM_OK;
}

static int32_t remap(lbmdem_domain* dom, bool reconstruct) {
  dom->d.P = (int)dom->hR.size();
  if (dom->d.fused) {
    timed(dom, 2, dom->stream, [&] { launch_mapping_geo(dom->d, reconstruct, dom->stream); });
    HIPCHK(dom, hipGetLastError());
    return LBMDEM_OK;
  }
  if (int32_t rc = refresh_order(dom)) return rc;
  timed(dom, 2, dom->stream, [&] { launch_mapping(dom->d, reconstruct, dom->stream); });
  HIPCHK(dom, hipGetLastError());
  return LBMDEM_OK;
}

// ---- static device scratch of the allocation-free probe ----------------------
// Staging of lbmdem_probe_density_static: the probe points and their results
// live in this file-scope device array instead of the domain region.  Each
// GPU holds its own copy for the life of the process.  In host code the name
// `scratch` is only a host-side stand-in: its device address is looked up once
// per device, with that device current, when a domain is created there, and
// only that address is ever passed to kernels or copies.
constexpr int PROBE_STATIC_MAX = 65536;  // points per call (4 doubles each: 2 MiB)
static __device__ __align__(256) double scratch[4 * (size_t)PROBE_STATIC_MAX];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[MAX_DEVICES] = {};

// Resolves the device address of `scratch` on device `dev` (current).
static hipError_t init_static_scratch(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = (double*)ptr;
  return hipSuccess;
}

static double* static_scratch(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[dev];
}

extern "C" {

int32_t lbmdem_config_init(lbmdem_config* c) {
  if (!c) return LBMDEM_EINVAL;
  std::memset(c, 0, sizeof(*c));
  c->nx = c->ny = c->nz = 32;
  c->walls[2] = 1;
  c->nu = 0.01;
  c->magic_lambda = 3.0 / 16.0;
  c->lambda_b = 100.0;
  c->delta_ab = 2.0;
  c->collision = LBMDEM_TRT_AB;
  c->boundary = LBMDEM_BC_CLI;
  c->storage = LBMDEM_STORE_F32;
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
  c->dem_kernel = 0;
  c->map_kernel = 0;
  c->overlap = 1;
  return LBMDEM_OK;
}

size_t lbmdem_footprint_bytes(const lbmdem_config* cfg) {
  if (check_config(cfg)) return 0;
  return make_layout(*cfg).total;
}

int32_t lbmdem_create(const lbmdem_config* cfg, void* dev_buf, size_t dev_bytes, void* hip_stream,
                      lbmdem_domain** out) {
  if (!out) return fail(nullptr, LBMDEM_EINVAL, "out is NULL");
  *out = nullptr;
  if (const char* e = check_config(cfg)) return fail(nullptr, LBMDEM_EINVAL, e);
  Layout L = make_layout(*cfg);
  if (dev_buf && dev_bytes < L.total)
    return fail(nullptr, LBMDEM_ENOMEM, "device region smaller than lbmdem_footprint_bytes()");
  if (dev_buf && ((uintptr_t)dev_buf & 255))
    return fail(nullptr, LBMDEM_EINVAL, "device region must be 256-byte aligned");
  lbmdem_domain* dom = new (std::nothrow) lbmdem_domain();
  if (!dom) return fail(nullptr, LBMDEM_ENOMEM, "host allocation failed");
  dom->cfg = *cfg;
  dom->L = L;
  dom->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&dom->device) != hipSuccess || init_static_scratch(dom->device) != hipSuccess) {
    delete dom;
    return fail(nullptr, LBMDEM_EDEVICE, "device query or static scratch lookup failed");
  }
  if (dev_buf) {
    dom->region = dev_buf;
  } else {
    if (hipMalloc(&dom->region, L.total) != hipSuccess) {
      delete dom;
      return fail(nullptr, LBMDEM_ENOMEM, "hipMalloc of the domain region failed");
    }
    dom->owns = true;
  }
  char* base = (char*)dom->region;
  DevDomain& d = dom->d;
  std::memset(&d, 0, sizeof(d));
  d.nx = cfg->nx;
  d.ny = cfg->ny;
  d.nz = cfg->nz;
  d.N = (long long)cfg->nx * cfg->ny * cfg->nz;
  for (int a = 0; a < 3; ++a) {
    d.walls[a] = cfg->walls[a];
    d.wall_u_lo[a] = cfg->wall_u_lo[a];
    d.wall_u_hi[a] = cfg->wall_u_hi[a];
    d.force[a] = cfg->body_force[a];
    d.gravity[a] = cfg->gravity[a];
  }
  d.storage = cfg->storage;
  d.forced = (cfg->body_force[0] != 0.0 || cfg->body_force[1] != 0.0 || cfg->body_force[2] != 0.0) ? 1 : 0;
  d.boundary = cfg->boundary;
  // Eq. (Viscosity), Eq. (MagicParameter), Eq. (lambda_b)
  const double snu = 1.0 / (3.0 * cfg->nu + 0.5);
  const double tau = 1.0 / snu - 0.5;
  const double smi = 1.0 / (0.5 + cfg->magic_lambda / tau);
  const double sb = 1.0 / (0.5 + cfg->lambda_b * tau);
  d.s_nu = snu;
  d.s_plus = snu;
  d.s_minus = smi;
  switch (cfg->collision) {
    case LBMDEM_TRT_AB: d.s_bulk_shell = sb; d.s_bulk_other = snu; break;
    case LBMDEM_TRT_B: d.s_bulk_shell = sb; d.s_bulk_other = sb; break;
    case LBMDEM_TRT: d.s_bulk_shell = snu; d.s_bulk_other = snu; break;
    default: d.s_minus = snu; d.s_bulk_shell = snu; d.s_bulk_other = snu; break;
  }
  d.delta_ab = cfg->delta_ab;
  d.pdf[0] = base + L.pdf0;
  d.pdf[1] = base + L.pdf1;
  d.flags = (uint8_t*)(base + L.flags);
  d.owner = (int32_t*)(base + L.owner);
  const bool claims = !use_ball(*cfg) && !use_fused(*cfg);
  d.claim = claims ? (unsigned long long*)(base + L.claim) : nullptr;
  d.shellstamp = claims ? (uint32_t*)(base + L.shellstamp) : nullptr;
  d.cellw = use_fused(*cfg) || use_ball(*cfg) ? (uint32_t*)(base + L.cellw) : nullptr;
  DevParticles& p = d.p;
  p.x = (double*)(base + L.x);
  p.u = (double*)(base + L.u);
  p.w = (double*)(base + L.w);
  p.xmap = (double*)(base + L.xmap);
  p.R = (double*)(base + L.R);
  p.rho = (double*)(base + L.rho);
  p.m = (double*)(base + L.m);
  p.I = (double*)(base + L.I);
  p.mode = (int*)(base + L.mode);
  p.presc = (double*)(base + L.presc);
  p.tpresc = (double*)(base + L.tpresc);
  p.Fprev = (double*)(base + L.Fprev);
  p.prev_valid = (int*)(base + L.prev_valid);
  p.Ffp = (double*)(base + L.Ffp);
  p.Fraw = (double*)(base + L.Fraw);
  p.Fold = (double*)(base + L.Fold);
  p.old_valid = (int*)(base + L.old_valid);
  p.diag = (double*)(base + L.diag);
  p.Fnew = (double*)(base + L.Fnew);
  p.hist_id = (int*)(base + L.hist_id);
  p.hist_d = (double*)(base + L.hist_d);
  p.nbr = (int*)(base + L.nbr);
  p.nbr_n = (int*)(base + L.nbr_n);
  p.x2 = (double*)(base + L.x2);
  p.u2 = (double*)(base + L.u2);
  p.w2 = (double*)(base + L.w2);
  p.order = (int*)(base + L.order);
  bin_dims(*cfg, d.bins.n);
  d.bins.cell = (int*)(base + L.bins);
  d.ctl = (DevCtl*)(base + L.ctl);
  d.P = 0;
  d.ZB = zblocks(*cfg);
  d.RB = rowblocks(*cfg);
  d.map_ball = use_ball(*cfg) ? 1 : 0;
  d.stage_edge = stage_edge(*cfg);
  d.list_cap = list_cap(*cfg);
  d.partial = (double*)(base + L.partial);
  d.fused = use_fused(*cfg) ? 1 : 0;
  {
    const FusedGeom g = fused_geom(*cfg);
    d.fbx = g.bx;
    d.fby = g.by;
    d.fgx = g.gx;
    d.fgy = g.gy;
    d.sl_E = g.E;
    d.sl_nx = g.snx;
    d.sl_ny = g.sny;
    d.sl_nz = g.snz;
    d.sl_per = d.fused ? g.snx * g.sny * g.snz : 0;
    d.slot = (double*)(base + L.slot);
    d.slot_stamp = (uint32_t*)(base + L.slot_stamp);
    if (d.fused || d.map_ball) mbin_dims(*cfg, d.mbins.n);
    else d.mbins.n[0] = d.mbins.n[1] = d.mbins.n[2] = 1;
    d.mbins.cell = (int*)(base + L.mbins);
    d.stage32 = (uint32_t*)(base + L.stage);
  }
  d.status = (int*)(base + L.status);
  d.n_sub = cfg->n_sub;
  d.force_averaging = cfg->force_averaging;
  d.e_dry = cfg->e_dry;
  d.poisson_ratio = cfg->poisson_ratio;
  d.friction = cfg->friction;
  d.tc = cfg->tc;
  d.dmin = cfg->dmin;
  d.cut_n = cfg->cut_n;
  d.cut_tt = cfg->cut_tt;
  d.cut_tr = cfg->cut_tr;
  d.lub_mask = cfg->lub_mask;
  d.nu = cfg->nu;
  d.skin = NBR_SKIN;
  hipStream_t s = dom->stream;
  const size_t Pm = (size_t)std::max(cfg->max_spheres, 1);

  // particle block and status are plain zeros except the free history slots
  int32_t rc = LBMDEM_OK;
  if (hipMemsetAsync(base + L.slot, 0, L.total - L.slot, s) != hipSuccess ||
      hipMemsetD32Async((hipDeviceptr_t)(base + L.hist_id), (int)0x80000000, Pm * HIST_SLOTS, s) !=
          hipSuccess)
    rc = fail(nullptr, LBMDEM_EDEVICE, "initialising the particle block failed");
  if (rc == LBMDEM_OK) {
    launch_fill_claims(d, s);
    if (hipGetLastError() != hipSuccess) rc = fail(nullptr, LBMDEM_EDEVICE, "init kernel launch failed");
  }
  if (rc == LBMDEM_OK && remap(dom, false) != LBMDEM_OK)
    rc = fail(nullptr, LBMDEM_EDEVICE, dom->err);
  if (rc == LBMDEM_OK && hipStreamSynchronize(s) != hipSuccess)
    rc = fail(nullptr, LBMDEM_EDEVICE, "initialisation failed on the device");
  if (rc != LBMDEM_OK) {
    if (dom->owns) (void)hipFree(dom->region);
    delete dom;
    return rc;
  }
  *out = dom;
  return LBMDEM_OK;
}

int32_t lbmdem_destroy(lbmdem_domain* dom) {
  if (!dom) return LBMDEM_OK;
  if (dom->batch) (void)lbmdem_batch_retire(dom->batch, dom);
  (void)hipStreamSynchronize(dom->stream);
  harvest(dom);
  for (auto e : dom->spare) (void)hipEventDestroy(e);
  if (dom->gexec) (void)hipGraphExecDestroy(dom->gexec);
  if (dom->graph) (void)hipGraphDestroy(dom->graph);
  if (dom->side) (void)hipStreamDestroy(dom->side);
  if (dom->ev_fork) (void)hipEventDestroy(dom->ev_fork);
  if (dom->ev_join) (void)hipEventDestroy(dom->ev_join);
  if (dom->owns) (void)hipFree(dom->region);
  delete dom;
  return LBMDEM_OK;
}

int32_t lbmdem_num_spheres(const lbmdem_domain* dom) { return dom ? (int32_t)dom->hR.size() : -1; }

static double min_wall_gap_h(const lbmdem_config& c, const double* x, double R) {
  const int n[3] = {c.nx, c.ny, c.nz};
  double g = 1e300;
  for (int a = 0; a < 3; ++a) {
    if (!c.walls[a]) continue;
    g = std::min(g, (x[a] - 1.0) - R);
    g = std::min(g, (((double)n[a] - 1.0) - x[a]) - R);
  }
  return g;
}

static double min_img_h(const lbmdem_config& c, int a, double v) {
  const int n[3] = {c.nx, c.ny, c.nz};
  if (c.walls[a]) return v;
  const double L = (double)n[a];
  if (v > 0.5 * L) return v - L;
  if (v < -0.5 * L) return v + L;
  return v;
}

static int32_t refresh_host_positions(lbmdem_domain* dom) {
  const size_t P = dom->hR.size();
  dom->hx.resize(3 * P);
  if (P) HIPCHK(dom, hipMemcpyAsync(dom->hx.data(), dom->d.p.x, 24 * P, hipMemcpyDeviceToHost, dom->stream));
  HIPCHK(dom, hipStreamSynchronize(dom->stream));
  return LBMDEM_OK;
}

int32_t lbmdem_add_spheres(lbmdem_domain* dom, int32_t n, const double* x, const double* u,
                           const double* w, const double* radius, const double* rho,
                           int32_t* ids_out) {
  if (!dom) return LBMDEM_EINVAL;
  if (dom->failed) return fail(dom, LBMDEM_ESTATE, "domain has failed");
  if (n < 0 || (n > 0 && (!x || !radius || !rho))) return fail(dom, LBMDEM_EINVAL, "bad arguments");
  if (n == 0) return LBMDEM_OK;
  const lbmdem_config& c = dom->cfg;
  const size_t P0 = dom->hR.size();
  if ((long long)P0 + n > c.max_spheres) return fail(dom, LBMDEM_ECAPACITY, "max_spheres exceeded");
  if (int32_t rc = refresh_host_positions(dom)) return rc;
  const int nn[3] = {c.nx, c.ny, c.nz};
  std::vector<double> ax(dom->hx), aR(dom->hR);
  for (int s = 0; s < n; ++s) {
    const double* xs = x + 3 * s;
    const double R = radius[s];
    if (!(R > 0.0) || R > c.max_radius || !(rho[s] > 0.0))
      return fail(dom, LBMDEM_EINVAL, "radius must lie in (0, max_radius] and density be positive");
    for (int a = 0; a < 3; ++a)
      if (!(xs[a] >= 0.0 && xs[a] < (double)nn[a]))
        return fail(dom, LBMDEM_EINVAL, "sphere centre outside the lattice");
    if (min_wall_gap_h(c, xs, R) < 0.0) return fail(dom, LBMDEM_EOVERLAP, "sphere crosses a wall plane");
    for (size_t j = 0; j < aR.size(); ++j) {
      double dd[3];
      for (int a = 0; a < 3; ++a) dd[a] = min_img_h(c, a, xs[a] - ax[3 * j + a]);
      const double dist = std::sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
      if (dist - (R + aR[j]) < 0.0) return fail(dom, LBMDEM_EOVERLAP, "spheres overlap");
    }
    for (int a = 0; a < 3; ++a) ax.push_back(xs[a]);
    aR.push_back(R);
  }
  std::vector<double> hu(3 * n, 0.0), hw(3 * n, 0.0), hm(n), hI(n);
  for (int s = 0; s < n; ++s) {
    for (int a = 0; a < 3; ++a) {
      if (u) hu[3 * s + a] = u[3 * s + a];
      if (w) hw[3 * s + a] = w[3 * s + a];
    }
    const double R = radius[s];
    hm[s] = rho[s] * (4.0 / 3.0) * PI_H * R * R * R;
    hI[s] = 0.4 * hm[s] * R * R;
  }
  DevParticles& p = dom->d.p;
  hipStream_t st = dom->stream;
  HIPCHK(dom, hipMemcpyAsync(p.x + 3 * P0, x, 24 * (size_t)n, hipMemcpyHostToDevice, st));
  HIPCHK(dom, hipMemcpyAsync(p.xmap + 3 * P0, x, 24 * (size_t)n, hipMemcpyHostToDevice, st));
  HIPCHK(dom, hipMemcpyAsync(p.u + 3 * P0, hu.data(), 24 * (size_t)n, hipMemcpyHostToDevice, st));
  HIPCHK(dom, hipMemcpyAsync(p.w + 3 * P0, hw.data(), 24 * (size_t)n, hipMemcpyHostToDevice, st));
  HIPCHK(dom, hipMemcpyAsync(p.R + P0, radius, 8 * (size_t)n, hipMemcpyHostToDevice, st));
  HIPCHK(dom, hipMemcpyAsync(p.rho + P0, rho, 8 * (size_t)n, hipMemcpyHostToDevice, st));
  HIPCHK(dom, hipMemcpyAsync(p.m + P0, hm.data(), 8 * (size_t)n, hipMemcpyHostToDevice, st));
  HIPCHK(dom, hipMemcpyAsync(p.I + P0, hI.data(), 8 * (size_t)n, hipMemcpyHostToDevice, st));
  HIPCHK(dom, hipStreamSynchronize(st));
  for (int s = 0; s < n; ++s) {
    dom->hR.push_back(radius[s]);
    if (ids_out) ids_out[s] = (int32_t)(P0 + s);
  }
  return remap(dom, true);
}

// positions the next mapping starts from = current positions
static int32_t pin_mapped_positions(lbmdem_domain* dom) {
  const size_t P = dom->hR.size();
  if (P) launch_copy(dom->d.p.xmap, dom->d.p.x, 24 * P, dom->stream);
  HIPCHK(dom, hipGetLastError());
  return LBMDEM_OK;
}

int32_t lbmdem_update_spheres(lbmdem_domain* dom, int32_t n, const int32_t* ids, const double* x,
                              const double* u, const double* w, int32_t mask) {
  if (!dom) return LBMDEM_EINVAL;
  if (dom->failed) return fail(dom, LBMDEM_ESTATE, "domain has failed");
  if (n < 0 || (n > 0 && !ids)) return fail(dom, LBMDEM_EINVAL, "bad arguments");
  if (((mask & 1) && !x) || ((mask & 2) && !u) || ((mask & 4) && !w))
    return fail(dom, LBMDEM_EINVAL, "masked field pointer is NULL");
  const int nn[3] = {dom->cfg.nx, dom->cfg.ny, dom->cfg.nz};
  for (int s = 0; s < n; ++s) {
    if (ids[s] < 0 || ids[s] >= (int32_t)dom->hR.size()) return fail(dom, LBMDEM_EINVAL, "bad sphere id");
    if (mask & 1)
      for (int a = 0; a < 3; ++a)
        if (!(x[3 * s + a] >= 0.0 && x[3 * s + a] < (double)nn[a]))
          return fail(dom, LBMDEM_EINVAL, "sphere centre outside the lattice");
  }
  if (int32_t rc = pin_mapped_positions(dom)) return rc;
  DevParticles& p = dom->d.p;
  hipStream_t st = dom->stream;
  const int zero = 0;
  for (int s = 0; s < n; ++s) {
    const int i = ids[s];
    if (mask & 1) HIPCHK(dom, hipMemcpyAsync(p.x + 3 * i, x + 3 * s, 24, hipMemcpyHostToDevice, st));
    if (mask & 2) HIPCHK(dom, hipMemcpyAsync(p.u + 3 * i, u + 3 * s, 24, hipMemcpyHostToDevice, st));
    if (mask & 4) HIPCHK(dom, hipMemcpyAsync(p.w + 3 * i, w + 3 * s, 24, hipMemcpyHostToDevice, st));
    HIPCHK(dom, hipMemcpyAsync(p.old_valid + i, &zero, 4, hipMemcpyHostToDevice, st));
  }
  HIPCHK(dom, hipStreamSynchronize(st));
  return remap(dom, true);
}

int32_t lbmdem_set_sphere_mode(lbmdem_domain* dom, int32_t id, int32_t mode, const double* u_target,
                               double c_acc, double t_st, double release_gap) {
  if (!dom) return LBMDEM_EINVAL;
  if (dom->failed) return fail(dom, LBMDEM_ESTATE, "domain has failed");
  if (id < 0 || id >= (int32_t)dom->hR.size() || mode < 0 || mode > 2)
    return fail(dom, LBMDEM_EINVAL, "bad sphere id or mode");
  if (mode == LBMDEM_PRESCRIBED && (!u_target || !(t_st > 0.0)))
    return fail(dom, LBMDEM_EINVAL, "prescribed mode needs u_target and t_st > 0");
  if (int32_t rc = pin_mapped_positions(dom)) return rc;
  DevParticles& p = dom->d.p;
  hipStream_t st = dom->stream;
  const int zero = 0;
  HIPCHK(dom, hipMemcpyAsync(p.mode + id, &mode, 4, hipMemcpyHostToDevice, st));
  HIPCHK(dom, hipMemcpyAsync(p.old_valid + id, &zero, 4, hipMemcpyHostToDevice, st));
  if (mode == LBMDEM_PRESCRIBED) {
    dom->may_prescribe = true;
    const double pr[6] = {u_target[0], u_target[1], u_target[2], c_acc, t_st, release_gap};
    const double z3[3] = {0, 0, 0};
    const double t0 = 0.0;
    HIPCHK(dom, hipMemcpyAsync(p.presc + 6 * id, pr, 48, hipMemcpyHostToDevice, st));
    HIPCHK(dom, hipMemcpyAsync(p.tpresc + id, &t0, 8, hipMemcpyHostToDevice, st));
    HIPCHK(dom, hipMemcpyAsync(p.u + 3 * id, z3, 24, hipMemcpyHostToDevice, st));
    HIPCHK(dom, hipMemcpyAsync(p.w + 3 * id, z3, 24, hipMemcpyHostToDevice, st));
  }
  HIPCHK(dom, hipStreamSynchronize(st));
  return remap(dom, true);
}

// The DEM sub-cycles and the claims of step t need the forces formed by the
// boundary pass of step t - 1 and the particle state, not the sweep of step
// t, so they can run on a second stream while the sweep runs.
static bool overlap_step(const lbmdem_domain* dom) { return dom->cfg.overlap && dom->d.P > 0; }

static int32_t ensure_side(lbmdem_domain* dom) {
  if (dom->side) return LBMDEM_OK;
  HIPCHK(dom, hipEventCreateWithFlags(&dom->ev_fork, hipEventDisableTiming));
  HIPCHK(dom, hipEventCreateWithFlags(&dom->ev_join, hipEventDisableTiming));
  HIPCHK(dom, hipStreamCreateWithFlags(&dom->side, hipStreamNonBlocking));
  return LBMDEM_OK;
}

static void drop_step_graph(lbmdem_domain* dom) {
  if (dom->gexec) (void)hipGraphExecDestroy(dom->gexec);
  if (dom->graph) (void)hipGraphDestroy(dom->graph);
  dom->gexec = nullptr;
  dom->graph = nullptr;
  dom->g_P = dom->g_presc = -1;
}

// the launches of nsteps steps, enqueued directly
static int32_t step_direct(lbmdem_domain* dom, int32_t nsteps) {
  hipStream_t s0 = dom->stream;
  if (dom->d.fused) {
    // Alg. 1 in order on one stream: the sweep with the link boundary values
    // and momentum exchange, the per-sphere sums, the DEM sub-cycles, then the
    // mapping update with reconstruction and the step control
    for (int k = 0; k < nsteps; ++k) {
      hipError_t e = hipSuccess;
      timed(dom, 0, s0, [&] { launch_sweep_fused(dom->d, s0); });
      timed(dom, 1, s0, [&] {
        launch_force_reduce(dom->d, s0);
        e = launch_dem(dom->d, dom->cfg.dem_kernel, !dom->may_prescribe, s0);
      });
      if (e != hipSuccess) {
        dom->failed = 1;
        return fail(dom, LBMDEM_EDEVICE, std::string("DEM launch failed: ") + hipGetErrorString(e));
      }
      timed(dom, 2, s0, [&] { launch_update_fused(dom->d, s0); });
    }
    HIPCHK(dom, hipGetLastError());
    return LBMDEM_OK;
  }
  const bool ov = overlap_step(dom);
  if (ov && nsteps > 0)
    if (int32_t rc = ensure_side(dom)) return rc;
  hipStream_t s = dom->stream;
  // Per step: the sweep (A -> B) and, beside it or after it, the DEM
  // sub-cycles and the claims of the new positions; then reconstruction, the
  // boundary pass (mapping, boundary values and momentum-exchange partials of
  // the next step, written into B) and the step control (B becomes current).
  for (int k = 0; k < nsteps; ++k) {
    hipError_t e = hipSuccess;
    hipStream_t ds = s;
    // With the sweep timed, the event that opens its timing also releases the
    // second stream (each recorded event costs the queue a few microseconds).
    lbmdem_domain::Ev sw{nullptr, nullptr, 0};
    if (ov && dom->prof >= 1) {
      if (dom->pending.size() > 4096) {
        HIPCHK(dom, hipStreamSynchronize(s));
        harvest(dom);
      }
      sw = {get_event(dom), get_event(dom), 0};
      if (!sw.a || !sw.b) return fail(dom, LBMDEM_EDEVICE, "event creation failed");
    }
    if (ov) {
      hipEvent_t fork = sw.a ? sw.a : dom->ev_fork;
      HIPCHK(dom, hipEventRecord(fork, s));
      HIPCHK(dom, hipStreamWaitEvent(dom->side, fork, 0));
      ds = dom->side;
    }
    auto dem = [&] {
      timed(dom, 1, ds, [&] {
        e = launch_dem(dom->d, dom->cfg.dem_kernel, !dom->may_prescribe, ds);
        launch_map_prepare(dom->d, dem_many(dom->d, dom->cfg.dem_kernel), ds);
      });
    };
    if (!ov) {
      timed(dom, 0, s, [&] { launch_sweep(dom->d, s); });
      dem();
    } else {
      dem();
      if (sw.a) {
        launch_sweep(dom->d, s);
        HIPCHK(dom, hipEventRecord(sw.b, s));
        dom->pending.push_back(sw);
      } else {
        launch_sweep(dom->d, s);
      }
      HIPCHK(dom, hipEventRecord(dom->ev_join, ds));
      HIPCHK(dom, hipStreamWaitEvent(s, dom->ev_join, 0));
    }
    if (e != hipSuccess) {
      dom->failed = 1;
      return fail(dom, LBMDEM_EDEVICE, std::string("DEM launch failed: ") + hipGetErrorString(e));
    }
    timed(dom, 2, s, [&] { launch_update_and_advance(dom->d, s); });
  }
  HIPCHK(dom, hipGetLastError());
  return LBMDEM_OK;
}

int32_t lbmdem_step(lbmdem_domain* dom, int32_t nsteps) {
  if (!dom || nsteps < 0) return LBMDEM_EINVAL;
  if (dom->failed) return fail(dom, LBMDEM_ESTATE, "domain has failed");
  if (dom->batch) return fail(dom, LBMDEM_EINVAL, "domain is stepped by its batch");
  dom->d.P = (int)dom->hR.size();
  if (!dom->use_graph || dom->prof != 0 || nsteps == 0) return step_direct(dom, nsteps);
  // every kernel reads its step state (buffer parity, stamp, step count) from
  // device memory, so one captured step serves every step
  const int presc = dom->may_prescribe ? 1 : 0;
  if (!dom->gexec || dom->g_P != dom->d.P || dom->g_presc != presc) {
    drop_step_graph(dom);
    if (overlap_step(dom))
      if (int32_t rc = ensure_side(dom)) return rc;
    HIPCHK(dom, hipStreamBeginCapture(dom->stream, hipStreamCaptureModeThreadLocal));
    const int32_t rc = step_direct(dom, 1);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(dom->stream, &g);
    if (rc != LBMDEM_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      if (rc != LBMDEM_OK) return rc;
      return fail(dom, LBMDEM_EDEVICE, std::string("step graph capture: ") + hipGetErrorString(e));
    }
    dom->graph = g;
    HIPCHK(dom, hipGraphInstantiate(&dom->gexec, dom->graph, nullptr, nullptr, 0));
    dom->g_P = dom->d.P;
    dom->g_presc = presc;
  }
  for (int k = 0; k < nsteps; ++k) HIPCHK(dom, hipGraphLaunch(dom->gexec, dom->stream));
  return LBMDEM_OK;
}

int32_t lbmdem_set_graph(lbmdem_domain* dom, int32_t use_graph) {
  if (!dom) return LBMDEM_EINVAL;
  if (use_graph && !dom->stream) return fail(dom, LBMDEM_EINVAL, "step graphs need a stream other than the null stream");
  drop_step_graph(dom);
  dom->use_graph = use_graph ? 1 : 0;
  return LBMDEM_OK;
}

int32_t lbmdem_sync(lbmdem_domain* dom) {
  if (!dom) return LBMDEM_EINVAL;
  if (!dom->failed) launch_density_check(dom->d, dom->stream);
  HIPCHK(dom, hipStreamSynchronize(dom->stream));
  int st = 0;
  HIPCHK(dom, hipMemcpy(&st, dom->d.status, 4, hipMemcpyDeviceToHost));
  if (st & ST_NONFINITE) {
    dom->failed = 1;
    return fail(dom, LBMDEM_EUNSTABLE, "non-finite particle state");
  }
  if (st & ST_DENSITY) {
    dom->failed = 1;
    return fail(dom, LBMDEM_EUNSTABLE, "a sampled fluid density left (0.5, 1.5)");
  }
  if (st & (ST_HIST_FULL | ST_NBR_FULL | ST_TILE_FULL)) {
    dom->failed = 1;
    return fail(dom, LBMDEM_ECAPACITY,
                (st & ST_TILE_FULL) ? "a sweep tile met more spheres than its table holds"
                                    : "contact-history, neighbour-list or bin slots exhausted");
  }
  return dom->failed ? LBMDEM_ESTATE : LBMDEM_OK;
}

int32_t lbmdem_get_sphere_state(lbmdem_domain* dom, int32_t id, double* out) {
  if (!dom || !out) return LBMDEM_EINVAL;
  if (id < 0 || id >= (int32_t)dom->hR.size()) return fail(dom, LBMDEM_EINVAL, "bad sphere id");
  const DevParticles& p = dom->d.p;
  hipStream_t st = dom->stream;
  double ffp[6], dg[18], fr[6], rr[2];
  int mode = 0;
  HIPCHK(dom, hipMemcpyAsync(out + 0, p.x + 3 * id, 24, hipMemcpyDeviceToHost, st));
  HIPCHK(dom, hipMemcpyAsync(out + 3, p.u + 3 * id, 24, hipMemcpyDeviceToHost, st));
  HIPCHK(dom, hipMemcpyAsync(out + 6, p.w + 3 * id, 24, hipMemcpyDeviceToHost, st));
  HIPCHK(dom, hipMemcpyAsync(ffp, p.Ffp + 6 * id, 48, hipMemcpyDeviceToHost, st));
  HIPCHK(dom, hipMemcpyAsync(dg, p.diag + 18 * id, 144, hipMemcpyDeviceToHost, st));
  HIPCHK(dom, hipMemcpyAsync(fr, p.Fraw + 6 * id, 48, hipMemcpyDeviceToHost, st));
  HIPCHK(dom, hipMemcpyAsync(&mode, p.mode + id, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(dom, hipMemcpyAsync(&rr[0], p.R + id, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(dom, hipMemcpyAsync(&rr[1], p.rho + id, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(dom, hipStreamSynchronize(st));
  for (int k = 0; k < 6; ++k) out[9 + k] = ffp[k];
  for (int k = 0; k < 18; ++k) out[15 + k] = dg[k];
  out[33] = (double)mode;
  out[34] = rr[0];
  out[35] = rr[1];
  for (int k = 0; k < 6; ++k) out[36 + k] = fr[k];
  return LBMDEM_OK;
}

int32_t lbmdem_get_spheres(lbmdem_domain* dom, int32_t n, const int32_t* ids, double* x, double* u,
                           double* w, double* F_fp, double* T_fp, double* F_tot, double* T_tot) {
  if (!dom || n < 0) return LBMDEM_EINVAL;
  const int32_t P = (int32_t)dom->hR.size();
  if (!ids && n > P) return fail(dom, LBMDEM_EINVAL, "n exceeds the number of spheres");
  for (int32_t s = 0; ids && s < n; ++s)
    if (ids[s] < 0 || ids[s] >= P) return fail(dom, LBMDEM_EINVAL, "bad sphere id");
  if (n == 0) return LBMDEM_OK;
  const DevParticles& p = dom->d.p;
  hipStream_t st = dom->stream;
  std::vector<double> hx, hu, hw, hf, hd;
  auto pull = [&](std::vector<double>& h, const double* src, size_t per) -> hipError_t {
    h.resize(per * (size_t)P);
    return hipMemcpyAsync(h.data(), src, 8 * per * (size_t)P, hipMemcpyDeviceToHost, st);
  };
  if (x) HIPCHK(dom, pull(hx, p.x, 3));
  if (u) HIPCHK(dom, pull(hu, p.u, 3));
  if (w) HIPCHK(dom, pull(hw, p.w, 3));
  if (F_fp || T_fp) HIPCHK(dom, pull(hf, p.Ffp, 6));
  if (F_tot || T_tot) HIPCHK(dom, pull(hd, p.diag, 18));
  HIPCHK(dom, hipStreamSynchronize(st));
  for (int32_t s = 0; s < n; ++s) {
    const size_t i = (size_t)(ids ? ids[s] : s);
    for (int a = 0; a < 3; ++a) {
      if (x) x[3 * s + a] = hx[3 * i + a];
      if (u) u[3 * s + a] = hu[3 * i + a];
      if (w) w[3 * s + a] = hw[3 * i + a];
      if (F_fp) F_fp[3 * s + a] = hf[6 * i + a];
      if (T_fp) T_fp[3 * s + a] = hf[6 * i + 3 + a];
      if (F_tot) F_tot[3 * s + a] = hd[18 * i + a];
      if (T_tot) T_tot[3 * s + a] = hd[18 * i + 3 + a];
    }
  }
  return LBMDEM_OK;
}

int32_t lbmdem_probe_density(lbmdem_domain* dom, int32_t n, const double* xyz, double* out) {
  if (!dom || n < 0 || (n > 0 && (!xyz || !out))) return LBMDEM_EINVAL;
  if ((size_t)n * 4 > (size_t)dom->d.N) return fail(dom, LBMDEM_EINVAL, "too many probe points (at most N/4)");
  if (n == 0) return LBMDEM_OK;
  double* stage = (double*)((char*)dom->region + dom->L.stage);
  hipStream_t st = dom->stream;
  HIPCHK(dom, hipMemcpyAsync(stage, xyz, 24 * (size_t)n, hipMemcpyHostToDevice, st));
  launch_probe_density(dom->d, stage, n, st);
  HIPCHK(dom, hipGetLastError());
  HIPCHK(dom, hipMemcpyAsync(out, stage + 3 * (size_t)n, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
  HIPCHK(dom, hipStreamSynchronize(st));
  return LBMDEM_OK;
}

int32_t lbmdem_probe_density_static(lbmdem_domain* dom, int32_t n, const double* xyz, double* out) {
  if (!dom || n < 0 || (n > 0 && (!xyz || !out))) return LBMDEM_EINVAL;
  if (n > PROBE_STATIC_MAX)
    return fail(dom, LBMDEM_EINVAL, "too many probe points for the static scratch (at most 65536)");
  if (n == 0) return LBMDEM_OK;
  double* ptr = static_scratch(dom->device);
  if (!ptr) return fail(dom, LBMDEM_EDEVICE, "static scratch not resolved on this device");
  hipStream_t st = dom->stream;
  HIPCHK(dom, hipMemcpyAsync(ptr, xyz, 24 * (size_t)n, hipMemcpyDeviceToDevice, st));
  launch_probe_density(dom->d, ptr, n, st);
  HIPCHK(dom, hipGetLastError());
  HIPCHK(dom, hipMemcpyAsync(out, ptr + 3 * (size_t)n, 8 * (size_t)n, hipMemcpyDeviceToDevice, st));
  return LBMDEM_OK;
}

int32_t lbmdem_get_field(lbmdem_domain* dom, int32_t field, void* dst, size_t bytes,
                         int32_t dst_is_device) {
  if (!dom || !dst) return LBMDEM_EINVAL;
  const size_t N = (size_t)dom->d.N;
  size_t need = 0;
  int first = 0, planes = 0;
  switch (field) {
    case LBMDEM_FIELD_RHO: need = 8 * N; first = 0; planes = 1; break;
    case LBMDEM_FIELD_VEL: need = 24 * N; first = 1; planes = 3; break;
    case LBMDEM_FIELD_PDF: need = 8 * N * Q; first = 10; planes = Q; break;
    case LBMDEM_FIELD_FLAGS: need = N; first = 40; planes = 1; break;
    case LBMDEM_FIELD_OWNER: need = 4 * N; first = 41; planes = 1; break;
    case LBMDEM_FIELD_PDF_RAW: need = 8 * N * Q; first = 60; planes = Q; break;
    default: return fail(dom, LBMDEM_EINVAL, "unknown field");
  }
  if (bytes < need) return fail(dom, LBMDEM_EINVAL, "destination too small");
  double* stage = (double*)((char*)dom->region + dom->L.stage);
  hipStream_t st = dom->stream;
  const hipMemcpyKind kind = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (field == LBMDEM_FIELD_FLAGS || field == LBMDEM_FIELD_OWNER) {
    std::vector<double> h(N);
    launch_fields(dom->d, first, stage, st);
    HIPCHK(dom, hipGetLastError());
    HIPCHK(dom, hipMemcpyAsync(h.data(), stage, 8 * N, hipMemcpyDeviceToHost, st));
    HIPCHK(dom, hipStreamSynchronize(st));
    if (field == LBMDEM_FIELD_FLAGS) {
      std::vector<uint8_t> o(N);
      for (size_t c = 0; c < N; ++c) o[c] = (uint8_t)h[c];
      HIPCHK(dom, hipMemcpy(dst, o.data(), N, dst_is_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
    } else {
      std::vector<int32_t> o(N);
      for (size_t c = 0; c < N; ++c) o[c] = (int32_t)h[c];
      HIPCHK(dom, hipMemcpy(dst, o.data(), 4 * N, dst_is_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
    }
    return LBMDEM_OK;
  }
  for (int k = 0; k < planes; ++k) {
    launch_fields(dom->d, first + k, stage, st);
    HIPCHK(dom, hipGetLastError());
    HIPCHK(dom, hipMemcpyAsync((char*)dst + 8 * N * (size_t)k, stage, 8 * N, kind, st));
    HIPCHK(dom, hipStreamSynchronize(st));
  }
  return LBMDEM_OK;
}

int32_t lbmdem_set_pdf(lbmdem_domain* dom, const double* f) {
  if (!dom || !f) return LBMDEM_EINVAL;
  if (dom->failed) return fail(dom, LBMDEM_ESTATE, "domain has failed");
  const size_t N = (size_t)dom->d.N;
  double* stage = (double*)((char*)dom->region + dom->L.stage);
  hipStream_t st = dom->stream;
  for (int q = 0; q < Q; ++q) {
    HIPCHK(dom, hipMemcpyAsync(stage, f + (size_t)q * N, 8 * N, hipMemcpyHostToDevice, st));
    launch_set_pdf(dom->d, q, stage, st);
    HIPCHK(dom, hipGetLastError());
    HIPCHK(dom, hipStreamSynchronize(st));
  }
  if (dom->d.fused) return LBMDEM_OK;  // links are formed by the next sweep
  if (int32_t rc = pin_mapped_positions(dom)) return rc;
  return remap(dom, false);
}

// ---- checkpoint ------------------------------------------------------------

namespace {

constexpr char CK_MAGIC[8] = {'L', 'B', 'M', 'D', 'E', 'M', 'C', 'K'};
constexpr uint32_t CK_VERSION = 3;

struct CkHeader {
  char magic[8];
  uint32_t version;
  uint32_t cfg_bytes;
  lbmdem_config cfg;
  int32_t cur;
  int32_t P;
  int32_t pad;
  uint64_t seg[3];  // bytes of: current PDF buffer, cell arrays, particle block
};

bool same_config(const lbmdem_config& a, const lbmdem_config& b) {
  bool eq = a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.collision == b.collision &&
            a.boundary == b.boundary && a.storage == b.storage && a.n_sub == b.n_sub &&
            a.force_averaging == b.force_averaging && a.lub_mask == b.lub_mask &&
            a.max_spheres == b.max_spheres && a.dem_kernel == b.dem_kernel && a.map_kernel == b.map_kernel;
  for (int k = 0; k < 3; ++k)
    eq = eq && a.walls[k] == b.walls[k] && a.wall_u_lo[k] == b.wall_u_lo[k] && a.wall_u_hi[k] == b.wall_u_hi[k] &&
         a.gravity[k] == b.gravity[k] && a.body_force[k] == b.body_force[k];
  eq = eq && a.nu == b.nu && a.magic_lambda == b.magic_lambda && a.lambda_b == b.lambda_b &&
       a.delta_ab == b.delta_ab && a.e_dry == b.e_dry && a.poisson_ratio == b.poisson_ratio &&
       a.friction == b.friction && a.tc == b.tc && a.dmin == b.dmin && a.cut_n == b.cut_n &&
       a.cut_tt == b.cut_tt && a.cut_tr == b.cut_tr && a.max_radius == b.max_radius;
  return eq;
}

// device segments of a checkpoint: the current PDF buffer, the cell arrays
// (flags, owners and, where the domain has them, claims, shell stamps and
// cell words) and the particle block
void ck_segments(const lbmdem_domain* dom, int cur, char** at, size_t* len) {
  char* base = (char*)dom->region;
  const Layout& L = dom->L;
  at[0] = base + (cur ? L.pdf1 : L.pdf0);
  len[0] = L.pdf1 - L.pdf0;
  at[1] = base + L.flags;
  len[1] = L.stage - L.flags;
  at[2] = base + L.x;
  len[2] = L.total - L.x;
}

}  // namespace

static int32_t read_ctl(lbmdem_domain* dom, DevCtl* c) {
  HIPCHK(dom, hipMemcpyAsync(c, dom->d.ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, dom->stream));
  HIPCHK(dom, hipStreamSynchronize(dom->stream));
  return LBMDEM_OK;
}

int32_t lbmdem_save(lbmdem_domain* dom, void* host_blob, size_t* bytes) {
  if (!dom || !bytes) return LBMDEM_EINVAL;
  DevCtl c;
  if (int32_t rc = read_ctl(dom, &c)) return rc;
  char* at[3];
  size_t len[3];
  ck_segments(dom, c.cur, at, len);
  const size_t P = dom->hR.size();
  const size_t need = sizeof(CkHeader) + 8 * P + len[0] + len[1] + len[2];
  if (!host_blob) {
    *bytes = need;
    return LBMDEM_OK;
  }
  if (*bytes < need) {
    *bytes = need;
    return fail(dom, LBMDEM_EINVAL, "checkpoint buffer too small");
  }
  CkHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, CK_MAGIC, 8);
  h.version = CK_VERSION;
  h.cfg_bytes = sizeof(lbmdem_config);
  h.cfg = dom->cfg;
  h.cur = c.cur;
  h.P = (int32_t)P;
  for (int k = 0; k < 3; ++k) h.seg[k] = len[k];
  char* out = (char*)host_blob;
  std::memcpy(out, &h, sizeof(h));
  out += sizeof(h);
  if (P) std::memcpy(out, dom->hR.data(), 8 * P);
  out += 8 * P;
  for (int k = 0; k < 3; ++k) {
    HIPCHK(dom, hipMemcpyAsync(out, at[k], len[k], hipMemcpyDeviceToHost, dom->stream));
    out += len[k];
  }
  HIPCHK(dom, hipStreamSynchronize(dom->stream));
  *bytes = need;
  return LBMDEM_OK;
}

int32_t lbmdem_restore(lbmdem_domain* dom, const void* host_blob, size_t bytes) {
  if (!dom || !host_blob) return LBMDEM_EINVAL;
  CkHeader h;
  if (bytes < sizeof(h)) return fail(dom, LBMDEM_EINVAL, "checkpoint truncated");
  std::memcpy(&h, host_blob, sizeof(h));
  if (std::memcmp(h.magic, CK_MAGIC, 8) != 0 || h.version != CK_VERSION || h.cfg_bytes != sizeof(lbmdem_config))
    return fail(dom, LBMDEM_EINVAL, "not a checkpoint of this library version");
  if (!same_config(h.cfg, dom->cfg)) return fail(dom, LBMDEM_EINVAL, "checkpoint of a different configuration");
  if (h.P < 0 || h.P > dom->cfg.max_spheres || (h.cur != 0 && h.cur != 1))
    return fail(dom, LBMDEM_EINVAL, "corrupt checkpoint header");
  HIPCHK(dom, hipStreamSynchronize(dom->stream));
  harvest(dom);
  char* at[3];
  size_t len[3];
  ck_segments(dom, h.cur, at, len);
  const size_t need = sizeof(CkHeader) + 8 * (size_t)h.P + len[0] + len[1] + len[2];
  if (bytes < need || h.seg[0] != len[0] || h.seg[1] != len[1] || h.seg[2] != len[2])
    return fail(dom, LBMDEM_EINVAL, "checkpoint size does not match this domain");
  const char* in = (const char*)host_blob + sizeof(h);
  dom->hR.assign((const double*)in, (const double*)in + h.P);
  in += 8 * (size_t)h.P;
  // the step state (current buffer, stamp, step count) is part of the
  // particle block
  for (int k = 0; k < 3; ++k) {
    HIPCHK(dom, hipMemcpyAsync(at[k], in, len[k], hipMemcpyHostToDevice, dom->stream));
    in += len[k];
  }
  HIPCHK(dom, hipStreamSynchronize(dom->stream));
  dom->d.P = h.P;
  dom->may_prescribe = true;  // the restored spheres' modes are not known here
  dom->failed = 0;
  return LBMDEM_OK;
}

int32_t lbmdem_set_stop_rule(lbmdem_domain* dom, int32_t rule, int64_t max_steps) {
  if (!dom) return LBMDEM_EINVAL;
  if (rule != STOP_NONE && rule != STOP_REBOUND) return fail(dom, LBMDEM_EINVAL, "unknown stop rule");
  DevCtl c;
  if (int32_t rc = read_ctl(dom, &c)) return rc;
  c.stop_rule = rule;
  c.max_steps = max_steps;
  c.stop_req = 0;
  c.frozen = 0;
  c.rb_phase = 0;
  HIPCHK(dom, hipMemcpyAsync(dom->d.ctl, &c, sizeof(DevCtl), hipMemcpyHostToDevice, dom->stream));
  HIPCHK(dom, hipStreamSynchronize(dom->stream));
  return LBMDEM_OK;
}

int32_t lbmdem_get_progress(lbmdem_domain* dom, int64_t* steps, int32_t* stopped) {
  if (!dom) return LBMDEM_EINVAL;
  DevCtl c;
  if (int32_t rc = read_ctl(dom, &c)) return rc;
  if (steps) *steps = c.steps;
  if (stopped) *stopped = (c.frozen || c.stop_req) ? 1 : 0;
  return LBMDEM_OK;
}

int32_t lbmdem_set_profiling(lbmdem_domain* dom, int32_t enable) {
  if (!dom) return LBMDEM_EINVAL;
  HIPCHK(dom, hipStreamSynchronize(dom->stream));
  harvest(dom);
  dom->prof = enable < 0 ? 0 : (enable > 2 ? 2 : enable);
  for (int k = 0; k < 3; ++k) {
    dom->ms[k] = 0.0;
    dom->cnt[k] = 0;
  }
  return LBMDEM_OK;
}

int32_t lbmdem_get_profile(lbmdem_domain* dom, int32_t kernel, double* total_ms, int64_t* count) {
  if (!dom || kernel < 0 || kernel > 2) return LBMDEM_EINVAL;
  HIPCHK(dom, hipStreamSynchronize(dom->stream));
  harvest(dom);
  if (total_ms) *total_ms = dom->ms[kernel];
  if (count) *count = dom->cnt[kernel];
  return LBMDEM_OK;
}

double lbmdem_sweep_bytes(const lbmdem_domain* dom) {
  if (!dom) return 0.0;
  return (2.0 * Q * (double)storage_size(dom->cfg.storage) + 1.0) * (double)dom->d.N;
}

int32_t lbmdem_device_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (!dst || !src) return LBMDEM_EINVAL;
  launch_copy(dst, src, bytes, (hipStream_t)hip_stream);
  return hipGetLastError() == hipSuccess ? LBMDEM_OK : LBMDEM_EDEVICE;
}

const char* lbmdem_last_error(const lbmdem_domain* dom) {
  return dom ? dom->err.c_str() : g_create_error.c_str();
}

}  // extern "C"

// ---- batches ------------------------------------------------------------------

__global__ void k_batch_status(const DevDomain* __restrict__ tab, int ndom, long long* steps, int* stopped) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ndom) return;
  const DevCtl* c = tab[k].ctl;
  steps[k] = c->steps;
  stopped[k] = (c->frozen || c->stop_req) ? 1 : 0;
}

struct lbmdem_batch {
  hipStream_t stream = nullptr;
  size_t pool = 0, used = 0;
  int use_graph = 1;
  int storage = -1;
  std::vector<lbmdem_domain*> doms;
  std::vector<int32_t> slots;
  int32_t next_slot = 0;
  // device tables: descriptors, block starts of the three launch kinds, status
  void* dmem = nullptr;
  size_t dmem_bytes = 0;
  BatchTables t{};
  long long* d_steps = nullptr;
  int* d_stopped = nullptr;
  bool dirty = true;
  std::vector<int> built_P;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // side stream of the DEM and the claims beside the sweep, and the events
  // that fork and join it (also inside a captured graph)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::string err;
};

static int32_t bfail(lbmdem_batch* b, int32_t code, const std::string& msg) {
  if (b) b->err = msg;
  return code;
}

#define BHIPCHK(b, call)                                                                \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return bfail(b, LBMDEM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

static void drop_graph(lbmdem_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// rebuilds the device tables when the admitted domains or their sphere counts
// changed
static int32_t build_tables(lbmdem_batch* b) {
  const int nd = (int)b->doms.size();
  std::vector<int> P(nd);
  for (int k = 0; k < nd; ++k) P[k] = (int)b->doms[k]->hR.size();
  if (!b->dirty && P == b->built_P) return LBMDEM_OK;
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  drop_graph(b);
  std::vector<DevDomain> tab(nd);
  std::vector<int> ss(nd + 1, 0), cs(nd + 1, 0), ms(nd + 1, 0);
  for (int k = 0; k < nd; ++k) {
    lbmdem_domain* dom = b->doms[k];
    dom->d.P = P[k];
    tab[k] = dom->d;
    const DevDomain& d = dom->d;
    ss[k + 1] = ss[k] + (int)((d.N + 255) / 256);
    cs[k + 1] = cs[k] + d.P * d.ZB;
    ms[k + 1] = ms[k] + d.P * d.ZB * d.RB;
  }
  const size_t tb = align256(sizeof(DevDomain) * (size_t)std::max(nd, 1));
  const size_t ib = align256(4 * (size_t)(nd + 1));
  const size_t need = tb + 3 * ib + align256(8 * (size_t)std::max(nd, 1)) + align256(4 * (size_t)std::max(nd, 1));
  if (need > b->dmem_bytes) {
    if (b->dmem) BHIPCHK(b, hipFree(b->dmem));
    b->dmem = nullptr;
    b->dmem_bytes = 0;
    BHIPCHK(b, hipMalloc(&b->dmem, need));
    b->dmem_bytes = need;
  }
  char* m = (char*)b->dmem;
  if (nd) BHIPCHK(b, hipMemcpyAsync(m, tab.data(), sizeof(DevDomain) * nd, hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipMemcpyAsync(m + tb, ss.data(), 4 * (nd + 1), hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipMemcpyAsync(m + tb + ib, cs.data(), 4 * (nd + 1), hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipMemcpyAsync(m + tb + 2 * ib, ms.data(), 4 * (nd + 1), hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  b->t.tab = (const DevDomain*)m;
  b->t.sweep_start = (const int*)(m + tb);
  b->t.claim_start = (const int*)(m + tb + ib);
  b->t.commit_start = (const int*)(m + tb + 2 * ib);
  b->t.ndom = nd;
  b->t.sweep_blocks = ss[nd];
  b->t.claim_blocks = cs[nd];
  b->t.commit_blocks = ms[nd];
  b->t.storage = b->storage;
  b->d_steps = (long long*)(m + tb + 3 * ib);
  b->d_stopped = (int*)(m + tb + 3 * ib + align256(8 * (size_t)std::max(nd, 1)));
  b->built_P = P;
  b->dirty = false;
  return LBMDEM_OK;
}

// One step of every domain: the sweep and, beside it on the side stream, the
// DEM sub-cycles and the claims (they need the previous step's forces only);
// then reconstruction, the boundary pass and the step control.
static hipError_t launch_batch_step(lbmdem_batch* b) {
  hipError_t e = hipEventRecord(b->ev_fork, b->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->side, b->ev_fork, 0);
  if (e != hipSuccess) return e;
  launch_dem_batch(b->t, b->side);
  launch_claim_batch(b->t, b->side);
  launch_sweep_batch(b->t, b->stream);
  e = hipEventRecord(b->ev_join, b->side);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_join, 0);
  if (e != hipSuccess) return e;
  launch_update_batch(b->t, b->stream);
  launch_advance_batch(b->t, b->stream);
  return hipGetLastError();
}

extern "C" {

int32_t lbmdem_batch_create(void* hip_stream, size_t pool_bytes, lbmdem_batch** out) {
  if (!out) return LBMDEM_EINVAL;
  lbmdem_batch* b = new (std::nothrow) lbmdem_batch();
  if (!b) return LBMDEM_ENOMEM;
  b->stream = (hipStream_t)hip_stream;
  b->pool = pool_bytes;
  if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) != hipSuccess) {
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    delete b;
    return LBMDEM_EDEVICE;
  }
  *out = b;
  return LBMDEM_OK;
}

int32_t lbmdem_batch_destroy(lbmdem_batch* b) {
  if (!b) return LBMDEM_OK;
  (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  for (auto* d : b->doms) d->batch = nullptr;
  if (b->dmem) (void)hipFree(b->dmem);
  (void)hipStreamSynchronize(b->side);
  (void)hipStreamDestroy(b->side);
  (void)hipEventDestroy(b->ev_fork);
  (void)hipEventDestroy(b->ev_join);
  delete b;
  return LBMDEM_OK;
}

int32_t lbmdem_batch_set_graph(lbmdem_batch* b, int32_t use_graph) {
  if (!b) return LBMDEM_EINVAL;
  (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  b->use_graph = use_graph ? 1 : 0;
  return LBMDEM_OK;
}

int32_t lbmdem_batch_admit(lbmdem_batch* b, lbmdem_domain* dom, int32_t* slot) {
  if (!b || !dom) return LBMDEM_EINVAL;
  if (dom->failed) return bfail(b, LBMDEM_ESTATE, "domain has failed");
  if (dom->batch) return bfail(b, LBMDEM_EINVAL, "domain already belongs to a batch");
  if (dom->stream != b->stream) return bfail(b, LBMDEM_EINVAL, "domain was created on another stream");
  if (b->storage >= 0 && dom->cfg.storage != b->storage)
    return bfail(b, LBMDEM_EINVAL, "all domains of a batch share one storage precision");
  if (dom->d.map_ball || dom->d.fused)
    return bfail(b, LBMDEM_EINVAL, "batched domains use the slab boundary pass (map_kernel 1)");
  const size_t fp = dom->L.total;
  if (b->used + fp > b->pool) return bfail(b, LBMDEM_ENOMEM, "pool budget exceeded");
  b->storage = dom->cfg.storage;
  b->used += fp;
  b->doms.push_back(dom);
  b->slots.push_back(b->next_slot);
  if (slot) *slot = b->next_slot;
  b->next_slot++;
  dom->batch = b;
  b->dirty = true;
  return LBMDEM_OK;
}

int32_t lbmdem_batch_retire(lbmdem_batch* b, lbmdem_domain* dom) {
  if (!b || !dom) return LBMDEM_EINVAL;
  for (size_t k = 0; k < b->doms.size(); ++k)
    if (b->doms[k] == dom) {
      b->doms.erase(b->doms.begin() + k);
      b->slots.erase(b->slots.begin() + k);
      b->used -= dom->L.total;
      dom->batch = nullptr;
      b->dirty = true;
      return LBMDEM_OK;
    }
  return bfail(b, LBMDEM_EINVAL, "domain is not in this batch");
}

int32_t lbmdem_batch_step(lbmdem_batch* b, int32_t nsteps) {
  if (!b || nsteps < 0) return LBMDEM_EINVAL;
  if (int32_t rc = build_tables(b)) return rc;
  if (b->t.ndom == 0 || nsteps == 0) return LBMDEM_OK;
  if (!b->use_graph) {
    for (int s = 0; s < nsteps; ++s) BHIPCHK(b, launch_batch_step(b));
    return LBMDEM_OK;
  }
  if (!b->exec) {
    BHIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const hipError_t el = launch_batch_step(b);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (e == hipSuccess && el != hipSuccess) e = el;
    if (e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return bfail(b, LBMDEM_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    b->graph = g;
    BHIPCHK(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  for (int s = 0; s < nsteps; ++s) BHIPCHK(b, hipGraphLaunch(b->exec, b->stream));
  return LBMDEM_OK;
}

int32_t lbmdem_batch_status(lbmdem_batch* b, int32_t* slots, int64_t* steps, int32_t* stopped, int32_t* n) {
  if (!b || !n) return LBMDEM_EINVAL;
  if (int32_t rc = build_tables(b)) return rc;
  const int nd = b->t.ndom;
  if (*n < nd) {
    *n = nd;
    return bfail(b, LBMDEM_EINVAL, "output arrays too small");
  }
  std::vector<long long> hs(nd);
  std::vector<int> hf(nd);
  if (nd) {
    hipLaunchKernelGGL(k_batch_status, dim3((nd + 255) / 256), dim3(256), 0, b->stream, b->t.tab, nd, b->d_steps,
                       b->d_stopped);
    BHIPCHK(b, hipGetLastError());
    BHIPCHK(b, hipMemcpyAsync(hs.data(), b->d_steps, 8 * nd, hipMemcpyDeviceToHost, b->stream));
    BHIPCHK(b, hipMemcpyAsync(hf.data(), b->d_stopped, 4 * nd, hipMemcpyDeviceToHost, b->stream));
  }
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  for (int k = 0; k < nd; ++k) {
    if (slots) slots[k] = b->slots[k];
    if (steps) steps[k] = hs[k];
    if (stopped) stopped[k] = hf[k];
  }
  *n = nd;
  return LBMDEM_OK;
}

int32_t lbmdem_batch_done(lbmdem_batch* b, int32_t* slots, int32_t* n) {
  if (!b || !n || (*n > 0 && !slots)) return LBMDEM_EINVAL;
  const int cap = *n;
  int32_t nd = (int32_t)b->doms.size();
  std::vector<int32_t> sl(nd), st(nd);
  if (int32_t rc = lbmdem_batch_status(b, sl.data(), nullptr, st.data(), &nd)) return rc;
  int m = 0;
  for (int k = 0; k < nd; ++k)
    if (st[k]) {
      if (m < cap) slots[m] = sl[k];
      ++m;
    }
  *n = m;
  return m > cap ? bfail(b, LBMDEM_EINVAL, "output array too small") : LBMDEM_OK;
}

const char* lbmdem_batch_last_error(const lbmdem_batch* b) { return b ? b->err.c_str() : ""; }

}  // extern "C"
