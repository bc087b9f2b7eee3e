// Fused D3Q19 pull stream + TRT+aB collide of one cell (Eqs. LBM_Stream,
// LBM_Collide, MRT with the rates of Eqs. TRTmatrix / TRTbulkmatrix, adaptive
// shell of Sec. 2.3.2), shared by the plain sweep and the sweep that also forms
// the particle-link boundary values.  See sweep.hip for the arithmetic.
#pragma once

#include "internal.hpp"

namespace lbmdem {

template <typename T>
struct Store;

template <>
struct Store<double> {
  using C = double;
  __device__ static inline double load(const double* p) { return *p; }
  __device__ static inline double load_nt(const double* p) { return __builtin_nontemporal_load(p); }
  __device__ static inline void store(double* p, double v) { __builtin_nontemporal_store(v, p); }
};

template <>
struct Store<float> {
  using C = float;
  __device__ static inline float load(const float* p) { return *p; }
  __device__ static inline float load_nt(const float* p) { return __builtin_nontemporal_load(p); }
  __device__ static inline void store(float* p, float v) { __builtin_nontemporal_store(v, p); }
};

template <>
struct Store<__half> {
  using C = float;
  __device__ static inline float load(const __half* p) { return __half2float(*p); }
  __device__ static inline float load_nt(const __half* p) {
    const unsigned short b = __builtin_nontemporal_load(reinterpret_cast<const unsigned short*>(p));
    return __half2float(*reinterpret_cast<const __half*>(&b));
  }
  __device__ static inline void store(__half* p, float v) {
    __half h = __float2half_rn(v);
    __builtin_nontemporal_store(*reinterpret_cast<unsigned short*>(&h),
                                reinterpret_cast<unsigned short*>(p));
  }
};

// Moving-wall bounce-back of direction q (c = (cx, cy, cz), weight w, opposite
// qb): the value pulled from the wall cell x - c_q becomes
// f~_qb(x) + 6 w (u_w . c_q); in deviations the weights cancel.
#define WALL_BB(q, qb, w, cx, cy, cz, ux, uy, uz)                                         \
  g[q] = (C)((double)Store<T>::load(src + (size_t)(qb) * NN + idx) +                       \
             6.0 * (w) * ((ux) * (cx) + (uy) * (cy) + (uz) * (cz)))

// The five directions whose source lies across one wall layer, per side.  The
// x and y layers rest; a value from an edge cell shared with a z layer takes
// that layer's velocity (the z rules run last).
#define WALLS_XP(ux, uy, uz)                                              \
  WALL_BB(4, 3, W1, 1, 0, 0, ux, uy, uz); WALL_BB(8, 9, W2, 1, 1, 0, ux, uy, uz); \
  WALL_BB(10, 7, W2, 1, -1, 0, ux, uy, uz); WALL_BB(14, 17, W2, 1, 0, 1, ux, uy, uz); \
  WALL_BB(18, 13, W2, 1, 0, -1, ux, uy, uz)
#define WALLS_XM(ux, uy, uz)                                              \
  WALL_BB(3, 4, W1, -1, 0, 0, ux, uy, uz); WALL_BB(7, 10, W2, -1, 1, 0, ux, uy, uz); \
  WALL_BB(9, 8, W2, -1, -1, 0, ux, uy, uz); WALL_BB(13, 18, W2, -1, 0, 1, ux, uy, uz); \
  WALL_BB(17, 14, W2, -1, 0, -1, ux, uy, uz)
#define WALLS_YP(ux, uy, uz)                                              \
  WALL_BB(1, 2, W1, 0, 1, 0, ux, uy, uz); WALL_BB(7, 10, W2, -1, 1, 0, ux, uy, uz); \
  WALL_BB(8, 9, W2, 1, 1, 0, ux, uy, uz); WALL_BB(11, 16, W2, 0, 1, 1, ux, uy, uz); \
  WALL_BB(15, 12, W2, 0, 1, -1, ux, uy, uz)
#define WALLS_YM(ux, uy, uz)                                              \
  WALL_BB(2, 1, W1, 0, -1, 0, ux, uy, uz); WALL_BB(9, 8, W2, -1, -1, 0, ux, uy, uz); \
  WALL_BB(10, 7, W2, 1, -1, 0, ux, uy, uz); WALL_BB(12, 15, W2, 0, -1, 1, ux, uy, uz); \
  WALL_BB(16, 11, W2, 0, -1, -1, ux, uy, uz)
#define WALLS_ZP(ux, uy, uz)                                              \
  WALL_BB(5, 6, W1, 0, 0, 1, ux, uy, uz); WALL_BB(11, 16, W2, 0, 1, 1, ux, uy, uz); \
  WALL_BB(12, 15, W2, 0, -1, 1, ux, uy, uz); WALL_BB(13, 18, W2, -1, 0, 1, ux, uy, uz); \
  WALL_BB(14, 17, W2, 1, 0, 1, ux, uy, uz)
#define WALLS_ZM(ux, uy, uz)                                              \
  WALL_BB(6, 5, W1, 0, 0, -1, ux, uy, uz); WALL_BB(15, 12, W2, 0, 1, -1, ux, uy, uz); \
  WALL_BB(16, 11, W2, 0, -1, -1, ux, uy, uz); WALL_BB(17, 14, W2, -1, 0, -1, ux, uy, uz); \
  WALL_BB(18, 13, W2, 1, 0, -1, ux, uy, uz)

// FORCED: a fluid body force a by Guo's scheme, written in velocity space:
// the equilibrium takes u = j + a/2, and the collision adds
// (1 - s+/2) F+ + (1 - s-/2) F- with F+_q = w_q (9 (c.u)(c.a) - 3 u.a) and
// F-_q = 3 w_q c.a (the even and odd parts of Guo's source term); of the two
// bulk rows only the kinetic-energy row sees F+ (M_4 . F+ = 2 u.a, M_5 . F+ =
// 0), which adds -3/2 (s_b - s+) u.a to that row's correction.  On the
// conserved momentum TRT's odd rate and the moment-space rate 0 give the same
// j + a.
// Pull of the 19 values of cell (x, y, z) (index idx) from the source buffer,
// with the values that come from a wall layer replaced by the moving-wall
// bounce-back of Sec. 2.2.
template <typename T, bool NTLOAD = false>
__device__ __forceinline__ void pull_cell(const DevDomain& d, const T* __restrict__ src, int x, int y, int z,
                                          unsigned int idx, typename Store<T>::C* g) {
  using C = typename Store<T>::C;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const unsigned int nxy = (unsigned int)nx * (unsigned int)ny;

  // source of direction q is x - c_q: index [1 - c] of these triples
  const unsigned int X0 = (unsigned int)(x == 0 ? nx - 1 : x - 1), X1 = (unsigned int)x,
                     X2 = (unsigned int)(x == nx - 1 ? 0 : x + 1);
  const unsigned int Y0 = (unsigned int)(y == 0 ? ny - 1 : y - 1) * (unsigned int)nx,
                     Y1 = (unsigned int)y * (unsigned int)nx,
                     Y2 = (unsigned int)(y == ny - 1 ? 0 : y + 1) * (unsigned int)nx;
  const unsigned int Z0 = (unsigned int)(z == 0 ? nz - 1 : z - 1) * nxy, Z1 = (unsigned int)z * nxy,
                     Z2 = (unsigned int)(z == nz - 1 ? 0 : z + 1) * nxy;

  const size_t NN = (size_t)d.N;
#define LD(q, xs, ys, zs) \
  (NTLOAD ? Store<T>::load_nt(src + (size_t)(q) * NN + (xs + ys + zs)) : Store<T>::load(src + (size_t)(q) * NN + (xs + ys + zs)))
  g[0] = LD(0, X1, Y1, Z1);
  g[1] = LD(1, X1, Y0, Z1);    // c = ( 0, 1, 0)
  g[2] = LD(2, X1, Y2, Z1);    // c = ( 0,-1, 0)
  g[3] = LD(3, X2, Y1, Z1);    // c = (-1, 0, 0)
  g[4] = LD(4, X0, Y1, Z1);    // c = ( 1, 0, 0)
  g[5] = LD(5, X1, Y1, Z0);    // c = ( 0, 0, 1)
  g[6] = LD(6, X1, Y1, Z2);    // c = ( 0, 0,-1)
  g[7] = LD(7, X2, Y0, Z1);    // c = (-1, 1, 0)
  g[8] = LD(8, X0, Y0, Z1);    // c = ( 1, 1, 0)
  g[9] = LD(9, X2, Y2, Z1);    // c = (-1,-1, 0)
  g[10] = LD(10, X0, Y2, Z1);  // c = ( 1,-1, 0)
  g[11] = LD(11, X1, Y0, Z0);  // c = ( 0, 1, 1)
  g[12] = LD(12, X1, Y2, Z0);  // c = ( 0,-1, 1)
  g[13] = LD(13, X2, Y1, Z0);  // c = (-1, 0, 1)
  g[14] = LD(14, X0, Y1, Z0);  // c = ( 1, 0, 1)
  g[15] = LD(15, X1, Y0, Z2);  // c = ( 0, 1,-1)
  g[16] = LD(16, X1, Y2, Z2);  // c = ( 0,-1,-1)
  g[17] = LD(17, X2, Y1, Z2);  // c = (-1, 0,-1)
  g[18] = LD(18, X0, Y1, Z2);  // c = ( 1, 0,-1)
#undef LD

  {
    // cells next to a wall layer (block-uniform for z walls)
    constexpr double W1 = 1.0 / 18.0, W2 = 1.0 / 36.0;
    if (d.walls[0]) {
      if (x == 1) { WALLS_XP(0.0, 0.0, 0.0); }
      if (x == nx - 2) { WALLS_XM(0.0, 0.0, 0.0); }
    }
    if (d.walls[1]) {
      if (y == 1) { WALLS_YP(0.0, 0.0, 0.0); }
      if (y == ny - 2) { WALLS_YM(0.0, 0.0, 0.0); }
    }
    if (d.walls[2]) {
      if (z == 1) { WALLS_ZP(d.wall_u_lo[0], d.wall_u_lo[1], d.wall_u_lo[2]); }
      if (z == nz - 2) { WALLS_ZM(d.wall_u_hi[0], d.wall_u_hi[1], d.wall_u_hi[2]); }
    }
  }
}

// TRT+aB collision of the pulled values g (deviations) of the cell with flag
// byte fl and storage of the results into slot idx of dst.
template <typename T, bool FORCED>
__device__ __forceinline__ void collide_store(const DevDomain& d, T* __restrict__ dst, unsigned int idx, uint8_t fl,
                                              typename Store<T>::C* g, typename Store<T>::C sp,
                                              typename Store<T>::C sm, typename Store<T>::C db_shell,
                                              typename Store<T>::C db_other) {
  using C = typename Store<T>::C;
  const size_t NN = (size_t)d.N;
  // moments (rho0 = 1: u = j; deviations carry no mass or momentum of w_q)
  const C sumd = ((g[7] + g[8]) + (g[9] + g[10])) + ((g[11] + g[12]) + (g[13] + g[14])) +
                 ((g[15] + g[16]) + (g[17] + g[18]));
  const C suma = ((g[1] + g[2]) + (g[3] + g[4])) + (g[5] + g[6]);
  const C rho = (g[0] + suma) + sumd;  // rho - 1
  C ux = ((g[4] - g[3]) + (g[8] - g[7])) + ((g[10] - g[9]) + (g[14] - g[13])) + (g[18] - g[17]);
  C uy = ((g[1] - g[2]) + (g[7] + g[8])) - ((g[9] + g[10]) - (g[11] - g[12])) + (g[15] - g[16]);
  C uz = ((g[5] - g[6]) + (g[11] + g[12])) + ((g[13] + g[14]) - (g[15] + g[16])) - (g[17] + g[18]);
  C ax = C(0), ay = C(0), az = C(0), ua = C(0);
  if (FORCED) {
    ax = (C)d.force[0];
    ay = (C)d.force[1];
    az = (C)d.force[2];
    ux += C(0.5) * ax;
    uy += C(0.5) * ay;
    uz += C(0.5) * az;
    ua = ux * ax + uy * ay + uz * az;
  }
  const C usq = ux * ux + uy * uy + uz * uz;

  // bulk correction amplitudes (rows 4 and 5 of M, 0-based)
  const C db = (fl & F_SHELL) ? db_shell : db_other;  // s_b - s+
  const C m4 = sumd - g[0];
  const C m5 = (g[0] - C(2) * suma) + sumd;
  const C A4 = db * (C(1.5) * (FORCED ? (usq - m4) - ua : usq - m4));
  const C A5 = db * (C(-0.5) * m5);

  const C w0 = C(1.0 / 3.0), w1 = C(1.0 / 18.0), w2 = C(1.0 / 36.0);
  C o[Q];
  {
    const C e0 = w0 * (rho - C(1.5) * usq);
    o[0] = (g[0] - sp * (g[0] - e0)) + w0 * (A5 - A4);
  }
  const C ba = C(-2) * w1 * A5;
  const C bd = w2 * (A4 + A5);
  const C base1 = w1 * (rho - C(1.5) * usq);
  const C base2 = w2 * (rho - C(1.5) * usq);
#define PAIR(a, b, w, base, cu, bulk)                 \
  {                                                   \
    const C cu_ = (cu);                               \
    const C ep = (base) + C(4.5) * (w) * cu_ * cu_;   \
    const C em = C(3) * (w) * cu_;                    \
    const C gp = C(0.5) * (g[a] + g[b]);              \
    const C gm = C(0.5) * (g[a] - g[b]);              \
    const C dp = sp * (gp - ep);                      \
    const C dm = sm * (gm - em);                      \
    o[a] = ((g[a] - dp) - dm) + (bulk);               \
    o[b] = ((g[b] - dp) + dm) + (bulk);               \
  }
  PAIR(1, 2, w1, base1, uy, ba)
  PAIR(4, 3, w1, base1, ux, ba)
  PAIR(5, 6, w1, base1, uz, ba)
  PAIR(7, 10, w2, base2, uy - ux, bd)
  PAIR(8, 9, w2, base2, ux + uy, bd)
  PAIR(11, 16, w2, base2, uy + uz, bd)
  PAIR(12, 15, w2, base2, uz - uy, bd)
  PAIR(13, 18, w2, base2, uz - ux, bd)
  PAIR(14, 17, w2, base2, ux + uz, bd)
#undef PAIR

  if (FORCED) {
    const C cp = C(1) - C(0.5) * sp, cm = C(1) - C(0.5) * sm;
    o[0] += cp * (w0 * (C(-3) * ua));
#define FPAIR(a, b, w, cu, ca)                                 \
  {                                                            \
    const C ca_ = (ca);                                        \
    const C fp = cp * ((w) * (C(9) * (cu) * ca_ - C(3) * ua)); \
    const C fm = cm * ((w) * (C(3) * ca_));                    \
    o[a] += fp + fm;                                           \
    o[b] += fp - fm;                                           \
  }
    FPAIR(1, 2, w1, uy, ay)
    FPAIR(4, 3, w1, ux, ax)
    FPAIR(5, 6, w1, uz, az)
    FPAIR(7, 10, w2, uy - ux, ay - ax)
    FPAIR(8, 9, w2, ux + uy, ax + ay)
    FPAIR(11, 16, w2, uy + uz, ay + az)
    FPAIR(12, 15, w2, uz - uy, az - ay)
    FPAIR(13, 18, w2, uz - ux, az - ax)
    FPAIR(14, 17, w2, ux + uz, ax + az)
#undef FPAIR
  }

#pragma unroll
  for (int q = 0; q < Q; ++q) Store<T>::store(dst + (size_t)q * NN + idx, o[q]);
}

template <typename T, bool FORCED, bool NTLOAD = false>
__device__ __forceinline__ void sweep_cell(const DevDomain& d, const T* __restrict__ src, T* __restrict__ dst,
                                           int x, int y, int z, typename Store<T>::C sp,
                                           typename Store<T>::C sm, typename Store<T>::C db_shell,
                                           typename Store<T>::C db_other) {
  using C = typename Store<T>::C;
  const unsigned int idx = (unsigned int)x + (unsigned int)d.nx * (unsigned int)y +
                           (unsigned int)d.nx * (unsigned int)d.ny * (unsigned int)z;
  const uint8_t fl = d.flags[idx];
  C g[Q];
  pull_cell<T, NTLOAD>(d, src, x, y, z, idx, g);
  collide_store<T, FORCED>(d, dst, idx, fl, g, sp, sm, db_shell, db_other);
}
#undef WALL_BB
#undef WALLS_XP
#undef WALLS_XM
#undef WALLS_YP
#undef WALLS_YM
#undef WALLS_ZP
#undef WALLS_ZM


}  // namespace lbmdem
