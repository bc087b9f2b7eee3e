// Domain initialisation, field read-out/write-in and a plain copy kernel.
#include "internal.hpp"

namespace lbmdem {

// fluid at rest (deviation 0), wall layers flagged, claims cleared
template <typename T>
__global__ void k_init(DevDomain d) {
  const size_t N = (size_t)d.N;
  T* a = (T*)d.pdf[0];
  T* b = (T*)d.pdf[1];
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N;
       c += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % d.nx);
    const int j = (int)((c / d.nx) % d.ny);
    const int k = (int)(c / ((size_t)d.nx * d.ny));
    const bool wall = (d.walls[0] && (i == 0 || i == d.nx - 1)) ||
                      (d.walls[1] && (j == 0 || j == d.ny - 1)) ||
                      (d.walls[2] && (k == 0 || k == d.nz - 1));
    d.flags[c] = wall ? F_WALL : 0;
    d.owner[c] = -1;
    if (d.claim) {
      d.claim[c] = 0ull;
      d.shellstamp[c] = 0u;
    }
    if (d.cellw) d.cellw[c] = wall ? F_WALL : 0u;
    for (int q = 0; q < Q; ++q) {
      a[(size_t)q * N + c] = T(0.0f);
      b[(size_t)q * N + c] = T(0.0f);
    }
  }
}

template <typename T>
__device__ inline double to_d(T v) {
  return (double)v;
}
template <>
__device__ inline double to_d<__half>(__half v) {
  return (double)__half2float(v);
}

// which: 0 rho, 1..3 velocity component, 10+q PDF plane q (full f),
// 40 canonical flags, 41 owner (as double), 60+q plane q as stored (full f)
// in every cell, solid and wall cells included
template <typename T>
__global__ void k_get_plane(DevDomain d, int which, double* dst) {
  const int cur = d.ctl->cur;
  const size_t N = (size_t)d.N;
  const T* f = (const T*)d.pdf[cur];
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N;
       c += (size_t)gridDim.x * blockDim.x) {
    const uint8_t fl = d.flags[c];
    const bool fluid = !(fl & (F_SOLID | F_WALL));
    double v = 0.0;
    if (which == 40) {
      v = (fl & F_WALL) ? 3.0 : ((fl & F_SOLID) ? 2.0 : ((fl & F_SHELL) ? 1.0 : 0.0));
    } else if (which == 41) {
      v = (fl & F_SOLID) ? (double)d.owner[c] : -1.0;
    } else if (which >= 60) {
      const int q = which - 60;
      v = to_d<T>(f[(size_t)q * N + c]) + WQ[q];
    } else if (fluid) {
      if (which >= 10) {
        const int q = which - 10;
        v = to_d<T>(f[(size_t)q * N + c]) + WQ[q];
      } else {
        double s = 0.0;
        for (int q = 0; q < Q; ++q) {
          const double g = to_d<T>(f[(size_t)q * N + c]);
          const int cq = which == 0 ? 1 : (which == 1 ? CX[q] : (which == 2 ? CY[q] : CZ[q]));
          s += g * cq;
        }
        // with a body force the stored (post-collision) momentum holds the
        // whole impulse a; the velocity is half-way
        const double a = which == 1 ? d.force[0] : (which == 2 ? d.force[1] : d.force[2]);
        v = which == 0 ? 1.0 + s : s - 0.5 * a;
      }
    }
    dst[c] = v;
  }
}

template <typename T>
__device__ inline T from_d(double v) {
  return (T)v;
}
template <>
__device__ inline __half from_d<__half>(double v) {
  return __float2half_rn((float)v);
}

template <typename T>
__global__ void k_set_plane(DevDomain d, int q, const double* src) {
  const int cur = d.ctl->cur;
  const size_t N = (size_t)d.N;
  T* f = (T*)d.pdf[cur];
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N;
       c += (size_t)gridDim.x * blockDim.x)
    f[(size_t)q * N + c] = from_d<T>(src[c] - WQ[q]);
}

__global__ void k_copy16(uint4* __restrict__ dst, const uint4* __restrict__ src, size_t n16) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void k_copy1(uint8_t* dst, const uint8_t* src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Density at points (xyz[3n], lattice units) by trilinear interpolation of
// the cell-centre densities of the current state (periodic axes wrap); NaN
// when one of the eight cells is not fluid or lies outside a walled axis.
// Buffer io: the 3n coordinates, then the n results.
template <typename T>
__global__ void k_probe_density(DevDomain d, double* io, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const size_t N = (size_t)d.N;
  const T* f = (const T*)(d.ctl->cur ? d.pdf[1] : d.pdf[0]);
  const int nn[3] = {d.nx, d.ny, d.nz};
  int i0[3];
  double t[3];
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double s = io[3 * k + a] - 0.5;
    const double fl = floor(s);
    i0[a] = (int)fl;
    t[a] = s - fl;
    if (d.walls[a]) ok = ok && i0[a] >= 0 && i0[a] + 1 < nn[a];
  }
  double r = 0.0;
  if (ok) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      int ijk[3];
      double w = 1.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int o = (c >> a) & 1;
        ijk[a] = d.walls[a] ? i0[a] + o : wrapmod(i0[a] + o, nn[a]);
        w *= o ? t[a] : 1.0 - t[a];
      }
      const size_t cc = (size_t)cidx(d, ijk[0], ijk[1], ijk[2]);
      if (d.flags[cc] & (F_SOLID | F_WALL)) ok = false;
      double rho = 1.0;
      for (int q = 0; q < Q; ++q) rho += to_d<T>(f[(size_t)q * N + cc]);
      r += w * rho;
    }
  }
  io[3 * (size_t)n + k] = ok ? r : __builtin_nan("");
}

void launch_probe_density(const DevDomain& d, double* io, int n, hipStream_t s) {
  const dim3 g((unsigned)((n + 255) / 256));
  if (d.storage == 0)
    hipLaunchKernelGGL(k_probe_density<double>, g, dim3(256), 0, s, d, io, n);
  else if (d.storage == 1)
    hipLaunchKernelGGL(k_probe_density<float>, g, dim3(256), 0, s, d, io, n);
  else
    hipLaunchKernelGGL(k_probe_density<__half>, g, dim3(256), 0, s, d, io, n);
}

// Health check of the fluid: the density 1 + sum_q g_q of up to
// DENSITY_SAMPLES fluid cells spread over the lattice by a multiplicative
// hash (the same cells on every call); one outside (0.5, 1.5), or not finite,
// raises ST_DENSITY.
constexpr int DENSITY_SAMPLES = 65536;
template <typename T>
__global__ void k_density_check(DevDomain d, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const size_t N = (size_t)d.N;
  const size_t c = n == (int)N ? (size_t)k : (size_t)(((unsigned long long)k * 2654435761ull) % N);
  if (d.flags[c] & (F_SOLID | F_WALL)) return;
  const T* f = (const T*)(d.ctl->cur ? d.pdf[1] : d.pdf[0]);
  double rho = 1.0;
  for (int q = 0; q < Q; ++q) rho += to_d<T>(f[(size_t)q * N + c]);
  if (!(rho > 0.5 && rho < 1.5)) atomicOr(d.status, ST_DENSITY);
}

void launch_density_check(const DevDomain& d, hipStream_t s) {
  const int n = d.N < (long long)DENSITY_SAMPLES ? (int)d.N : DENSITY_SAMPLES;
  const dim3 g((unsigned)((n + 255) / 256));
  if (d.storage == 0)
    hipLaunchKernelGGL(k_density_check<double>, g, dim3(256), 0, s, d, n);
  else if (d.storage == 1)
    hipLaunchKernelGGL(k_density_check<float>, g, dim3(256), 0, s, d, n);
  else
    hipLaunchKernelGGL(k_density_check<__half>, g, dim3(256), 0, s, d, n);
}

static dim3 grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

void launch_fill_claims(const DevDomain& d, hipStream_t s) {
  if (d.storage == 0)
    hipLaunchKernelGGL(k_init<double>, grid_for(d.N), dim3(256), 0, s, d);
  else if (d.storage == 1)
    hipLaunchKernelGGL(k_init<float>, grid_for(d.N), dim3(256), 0, s, d);
  else
    hipLaunchKernelGGL(k_init<__half>, grid_for(d.N), dim3(256), 0, s, d);
}

void launch_fields(const DevDomain& d, int which, double* dst, hipStream_t s) {
  if (d.storage == 0)
    hipLaunchKernelGGL(k_get_plane<double>, grid_for(d.N), dim3(256), 0, s, d, which, dst);
  else if (d.storage == 1)
    hipLaunchKernelGGL(k_get_plane<float>, grid_for(d.N), dim3(256), 0, s, d, which, dst);
  else
    hipLaunchKernelGGL(k_get_plane<__half>, grid_for(d.N), dim3(256), 0, s, d, which, dst);
}

// src: the full distribution of direction q on every cell
void launch_set_pdf(const DevDomain& d, int q, const double* src, hipStream_t s) {
  if (d.storage == 0)
    hipLaunchKernelGGL(k_set_plane<double>, grid_for(d.N), dim3(256), 0, s, d, q, src);
  else if (d.storage == 1)
    hipLaunchKernelGGL(k_set_plane<float>, grid_for(d.N), dim3(256), 0, s, d, q, src);
  else
    hipLaunchKernelGGL(k_set_plane<__half>, grid_for(d.N), dim3(256), 0, s, d, q, src);
}

void launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  if (n16 > 0) {
    size_t b = (n16 + 255) / 256;
    if (b > 16384) b = 16384;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)b), dim3(256), 0, s, (uint4*)dst, (const uint4*)src, n16);
  }
  const size_t tail = bytes - n16 * 16;
  if (tail)
    hipLaunchKernelGGL(k_copy1, dim3(1), dim3(256), 0, s, (uint8_t*)dst + n16 * 16,
                       (const uint8_t*)src + n16 * 16, tail);
}

}  // namespace lbmdem
