// Transport operator and splitting kernels (Sec. 3.3, the Simpler balanced splitting
// around the reaction substep).
//
// The transport operator of the model problem is linear advection along x plus isotropic
// diffusion on an nx x ny x nz grid of cubic cells:
//   T(U)_r = -a (U_{x+1} - U_{x-1}) / (2 dx) + D (sum of the six neighbours - 6 U) / dx^2
// for every state row r (species mass fractions and temperature), second-order central
// differences.  Cell c = x + nx (y + ny z).  y and z are periodic; x is periodic, or open:
// the neighbour before x = 0 is the inflow ghost value of the row, the neighbour after
// x = nx - 1 is that cell itself (zero-gradient outflow).  A state is addressed by rows:
// row r < ns is y + r n, row ns is t (the ABI's Y / T arrays, or a contiguous [N][n]
// workspace with t = y + ns n).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rok4e {

struct GridDev {
  int nx, ny, nz;
  double inv2dx, invdx2;   // 1 / (2 dx), 1 / dx^2
  double vel, diff;        // a, D
  const double* inflow;    // open x boundary: ghost value per row; null: periodic x
};

struct RowsC {
  const double* y;
  const double* t;
  __device__ __forceinline__ const double* row(int r, int ns, int64_t n) const {
    return r < ns ? y + (int64_t)r * n : t;
  }
};
struct RowsW {
  double* y;
  double* t;
  __device__ __forceinline__ double* row(int r, int ns, int64_t n) const {
    return r < ns ? y + (int64_t)r * n : t;
  }
};

// T(U) at cell c of row r.
__device__ __forceinline__ double transport_at(const GridDev& g, const double* u, int r, int x, int y, int z) {
  const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
  const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny;
  const int64_t line = sy * y + sz * z;
  const int64_t c = x + line;
  const double uc = u[c];
  double uxm, uxp;
  if (g.inflow) {
    uxm = x == 0 ? g.inflow[r] : u[c - 1];
    uxp = x == g.nx - 1 ? uc : u[c + 1];
  } else {
    uxm = u[(x == 0 ? g.nx - 1 : x - 1) + line];
    uxp = u[(x == g.nx - 1 ? 0 : x + 1) + line];
  }
  const double uym = u[x + sy * ym + sz * z], uyp = u[x + sy * yp + sz * z];
  const double uzm = u[x + sy * y + sz * zm], uzp = u[x + sy * y + sz * zp];
  const double adv = -g.vel * (uxp - uxm) * g.inv2dx;
  const double dif = g.diff * (((uxm + uxp) + (uym + uyp)) + (uzm + uzp) - 6.0 * uc) * g.invdx2;
  return adv + dif;
}

// out = T(src) (+ optionally a second output out2 = T(src) + add), one thread per (row,
// cell), cells fastest so that x-neighbours are coalesced.
__global__ void __launch_bounds__(256) k_transport(GridDev g, int ns, RowsC src, double* out, const double* add,
                                                   double* out2) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const int64_t total = n * (ns + 1);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / n);
    const int64_t c = i - (int64_t)r * n;
    const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / ((int64_t)g.nx * g.ny));
    const double v = transport_at(g, src.row(r, ns, n), r, x, y, z);
    out[i] = v;
    if (out2) out2[i] = add ? v + add[i] : v;
  }
}

// One stage of the classical Runge-Kutta method on u' = T(u) - s0 (s0 may be null):
// k = T(src) - s0; acc = (init ? base : acc) + wacc k; next = base + wnext k (next may be
// null).  On the last stage acc is the new state (written through dst rows when given).
__global__ void __launch_bounds__(256) k_rk4_stage(GridDev g, int ns, RowsC src, const double* s0, RowsC base,
                                                   double* acc, int init, double wacc, double* next, double wnext,
                                                   RowsW dst) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const int64_t total = n * (ns + 1);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / n);
    const int64_t c = i - (int64_t)r * n;
    const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / ((int64_t)g.nx * g.ny));
    double k = transport_at(g, src.row(r, ns, n), r, x, y, z);
    if (s0) k = k - s0[i];
    const double b = base.row(r, ns, n)[c];
    const double a = (init ? b : acc[i]) + wacc * k;
    if (dst.y) dst.row(r, ns, n)[c] = a;
    else acc[i] = a;
    if (next) next[i] = b + wnext * k;
  }
}

// dst rows = src rows (state copy into a contiguous workspace).
__global__ void __launch_bounds__(256) k_copy_rows(int64_t n, int ns, RowsC src, double* dst) {
  const int64_t total = n * (ns + 1);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / n);
    const int64_t c = i - (int64_t)r * n;
    dst[i] = src.row(r, ns, n)[c];
  }
}

}  // namespace rok4e
