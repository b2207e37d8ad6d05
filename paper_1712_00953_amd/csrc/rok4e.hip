// Batched ROK4E reaction substep: kernels and the C ABI declared in include/rok4e.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "rok4e.h"
#include "rok4e_integrator.hpp"
#include "rok4e_placement.hpp"
#include "rok4e_split.hpp"

namespace rok4e {

// ------------------------------------------------------------------ kernels ----

__global__ void k_zero_u32(unsigned int* x) { *x = 0u; }

// FP64 FMA throughput probe: eight independent chains per thread (enough to cover the
// FMA latency with a few waves per SIMD), each round eight FMAs.
__global__ void __launch_bounds__(256) k_fma_probe(int iters, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double b = 0.9999999999, c = 1e-12 * (double)(threadIdx.x + 1);
  double a[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) a[q] = 1.0 + 0.125 * q;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = fma(a[q], b, c);
  out[i] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// ---------------------------------------------------------- cell order ----
// Hottest-first order of the persistent queue: a counting sort of the cells by
// temperature bin (16 K wide, bin 0 the hottest; non-finite or non-positive T in the
// last bin).  Within a bin the order is whatever the atomics give; the results do not
// depend on it.
constexpr int kOrderBins = 256;

__device__ __forceinline__ int order_bin(double T) {
  if (!(T > 0.0) || !__builtin_isfinite(T)) return kOrderBins - 1;
  const int b = (int)((4096.0 - fmin(T, 4095.5)) * (1.0 / 16.0));
  return b < 0 ? 0 : (b > kOrderBins - 1 ? kOrderBins - 1 : b);
}

__global__ void __launch_bounds__(256) k_fill_u32(unsigned int* x, int n, unsigned int v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] = v;
}

__global__ void __launch_bounds__(256) k_order_hist(const double* T, int64_t n, unsigned int* bins) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&bins[order_bin(T[c])], 1u);
}

// Exclusive prefix sum of the kOrderBins counts in place (one block of kOrderBins threads).
__global__ void __launch_bounds__(kOrderBins) k_order_scan(unsigned int* bins) {
  __shared__ unsigned int s[kOrderBins];
  const int i = threadIdx.x;
  const unsigned int own = bins[i];
  s[i] = own;
  __syncthreads();
  for (int d = 1; d < kOrderBins; d <<= 1) {
    const unsigned int add = i >= d ? s[i - d] : 0u;
    __syncthreads();
    s[i] += add;
    __syncthreads();
  }
  bins[i] = s[i] - own;
}

__global__ void __launch_bounds__(256) k_order_scatter(const double* T, int64_t n, unsigned int* bins,
                                                       int32_t* order) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    const unsigned int pos = atomicAdd(&bins[order_bin(T[c])], 1u);
    order[pos] = (int32_t)c;
  }
}

// Persistent integrator: every segment of L lanes pulls cells from a device counter
// until the batch is exhausted, so cells with 1 and 1000 attempts share the chip
// without waiting on each other.
// Waves per SIMD the register allocation is held to: three for one row slot per lane
// (no spills), two for larger layouts.
#ifndef ROK4E_OCC_ROWS1
#define ROK4E_OCC_ROWS1 3
#endif
template <int ROWS>
constexpr int occupancy() { return ROWS == 1 ? ROK4E_OCC_ROWS1 : 2; }
// Largest block of the persistent integrator: four waves for one row slot per lane, eight
// for larger layouts (eight waves over the four SIMDs at two waves per SIMD: one block,
// one copy of the mechanism tables in LDS, fills a compute unit).
template <int ROWS>
constexpr int integrate_max_threads() { return ROWS == 1 ? 256 : 512; }

// FORM selects the state: the 0-D reactor (Y, T; p per cell) or the conservative
// variables with the auxiliary temperature (P.Y = U, P.T = the final temperatures or
// null; FP64; no carried steps).
//
// With one segment per wave, each cell is integrated to the end before the next is
// taken.  With several segments per wave, one loop over attempts: on every pass each
// segment makes one attempt on its cell, and a segment whose cell is done first stores it
// and takes the next cell from the queue, so the segments stay in step attempt by attempt
// instead of the wave waiting for its slowest cell before any segment takes a new one; the
// wave leaves the loop when none of its segments holds a cell.
// GATHER: the Jacobian-vector products read the base concentrations from a per-basis
// gather into lane-private memory instead of LDS (layouts with has_gather only).
// OCC4: registers held to four waves per SIMD (128 VGPRs, more spills) with blocks of up
// to 16 waves, one-slot layouts (a launch-tuner candidate).
template <int L, int ROWS, int MMAX, class RT, int FORM = kFormReactor, int GATHER = 0, int OCC4 = 0>
__global__ void __launch_bounds__(OCC4 ? 1024 : integrate_max_threads<ROWS>(), OCC4 ? 4 : occupancy<ROWS>())
    k_integrate(DevMech m, Launch P) {
  extern __shared__ __align__(16) char smem[];
  const MechLds t = load_mech_lds<L>(m, smem);
  const int lane = (int)(threadIdx.x % L);
  char* seg = smem + m.image_bytes + (threadIdx.x / L) * P.seg_bytes;
  const SegLds<RT> S = seg_lds<RT>(seg, P);
  init_seg<RT>(m, S);
  if constexpr (L == 64) {
    // one segment per wave: each cell integrated to the end before the next is taken
    while (true) {
      const unsigned int ticket = atomicAdd(P.queue, lane == 0 ? 1u : 0u);
      const int tk = seg_bcast<L>((int)ticket, 0);
      if (tk < 0 || (int64_t)tk >= P.n_cells) break;
      const int cell = P.order ? P.order[tk] : tk;
      double u[ROWS], s[ROWS], p = 0.0;
      CellState c{};
      c.status = 3;
      if constexpr (FORM == kFormConservative) {
        if (load_cell_cons<L, ROWS>(m, t, P, cell, lane, u, s)) {
          c = integrate_cell<L, ROWS, MMAX, RT, FORM, GATHER>(m, t, P, u, p, s, S, lane);
          store_cell_cons<L, ROWS>(m, P, cell, lane, u);
        }
      } else if (load_cell<L, ROWS>(m, P, cell, lane, u, s, p)) {
        c = integrate_cell<L, ROWS, MMAX, RT, FORM, GATHER>(m, t, P, u, p, s, S, lane, P.hio ? P.hio[cell] : 0.0);
        store_cell<L, ROWS>(m, P, cell, lane, u);
        if (P.hio) P.hio[cell] = c.hnext;
      }
      P.acc[cell] = c.accepted;
      P.rej[cell] = c.rejected;
      P.status[cell] = c.status;
    }
    return;
  }
  double u[ROWS], s[ROWS], fn[ROWS], Q[ROWS][MMAX];
  double p = 0.0;
  CellState c{};
  int cell = -1;          // the segment's cell (segment-uniform), -1 for none
  bool drained = false;   // the queue has run out for this segment
  while (true) {
    if (cell >= 0 && !cell_running(P, c)) {
      if constexpr (FORM == kFormConservative) {
        store_cell_cons<L, ROWS>(m, P, cell, lane, u);
      } else {
        store_cell<L, ROWS>(m, P, cell, lane, u);
        if (P.hio) P.hio[cell] = c.hnext;
      }
      // every lane of the segment stores the same (segment-uniform) values
      P.acc[cell] = c.accepted;
      P.rej[cell] = c.rejected;
      P.status[cell] = c.status;
      cell = -1;
    }
    while (cell < 0 && !drained) {
      // Every lane takes part in the atomic (the segment's first lane adds 1, the others
      // 0), so no lane-dependent branch surrounds the value that is then broadcast.
      const unsigned int ticket = atomicAdd(P.queue, lane == 0 ? 1u : 0u);
      const int tk = seg_bcast<L>((int)ticket, 0);
      if (tk < 0 || (int64_t)tk >= P.n_cells) {
        drained = true;
        break;
      }
      const int cand = P.order ? P.order[tk] : tk;
      bool ok;
      if constexpr (FORM == kFormConservative) ok = load_cell_cons<L, ROWS>(m, t, P, cand, lane, u, s);
      else ok = load_cell<L, ROWS>(m, P, cand, lane, u, s, p);
      if (ok) {
        cell = cand;
        // a new cell always needs an attempt (t = 0 < dt, no attempt made yet)
        cell_start(P, c, (FORM == kFormReactor && P.hio) ? P.hio[cand] : 0.0);
      } else {
        // invalid input: the state is left as it is
        P.acc[cand] = 0;
        P.rej[cand] = 0;
        P.status[cand] = 3;
      }
    }
    if (!__any(cell >= 0)) break;
    if (cell >= 0) cell_attempt<L, ROWS, MMAX, RT, FORM, GATHER>(m, t, P, u, p, s, S, lane, c, fn, Q);
  }
}

// Explicit Dormand-Prince 5(4) reference integrator over the same persistent queue.
template <int L, int ROWS, class RT>
__global__ void __launch_bounds__(256, occupancy<ROWS>()) k_rkdp(DevMech m, Launch P) {
  extern __shared__ __align__(16) char smem[];
  const MechLds t = load_mech_lds<L>(m, smem);
  const int lane = (int)(threadIdx.x % L);
  char* seg = smem + m.image_bytes + (threadIdx.x / L) * P.seg_bytes;
  const SegLds<RT> S = seg_lds<RT>(seg, P);
  init_seg<RT>(m, S);
  while (true) {
    const unsigned int ticket = atomicAdd(P.queue, lane == 0 ? 1u : 0u);
    const int tk = seg_bcast<L>((int)ticket, 0);
    if (tk < 0 || (int64_t)tk >= P.n_cells) break;
    const int cell = P.order ? P.order[tk] : tk;
    double u[ROWS], s[ROWS], p;
    CellState c{};
    c.status = 3;
    if (load_cell<L, ROWS>(m, P, cell, lane, u, s, p)) {
      c = rkdp_cell<L, ROWS, RT>(m, t, P, u, p, s, S, lane);
      store_cell<L, ROWS>(m, P, cell, lane, u);
    }
    P.acc[cell] = c.accepted;
    P.rej[cell] = c.rejected;
    P.status[cell] = c.status;
  }
}

// Device buffers of the per-attempt schedule: the state each active cell carries from
// one launch to the next (cell-major, so a segment's lanes read contiguous rows).
struct AttemptWork {
  CellState* st;          // [n]
  double* fnq;            // [n][1 + MMAX][LP]: f(u_n) and the Krylov basis
  double* H;              // [n][MMAX * MMAX]
  const int32_t* act_in;  // cells active before this launch (unused on the first launch)
  const unsigned int* n_in;
  int32_t* act_out;       // cells still active after it
  unsigned int* n_out;
  int first;              // 1: every cell, starting from its initial state
};

// Per-attempt schedule: each launch performs one attempt of every active cell (the same
// cell_attempt as the persistent kernel, so the results are bitwise identical) and
// appends the cells that need another attempt to act_out.  The host relaunches until no
// cell is active.
template <int L, int ROWS, int MMAX, class RT>
__global__ void __launch_bounds__(256, occupancy<ROWS>()) k_attempt(DevMech m, Launch P, AttemptWork W) {
  extern __shared__ __align__(16) char smem[];
  const MechLds t = load_mech_lds<L>(m, smem);
  const int lane = (int)(threadIdx.x % L);
  char* seg = smem + m.image_bytes + (threadIdx.x / L) * P.seg_bytes;
  const SegLds<RT> S = seg_lds<RT>(seg, P);
  init_seg<RT>(m, S);
  constexpr int LP = L * ROWS;
  const int64_t nact = W.first ? P.n_cells : (int64_t)*W.n_in;
  const int64_t nseg = (int64_t)gridDim.x * (blockDim.x / L);
  for (int64_t idx = (int64_t)blockIdx.x * (blockDim.x / L) + threadIdx.x / L; idx < nact; idx += nseg) {
    const int64_t cell = W.first ? idx : (int64_t)W.act_in[idx];
    double u[ROWS], s[ROWS], p, fn[ROWS], Q[ROWS][MMAX];
    const bool valid = load_cell<L, ROWS>(m, P, cell, lane, u, s, p);
    double* fq = W.fnq + cell * (int64_t)((1 + MMAX) * LP);
    double* Hc = W.H + cell * (int64_t)(MMAX * MMAX);
    CellState c{};
    bool run = false;
    if (W.first) {
      c.status = 3;
      if (valid) {
        cell_start(P, c, P.hio ? P.hio[cell] : 0.0);
        run = cell_running(P, c);
      }
    } else {
      c = W.st[cell];
      run = true;
#pragma unroll
      for (int i = 0; i < ROWS; ++i) {
        fn[i] = fq[i * L + lane];
#pragma unroll
        for (int j = 0; j < MMAX; ++j) Q[i][j] = fq[(1 + j) * LP + i * L + lane];
      }
      for (int i = lane; i < MMAX * MMAX; i += L) S.H[i] = Hc[i];
      lds_sync();
    }
    if (run) {
      cell_attempt<L, ROWS, MMAX, RT>(m, t, P, u, p, s, S, lane, c, fn, Q);
      store_cell<L, ROWS>(m, P, cell, lane, u);
      run = cell_running(P, c);
    }
    if (run) {
#pragma unroll
      for (int i = 0; i < ROWS; ++i) {
        fq[i * L + lane] = fn[i];
#pragma unroll
        for (int j = 0; j < MMAX; ++j) fq[(1 + j) * LP + i * L + lane] = Q[i][j];
      }
      for (int i = lane; i < MMAX * MMAX; i += L) Hc[i] = S.H[i];
      // every lane writes the same state; the segment's first lane appends the cell
      W.st[cell] = c;
      const unsigned int slot = atomicAdd(W.n_out, lane == 0 ? 1u : 0u);
      const int pos = seg_bcast<L>((int)slot, 0);
      W.act_out[pos] = (int32_t)cell;
    } else {
      P.acc[cell] = c.accepted;
      P.rej[cell] = c.rejected;
      P.status[cell] = c.status;
      if (P.hio && valid) P.hio[cell] = c.hnext;
    }
    lds_sync();
  }
}

// f(u) for every cell (grid-stride over cells, one cell per segment).
template <int L, int ROWS, class RT>
__global__ void __launch_bounds__(256, 4) k_rhs(DevMech m, Launch P, double* dY, double* dT) {
  extern __shared__ __align__(16) char smem[];
  const MechLds t = load_mech_lds<L>(m, smem);
  const int lane = (int)(threadIdx.x % L);
  char* seg = smem + m.image_bytes + (threadIdx.x / L) * P.seg_bytes;
  const SegLds<RT> S = seg_lds<RT>(seg, P);
  init_seg<RT>(m, S);
  const int64_t nseg = (int64_t)gridDim.x * (blockDim.x / L);
  const int64_t n = P.n_cells;
  const int ns = m.ns;
  for (int64_t cell = (int64_t)blockIdx.x * (blockDim.x / L) + threadIdx.x / L; cell < n; cell += nseg) {
    double u[ROWS], f[ROWS];
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const int r = i * L + lane;
      u[i] = r < ns ? P.Y[(int64_t)r * n + cell] : (r == ns ? P.T[cell] : 0.0);
    }
    double w[ROWS];
    rhs<L, ROWS, RT, false>(m, t, u, P.p[cell], f, S.r, lane, nullptr, w);
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const int r = i * L + lane;
      if (r < ns) dY[(int64_t)r * n + cell] = f[i];
      else if (r == ns) dT[cell] = f[i];
    }
  }
}

// Arnoldi basis at every cell's state (diagnostics and step-level parity).
// The standalone basis kernel of the one-slot layouts with M <= 8 runs four waves per SIMD
// in one 16-wave block per compute unit (measured 10 % faster than three waves in 4-wave
// blocks on the 53-species flame slice); the other layouts run three waves per SIMD in
// 4-wave blocks.
template <int ROWS, int MMAX>
constexpr bool arnoldi_occ4() { return ROWS == 1 && MMAX <= 8; }

template <int L, int ROWS, int MMAX, class RT>
__global__ void __launch_bounds__((arnoldi_occ4<ROWS, MMAX>() ? 1024 : 256), (arnoldi_occ4<ROWS, MMAX>() ? 4 : 3))
    k_arnoldi(DevMech m, Launch P, double* Qo, double* Ho, int32_t* Mo) {
  extern __shared__ __align__(16) char smem[];
  const MechLds t = load_mech_lds<L>(m, smem);
  const int lane = (int)(threadIdx.x % L);
  char* seg = smem + m.image_bytes + (threadIdx.x / L) * P.seg_bytes;
  const SegLds<RT> S = seg_lds<RT>(seg, P);
  init_seg<RT>(m, S);
  const int64_t nseg = (int64_t)gridDim.x * (blockDim.x / L);
  const int64_t n = P.n_cells;
  const int N = m.ns + 1, M = P.M;
  for (int64_t cell = (int64_t)blockIdx.x * (blockDim.x / L) + threadIdx.x / L; cell < n; cell += nseg) {
    double u[ROWS], s[ROWS], fn[ROWS], p;
    load_cell<L, ROWS>(m, P, cell, lane, u, s, p);
    RhsBase base;
    double w[ROWS];
    rhs_forced<L, ROWS, RT, true>(m, t, u, p, s, fn, S, lane, &base, w);
    double Q[ROWS][MMAX];
    const int Meff = arnoldi<L, ROWS, MMAX, RT>(m, t, P, u, fn, base, w, Q, S, lane);
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const int r = i * L + lane;
      if (r < N)
#pragma unroll
        for (int j = 0; j < MMAX; ++j)
          if (j < M) Qo[((int64_t)cell * M + j) * N + r] = Q[i][j];
    }
    // H: the lanes of the segment store its M x M entries, one entry each per pass
    for (int e = lane; e < M * M; e += L) {
      const int i = e / M, j = e % M;
      Ho[(int64_t)cell * M * M + e] =
          (i < MMAX && j < MMAX && i <= j + 1 && i < Meff && j < Meff) ? S.H[i * MMAX + j] : 0.0;
    }
    if (lane == 0) Mo[cell] = Meff;
    lds_sync();
  }
}

// ------------------------------------------------------------ variant table ----

using IntegrateFn = void (*)(DevMech, Launch);
using AttemptFn = void (*)(DevMech, Launch, AttemptWork);
using RhsFn = void (*)(DevMech, Launch, double*, double*);
using ArnoldiFn = void (*)(DevMech, Launch, double*, double*, int32_t*);

struct Variant {
  int L, rows, mmax, prec;
  IntegrateFn integrate;
  IntegrateFn integrate_gather;   // the same with the JVP base-concentration gather (or null)
  IntegrateFn integrate_occ4;     // the same held to four waves per SIMD (or null)
  IntegrateFn integrate_cons;   // conservative variables (FP64 variants; null otherwise)
  IntegrateFn rkdp;
  AttemptFn attempt;
  ArnoldiFn arnoldi;
  RhsFn rhs;
};

template <int L, int ROWS, int MMAX, class RT>
constexpr IntegrateFn gather_kernel() {
  if constexpr (has_gather<L, ROWS, MMAX>()) return k_integrate<L, ROWS, MMAX, RT, kFormReactor, 1>;
  else return nullptr;
}

template <int L, int ROWS, int MMAX, class RT>
constexpr IntegrateFn occ4_kernel() {
  if constexpr (L == 64 && ROWS == 1 && MMAX <= 8) return k_integrate<L, ROWS, MMAX, RT, kFormReactor, 0, 1>;
  else return nullptr;
}

template <int L, int ROWS, int MMAX, class RT>
constexpr IntegrateFn cons_kernel() {
  if constexpr (sizeof(RT) == 8) return k_integrate<L, ROWS, MMAX, RT, kFormConservative>;
  else return nullptr;
}

#define ROK4E_VARIANT(Lv, Rv, Mv, T, P)                                                       \
  Variant{Lv, Rv, Mv, P, k_integrate<Lv, Rv, Mv, T>, gather_kernel<Lv, Rv, Mv, T>(),          \
          occ4_kernel<Lv, Rv, Mv, T>(),                                                        \
          cons_kernel<Lv, Rv, Mv, T>(),                                                        \
          k_rkdp<Lv, Rv, T>, k_attempt<Lv, Rv, Mv, T>,                                         \
          k_arnoldi<Lv, Rv, Mv, T>,                                                             \
          k_rhs<Lv, Rv, T>}

static const Variant kVariants[] = {
    ROK4E_VARIANT(16, 1, 4, double, ROK4E_FP64),  ROK4E_VARIANT(16, 1, 8, double, ROK4E_FP64),
    ROK4E_VARIANT(32, 1, 8, double, ROK4E_FP64),  ROK4E_VARIANT(32, 2, 8, double, ROK4E_FP64),
    ROK4E_VARIANT(64, 1, 4, double, ROK4E_FP64),  ROK4E_VARIANT(64, 1, 8, double, ROK4E_FP64),
    ROK4E_VARIANT(64, 1, 12, double, ROK4E_FP64), ROK4E_VARIANT(64, 1, 16, double, ROK4E_FP64),
    ROK4E_VARIANT(64, 2, 8, double, ROK4E_FP64),  ROK4E_VARIANT(64, 2, 12, double, ROK4E_FP64),
    ROK4E_VARIANT(64, 2, 16, double, ROK4E_FP64),
    ROK4E_VARIANT(16, 1, 4, float, ROK4E_MIXED),  ROK4E_VARIANT(16, 1, 8, float, ROK4E_MIXED),
    ROK4E_VARIANT(32, 1, 8, float, ROK4E_MIXED),  ROK4E_VARIANT(32, 2, 8, float, ROK4E_MIXED),
    ROK4E_VARIANT(64, 1, 4, float, ROK4E_MIXED),  ROK4E_VARIANT(64, 1, 8, float, ROK4E_MIXED),
    ROK4E_VARIANT(64, 1, 12, float, ROK4E_MIXED), ROK4E_VARIANT(64, 1, 16, float, ROK4E_MIXED),
    ROK4E_VARIANT(64, 2, 8, float, ROK4E_MIXED),  ROK4E_VARIANT(64, 2, 12, float, ROK4E_MIXED),
    ROK4E_VARIANT(64, 2, 16, float, ROK4E_MIXED),
};

// Largest block of a variant's persistent integrator, in waves.
inline int integrate_waves(const Variant& v) { return v.rows == 1 ? 4 : 8; }

}  // namespace rok4e

using namespace rok4e;

// ----------------------------------------------------- static scratch ----
// Device scratch of the allocation-free entry point rok4e_integrate_static, one copy per
// GPU for the life of the process: word 0 the work-queue counter, words
// [kScratchBins, kScratchBins + kOrderBins) the temperature-bin counters of the queue
// order, and from kScratchOrder the queue order of up to ROK4E_STATIC_MAX_CELLS cells
// (8 MiB in all).  Host code never passes the symbol itself to a kernel or a copy: the
// device address of each GPU's copy comes from hipGetSymbolAddress (scratch_ptr).
namespace rok4e {
constexpr int kScratchBins = 64, kScratchOrder = 64 + kOrderBins;
static __device__ __align__(256) unsigned int scratch[kScratchOrder + ROK4E_STATIC_MAX_CELLS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned int* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of scratch, looked up once per device
// (the caller has made `device` current); null if the lookup fails.
unsigned int* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[device] = (unsigned int*)ptr;
  }
  return g_scratch_ptr[device];
}
}  // namespace rok4e

// ------------------------------------------------------------------- handle ----

struct rok4e_mech {
  int device = 0;
  int ns = 0, nr = 0;
  rok4e_options opt{};
  const Variant* var = nullptr;
  int cu_count = 0;
  std::string arch;   // GPU architecture name (gcnArchName), part of the tuning-cache key
  size_t lds_per_block_max = 0;
  // host copy of the mechanism
  std::vector<double> W, cp, hf, par;          // par: 6 x nr
  std::vector<int> reac, prod;                 // 2 x nr
  // device table image for the current layout
  int image_key = -1;
  DevMech dm{};
  void* d_image = nullptr;
  // layout and image of the conservative-variable form when the current layout holds
  // fewer than ns + 6 rows
  const Variant* cons_var = nullptr;
  int cons_image_key = -1;
  DevMech cons_dm{};
  void* d_cons_image = nullptr;
  unsigned int* d_queue = nullptr;
  unsigned int* scratch = nullptr;   // this device's static scratch (rok4e_integrate_static)
  // per-cell workspace
  int64_t cap = 0;
  int32_t* d_acc = nullptr;
  int32_t* d_rej = nullptr;
  int32_t* d_status = nullptr;
  int32_t* d_order = nullptr;      // [cap] queue order of the persistent schedule
  unsigned int* d_bins = nullptr;  // [kOrderBins] temperature-bin counts / offsets
  int64_t last_n = 0;
  // per-attempt schedule: carried cell state, active lists and their counters
  int64_t att_cap = 0;
  const Variant* att_var = nullptr;   // layout the buffers are sized for
  CellState* d_st = nullptr;
  double* d_fnq = nullptr;
  double* d_H = nullptr;
  int32_t* d_act[2] = {nullptr, nullptr};
  unsigned int* d_cnt = nullptr;   // [2]
  unsigned int* h_cnt = nullptr;   // pinned host copy of one counter
};

namespace {

int hip_fail(hipError_t e) { return e == hipErrorOutOfMemory ? ROK4E_ENOMEM : ROK4E_EHIP; }

bool options_ok(const rok4e_options& o) {
  if (o.M < 1 || o.M > 16) return false;
  if (o.precision != ROK4E_FP64 && o.precision != ROK4E_MIXED) return false;
  if (o.fixed_steps < 0) return false;
  if (o.lanes_per_cell != 0 && o.lanes_per_cell != 16 && o.lanes_per_cell != 32 && o.lanes_per_cell != 64)
    return false;
  if (o.waves_per_block < 0 || o.waves_per_block > 16) return false;
  if (o.waves_per_simd != 0 && o.waves_per_simd != 3 && o.waves_per_simd != 4) return false;
  if (o.blocks_per_cu < 0 || o.blocks_per_cu > 64) return false;
  if (o.scheduling != ROK4E_PERSISTENT && o.scheduling != ROK4E_PER_ATTEMPT) return false;
  if (o.method != ROK4E_METHOD_ROK4E && o.method != ROK4E_METHOD_RKDP45) return false;
  if (o.cell_order != ROK4E_ORDER_HOT_FIRST && o.cell_order != ROK4E_ORDER_ARRAY) return false;
  if (o.jvp_gather != ROK4E_GATHER_AUTO && o.jvp_gather != ROK4E_GATHER_LDS && o.jvp_gather != ROK4E_GATHER_PRIVATE)
    return false;
  if (!std::isfinite(o.h0)) return false;
  return true;
}

// Smallest instantiated variant that holds ns + extra rows (the reactor state: extra = 1)
// and M Krylov vectors.
const Variant* pick_variant(int ns, const rok4e_options& o, int extra = 1) {
  const int N = ns + extra;
  const Variant* best = nullptr;
  for (const Variant& v : kVariants) {
    if (v.prec != o.precision || v.mmax < o.M || v.L * v.rows < N) continue;
    if (o.lanes_per_cell != 0 && v.L != o.lanes_per_cell) continue;
    if (o.lanes_per_cell == 0) {
      // automatic: fewest lanes that hold the state in one slot, then smallest MMAX
      if (!best) { best = &v; continue; }
      auto key = [&](const Variant* x) { return std::make_tuple(x->rows, x->L * x->rows, x->mmax); };
      if (key(&v) < key(best)) best = &v;
    } else {
      if (!best || std::make_tuple(v.rows, v.mmax) < std::make_tuple(best->rows, best->mmax)) best = &v;
    }
  }
  return best;
}

// Per-segment LDS: concentrations [LP] in the rate type, their increments [LP] in FP64,
// the production accumulators [LP] in FP64 (two copies LP + 8 entries apart in the mixed
// form), the rate-constant pairs [NRP] in the rate type, H, LU [MMAX^2] and 1/diag(U)
// [MMAX] in FP64.
struct SegLayout {
  int bytes, off_k, off_H, off_LU, off_rdiag;
};

int n_rx_padded(int nr) { return (std::max(nr, 1) + 1) & ~1; }

int al16(int x) { return (x + 15) & ~15; }

int rate_bytes(int prec) { return prec == ROK4E_FP64 ? 8 : 4; }

SegLayout seg_layout(int nr, const Variant& v) {
  const int rt = rate_bytes(v.prec);
  const int lp = v.L * v.rows;
  SegLayout s{};
  // concentrations (rate type), FP64 increments, accumulators (two copies in the mixed
  // form)
  int off = al16(lp * rt + lp * 8 + (rt == 4 ? 2 * lp + 8 : lp) * 8);
  s.off_k = off;
  off = al16(off + n_rx_padded(nr) * 2 * rt);
  s.off_H = off;
  off = al16(off + v.mmax * v.mmax * 8);
  s.off_LU = off;
  off = al16(off + v.mmax * v.mmax * 8);
  s.off_rdiag = off;
  off = al16(off + v.mmax * 8);
  s.bytes = off;
  return s;
}

// Annealing steps of the reaction / species placement (about 10 us each at 53 species).
constexpr long kPlacementSteps = 60000;

// Builds (or reuses) the table image for the handle's current layout and rate type; see
// DevMech.
// Builds the table image of layout var into *d_image / *dm (kept while *image_key matches).
int build_image(rok4e_mech* m, const Variant* var, DevMech* dm, void** d_image, int* image_key) {
  const int lp = var->L * var->rows;
  const int rb = rate_bytes(var->prec);
  const int key = lp * 64 + rb;
  if (*image_key == key && *d_image) return ROK4E_OK;
  const int ns = m->ns, nr = m->nr;
  const int nrp = n_rx_padded(nr);
  // placement of reactions on (iteration, lane) positions and of species in LDS
  std::vector<int> slots(4 * (size_t)nr);
  for (int j = 0; j < nr; ++j) {
    const int sl[4] = {m->reac[2 * j], m->reac[2 * j + 1], m->prod[2 * j], m->prod[2 * j + 1]};
    for (int a = 0; a < 4; ++a) slots[4 * j + a] = sl[a] < 0 ? ns : sl[a];
  }
  PlacementSearch search(ns, nr, slots, var->L, rb, rb == 4 ? 2 * lp + 16 : 0);
  const Placement pl = search.run(kPlacementSteps, 0x5eed0000ull + (uint64_t)key);
  const int off_spec = al16(3 * nrp * 16);
  const int off_rxo = al16(off_spec + 4 * lp * 8);
  const int off_spos = al16(off_rxo + nrp * 8);
  const int bytes = al16(off_spos + lp * 4);
  std::vector<char> img(bytes, 0);
  // (ln A_f, ln A_r), (b_f, E_f), (b_r, E_r); m->par holds ln A_f, b_f, E_f, ln A_r,
  // b_r, E_r, each [nr]
  double* par = (double*)img.data();
  const int pair_q[3][2] = {{0, 3}, {1, 2}, {4, 5}};
  for (int a = 0; a < 3; ++a)
    for (int q = 0; q < nr; ++q) {
      const int j = pl.order[q];
      par[(a * nrp + q) * 2] = m->par[pair_q[a][0] * nr + j];
      par[(a * nrp + q) * 2 + 1] = m->par[pair_q[a][1] * nr + j];
    }
  double* sp = (double*)(img.data() + off_spec);
  for (int r = 0; r < lp; ++r) {
    const bool spc = r < ns;
    sp[r] = spc ? m->W[r] : 1.0;
    sp[lp + r] = spc ? 1.0 / m->W[r] : 0.0;
    sp[2 * lp + r] = spc ? m->cp[r] : 0.0;
    sp[3 * lp + r] = spc ? m->hf[r] : 0.0;
  }
  uint32_t* rxo = (uint32_t*)(img.data() + off_rxo);
  auto off = [&](int k) { return (uint32_t)(pl.pos[k] * rb); };
  for (int q = 0; q < nr; ++q) {
    const int* sl = &slots[4 * (size_t)pl.order[q]];
    rxo[2 * q] = off(sl[0]) | off(sl[1]) << 16;
    rxo[2 * q + 1] = off(sl[2]) | off(sl[3]) << 16;
  }
  int* spos = (int*)(img.data() + off_spos);
  for (int r = 0; r < lp; ++r) spos[r] = r < ns ? pl.pos[r] : ns;
  if (*d_image) (void)hipFree(*d_image);
  *d_image = nullptr;
  *image_key = -1;
  hipError_t e = hipMalloc(d_image, bytes);
  if (e == hipSuccess) e = hipMemcpy(*d_image, img.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e);
  *dm = DevMech{ns, nr, nrp, lp, off_spec, off_rxo, off_spos, bytes, (const int4*)*d_image};
  *image_key = key;
  return ROK4E_OK;
}

int ensure_image(rok4e_mech* m) { return build_image(m, m->var, &m->dm, &m->d_image, &m->image_key); }

struct LaunchShape {
  int block, grid, segs_per_block, lds;
};

// Launch shape: blocks of `waves_per_block` waves (fewer if the block's LDS would not
// fit), as many blocks per CU as occupancy allows for a persistent launch, never more
// segments than cells.
// max_wpb: the kernel's largest block in waves (its launch bounds).
int shape_for(const rok4e_mech* m, const SegLayout& sl, int64_t n_cells, const void* kernel,
              bool persistent, LaunchShape* out, const Variant* var = nullptr, const DevMech* dmp = nullptr,
              int max_wpb = 4) {
  const Variant& v = var ? *var : *m->var;
  const DevMech& dm = dmp ? *dmp : m->dm;
  int wpb = std::min(m->opt.waves_per_block > 0 ? m->opt.waves_per_block : max_wpb, max_wpb);
  const int segs_per_wave = 64 / v.L;
  while (wpb > 1 && (size_t)(dm.image_bytes + wpb * segs_per_wave * sl.bytes) > m->lds_per_block_max) --wpb;
  LaunchShape s{};
  s.block = 64 * wpb;
  s.segs_per_block = wpb * segs_per_wave;
  s.lds = dm.image_bytes + s.segs_per_block * sl.bytes;
  if ((size_t)s.lds > m->lds_per_block_max) return ROK4E_ENOTSUP;
  const int64_t need = (n_cells + s.segs_per_block - 1) / s.segs_per_block;
  int per_cu = 1;
  if (persistent && m->opt.blocks_per_cu > 0) {
    per_cu = m->opt.blocks_per_cu;
  } else {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, s.block, s.lds) != hipSuccess || occ < 1)
      occ = 1;
    per_cu = occ;
  }
  int64_t grid = (int64_t)per_cu * m->cu_count;
  if (!persistent) grid = std::min<int64_t>(grid * 4, need);
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  s.grid = (int)grid;
  *out = s;
  return ROK4E_OK;
}

// Buffers of the per-attempt schedule for n cells of the current layout.
int ensure_attempt_work(rok4e_mech* m, int64_t n) {
  const size_t per_cell = (size_t)(1 + m->var->mmax) * m->var->L * m->var->rows;
  if (n <= m->att_cap && m->att_var == m->var) return ROK4E_OK;
  void* bufs[] = {m->d_st, m->d_fnq, m->d_H, m->d_act[0], m->d_act[1]};
  for (void* b : bufs) (void)hipFree(b);
  m->d_st = nullptr;
  m->d_fnq = m->d_H = nullptr;
  m->d_act[0] = m->d_act[1] = nullptr;
  m->att_cap = 0;
  const int64_t cap = std::max(n, m->cap);
  const size_t mm = (size_t)m->var->mmax * m->var->mmax;
  hipError_t e = hipMalloc((void**)&m->d_st, cap * sizeof(CellState));
  if (e == hipSuccess) e = hipMalloc((void**)&m->d_fnq, cap * per_cell * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&m->d_H, cap * mm * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&m->d_act[0], cap * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&m->d_act[1], cap * sizeof(int32_t));
  if (e == hipSuccess && !m->d_cnt) e = hipMalloc((void**)&m->d_cnt, 2 * sizeof(unsigned int));
  if (e == hipSuccess && !m->h_cnt) e = hipHostMalloc((void**)&m->h_cnt, sizeof(unsigned int));
  if (e != hipSuccess) return hip_fail(e);
  m->att_cap = cap;
  m->att_var = m->var;
  return ROK4E_OK;
}

int ensure_workspace(rok4e_mech* m, int64_t n, hipStream_t stream) {
  if (n <= m->cap) return ROK4E_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return ROK4E_ECAPTURE;
  return rok4e_reserve(m, n);
}

// Queue order of the persistent schedule (hottest first unless the options ask for
// array order): four small kernels on the launch stream, none of them a memset, so a
// captured launch replays them too.  Sets P.order.  Skipped for batches of fewer than
// eight cells per segment in flight, where most cells start at once and the order
// cannot shorten the tail by more than the kernels cost.
// bins (kOrderBins counters) and order (n entries) are device buffers: the handle's, or
// the static scratch of rok4e_integrate_static.
void launch_order(rok4e_mech* m, const double* T, int64_t n, int64_t segments, hipStream_t st, Launch& P,
                  unsigned int* bins, int32_t* order) {
  P.order = nullptr;
  if (m->opt.cell_order != ROK4E_ORDER_HOT_FIRST || n < 8 * segments) return;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, (int64_t)m->cu_count * 8);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, bins, kOrderBins, 0u);
  hipLaunchKernelGGL(k_order_hist, dim3(grid), dim3(256), 0, st, T, n, bins);
  hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(kOrderBins), 0, st, bins);
  hipLaunchKernelGGL(k_order_scatter, dim3(grid), dim3(256), 0, st, T, n, bins, order);
  P.order = order;
}

// Whether the persistent ROK4E kernel runs four waves per SIMD: when asked for, and by
// default for the FP64 layouts that have that build when the block shape is left
// automatic (on the 53-species workloads it is the fastest layout: 114 against 118 ms on
// the flame slice, 217 against 222 ms on the bimodal batch).
bool use_occ4(const rok4e_mech* m) {
  if (!m->var->integrate_occ4 || m->opt.jvp_gather == ROK4E_GATHER_PRIVATE) return false;
  if (m->opt.waves_per_simd == 4) return true;
  return m->opt.waves_per_simd == 0 && m->opt.waves_per_block == 0 && m->opt.blocks_per_cu == 0 &&
         m->opt.precision == ROK4E_FP64;
}

// The persistent ROK4E kernel of the handle's layout, gather and occupancy options, and its
// largest block in waves.
IntegrateFn integrate_fn(const rok4e_mech* m) {
  if (m->opt.jvp_gather == ROK4E_GATHER_PRIVATE && m->var->integrate_gather) return m->var->integrate_gather;
  if (use_occ4(m)) return m->var->integrate_occ4;
  return m->var->integrate;
}
int integrate_fn_waves(const rok4e_mech* m) {
  if (m->opt.jvp_gather == ROK4E_GATHER_PRIVATE && m->var->integrate_gather) return integrate_waves(*m->var);
  if (use_occ4(m)) return 16;
  return integrate_waves(*m->var);
}

int check_state_args(int64_t n, rok4e_mech* mech, const void* Y, const void* T, const void* p) {
  if (!mech || n < 0) return ROK4E_EINVAL;
  if (n > 0 && (!Y || !T || !p)) return ROK4E_EINVAL;
  if (n > INT32_MAX - 1) return ROK4E_EINVAL;
  return ROK4E_OK;
}

Launch base_launch(rok4e_mech* m, int64_t n, double* Y, double* T, const double* p, const double* S,
                   const SegLayout& sl) {
  Launch P{};
  P.n_cells = n;
  P.Y = Y;
  P.T = T;
  P.p = p;
  P.S = S;
  P.M = m->opt.M;
  P.max_attempts = m->opt.max_attempts;
  P.fixed_steps = m->opt.fixed_steps;
  P.h0 = m->opt.h0;
  // FD increment delta = sqrt(eps (1 + |u|)) with eps = 2^-52 in both precisions: the
  // difference-form numerator carries no 1/delta rounding amplification to balance.
  P.eps_fd = std::ldexp(1.0, -52);
  P.queue = m->d_queue;
  P.acc = m->d_acc;
  P.rej = m->d_rej;
  P.status = m->d_status;
  P.seg_bytes = sl.bytes;
  P.off_k = sl.off_k;
  P.off_H = sl.off_H;
  P.off_LU = sl.off_LU;
  P.off_rdiag = sl.off_rdiag;
  return P;
}

// Per-attempt schedule: launch one attempt of every active cell, read back how many
// remain, repeat (the stream is synchronised once per launch; not capturable).
int run_per_attempt(rok4e_mech* m, const Launch& P, const SegLayout& sl, int64_t n_cells, hipStream_t st) {
  AttemptWork W{};
  W.st = m->d_st;
  W.fnq = m->d_fnq;
  W.H = m->d_H;
  int cur = 0;
  int64_t active = n_cells;
  for (int launch = 0; active > 0; ++launch) {
    LaunchShape sh;
    int rc = shape_for(m, sl, active, (const void*)m->var->attempt, false, &sh);
    if (rc) return rc;
    W.first = launch == 0 ? 1 : 0;
    W.act_in = m->d_act[cur];
    W.n_in = m->d_cnt + cur;
    W.act_out = m->d_act[cur ^ 1];
    W.n_out = m->d_cnt + (cur ^ 1);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, W.n_out);
    hipLaunchKernelGGL(m->var->attempt, dim3(sh.grid), dim3(sh.block), sh.lds, st, m->dm, P, W);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(m->h_cnt, W.n_out, sizeof(unsigned int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e);
    active = *m->h_cnt;
    cur ^= 1;
  }
  return ROK4E_OK;
}

// ------------------------------------------------------------- tuning cache ----
// Choices of rok4e_tune, kept for the life of the process and shared by all handles:
// key (GPU architecture, compute units, n_species, n_reactions, M, precision, method).
using TuneKey = std::tuple<std::string, int, int, int, int, int, int>;
struct TuneChoice {
  int lanes, waves, blocks, gather, simd;
  float ms;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice> g_tune_cache;

TuneKey tune_key(const rok4e_mech* m) {
  return TuneKey{m->arch, m->cu_count, m->ns, m->nr, m->opt.M, m->opt.precision, m->opt.method};
}

bool tune_lookup(const TuneKey& k, TuneChoice* c) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  const auto it = g_tune_cache.find(k);
  if (it == g_tune_cache.end()) return false;
  *c = it->second;
  return true;
}

void tune_store(const TuneKey& k, const TuneChoice& c) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_cache[k] = c;
}

// Sets the handle's launch options to a choice (its other options unchanged) and builds
// the tables of its layout.
int apply_choice(rok4e_mech* m, const TuneChoice& c) {
  rok4e_options o = m->opt;
  o.lanes_per_cell = c.lanes;
  o.waves_per_block = c.waves;
  o.blocks_per_cu = c.blocks;
  o.jvp_gather = c.gather;
  o.waves_per_simd = c.simd;
  const Variant* v = pick_variant(m->ns, o);
  if (!v) return ROK4E_ENOTSUP;
  m->opt = o;
  m->var = v;
  return ensure_image(m);
}

}  // namespace

extern "C" {

void rok4e_options_default(rok4e_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->M = 4;
  o->precision = ROK4E_FP64;
  o->scheduling = ROK4E_PERSISTENT;
}

const char* rok4e_strerror(int code) {
  switch (code) {
    case ROK4E_OK: return "ok";
    case ROK4E_EINVAL: return "invalid argument";
    case ROK4E_ENOMEM: return "device allocation failed";
    case ROK4E_EHIP: return "HIP runtime or launch error";
    case ROK4E_ECAPTURE: return "workspace too small during stream capture (call rok4e_reserve first)";
    case ROK4E_ENOTSUP: return "no kernel variant for this size, M, precision and layout";
    case ROK4E_ESTATIC: return "batch larger than the static scratch of rok4e_integrate_static";
    default: return "unknown error";
  }
}

int rok4e_mech_destroy(rok4e_mech* m) {
  if (!m) return ROK4E_OK;
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  void* bufs[] = {m->d_image, m->d_cons_image, m->d_queue, m->d_acc, m->d_rej, m->d_status, m->d_order, m->d_bins,
                  m->d_st, m->d_fnq, m->d_H,
                  m->d_act[0], m->d_act[1], m->d_cnt};
  for (void* b : bufs) (void)hipFree(b);
  if (m->h_cnt) (void)hipHostFree(m->h_cnt);
  (void)hipSetDevice(dev);
  delete m;
  return ROK4E_OK;
}

int rok4e_mech_create(const rok4e_mech_desc* d, const rok4e_options* o, rok4e_mech** out) {
  if (!d || !out) return ROK4E_EINVAL;
  *out = nullptr;
  const int ns = d->n_species, nr = d->n_reactions;
  if (ns < 1 || nr < 0 || !d->W || !d->cp || !d->hf) return ROK4E_EINVAL;
  if (nr > 0 && (!d->reac || !d->prod || !d->lnAf || !d->bf || !d->Ef || !d->lnAr || !d->br || !d->Er))
    return ROK4E_EINVAL;
  rok4e_options opt;
  rok4e_options_default(&opt);
  if (o) opt = *o;
  if (!options_ok(opt)) return ROK4E_EINVAL;
  for (int k = 0; k < ns; ++k)
    if (!(d->W[k] > 0.0) || !(d->cp[k] > 0.0) || !std::isfinite(d->W[k]) || !std::isfinite(d->cp[k]) ||
        !std::isfinite(d->hf[k]))
      return ROK4E_EINVAL;
  for (int j = 0; j < nr; ++j) {
    const double v[6] = {d->lnAf[j], d->bf[j], d->Ef[j], d->lnAr[j], d->br[j], d->Er[j]};
    for (double x : v)
      if (!std::isfinite(x)) return ROK4E_EINVAL;
    for (int a = 0; a < 2; ++a) {
      const int r = d->reac[2 * j + a], q = d->prod[2 * j + a];
      if (r < -1 || r >= ns || q < -1 || q >= ns) return ROK4E_EINVAL;
    }
    if (d->reac[2 * j] < 0 || d->prod[2 * j] < 0) return ROK4E_EINVAL;   // first slot filled
  }
  // element balance of every reaction, when the caller gives the element table
  if (d->n_elements < 0 || (d->n_elements > 0 && !d->elem)) return ROK4E_EINVAL;
  for (int j = 0; j < nr && d->n_elements > 0; ++j)
    for (int e = 0; e < d->n_elements; ++e) {
      int net = 0;
      for (int a = 0; a < 2; ++a) {
        const int r = d->reac[2 * j + a], q = d->prod[2 * j + a];
        if (r >= 0) net += d->elem[(size_t)r * d->n_elements + e];
        if (q >= 0) net -= d->elem[(size_t)q * d->n_elements + e];
      }
      if (net != 0) return ROK4E_EINVAL;
    }
  if (ns > 254) return ROK4E_ENOTSUP;
  const Variant* var = pick_variant(ns, opt);
  if (!var) return ROK4E_ENOTSUP;

  rok4e_mech* m = new (std::nothrow) rok4e_mech();
  if (!m) return ROK4E_ENOMEM;
  (void)hipGetDevice(&m->device);
  m->ns = ns;
  m->nr = nr;
  m->opt = opt;
  m->var = var;
  m->W.assign(d->W, d->W + ns);
  m->cp.assign(d->cp, d->cp + ns);
  m->hf.assign(d->hf, d->hf + ns);
  m->par.assign((size_t)6 * nr, 0.0);
  const double* src[6] = {d->lnAf, d->bf, d->Ef, d->lnAr, d->br, d->Er};
  for (int q = 0; q < 6; ++q)
    for (int j = 0; j < nr; ++j) m->par[(size_t)q * nr + j] = src[q][j];
  if (nr > 0) {
    m->reac.assign(d->reac, d->reac + 2 * nr);
    m->prod.assign(d->prod, d->prod + 2 * nr);
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, m->device) != hipSuccess) {
    delete m;
    return ROK4E_EHIP;
  }
  m->cu_count = prop.multiProcessorCount;
  m->arch = prop.gcnArchName;
  m->lds_per_block_max = prop.sharedMemPerBlock;
  // the static scratch of this device: its address is looked up here, once per device,
  // with the handle's device current
  m->scratch = scratch_ptr(m->device);
  if (!m->scratch) {
    delete m;
    return ROK4E_EHIP;
  }
  hipError_t e = hipMalloc((void**)&m->d_queue, sizeof(unsigned int));
  if (e == hipSuccess) e = hipMemset(m->d_queue, 0, sizeof(unsigned int));
  int rc = e == hipSuccess ? ensure_image(m) : hip_fail(e);
  if (rc != ROK4E_OK) {
    rok4e_mech_destroy(m);
    return rc;
  }
  *out = m;
  return ROK4E_OK;
}

int rok4e_set_options(rok4e_mech* m, const rok4e_options* o) {
  if (!m || !o || !options_ok(*o)) return ROK4E_EINVAL;
  const Variant* var = pick_variant(m->ns, *o);
  if (!var) return ROK4E_ENOTSUP;
  m->opt = *o;
  m->var = var;
  return ensure_image(m);
}

int rok4e_get_options(const rok4e_mech* m, rok4e_options* o) {
  if (!m || !o) return ROK4E_EINVAL;
  *o = m->opt;
  o->lanes_per_cell = m->var->L;
  return ROK4E_OK;
}

int rok4e_reserve(rok4e_mech* m, int64_t max_cells) {
  if (!m || max_cells < 0 || max_cells > INT32_MAX - 1) return ROK4E_EINVAL;
  if (max_cells <= m->cap) return ROK4E_OK;
  (void)hipFree(m->d_acc);
  (void)hipFree(m->d_rej);
  (void)hipFree(m->d_status);
  (void)hipFree(m->d_order);
  m->d_acc = m->d_rej = m->d_status = m->d_order = nullptr;
  m->cap = 0;
  hipError_t e = hipMalloc((void**)&m->d_acc, max_cells * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&m->d_rej, max_cells * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&m->d_status, max_cells * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&m->d_order, max_cells * sizeof(int32_t));
  if (e == hipSuccess && !m->d_bins) e = hipMalloc((void**)&m->d_bins, kOrderBins * sizeof(unsigned int));
  if (e != hipSuccess) return hip_fail(e);
  m->cap = max_cells;
  return ROK4E_OK;
}

int rok4e_integrate_ex(int64_t n_cells, rok4e_mech* m, double* Y, double* T, const double* p,
                       const double* S, double* h_io, double dt, double rtol, double atol, void* stream) {
  int rc = check_state_args(n_cells, m, Y, T, p);
  if (rc) return rc;
  if (h_io && m->opt.method == ROK4E_METHOD_RKDP45) return ROK4E_ENOTSUP;
  if (!(dt > 0.0) || !std::isfinite(dt) || !(rtol > 0.0) || !(atol >= 0.0) || !std::isfinite(rtol) ||
      !std::isfinite(atol))
    return ROK4E_EINVAL;
  if (n_cells == 0) return ROK4E_OK;
  hipStream_t st = (hipStream_t)stream;
  rc = ensure_workspace(m, n_cells, st);
  if (rc) return rc;
  const SegLayout sl = seg_layout(m->nr, *m->var);
  Launch P = base_launch(m, n_cells, Y, T, p, S, sl);
  P.dt = dt;
  P.rtol = rtol;
  P.atol = atol;
  P.hio = h_io;
  LaunchShape sh;
  if (m->opt.method == ROK4E_METHOD_RKDP45) {
    if (m->opt.scheduling != ROK4E_PERSISTENT) return ROK4E_ENOTSUP;
    rc = shape_for(m, sl, n_cells, (const void*)m->var->rkdp, true, &sh);
    if (rc) return rc;
    launch_order(m, T, n_cells, (int64_t)sh.grid * sh.segs_per_block, st, P, m->d_bins, m->d_order);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, m->d_queue);
    hipLaunchKernelGGL(m->var->rkdp, dim3(sh.grid), dim3(sh.block), sh.lds, st, m->dm, P);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e);
    m->last_n = n_cells;
    return ROK4E_OK;
  }
  if (m->opt.scheduling == ROK4E_PER_ATTEMPT) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return ROK4E_ECAPTURE;
    rc = ensure_attempt_work(m, n_cells);
    if (rc) return rc;
    rc = run_per_attempt(m, P, sl, n_cells, st);
    if (rc) return rc;
    m->last_n = n_cells;
    return ROK4E_OK;
  }
  const IntegrateFn kern = integrate_fn(m);
  rc = shape_for(m, sl, n_cells, (const void*)kern, true, &sh, nullptr, nullptr, integrate_fn_waves(m));
  if (rc) return rc;
  launch_order(m, T, n_cells, (int64_t)sh.grid * sh.segs_per_block, st, P, m->d_bins, m->d_order);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, m->d_queue);
  hipLaunchKernelGGL(kern, dim3(sh.grid), dim3(sh.block), sh.lds, st, m->dm, P);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);
  m->last_n = n_cells;
  return ROK4E_OK;
}

int rok4e_integrate_conservative(int64_t n_cells, rok4e_mech* m, double* U, const double* S,
                                 double* T_aux, double dt, double rtol, double atol, void* stream) {
  if (!m || n_cells < 0 || n_cells > INT32_MAX - 1 || (n_cells > 0 && !U)) return ROK4E_EINVAL;
  if (!(dt > 0.0) || !std::isfinite(dt) || !(rtol > 0.0) || !(atol >= 0.0) || !std::isfinite(rtol) ||
      !std::isfinite(atol))
    return ROK4E_EINVAL;
  if (m->opt.precision != ROK4E_FP64 || m->opt.method != ROK4E_METHOD_ROK4E ||
      m->opt.scheduling != ROK4E_PERSISTENT)
    return ROK4E_ENOTSUP;
  if (n_cells == 0) return ROK4E_OK;
  hipStream_t st = (hipStream_t)stream;
  // the handle's layout if it holds the ns + 6 rows, else the smallest one that does
  // (same options), with its own table image
  const Variant* var = m->var;
  const DevMech* dm = &m->dm;
  if (var->L * var->rows < m->ns + 6) {
    var = pick_variant(m->ns, m->opt, 6);
    if (!var) return ROK4E_ENOTSUP;
    if (m->cons_var != var || m->cons_image_key < 0) {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return ROK4E_ECAPTURE;
      m->cons_image_key = -1;
      const int rc = build_image(m, var, &m->cons_dm, &m->d_cons_image, &m->cons_image_key);
      if (rc) return rc;
      m->cons_var = var;
    }
    dm = &m->cons_dm;
  }
  if (!var->integrate_cons) return ROK4E_ENOTSUP;
  int rc = ensure_workspace(m, n_cells, st);
  if (rc) return rc;
  const SegLayout sl = seg_layout(m->nr, *var);
  Launch P = base_launch(m, n_cells, U, T_aux, nullptr, S, sl);
  P.dt = dt;
  P.rtol = rtol;
  P.atol = atol;
  LaunchShape sh;
  rc = shape_for(m, sl, n_cells, (const void*)var->integrate_cons, true, &sh, var, dm, integrate_waves(*var));
  if (rc) return rc;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, m->d_queue);
  hipLaunchKernelGGL(var->integrate_cons, dim3(sh.grid), dim3(sh.block), sh.lds, st, *dm, P);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);
  m->last_n = n_cells;
  return ROK4E_OK;
}

int rok4e_integrate_forced(int64_t n_cells, rok4e_mech* m, double* Y, double* T, const double* p,
                           const double* S, double dt, double rtol, double atol, void* stream) {
  return rok4e_integrate_ex(n_cells, m, Y, T, p, S, nullptr, dt, rtol, atol, stream);
}

int rok4e_integrate(int64_t n_cells, rok4e_mech* m, double* Y, double* T, const double* p, double dt,
                    double rtol, double atol, void* stream) {
  return rok4e_integrate_ex(n_cells, m, Y, T, p, nullptr, nullptr, dt, rtol, atol, stream);
}

int rok4e_integrate_static(int64_t n_cells, rok4e_mech* m, double* Y, double* T, const double* p,
                           const double* S, double dt, double rtol, double atol, int32_t* acc,
                           int32_t* rej, int32_t* status, void* stream) {
  int rc = check_state_args(n_cells, m, Y, T, p);
  if (rc) return rc;
  if (n_cells > 0 && (!acc || !rej || !status)) return ROK4E_EINVAL;
  if (!(dt > 0.0) || !std::isfinite(dt) || !(rtol > 0.0) || !(atol >= 0.0) || !std::isfinite(rtol) ||
      !std::isfinite(atol))
    return ROK4E_EINVAL;
  if (n_cells > ROK4E_STATIC_MAX_CELLS) return ROK4E_ESTATIC;
  if (n_cells == 0) return ROK4E_OK;
  if (!m->scratch) return ROK4E_EHIP;
  hipStream_t st = (hipStream_t)stream;
  const SegLayout sl = seg_layout(m->nr, *m->var);
  Launch P = base_launch(m, n_cells, Y, T, p, S, sl);
  P.dt = dt;
  P.rtol = rtol;
  P.atol = atol;
  P.queue = m->scratch;
  P.acc = acc;
  P.rej = rej;
  P.status = status;
  const bool rkdp = m->opt.method == ROK4E_METHOD_RKDP45;
  const IntegrateFn kern = rkdp ? m->var->rkdp : integrate_fn(m);
  LaunchShape sh;
  rc = shape_for(m, sl, n_cells, (const void*)kern, true, &sh, nullptr, nullptr, rkdp ? 4 : integrate_fn_waves(m));
  if (rc) return rc;
  launch_order(m, T, n_cells, (int64_t)sh.grid * sh.segs_per_block, st, P, m->scratch + kScratchBins,
               (int32_t*)(m->scratch + kScratchOrder));
  // the queue counter starts at zero: a one-thread kernel clears it (no memset node)
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, m->scratch);
  hipLaunchKernelGGL(kern, dim3(sh.grid), dim3(sh.block), sh.lds, st, m->dm, P);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);
  return ROK4E_OK;
}

int rok4e_tune(int64_t n_cells, rok4e_mech* m, const double* Y, const double* T, const double* p,
               double dt, double rtol, double atol, int32_t force, rok4e_tune_result* out, void* stream) {
  int rc = check_state_args(n_cells, m, Y, T, p);
  if (rc) return rc;
  if (n_cells == 0) return ROK4E_EINVAL;
  if (!(dt > 0.0) || !std::isfinite(dt) || !(rtol > 0.0) || !(atol >= 0.0) || !std::isfinite(rtol) ||
      !std::isfinite(atol))
    return ROK4E_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return ROK4E_ECAPTURE;
  rok4e_tune_result res{};
  const TuneKey key = tune_key(m);
  TuneChoice cached{};
  if (!force && tune_lookup(key, &cached)) {
    rc = apply_choice(m, cached);
    if (rc) return rc;
    res.lanes_per_cell = cached.lanes;
    res.waves_per_block = cached.waves;
    res.blocks_per_cu = cached.blocks;
    res.jvp_gather = cached.gather;
    res.waves_per_simd = cached.simd;
    res.ms = cached.ms;
    res.from_cache = 1;
    if (out) *out = res;
    return ROK4E_OK;
  }
  rc = ensure_workspace(m, n_cells, st);
  if (rc) return rc;
  // candidates, grouped by lane layout (each layout's tables are built once)
  std::vector<TuneChoice> cand;
  for (int L : {64, 32, 16}) {
    rok4e_options o = m->opt;
    o.lanes_per_cell = L;
    const Variant* v = pick_variant(m->ns, o);
    if (!v) continue;
    const int wmax = integrate_waves(*v);
    for (int wpb : {wmax, wmax / 2}) {
      if (wpb < 1) continue;
      cand.push_back(TuneChoice{L, wpb, 0, ROK4E_GATHER_LDS, 0, 0.0f});
      if (v->integrate_gather && m->opt.method == ROK4E_METHOD_ROK4E)
        cand.push_back(TuneChoice{L, wpb, 0, ROK4E_GATHER_PRIVATE, 0, 0.0f});
    }
    if (v->integrate_occ4 && m->opt.method == ROK4E_METHOD_ROK4E)
      cand.push_back(TuneChoice{L, 16, 0, ROK4E_GATHER_LDS, 4, 0.0f});
  }
  const size_t ny = (size_t)m->ns * n_cells;
  double *Y2 = nullptr, *T2 = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc((void**)&Y2, ny * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&T2, n_cells * sizeof(double));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // one timing: the faster of two runs after a warm-up run
  auto time_once = [&](float* best) {
    *best = 0.0f;
    for (int rep = 0; rep < 3 && e == hipSuccess && rc == ROK4E_OK; ++rep) {
      float ms = 0.0f;
      e = hipMemcpyAsync(Y2, Y, ny * sizeof(double), hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(T2, T, n_cells * sizeof(double), hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      if (e == hipSuccess) rc = rok4e_integrate(n_cells, m, Y2, T2, p, dt, rtol, atol, stream);
      if (e == hipSuccess && rc == ROK4E_OK) e = hipEventRecord(e1, st);
      if (e == hipSuccess && rc == ROK4E_OK) e = hipEventSynchronize(e1);
      if (e == hipSuccess && rc == ROK4E_OK) e = hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0 && (rep == 1 || ms < *best)) *best = ms;
    }
  };
  const rok4e_options saved = m->opt;
  const Variant* saved_var = m->var;
  float t_default = 0.0f;
  time_once(&t_default);
  TuneChoice best{};
  bool have = false;
  for (const TuneChoice& c : cand) {
    if (e != hipSuccess || rc != ROK4E_OK) break;
    rc = apply_choice(m, c);
    if (rc) break;
    float ms = 0.0f;
    time_once(&ms);
    if (e == hipSuccess && rc == ROK4E_OK && (!have || ms < best.ms)) {
      best = c;
      best.ms = ms;
      have = true;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(Y2);
  (void)hipFree(T2);
  if (e != hipSuccess || rc != ROK4E_OK || !have) {
    m->opt = saved;
    m->var = saved_var;
    const int rc2 = ensure_image(m);
    if (e != hipSuccess) return hip_fail(e);
    return rc ? rc : (rc2 ? rc2 : ROK4E_EHIP);
  }
  rc = apply_choice(m, best);
  if (rc) return rc;
  tune_store(key, best);
  res.lanes_per_cell = best.lanes;
  res.waves_per_block = best.waves;
  res.blocks_per_cu = best.blocks;
  res.jvp_gather = best.gather;
  res.waves_per_simd = best.simd;
  res.ms = best.ms;
  res.ms_default = t_default;
  res.candidates = (int32_t)cand.size();
  if (out) *out = res;
  return ROK4E_OK;
}

int rok4e_fma_probe(int64_t n_threads, int32_t iters, double* out, void* stream) {
  if (n_threads < 256 || n_threads % 256 || n_threads / 256 > INT32_MAX || iters < 1 || !out)
    return ROK4E_EINVAL;
  hipLaunchKernelGGL(k_fma_probe, dim3((unsigned)(n_threads / 256)), dim3(256), 0, (hipStream_t)stream, iters, out);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? ROK4E_OK : hip_fail(e);
}

int rok4e_rhs(int64_t n_cells, rok4e_mech* m, const double* Y, const double* T, const double* p,
              double* dY, double* dT, void* stream) {
  int rc = check_state_args(n_cells, m, Y, T, p);
  if (rc) return rc;
  if (n_cells > 0 && (!dY || !dT)) return ROK4E_EINVAL;
  if (n_cells == 0) return ROK4E_OK;
  // f alone needs only the concentrations, increments and accumulators of each segment:
  // the smaller footprint lets more segments share a compute unit
  SegLayout sl = seg_layout(m->nr, *m->var);
  sl.bytes = sl.off_k;
  Launch P = base_launch(m, n_cells, const_cast<double*>(Y), const_cast<double*>(T), p, nullptr, sl);
  LaunchShape sh;
  rc = shape_for(m, sl, n_cells, (const void*)m->var->rhs, true, &sh);
  if (rc) return rc;
  hipLaunchKernelGGL(m->var->rhs, dim3(sh.grid), dim3(sh.block), sh.lds, (hipStream_t)stream, m->dm, P, dY, dT);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? ROK4E_OK : hip_fail(e);
}

int rok4e_arnoldi(int64_t n_cells, rok4e_mech* m, const double* Y, const double* T, const double* p,
                  double* Q, double* H, int32_t* Meff, void* stream) {
  int rc = check_state_args(n_cells, m, Y, T, p);
  if (rc) return rc;
  if (n_cells > 0 && (!Q || !H || !Meff)) return ROK4E_EINVAL;
  if (n_cells == 0) return ROK4E_OK;
  const SegLayout sl = seg_layout(m->nr, *m->var);
  Launch P = base_launch(m, n_cells, const_cast<double*>(Y), const_cast<double*>(T), p, nullptr, sl);
  LaunchShape sh;
  rc = shape_for(m, sl, n_cells, (const void*)m->var->arnoldi, true, &sh, nullptr, nullptr,
                 m->var->rows == 1 && m->var->mmax <= 8 ? 16 : 4);
  if (rc) return rc;
  hipLaunchKernelGGL(m->var->arnoldi, dim3(sh.grid), dim3(sh.block), sh.lds, (hipStream_t)stream, m->dm, P, Q, H,
                     Meff);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? ROK4E_OK : hip_fail(e);
}

size_t rok4e_split_workspace_bytes(const rok4e_grid* g, int32_t n_species) {
  if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1 || n_species < 1) return 0;
  const size_t n = (size_t)g->nx * g->ny * g->nz;
  return 6 * (size_t)(n_species + 1) * n * sizeof(double);
}

}  // extern "C"

namespace {

bool grid_ok(const rok4e_grid* g) {
  if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1) return false;
  if ((int64_t)g->nx * g->ny * g->nz > INT32_MAX - 1) return false;
  if (g->x_boundary == ROK4E_X_PERIODIC ? g->inflow != nullptr
                                        : (g->x_boundary != ROK4E_X_INFLOW_OUTFLOW || !g->inflow))
    return false;
  return g->dx > 0.0 && std::isfinite(g->dx) && std::isfinite(g->vel) && g->diff >= 0.0 &&
         std::isfinite(g->diff);
}

GridDev grid_dev(const rok4e_grid* g) {
  return GridDev{g->nx, g->ny, g->nz, 0.5 / g->dx, 1.0 / (g->dx * g->dx), g->vel, g->diff,
                 g->x_boundary == ROK4E_X_INFLOW_OUTFLOW ? g->inflow : nullptr};
}

int elementwise_grid(int64_t total) { return (int)std::min<int64_t>((total + 255) / 256, 65536); }

// h_total of u' = T(u) - s0 (s0 may be null) in nsub classical Runge-Kutta steps, in place
// in the state rows (Y, T).  w: five [N][n] workspace arrays (base, two stage points, acc).
int transport_rk4(const GridDev& gd, int ns, double* Y, double* T, const double* s0, double h_total, int nsub,
                  double* w, hipStream_t st) {
  const int64_t n = (int64_t)gd.nx * gd.ny * gd.nz;
  const int64_t tot = n * (ns + 1);
  double* base = w;
  double* sa = w + tot;
  double* sb = w + 2 * tot;
  double* acc = w + 3 * tot;
  const RowsC state{Y, T};
  const RowsC rb{base, base + (int64_t)ns * n}, ra{sa, sa + (int64_t)ns * n}, rbb{sb, sb + (int64_t)ns * n};
  const RowsW none{nullptr, nullptr}, out{Y, T};
  const int grid = elementwise_grid(tot);
  const double dt = h_total / nsub;
  for (int k = 0; k < nsub; ++k) {
    hipLaunchKernelGGL(k_copy_rows, dim3(grid), dim3(256), 0, st, n, ns, state, base);
    hipLaunchKernelGGL(k_rk4_stage, dim3(grid), dim3(256), 0, st, gd, ns, rb, s0, rb, acc, 1, dt / 6.0, sa,
                       0.5 * dt, none);
    hipLaunchKernelGGL(k_rk4_stage, dim3(grid), dim3(256), 0, st, gd, ns, ra, s0, rb, acc, 0, dt / 3.0, sb,
                       0.5 * dt, none);
    hipLaunchKernelGGL(k_rk4_stage, dim3(grid), dim3(256), 0, st, gd, ns, rbb, s0, rb, acc, 0, dt / 3.0, sa, dt,
                       none);
    hipLaunchKernelGGL(k_rk4_stage, dim3(grid), dim3(256), 0, st, gd, ns, ra, s0, rb, acc, 0, dt / 6.0,
                       (double*)nullptr, 0.0, out);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? ROK4E_OK : hip_fail(e);
}

}  // namespace

extern "C" {

int rok4e_transport(const rok4e_grid* g, int32_t n_species, const double* Y, const double* T, double* S,
                    void* stream) {
  if (!grid_ok(g) || n_species < 1 || !Y || !T || !S) return ROK4E_EINVAL;
  const GridDev gd = grid_dev(g);
  const int64_t tot = (int64_t)g->nx * g->ny * g->nz * (n_species + 1);
  hipLaunchKernelGGL(k_transport, dim3(elementwise_grid(tot)), dim3(256), 0, (hipStream_t)stream, gd, n_species,
                     RowsC{Y, T}, S, (const double*)nullptr, (double*)nullptr);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? ROK4E_OK : hip_fail(e);
}

int rok4e_split_step(rok4e_mech* m, const rok4e_grid* g, int32_t scheme, double* Y, double* T, const double* p,
                     const double* src, double h, double rtol, double atol, int32_t nsub, void* work,
                     size_t work_bytes, void* stream) {
  if (!m || !grid_ok(g) || !Y || !T || !p || !work) return ROK4E_EINVAL;
  if (scheme != ROK4E_SPLIT_SIMPLER && scheme != ROK4E_SPLIT_STRANG) return ROK4E_EINVAL;
  if (!(h > 0.0) || !std::isfinite(h) || nsub < 1) return ROK4E_EINVAL;
  if (work_bytes < rok4e_split_workspace_bytes(g, m->ns)) return ROK4E_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int ns = m->ns;
  const int64_t n = (int64_t)g->nx * g->ny * g->nz;
  const int64_t tot = n * (ns + 1);
  const GridDev gd = grid_dev(g);
  double* s0 = (double*)work;     // T(U_n)
  double* f = s0 + tot;           // forcing of the reaction substep
  double* w = f + tot;            // transport workspace (4 arrays)
  int rc;
  if (scheme == ROK4E_SPLIT_SIMPLER) {
    // c_n = -T(U_n); reaction u' = R(u) + src - c_n over h; transport u' = T(u) + c_n over h/2
    hipLaunchKernelGGL(k_transport, dim3(elementwise_grid(tot)), dim3(256), 0, st, gd, ns, RowsC{Y, T}, s0, src, f);
    rc = rok4e_integrate_forced(n, m, Y, T, p, f, h, rtol, atol, stream);
    if (rc) return rc;
    return transport_rk4(gd, ns, Y, T, s0, 0.5 * h, nsub, w, st);
  }
  // Strang: transport h/2, reaction h, transport h/2
  rc = transport_rk4(gd, ns, Y, T, nullptr, 0.5 * h, nsub, w, st);
  if (rc) return rc;
  rc = rok4e_integrate_forced(n, m, Y, T, p, src, h, rtol, atol, stream);
  if (rc) return rc;
  return transport_rk4(gd, ns, Y, T, nullptr, 0.5 * h, nsub, w, st);
}

int rok4e_cell_stats_ptr(rok4e_mech* m, const int32_t** acc, const int32_t** rej, const int32_t** status) {
  if (!m) return ROK4E_EINVAL;
  if (acc) *acc = m->d_acc;
  if (rej) *rej = m->d_rej;
  if (status) *status = m->d_status;
  return ROK4E_OK;
}

int rok4e_copy_cell_stats(rok4e_mech* m, int32_t* acc, int32_t* rej, int32_t* status, void* stream) {
  if (!m) return ROK4E_EINVAL;
  const int64_t n = m->last_n;
  if (n == 0) return ROK4E_OK;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (acc) e = hipMemcpyAsync(acc, m->d_acc, n * 4, hipMemcpyDefault, st);
  if (e == hipSuccess && rej) e = hipMemcpyAsync(rej, m->d_rej, n * 4, hipMemcpyDefault, st);
  if (e == hipSuccess && status) e = hipMemcpyAsync(status, m->d_status, n * 4, hipMemcpyDefault, st);
  return e == hipSuccess ? ROK4E_OK : hip_fail(e);
}

int rok4e_get_stats(rok4e_mech* m, rok4e_stats* out, void* stream) {
  if (!m || !out) return ROK4E_EINVAL;
  std::memset(out, 0, sizeof(*out));
  const int64_t n = m->last_n;
  out->n_cells = n;
  if (n == 0) return ROK4E_OK;
  std::vector<int32_t> a(n), r(n), s(n);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(a.data(), m->d_acc, n * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(r.data(), m->d_rej, n * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(s.data(), m->d_status, n * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e);
  for (int64_t i = 0; i < n; ++i) {
    out->accepted += a[i];
    out->rejected += r[i];
    const int64_t att = (int64_t)a[i] + r[i];
    out->max_attempts = std::max<int64_t>(out->max_attempts, att);
    if (s[i] >= 0 && s[i] < 4) out->status_count[s[i]]++;
    int bin = 0;
    while (bin < ROK4E_HIST_BINS - 1 && att >= ((int64_t)1 << bin)) ++bin;
    out->attempt_histogram[bin]++;
  }
  return ROK4E_OK;
}

}  // extern "C"
