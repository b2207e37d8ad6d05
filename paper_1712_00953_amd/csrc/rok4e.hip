// Batched ROK4E reaction substep: kernels and the C ABI declared in include/rok4e.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "rok4e.h"
#include "rok4e_integrator.hpp"

namespace rok4e {

// ------------------------------------------------------------------ kernels ----

__global__ void k_zero_u32(unsigned int* x) { *x = 0u; }

// Persistent integrator: every segment of L lanes pulls cells from a device counter
// until the batch is exhausted, so cells with 1 and 1000 attempts share the chip
// without waiting on each other.
template <int L, int ROWS, int MMAX, class RT>
__global__ void __launch_bounds__(256, 2) k_integrate(DevMech m, Launch P) {
  extern __shared__ __align__(16) char smem[];
  const int lane = (int)(threadIdx.x % L);
  char* seg = smem + (threadIdx.x / L) * P.seg_bytes;
  const SegLds<RT> S = seg_lds<RT>(seg, P);
  while (true) {
    // Every lane takes part in the atomic (the segment's first lane adds 1, the others
    // 0), so no lane-dependent branch surrounds the value that is then broadcast.
    const unsigned int ticket = atomicAdd(P.queue, lane == 0 ? 1u : 0u);
    const int cell = seg_bcast<L>((int)ticket, 0);
    if (cell < 0 || (int64_t)cell >= P.n_cells) break;
    double u[ROWS], s[ROWS], p;
    CellResult r{3, 0, 0};
    if (load_cell<L, ROWS>(m, P, cell, lane, u, s, p)) {
      r = integrate_cell<L, ROWS, MMAX, RT>(m, P, u, p, s, S, lane);
      store_cell<L, ROWS>(m, P, cell, lane, u);
    }
    // every lane of the segment stores the same (segment-uniform) values
    P.acc[cell] = r.accepted;
    P.rej[cell] = r.rejected;
    P.status[cell] = r.status;
  }
}

// f(u) for every cell (grid-stride over cells, one cell per segment).
template <int L, int ROWS, class RT>
__global__ void __launch_bounds__(256, 2) k_rhs(DevMech m, Launch P, double* dY, double* dT) {
  extern __shared__ __align__(16) char smem[];
  const int lane = (int)(threadIdx.x % L);
  char* seg = smem + (threadIdx.x / L) * P.seg_bytes;
  const SegLds<RT> S = seg_lds<RT>(seg, P);
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
    RT w[ROWS];
    rhs<L, ROWS, RT, false>(m, u, P.p[cell], f, S.r, lane, nullptr, w);
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const int r = i * L + lane;
      if (r < ns) dY[(int64_t)r * n + cell] = f[i];
      else if (r == ns) dT[cell] = f[i];
    }
  }
}

// Arnoldi basis at every cell's state (diagnostics and step-level parity).
template <int L, int ROWS, int MMAX, class RT>
__global__ void __launch_bounds__(256, 2) k_arnoldi(DevMech m, Launch P, double* Qo, double* Ho,
                                                  int32_t* Mo) {
  extern __shared__ __align__(16) char smem[];
  const int lane = (int)(threadIdx.x % L);
  char* seg = smem + (threadIdx.x / L) * P.seg_bytes;
  const SegLds<RT> S = seg_lds<RT>(seg, P);
  const int64_t nseg = (int64_t)gridDim.x * (blockDim.x / L);
  const int64_t n = P.n_cells;
  const int N = m.ns + 1, M = P.M;
  for (int64_t cell = (int64_t)blockIdx.x * (blockDim.x / L) + threadIdx.x / L; cell < n; cell += nseg) {
    double u[ROWS], s[ROWS], fn[ROWS], p;
    load_cell<L, ROWS>(m, P, cell, lane, u, s, p);
    RhsBase base;
    RT w[ROWS];
    rhs_forced<L, ROWS, RT, true>(m, u, p, s, fn, S, lane, &base, w);
    for (int i = 0; i < MMAX * MMAX; ++i) S.H[i] = 0.0;
    lds_sync();
    double Q[ROWS][MMAX];
    const int Meff = arnoldi<L, ROWS, MMAX, RT>(m, P, u, fn, base, w, Q, S, lane);
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const int r = i * L + lane;
      if (r < N)
#pragma unroll
        for (int j = 0; j < MMAX; ++j)
          if (j < M) Qo[((int64_t)cell * M + j) * N + r] = Q[i][j];
    }
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j)
        Ho[((int64_t)cell * M + i) * M + j] =
            (i < MMAX && j < MMAX && i <= j + 1 && i < Meff && j < Meff) ? S.H[i * MMAX + j] : 0.0;
    Mo[cell] = Meff;
    lds_sync();
  }
}

// ------------------------------------------------------------ variant table ----

using IntegrateFn = void (*)(DevMech, Launch);
using RhsFn = void (*)(DevMech, Launch, double*, double*);
using ArnoldiFn = void (*)(DevMech, Launch, double*, double*, int32_t*);

struct Variant {
  int L, rows, mmax, prec;
  IntegrateFn integrate;
  ArnoldiFn arnoldi;
  RhsFn rhs;
};

#define ROK4E_VARIANT(Lv, Rv, Mv, T, P) \
  Variant{Lv, Rv, Mv, P, k_integrate<Lv, Rv, Mv, T>, k_arnoldi<Lv, Rv, Mv, T>, k_rhs<Lv, Rv, T>}

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

}  // namespace rok4e

using namespace rok4e;

// ------------------------------------------------------------------- handle ----

struct rok4e_mech {
  int device = 0;
  int ns = 0, nr = 0, deg_max = 0;
  rok4e_options opt{};
  const Variant* var = nullptr;
  int cu_count = 0;
  // device tables
  double* d_par = nullptr;    // 6 * nr
  int4* d_rx = nullptr;
  double* d_spec = nullptr;   // 3 * ns: W, cp, hf
  int* d_prod_j = nullptr;
  int* d_prod_nu = nullptr;
  int* d_deg = nullptr;
  unsigned int* d_queue = nullptr;
  // per-cell workspace
  int64_t cap = 0;
  int32_t* d_acc = nullptr;
  int32_t* d_rej = nullptr;
  int32_t* d_status = nullptr;
  int64_t last_n = 0;
};

namespace {

int hip_fail(hipError_t e) { return e == hipErrorOutOfMemory ? ROK4E_ENOMEM : ROK4E_EHIP; }

bool options_ok(const rok4e_options& o) {
  if (o.M < 1 || o.M > 16) return false;
  if (o.precision != ROK4E_FP64 && o.precision != ROK4E_MIXED) return false;
  if (o.fixed_steps < 0) return false;
  if (o.lanes_per_cell != 0 && o.lanes_per_cell != 16 && o.lanes_per_cell != 32 && o.lanes_per_cell != 64)
    return false;
  if (o.waves_per_block < 0 || o.waves_per_block > 4) return false;
  if (o.blocks_per_cu < 0 || o.blocks_per_cu > 64) return false;
  if (o.scheduling != ROK4E_PERSISTENT && o.scheduling != ROK4E_PER_ATTEMPT) return false;
  if (!std::isfinite(o.h0)) return false;
  return true;
}

// Smallest instantiated variant that holds ns+1 rows and M Krylov vectors.
const Variant* pick_variant(int ns, const rok4e_options& o) {
  const int N = ns + 1;
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

// Per-segment LDS: c, dc [ns] and q, kf, kr [nr] in the rate type; H, LU [MMAX^2] FP64;
// piv [MMAX].
struct SegLayout {
  int bytes, off_dc, off_q, off_kf, off_kr, off_H, off_LU, off_piv;
};

SegLayout seg_layout(int ns, int nr, const Variant& v) {
  const int rt = v.prec == ROK4E_FP64 ? 8 : 4;
  const int nrr = std::max(nr, 1);
  auto al = [](int x) { return (x + 15) & ~15; };
  SegLayout s{};
  int off = al(ns * rt);
  s.off_dc = off;
  off = al(off + ns * rt);
  s.off_q = off;
  off = al(off + nrr * rt);
  s.off_kf = off;
  off = al(off + nrr * rt);
  s.off_kr = off;
  off = al(off + nrr * rt);
  s.off_H = off;
  off = al(off + v.mmax * v.mmax * 8);
  s.off_LU = off;
  off = al(off + v.mmax * v.mmax * 8);
  s.off_piv = off;
  off = al(off + v.mmax * 4);
  s.bytes = off;
  return s;
}

DevMech dev_mech(const rok4e_mech* m) {
  DevMech d{};
  d.ns = m->ns;
  d.nr = m->nr;
  d.deg_max = m->deg_max;
  const int nr = m->nr;
  d.lnAf = m->d_par;
  d.bf = m->d_par + nr;
  d.Ef = m->d_par + 2 * nr;
  d.lnAr = m->d_par + 3 * nr;
  d.br = m->d_par + 4 * nr;
  d.Er = m->d_par + 5 * nr;
  d.rx = m->d_rx;
  d.W = m->d_spec;
  d.cp = m->d_spec + m->ns;
  d.hf = m->d_spec + 2 * m->ns;
  d.prod_j = m->d_prod_j;
  d.prod_nu = m->d_prod_nu;
  d.deg = m->d_deg;
  return d;
}

struct LaunchShape {
  int block, grid, segs_per_block, lds;
};

int waves_per_block_for(const rok4e_mech* m) {
  return m->opt.waves_per_block > 0 ? m->opt.waves_per_block : 4;
}

LaunchShape shape_for(const rok4e_mech* m, const SegLayout& sl, int64_t n_cells, const void* kernel,
                      bool persistent) {
  LaunchShape s{};
  const Variant& v = *m->var;
  int wpb = waves_per_block_for(m);
  s.block = 64 * wpb;
  s.segs_per_block = s.block / v.L;
  s.lds = s.segs_per_block * sl.bytes;
  const int64_t need = (n_cells + s.segs_per_block - 1) / s.segs_per_block;
  int per_cu = 1;
  if (persistent) {
    if (m->opt.blocks_per_cu > 0) {
      per_cu = m->opt.blocks_per_cu;
    } else {
      int occ = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, s.block, s.lds) != hipSuccess || occ < 1)
        occ = 1;
      per_cu = occ;
    }
  } else {
    per_cu = 8;
  }
  int64_t grid = (int64_t)per_cu * m->cu_count;
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  s.grid = (int)grid;
  return s;
}

int ensure_workspace(rok4e_mech* m, int64_t n, hipStream_t stream) {
  if (n <= m->cap) return ROK4E_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return ROK4E_ECAPTURE;
  return rok4e_reserve(m, n);
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
  P.off_dc = sl.off_dc;
  P.off_q = sl.off_q;
  P.off_kf = sl.off_kf;
  P.off_kr = sl.off_kr;
  P.off_H = sl.off_H;
  P.off_LU = sl.off_LU;
  P.off_piv = sl.off_piv;
  return P;
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
    default: return "unknown error";
  }
}

int rok4e_mech_destroy(rok4e_mech* m) {
  if (!m) return ROK4E_OK;
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  void* bufs[] = {m->d_par, m->d_rx, m->d_spec, m->d_prod_j, m->d_prod_nu, m->d_deg,
                  m->d_queue, m->d_acc, m->d_rej, m->d_status};
  for (void* b : bufs) (void)hipFree(b);
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
  const Variant* var = pick_variant(ns, opt);
  if (!var) return ROK4E_ENOTSUP;

  // Species-major production lists: for species k, (reaction j, net coefficient) for
  // every reaction with a non-zero net coefficient, in increasing j.
  std::vector<std::vector<std::pair<int, int>>> lists(ns);
  for (int j = 0; j < nr; ++j) {
    int sp[4], nu[4], nsp = 0;
    auto add = [&](int r, int c) {
      if (r < 0) return;
      int i = 0;
      while (i < nsp && sp[i] != r) ++i;
      if (i == nsp) { sp[nsp] = r; nu[nsp] = 0; ++nsp; }
      nu[i] += c;
    };
    add(d->reac[2 * j], -1);
    add(d->reac[2 * j + 1], -1);
    add(d->prod[2 * j], +1);
    add(d->prod[2 * j + 1], +1);
    for (int i = 0; i < nsp; ++i)
      if (nu[i] != 0) lists[sp[i]].push_back({j, nu[i]});
  }
  int deg_max = 0;
  for (auto& l : lists) deg_max = std::max<int>(deg_max, (int)l.size());
  const int dmax = std::max(deg_max, 1);
  std::vector<int> pj((size_t)dmax * ns, 0), pn((size_t)dmax * ns, 0), deg(ns, 0);
  for (int k = 0; k < ns; ++k) {
    deg[k] = (int)lists[k].size();
    for (int i = 0; i < deg[k]; ++i) {
      pj[(size_t)i * ns + k] = lists[k][i].first;
      pn[(size_t)i * ns + k] = lists[k][i].second;
    }
  }
  std::vector<double> par((size_t)6 * std::max(nr, 1), 0.0);
  std::vector<int4> rx(std::max(nr, 1));
  for (int j = 0; j < nr; ++j) {
    par[j] = d->lnAf[j];
    par[nr + j] = d->bf[j];
    par[2 * nr + j] = d->Ef[j];
    par[3 * nr + j] = d->lnAr[j];
    par[4 * nr + j] = d->br[j];
    par[5 * nr + j] = d->Er[j];
    rx[j] = make_int4(d->reac[2 * j], d->reac[2 * j + 1], d->prod[2 * j], d->prod[2 * j + 1]);
  }
  std::vector<double> spec((size_t)3 * ns);
  for (int k = 0; k < ns; ++k) {
    spec[k] = d->W[k];
    spec[ns + k] = d->cp[k];
    spec[2 * ns + k] = d->hf[k];
  }

  rok4e_mech* m = new (std::nothrow) rok4e_mech();
  if (!m) return ROK4E_ENOMEM;
  (void)hipGetDevice(&m->device);
  m->ns = ns;
  m->nr = nr;
  m->deg_max = deg_max;
  m->opt = opt;
  m->var = var;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, m->device) != hipSuccess) {
    delete m;
    return ROK4E_EHIP;
  }
  m->cu_count = prop.multiProcessorCount;
  hipError_t e = hipSuccess;
  auto up = [&](void** dst, const void* src, size_t bytes) {
    if (e != hipSuccess) return;
    e = hipMalloc(dst, bytes);
    if (e == hipSuccess) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  up((void**)&m->d_par, par.data(), par.size() * sizeof(double));
  up((void**)&m->d_rx, rx.data(), rx.size() * sizeof(int4));
  up((void**)&m->d_spec, spec.data(), spec.size() * sizeof(double));
  up((void**)&m->d_prod_j, pj.data(), pj.size() * sizeof(int));
  up((void**)&m->d_prod_nu, pn.data(), pn.size() * sizeof(int));
  up((void**)&m->d_deg, deg.data(), deg.size() * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&m->d_queue, sizeof(unsigned int));
  if (e == hipSuccess) e = hipMemset(m->d_queue, 0, sizeof(unsigned int));
  if (e != hipSuccess) {
    const int rc = hip_fail(e);
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
  return ROK4E_OK;
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
  m->d_acc = m->d_rej = m->d_status = nullptr;
  m->cap = 0;
  hipError_t e = hipMalloc((void**)&m->d_acc, max_cells * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&m->d_rej, max_cells * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&m->d_status, max_cells * sizeof(int32_t));
  if (e != hipSuccess) return hip_fail(e);
  m->cap = max_cells;
  return ROK4E_OK;
}

int rok4e_integrate_forced(int64_t n_cells, rok4e_mech* m, double* Y, double* T, const double* p,
                           const double* S, double dt, double rtol, double atol, void* stream) {
  int rc = check_state_args(n_cells, m, Y, T, p);
  if (rc) return rc;
  if (!(dt > 0.0) || !std::isfinite(dt) || !(rtol > 0.0) || !(atol >= 0.0) || !std::isfinite(rtol) ||
      !std::isfinite(atol))
    return ROK4E_EINVAL;
  if (n_cells == 0) return ROK4E_OK;
  hipStream_t st = (hipStream_t)stream;
  rc = ensure_workspace(m, n_cells, st);
  if (rc) return rc;
  const SegLayout sl = seg_layout(m->ns, m->nr, *m->var);
  Launch P = base_launch(m, n_cells, Y, T, p, S, sl);
  P.dt = dt;
  P.rtol = rtol;
  P.atol = atol;
  const DevMech dm = dev_mech(m);
  const LaunchShape sh = shape_for(m, sl, n_cells, (const void*)m->var->integrate, true);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, m->d_queue);
  hipLaunchKernelGGL(m->var->integrate, dim3(sh.grid), dim3(sh.block), sh.lds, st, dm, P);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);
  m->last_n = n_cells;
  return ROK4E_OK;
}

int rok4e_integrate(int64_t n_cells, rok4e_mech* m, double* Y, double* T, const double* p, double dt,
                    double rtol, double atol, void* stream) {
  return rok4e_integrate_forced(n_cells, m, Y, T, p, nullptr, dt, rtol, atol, stream);
}

int rok4e_rhs(int64_t n_cells, rok4e_mech* m, const double* Y, const double* T, const double* p,
              double* dY, double* dT, void* stream) {
  int rc = check_state_args(n_cells, m, Y, T, p);
  if (rc) return rc;
  if (n_cells > 0 && (!dY || !dT)) return ROK4E_EINVAL;
  if (n_cells == 0) return ROK4E_OK;
  const SegLayout sl = seg_layout(m->ns, m->nr, *m->var);
  Launch P = base_launch(m, n_cells, const_cast<double*>(Y), const_cast<double*>(T), p, nullptr, sl);
  const LaunchShape sh = shape_for(m, sl, n_cells, (const void*)m->var->rhs, false);
  hipLaunchKernelGGL(m->var->rhs, dim3(sh.grid), dim3(sh.block), sh.lds, (hipStream_t)stream, dev_mech(m), P,
                     dY, dT);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? ROK4E_OK : hip_fail(e);
}

int rok4e_arnoldi(int64_t n_cells, rok4e_mech* m, const double* Y, const double* T, const double* p,
                  double* Q, double* H, int32_t* Meff, void* stream) {
  int rc = check_state_args(n_cells, m, Y, T, p);
  if (rc) return rc;
  if (n_cells > 0 && (!Q || !H || !Meff)) return ROK4E_EINVAL;
  if (n_cells == 0) return ROK4E_OK;
  const SegLayout sl = seg_layout(m->ns, m->nr, *m->var);
  Launch P = base_launch(m, n_cells, const_cast<double*>(Y), const_cast<double*>(T), p, nullptr, sl);
  const LaunchShape sh = shape_for(m, sl, n_cells, (const void*)m->var->arnoldi, false);
  hipLaunchKernelGGL(m->var->arnoldi, dim3(sh.grid), dim3(sh.block), sh.lds, (hipStream_t)stream, dev_mech(m),
                     P, Q, H, Meff);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? ROK4E_OK : hip_fail(e);
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
    out->max_attempts = std::max<int64_t>(out->max_attempts, (int64_t)a[i] + r[i]);
    if (s[i] >= 0 && s[i] < 4) out->status_count[s[i]]++;
  }
  return ROK4E_OK;
}

}  // extern "C"
