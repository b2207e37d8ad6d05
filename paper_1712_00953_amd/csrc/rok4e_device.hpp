// Device building blocks of the batched ROK4E reaction substep (gfx950, wave64).
//
// Layout: one cell per "segment" of L lanes (L = 16, 32 or 64).  State row r of a cell
// (species 0..ns-1, then T at row ns) lives in lane r % L, slot r / L of that segment
// (ROWS slots per lane).  Reactions are taken round-robin by the segment's lanes for
// the rate evaluation.  Concentrations and rates of progress are staged through a
// per-segment LDS region; the small M x M projected matrices live there too.
//
// Reductions over a segment follow one fixed tree (16-lane butterfly, then lane
// halves, then slots pairwise), so results do not depend on L or ROWS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rok4e {

constexpr double kRu = 8.314462618;    // J/(mol K)
constexpr double kTref = 298.15;       // K

// ROK4E coefficients, table t:coeff_rok4e (b row read as (b1, b2, 0, b4), b-hat row as
// (bh1, bh2, bh3, 0)).
constexpr double G = 0.572816062482135;
constexpr double G21 = -0.602765307997356;
constexpr double G31 = -1.389195789724843, G32 = 1.072950969011413;
constexpr double G41 = 0.992356412977094, G42 = -1.390032613873701, G43 = -0.440875890223325;
constexpr double A21 = 0.432364435748567;
constexpr double A31 = -0.514211316876170, A32 = 1.382271144617360;
constexpr double B1 = 0.194335256262729, B2 = 0.483167813989227, B4 = 0.322496929748044;
constexpr double BH1 = -0.217819895945721, BH2 = 1.03130847478467, BH3 = 0.186511421161047;
// Embedded minus main weights (b3 = 0, bh4 = 0).
constexpr double E1 = BH1 - B1, E2 = BH2 - B2, E3 = BH3 - 0.0, E4 = 0.0 - B4;

// Device view of a mechanism: one contiguous table image in global memory, copied to
// LDS once per block by the kernels.  Image layout (NRP = reaction count rounded to even,
// LP = lanes x slots of the layout, D = production-list length):
//   double par[6][NRP]   ln A_f, b_f, E_f, ln A_r, b_r, E_r
//   double spec[4][LP]   W, 1/W, c_p, h_f per state row (zeros/ones past the species)
//   int    rx[NRP]       species of reaction j packed in bytes (reac0, reac1, prod0,
//                        prod1); an absent slot holds ns, whose concentration is 1
//   int    gidx[D][LP]   production list of row r: indices into the signed rates
//                        qs = (q_0..q_{NRP-1}, -q_0..-q_{NRP-1}, 0); a coefficient of
//                        +-2 appears as two entries, padding points at the final 0
struct DevMech {
  int ns, nr, nrp, lp, D;
  int off_spec, off_rx, off_gidx, image_bytes;
  const int4* image;
};

// LDS view of the table image.
struct MechLds {
  const double* lnAf; const double* bf; const double* Ef;
  const double* lnAr; const double* br; const double* Er;
  const double* W; const double* invW; const double* cp; const double* hf;
  const int* rx;
  const int* gidx;
};

// Per-launch arguments of the integrator.
struct Launch {
  int64_t n_cells;
  double* Y; double* T; const double* p; const double* S;
  double dt, rtol, atol, h0, eps_fd;
  int M, max_attempts, fixed_steps;
  unsigned int* queue;
  int32_t* acc; int32_t* rej; int32_t* status;
  int seg_bytes, off_dc, off_q, off_kf, off_kr, off_H, off_LU, off_rdiag, off_piv;
};

// Copies the table image to the start of the block's LDS and returns the view.  All
// threads of the block take part; ends with a block barrier (kernel start only).
__device__ __forceinline__ MechLds load_mech_lds(const DevMech& m, char* lds) {
  int4* dst = (int4*)lds;
  for (int i = threadIdx.x; i < m.image_bytes / 16; i += blockDim.x) dst[i] = m.image[i];
  __syncthreads();
  const double* par = (const double*)lds;
  MechLds t;
  t.lnAf = par; t.bf = par + m.nrp; t.Ef = par + 2 * m.nrp;
  t.lnAr = par + 3 * m.nrp; t.br = par + 4 * m.nrp; t.Er = par + 5 * m.nrp;
  const double* sp = (const double*)(lds + m.off_spec);
  t.W = sp; t.invW = sp + m.lp; t.cp = sp + 2 * m.lp; t.hf = sp + 3 * m.lp;
  t.rx = (const int*)(lds + m.off_rx);
  t.gidx = (const int*)(lds + m.off_gidx);
  return t;
}

// ------------------------------------------------------------ cross-lane ----

__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}
// lane ^ 16 within each half of the wave
__device__ __forceinline__ double swz16(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_ds_swizzle(lo, 0x401F);
  hi = __builtin_amdgcn_ds_swizzle(hi, 0x401F);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float swz16(float x) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), 0x401F));
}
__device__ __forceinline__ double readlane(double x, int l) {
  int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ int readlane(int x, int l) { return __builtin_amdgcn_readlane(x, l); }

// Sum over the L lanes of a segment; every lane receives the result.
template <int L, class V>
__device__ __forceinline__ V seg_sum1(V x) {
  x = x + dpp<0xB1>(x);     // quad_perm [1,0,3,2]
  x = x + dpp<0x4E>(x);     // quad_perm [2,3,0,1]
  x = x + dpp<0x141>(x);    // row_half_mirror: pairs the two quads of each half-row
  x = x + dpp<0x140>(x);    // row_mirror: pairs the two half-rows of each row
  if constexpr (L >= 32) x = x + swz16(x);
  if constexpr (L == 64) x = readlane(x, 0) + readlane(x, 32);
  return x;
}

// Sum over all rows of a segment: per-slot lane reduction, then slots pairwise.
template <int L, int ROWS, class V>
__device__ __forceinline__ V seg_sum(const V (&x)[ROWS]) {
  if constexpr (ROWS == 1) {
    return seg_sum1<L>(x[0]);
  } else if constexpr (ROWS == 2) {
    return seg_sum1<L>(x[0]) + seg_sum1<L>(x[1]);
  } else {
    static_assert(ROWS == 4, "ROWS must be 1, 2 or 4");
    return (seg_sum1<L>(x[0]) + seg_sum1<L>(x[1])) + (seg_sum1<L>(x[2]) + seg_sum1<L>(x[3]));
  }
}

// Value of x in lane `src` of this segment.
template <int L, class V>
__device__ __forceinline__ V seg_bcast(V x, int src) {
  if constexpr (L == 64) {
    return readlane(x, src);
  } else {
    const int base = (int)(threadIdx.x & 63) & ~(L - 1);
    return __shfl(x, base + src, 64);
  }
}

// ----------------------------------------------------------- arithmetic ----

// Arrhenius rate exp(lnA + b lnT - E invRT) in the compute type.
__device__ __forceinline__ double arrhenius(double lnA, double b, double E, double lnT, double invRT,
                                            double) {
  return exp(lnA + b * lnT - E * invRT);
}
// FP32 rate: the exponent is formed in FP64 and split into an integer and a fraction so
// that the hardware exp2 only sees |r| <= 0.5 (relative error ~1 ulp of FP32).
__device__ __forceinline__ float arrhenius(double lnA, double b, double E, double lnT, double invRT,
                                           float) {
  const double x = (lnA + b * lnT - E * invRT) * 1.4426950408889634;   // log2(e)
  const double n = rint(x);
  const float r = (float)(x - n);
  return ldexpf(__builtin_amdgcn_exp2f(r), (int)fmax(fmin(n, 300.0), -300.0));
}

template <class V>
__device__ __forceinline__ bool finite_(V x) { return __builtin_isfinite(x); }

// -------------------------------------------------------- right-hand side ----

// Per-segment LDS scratch of the right-hand side.
template <class RT>
struct RhsLds {
  RT* c;    // [LP] concentrations of the base state; c[ns] = 1 (absent reaction slot)
  RT* dc;   // [LP] their increments (difference evaluation); dc[ns] = 0
  RT* qs;   // [2 NRP + 1] signed rates of progress (or increments), last entry 0
  RT* kf;   // [NRP] forward rate constants of the base state
  RT* kr;   // [NRP] reverse rate constants of the base state
};

// Cell-uniform quantities of a base evaluation f(u), kept for the difference evaluation.
struct RhsBase {
  double T, invT, sigma, cpbar, rho, invrho, hsum;
};

// expm1 for the small arguments of the difference evaluation (Taylor series to x^5,
// relative error below 2e-18 for |x| < 1e-3), the library routine otherwise.
__device__ __forceinline__ double expm1_small(double x) {
  if (fabs(x) < 1e-3)
    return x * (1.0 + x * (0.5 + x * (1.0 / 6.0 + x * (1.0 / 24.0 + x * (1.0 / 120.0)))));
  return expm1(x);
}

template <int L, int ROWS>
__device__ __forceinline__ double row_value(const double (&u)[ROWS], int slot) {
  double v = 0.0;
#pragma unroll
  for (int s = 0; s < ROWS; ++s)
    if (s == slot) v = u[s];
  return v;
}

// Sum of the signed rates listed for state row r (fixed order: increasing reaction
// index), i.e. sum_j nu_rj q_j.
template <class RT>
__device__ __forceinline__ RT production(const MechLds& t, const RT* qs, int D, int lp, int r) {
  const int* g = t.gidx + r;
  RT acc = 0;
#pragma unroll 8
  for (int d = 0; d < D; ++d) acc = acc + qs[g[d * lp]];
  return acc;
}

// f(u) of one cell held by a segment (Sec. 4.4, e:cv_reactor, constant-pressure
// reading): rho = p / (Ru T sum Y/W), c_k = 1e-6 rho Y_k / W_k (mol/cm^3),
// q_j = k_f prod c - k_r prod c, omega_k = 1e6 sum_j nu_kj q_j,
// dY_k/dt = W_k omega_k / rho, dT/dt = -sum_k h_k W_k omega_k / (rho cp_mix).
// RT is the type of the rate constants, concentrations and production sums.  With SAVE
// the rate constants go to LDS and the base quantities to *base / w for rhs_diff.
template <int L, int ROWS, class RT, bool SAVE>
__device__ __forceinline__ void rhs(const DevMech& m, const MechLds& t, const double (&u)[ROWS],
                                    double p, double (&f)[ROWS], const RhsLds<RT>& S, int lane,
                                    RhsBase* base, RT (&w)[ROWS]) {
  const int ns = m.ns, nrp = m.nrp;
  const int sT = ns / L, lT = ns % L;
  const double T = seg_bcast<L>(row_value<L, ROWS>(u, sT), lT);

  double ps[ROWS], pc[ROWS];
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = s * L + lane;          // rows past the species have invW = cp = 0
    ps[s] = (r < ns ? u[s] : 0.0) * t.invW[r];
    pc[s] = (r < ns ? u[s] : 0.0) * t.cp[r];
  }
  const double sigma = seg_sum<L, ROWS>(ps);
  const double cpbar = seg_sum<L, ROWS>(pc);
  const double rho = p / (kRu * T * sigma);
  const double invrho = 1.0 / rho;
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = s * L + lane;
    if (r < ns) S.c[r] = (RT)(1e-6 * rho * u[s] * t.invW[r]);
  }
  const double lnT = log(T);
  const double invRT = 1.0 / (kRu * T);
  lds_sync();
  for (int j = lane; j < m.nr; j += L) {
    const RT kf = arrhenius(t.lnAf[j], t.bf[j], t.Ef[j], lnT, invRT, RT(0));
    const RT kr = arrhenius(t.lnAr[j], t.br[j], t.Er[j], lnT, invRT, RT(0));
    if constexpr (SAVE) {
      S.kf[j] = kf;
      S.kr[j] = kr;
    }
    const int x = t.rx[j];
    const RT pf = S.c[x & 0xFF] * S.c[(x >> 8) & 0xFF];
    const RT pr = S.c[(x >> 16) & 0xFF] * S.c[(x >> 24) & 0xFF];
    const RT q = kf * pf - kr * pr;
    S.qs[j] = q;
    S.qs[nrp + j] = -q;
  }
  lds_sync();
  double ph[ROWS];
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = s * L + lane;
    const RT wk = (RT)1e6 * production<RT>(t, S.qs, m.D, m.lp, r);
    w[s] = wk;
    f[s] = (double)((RT)t.W[r] * wk * (RT)invrho);
    const RT hk = (RT)(t.hf[r] + t.cp[r] * (T - kTref));
    ph[s] = (double)(hk * (RT)t.W[r] * wk);
  }
  const double hsum = seg_sum<L, ROWS>(ph);
  const double fT = -hsum / (rho * cpbar);
#pragma unroll
  for (int s = 0; s < ROWS; ++s)
    if (s == sT && lane == lT) f[s] = fT;
  if constexpr (SAVE) *base = RhsBase{T, 1.0 / T, sigma, cpbar, rho, invrho, hsum};
  lds_sync();   // the LDS scratch is reused by the next evaluation
}

// df = f(u + du) - f(u) in difference form, given the base evaluation at u (base, w,
// S.c, S.kf, S.kr): every intermediate quantity is carried with its increment, formed
// from increments only, so the result has the relative accuracy of the compute type
// instead of the absolute accuracy eps |f| of a difference of two evaluations.
// The increments of the scalar state functions (rho, ln T, 1/(Ru T)) are FP64.
template <int L, int ROWS, class RT>
__device__ __forceinline__ void rhs_diff(const DevMech& m, const MechLds& t, const RhsBase& B,
                                         const RT (&w)[ROWS], const double (&u)[ROWS],
                                         const double (&du)[ROWS], double (&df)[ROWS],
                                         const RhsLds<RT>& S, int lane) {
  const int ns = m.ns, nrp = m.nrp;
  const int sT = ns / L, lT = ns % L;
  const double T = B.T;
  const double dT = seg_bcast<L>(row_value<L, ROWS>(du, sT), lT);
  const double T1 = T + dT;
  double ps[ROWS], pc[ROWS];
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = s * L + lane;
    ps[s] = (r < ns ? du[s] : 0.0) * t.invW[r];
    pc[s] = (r < ns ? du[s] : 0.0) * t.cp[r];
  }
  const double dsigma = seg_sum<L, ROWS>(ps);
  const double dcp = seg_sum<L, ROWS>(pc);
  const double sigma1 = B.sigma + dsigma, cp1 = B.cpbar + dcp;
  const double rho = B.rho;
  const double drho = -rho * (dT * sigma1 + T * dsigma) / (T1 * sigma1);
  const double rho1 = rho + drho;
  const double invrho1 = 1.0 / rho1;
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = s * L + lane;
    if (r < ns) S.dc[r] = (RT)(1e-6 * (rho1 * du[s] + drho * u[s]) * t.invW[r]);
  }
  const double dlnT = log1p(dT * B.invT);
  const double dinvRT = -dT / (kRu * T * T1);
  lds_sync();
  for (int j = lane; j < m.nr; j += L) {
    const RT kf = S.kf[j], kr = S.kr[j];
    const RT dkf = kf * (RT)expm1_small(t.bf[j] * dlnT - t.Ef[j] * dinvRT);
    const RT dkr = kr * (RT)expm1_small(t.br[j] * dlnT - t.Er[j] * dinvRT);
    const int x = t.rx[j];
    // products of concentrations with increments: d(ab) = (a + da) db + da b
    const int a0 = x & 0xFF, a1 = (x >> 8) & 0xFF, b0 = (x >> 16) & 0xFF, b1 = (x >> 24) & 0xFF;
    const RT ca = S.c[a0], dca = S.dc[a0], cb = S.c[a1], dcb = S.dc[a1];
    const RT pf = ca * cb, dpf = (ca + dca) * dcb + dca * cb;
    const RT cc = S.c[b0], dcc = S.dc[b0], cd = S.c[b1], dcd = S.dc[b1];
    const RT pr = cc * cd, dpr = (cc + dcc) * dcd + dcc * cd;
    const RT dq = ((kf + dkf) * dpf + dkf * pf) - ((kr + dkr) * dpr + dkr * pr);
    S.qs[j] = dq;
    S.qs[nrp + j] = -dq;
  }
  lds_sync();
  double ph[ROWS];
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = s * L + lane;
    const double dw = 1e6 * (double)production<RT>(t, S.qs, m.D, m.lp, r), wk = (double)w[s];
    df[s] = t.W[r] * (dw * invrho1 - wk * drho * B.invrho * invrho1);
    const double hk = t.hf[r] + t.cp[r] * (T - kTref), dhk = t.cp[r] * dT;
    ph[s] = t.W[r] * ((hk + dhk) * dw + dhk * wk);
  }
  const double dhsum = seg_sum<L, ROWS>(ph);
  const double D = rho * B.cpbar, dD = drho * cp1 + rho * dcp;
  const double dfT = -(dhsum / (D + dD) - B.hsum * dD / (D * (D + dD)));
#pragma unroll
  for (int s = 0; s < ROWS; ++s)
    if (s == sT && lane == lT) df[s] = dfT;
  lds_sync();
}

}  // namespace rok4e
