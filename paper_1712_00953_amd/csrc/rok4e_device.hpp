// Device building blocks of the batched ROK4E reaction substep (gfx950, wave64).
//
// Layout: one cell per "segment" of L lanes (L = 16, 32 or 64).  State row r of a cell
// (species 0..ns-1, then T at row ns) lives in lane r % L, slot r / L of that segment
// (ROWS slots per lane).  Reactions are taken round-robin by the segment's lanes for
// the rate evaluation.  The segment's LDS scratch holds per species the concentration,
// its increment and a production accumulator: the reaction lanes read the
// concentrations and add their signed rates of progress into the accumulators with LDS
// float atomics, so the production sums need no per-species gather.  The small M x M
// projected matrices live in the segment's scratch too.
//
// Reductions over a segment follow one fixed tree (16-lane butterfly, then rows
// pairwise, then slots pairwise).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef ROK4E_RX_UNROLL
#define ROK4E_RX_UNROLL 1
#endif

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
// LDS once per block by the kernels.  The Arrhenius parameters are stored as pairs that
// one evaluation uses together, so each pair is one 16-byte LDS load and consecutive
// reactions are contiguous (no bank conflicts).  Image layout (NRP = reaction count
// rounded to even, LP = lanes x slots of the layout):
//   double2 lnA[NRP]     (ln A_f, ln A_r)
//   double2 bEf[NRP]     (b_f, E_f)
//   double2 bEr[NRP]     (b_r, E_r)
//   double  spec[4][LP]  W, 1/W, c_p, h_f per state row (zeros/ones past the species)
//   uint2   rxo[NRP]     byte offsets (LDS position x size of the rate type) of the species
//                        of reaction j in the per-cell species arrays: .x = reac0 | reac1
//                        << 16, .y = prod0 | prod1 << 16; an absent slot holds the offset
//                        of entry ns (concentration 1, increment 0)
//   int     spos[LP]     LDS position of the species of state row r (ns past the species)
// Reaction j of the tables is the mechanism's reaction order[j] and species k sits at LDS
// position pos[k] (host-side placement that spreads LDS bank traffic; it changes only the
// order of the production sums).
struct DevMech {
  int ns, nr, nrp, lp;
  int off_spec, off_rxo, off_spos, image_bytes;
  const int4* image;
};

// LDS view of the table image.
struct MechLds {
  const double2* lnA; const double2* bEf; const double2* bEr;
  const double* W; const double* invW; const double* cp; const double* hf;
  const uint2* rxo;
  const int* spos;
  // this lane's state row (lane % L) of W, 1/W, cp, hf and the species position, read
  // once at kernel start: the one-row layouts take them from registers (or private
  // memory) instead of LDS in every evaluation
  double rW, rinvW, rcp, rhf;
  int rspos;
};

// A pair of rate-type values (the forward and reverse rate constants of a reaction).
template <class RT> struct Pair2;
template <> struct Pair2<double> { using type = double2; };
template <> struct Pair2<float> { using type = float2; };

// Per-launch arguments of the integrator.
struct Launch {
  int64_t n_cells;
  double* Y; double* T; const double* p; const double* S;
  double dt, rtol, atol, h0, eps_fd;
  int M, max_attempts, fixed_steps;
  unsigned int* queue;
  int32_t* acc; int32_t* rej; int32_t* status;
  double* hio;   // [n] per-cell first trial step in, step for the next call out (or null)
  const int32_t* order;   // [n] cell handed out for each queue ticket (or null: array order)
  int seg_bytes, off_k, off_H, off_LU, off_rdiag;
};

// Copies the table image to the start of the block's LDS and returns the view.  All
// threads of the block take part; ends with a block barrier (kernel start only).
template <int L>
__device__ __forceinline__ MechLds load_mech_lds(const DevMech& m, char* lds) {
  int4* dst = (int4*)lds;
  for (int i = threadIdx.x; i < m.image_bytes / 16; i += blockDim.x) dst[i] = m.image[i];
  __syncthreads();
  MechLds t;
  t.lnA = (const double2*)lds;
  t.bEf = t.lnA + m.nrp;
  t.bEr = t.bEf + m.nrp;
  const double* sp = (const double*)(lds + m.off_spec);
  t.W = sp; t.invW = sp + m.lp; t.cp = sp + 2 * m.lp; t.hf = sp + 3 * m.lp;
  t.rxo = (const uint2*)(lds + m.off_rxo);
  t.spos = (const int*)(lds + m.off_spos);
  const int r0 = (int)(threadIdx.x % L);
  t.rW = t.W[r0]; t.rinvW = t.invW[r0]; t.rcp = t.cp[r0]; t.rhf = t.hf[r0]; t.rspos = t.spos[r0];
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
// DPP move restricted to the rows in ROWMASK; the other rows receive +0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_rows(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_rows(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWMASK, 0xF, false));
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

// x + (x of lane i ^ 16) and x + (x of lane i ^ 32) in every lane, from the gfx950
// row-swap permutes (v_permlane16_swap / v_permlane32_swap of x with itself leave the two
// partners' values in two registers; their sum has the same bits in both lanes).
__device__ __forceinline__ double add_xor16(double x) {
  const unsigned lo = (unsigned)__double2loint(x), hi = (unsigned)__double2hiint(x);
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}
__device__ __forceinline__ float add_xor16(float x) {
  const auto v = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(v[0]) + __uint_as_float(v[1]);
}
__device__ __forceinline__ double add_xor32(double x) {
  const unsigned lo = (unsigned)__double2loint(x), hi = (unsigned)__double2hiint(x);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}
__device__ __forceinline__ float add_xor32(float x) {
  const auto v = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(v[0]) + __uint_as_float(v[1]);
}

// Split exchange of two values a, b across lane ^ 32 (D = 32) or lane ^ 16 (D = 16): one
// row-swap permute per 32-bit word moves the b of the lower partner and the a of the upper
// one across, so that the sum is a + a' in the lanes whose bit log2(D) is clear and
// b + b' in the others: two reductions advance one level for the cost of one.
template <int D>
__device__ __forceinline__ double swap_split(double a, double b) {
  const unsigned alo = (unsigned)__double2loint(a), ahi = (unsigned)__double2hiint(a);
  const unsigned blo = (unsigned)__double2loint(b), bhi = (unsigned)__double2hiint(b);
  if constexpr (D == 32) {
    const auto l = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
  } else {
    const auto l = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
  }
}
template <int D>
__device__ __forceinline__ float swap_split(float a, float b) {
  if constexpr (D == 32) {
    const auto v = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(v[0]) + __uint_as_float(v[1]);
  } else {
    const auto v = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(v[0]) + __uint_as_float(v[1]);
  }
}

// The levels of a segment reduction, each pairing every lane with the lane whose index
// differs by an XOR mask: lane ^ 32 and lane ^ 16 (row-swap permutes), then within a
// 16-lane row lane ^ 15 (row mirror), lane ^ 7 (half-row mirror), lane ^ 2 and lane ^ 1
// (quad permutes).  The masks span the lane index bits, so after all levels from the
// segment's first one every lane holds the segment sum; every level is symmetric and
// additions commute bit for bit, so every lane holds the same bits.
//   level 0: ^32, 1: ^16, 2: ^15, 3: ^7, 4: ^2, 5: ^1
// When a level splits a pair of values, the lanes keep the value selected by the level's
// bit (32: bit 5, 16: bit 4, 15: bit 3, 7: bit 2, 2: bit 1, 1: bit 0).
constexpr int kLevelBit[6] = {5, 4, 3, 2, 1, 0};
template <int LEVEL>
constexpr int level_dpp() { return LEVEL == 2 ? 0x140 : LEVEL == 3 ? 0x141 : LEVEL == 4 ? 0x4E : 0xB1; }

template <int LEVEL, class V>
__device__ __forceinline__ V level_full(V x) {
  if constexpr (LEVEL == 0) return add_xor32(x);
  else if constexpr (LEVEL == 1) return add_xor16(x);
  else return x + dpp<level_dpp<LEVEL>()>(x);
}

template <int LEVEL, class V>
__device__ __forceinline__ V level_split(V a, V b, int lid) {
  if constexpr (LEVEL == 0) return swap_split<32>(a, b);
  else if constexpr (LEVEL == 1) return swap_split<16>(a, b);
  else {
    const bool hi = ((lid >> kLevelBit[LEVEL]) & 1) != 0;
    const V keep = hi ? b : a, send = hi ? a : b;
    return keep + dpp<level_dpp<LEVEL>()>(send);
  }
}

// Levels LEVEL..5 applied to NV values (NV a power of two): the first log2(NV) levels
// split pairs, the rest sum fully.  On return each lane holds one partial: the sum of value
// i, i = sum over the splitting levels j of (lane bit of level j) << j, over the segment.
template <int LEVEL, int NV, class V>
__device__ __forceinline__ V seg_levels(const V (&v)[NV], int lid) {
  if constexpr (LEVEL == 6) {
    static_assert(NV == 1, "more values than split levels");
    return v[0];
  } else if constexpr (NV == 1) {
    V w[1] = {level_full<LEVEL>(v[0])};
    return seg_levels<LEVEL + 1, 1>(w, lid);
  } else {
    V w[NV / 2];
#pragma unroll
    for (int m = 0; m < NV / 2; ++m) w[m] = level_split<LEVEL>(v[2 * m], v[2 * m + 1], lid);
    return seg_levels<LEVEL + 1, NV / 2>(w, lid);
  }
}

template <int L>
constexpr int first_level() { return L == 64 ? 0 : (L == 32 ? 1 : 2); }

// Lane (within the segment) that holds the sum of value i after seg_levels from the
// segment's first level.
template <int L>
__device__ __forceinline__ constexpr int sum_lane(int i) {
  int lane = 0;
  for (int j = 0; (1 << j) <= i; ++j)
    if ((i >> j) & 1) lane |= 1 << kLevelBit[first_level<L>() + j];
  return lane;
}

// Sum over the L lanes of a segment; every lane receives the result (the same bits in
// every lane of the segment).
template <int L, class V>
__device__ __forceinline__ V seg_sum1(V x) {
  V v[1] = {x};
  return seg_levels<first_level<L>(), 1>(v, 0);
}

// Sum over all rows of a segment: the slots added in each lane, then one lane reduction.
template <int L, int ROWS, class V>
__device__ __forceinline__ V seg_sum(const V (&x)[ROWS]) {
  if constexpr (ROWS == 1) {
    return seg_sum1<L>(x[0]);
  } else if constexpr (ROWS == 2) {
    return seg_sum1<L>(x[0] + x[1]);
  } else {
    static_assert(ROWS == 4, "ROWS must be 1, 2 or 4");
    return seg_sum1<L>((x[0] + x[1]) + (x[2] + x[3]));
  }
}

// Sums over the L lanes of a segment of K values at once (K = 2, 4 or 8); every lane
// receives all K sums in x.  The first log2(K) levels split the values between partner
// lanes (a level costs one exchange and one add for two sums), the remaining levels sum
// the one partial left; sum i is then read from the lane that holds it.
template <int L, int K, class V>
__device__ __forceinline__ void seg_sum_k(V (&x)[K]) {
  static_assert(K == 2 || K == 4 || K == 8, "K must be 2, 4 or 8");
  const int lid = (int)(threadIdx.x & 63);
  const V z = seg_levels<first_level<L>(), K>(x, lid);
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const int q = sum_lane<L>(i);
    if constexpr (L == 64) {
      x[i] = readlane(z, q);
    } else if constexpr (L == 32) {
      const V a = readlane(z, q), c = readlane(z, 32 + q);
      x[i] = (lid & 32) ? c : a;
    } else {
      x[i] = __shfl(z, (lid & ~15) + q, 64);
    }
  }
}

// seg_sum_k over the ROWS slots of each of K values (slots added first).
template <int L, int ROWS, int K, class V>
__device__ __forceinline__ void seg_sum_rows_k(const V (&x)[ROWS][K], V (&out)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    V a = x[0][k];
#pragma unroll
    for (int s = 1; s < ROWS; ++s) a = a + x[s][k];
    out[k] = a;
  }
  seg_sum_k<L, K>(out);
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

// sqrt(x) and 1/sqrt(x) for positive x: the hardware reciprocal square root refined by two
// Newton steps, the root from it with one correction step (each within about one ulp; for
// the Arnoldi norms, in place of a square root and a division); the library routines for x
// outside [2^-1000, 2^1000].
__device__ __forceinline__ void sqrt_rsqrt(double x, double& root, double& rroot) {
  if (!(x >= 0x1p-1000 && x <= 0x1p1000)) {   // far from the normal range: library routines
    root = sqrt(x);
    rroot = 1.0 / root;
    return;
  }
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  const double r = x * y;
  root = fma(0.5 * y, fma(-r, r, x), r);
  rroot = y;
}

// 1/x for normal x of either sign: the hardware reciprocal refined by two Newton steps
// (within about one ulp; used for cell-uniform quantities such as rho and T, and the
// pivots of the projected factorisation).
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// -------------------------------------------------------- right-hand side ----

// Per-segment LDS scratch of the right-hand side.  spc holds the concentrations of the
// base state (LP entries in the rate type), then their FP64 increments for the difference
// evaluation (LP entries), then the FP64 production accumulators: species k sits at
// spc[k], inc[k] and acc(k) (consecutive species fall in different LDS banks).  In the
// mixed form the accumulators come in two copies, LP + 8 entries apart (half the banks
// over): the reaction lanes of even index add into the first, those of odd index into the
// second, and a species' production is the sum of its two entries.  Two lanes of one
// accumulate instruction that add into the same address are serialised by the LDS at a
// cost well above that of a bank conflict, and with the copies neighbouring lanes never
// do.  The FP64 layout keeps one copy: the second does not fit beside three blocks per CU.
// Entry ns is the absent reaction slot: concentration 1, increment 0, accumulators never
// read.
template <class RT>
struct RhsLds {
  RT* spc;                        // [LP] rate type, then double [LP] increments, then
                                  // double [LP] accumulators (x2 + 8 mixed)
  typename Pair2<RT>::type* k;    // [NRP] (k_f, k_r) of the base state
};

// Accumulator copies of the layout (2 in the mixed form, 1 in FP64) and the byte
// distance between them.
template <class RT>
constexpr int acc_copies() { return sizeof(RT) == 4 ? 2 : 1; }
template <int LP>
constexpr unsigned acc_copy_bytes() { return (LP + 8) * sizeof(double); }

// FP64 increment of the species at byte offset off (species x sizeof(RT)) of the
// concentration array that starts at rb.
template <int LP, class RT>
__device__ __forceinline__ double* inc_at(char* rb, unsigned off) {
  return (double*)(rb + LP * sizeof(RT) + off * (sizeof(double) / sizeof(RT)));
}
template <int LP, class RT>
__device__ __forceinline__ double inc_read(const char* rb, unsigned off) {
  return *(const double*)(rb + LP * sizeof(RT) + off * (sizeof(double) / sizeof(RT)));
}

// Accumulator (first copy) of the species at byte offset off (species x sizeof(RT)) of the
// concentration array that starts at rb.
template <int LP, class RT>
__device__ __forceinline__ double* acc_at(char* rb, unsigned off) {
  return (double*)(rb + LP * sizeof(RT) + LP * sizeof(double) + off * (sizeof(double) / sizeof(RT)));
}

// Clears the accumulator copies of a species.
template <int LP, class RT>
__device__ __forceinline__ void acc_clear(char* rb, unsigned off) {
  double* a = acc_at<LP, RT>(rb, off);
  a[0] = 0.0;
  if constexpr (acc_copies<RT>() == 2) a[acc_copy_bytes<LP>() / sizeof(double)] = 0.0;
}

// Production sum of a species: first copy (+ second copy).
template <int LP, class RT>
__device__ __forceinline__ double acc_sum(char* rb, unsigned off) {
  const double* a = acc_at<LP, RT>(rb, off);
  if constexpr (acc_copies<RT>() == 2) return a[0] + a[acc_copy_bytes<LP>() / sizeof(double)];
  return a[0];
}

// Base address for this lane's accumulates (its copy); concentrations are read from rb.
template <int LP, class RT>
__device__ __forceinline__ char* acc_base(char* rb, int lane) {
  if constexpr (acc_copies<RT>() == 2) return rb + ((lane & 1) ? acc_copy_bytes<LP>() : 0u);
  return rb;
}

// Cell-uniform quantities of a base evaluation f(u), kept for the difference evaluation.
struct RhsBase {
  double T, invT, invRT, sigma, cpbar, rho, invrho, invD, hsum;
};

// expm1 for the small arguments of the difference evaluation: Taylor series to x^3
// (relative truncation error about x^3/24, below 5e-17 for |x| < 1e-5), the library
// routine otherwise.  The arguments are increments of ln k for a state perturbation of
// relative size ~1e-8, so the series is the path taken.
__device__ __forceinline__ double expm1_small(double x) {
  double s = x * (1.0 + x * (0.5 + x * (1.0 / 6.0)));
  if (!(fabs(x) < 1e-5)) s = expm1(x);
  return s;
}

// log1p for the small arguments of the difference evaluation: alternating series to x^4
// (relative truncation error about x^4/5, below 3e-21 for |x| < 1e-5), the library
// routine otherwise.
__device__ __forceinline__ double log1p_small(double x) {
  if (fabs(x) < 1e-5) return x * (1.0 - x * (0.5 - x * (1.0 / 3.0 - x * 0.25)));
  return log1p(x);
}

template <int L, int ROWS>
__device__ __forceinline__ double row_value(const double (&u)[ROWS], int slot) {
  double v = 0.0;
#pragma unroll
  for (int s = 0; s < ROWS; ++s)
    if (s == slot) v = u[s];
  return v;
}

// LDS float atomic add (ds_add_f64 / ds_add_f32); the value is not returned.
template <class RT>
__device__ __forceinline__ void lds_add(RT* p, RT v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Adds -q to the accumulators of the reactants and +q to those of the products of one
// reaction (rb: the lane's accumulator base, acc_base): a repeated species receives the
// term twice, a species on both sides -q and +q.  An absent slot adds into the
// accumulator of entry ns, which is never read.
template <int LP, class RT, class V>
__device__ __forceinline__ void scatter_rate(char* rb, uint2 o, V qr) {
  const double q = (double)qr;
  lds_add(acc_at<LP, RT>(rb, o.x & 0xFFFFu), -q);
  lds_add(acc_at<LP, RT>(rb, o.x >> 16), -q);
  lds_add(acc_at<LP, RT>(rb, o.y & 0xFFFFu), q);
  lds_add(acc_at<LP, RT>(rb, o.y >> 16), q);
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
                                    RhsBase* base, double (&w)[ROWS]) {
  constexpr int LP = L * ROWS;
  const int ns = m.ns;
  const int sT = ns / L, lT = ns % L;
  const double T = seg_bcast<L>(row_value<L, ROWS>(u, sT), lT);

  double sc2[ROWS][2], sums[2];
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = s * L + lane;          // rows past the species have invW = cp = 0
    sc2[s][0] = (r < ns ? u[s] : 0.0) * (ROWS == 1 ? t.rinvW : t.invW[r]);
    sc2[s][1] = (r < ns ? u[s] : 0.0) * (ROWS == 1 ? t.rcp : t.cp[r]);
  }
  seg_sum_rows_k<L, ROWS, 2>(sc2, sums);
  const double sigma = sums[0], cpbar = sums[1];
  const double rho = p * rcp(kRu * T * sigma);
  const double invrho = rcp(rho);
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = s * L + lane;
    if (r < ns) {
      const int q = (ROWS == 1 ? t.rspos : t.spos[r]);
      S.spc[q] = (RT)(1e-6 * rho * u[s] * (ROWS == 1 ? t.rinvW : t.invW[r]));
      acc_clear<LP, RT>((char*)S.spc, q * sizeof(RT));
    }
  }
  const double lnT = log(T);
  const double invT = rcp(T);
  const double invRT = invT * (1.0 / kRu);
  char* rb = (char*)S.spc;
  char* ab = acc_base<LP, RT>(rb, lane);
  lds_sync();
  // species offsets one iteration ahead where the registers allow (as in rhs_diff)
  constexpr bool kPrefetch = !(L == 64 && ROWS == 1);
  uint2 on = t.rxo[lane < m.nr ? lane : 0];
#pragma unroll ROK4E_RX_UNROLL
  for (int j = lane; j < m.nr; j += L) {
    const double2 lnA = t.lnA[j], bEf = t.bEf[j], bEr = t.bEr[j];
    const RT kf = arrhenius(lnA.x, bEf.x, bEf.y, lnT, invRT, RT(0));
    const RT kr = arrhenius(lnA.y, bEr.x, bEr.y, lnT, invRT, RT(0));
    if constexpr (SAVE) S.k[j] = {kf, kr};
    uint2 o;
    if constexpr (kPrefetch) {
      o = on;
      on = t.rxo[min(j + L, m.nr - 1)];
    } else {
      o = t.rxo[j];
    }
    const RT pf = *(const RT*)(rb + (o.x & 0xFFFFu)) * *(const RT*)(rb + (o.x >> 16));
    const RT pr = *(const RT*)(rb + (o.y & 0xFFFFu)) * *(const RT*)(rb + (o.y >> 16));
    scatter_rate<LP, RT>(ab, o, kf * pf - kr * pr);
  }
  lds_sync();
  double ph[ROWS];
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = s * L + lane;
    // the production rates, the species derivatives and the heat release are formed in
    // FP64 from the FP64 sums in both forms: rounding them to FP32 would break the exact
    // balance of the production rates (mass and elements), which the FP32 rates of
    // progress keep
    const double wk = r < ns ? 1e6 * acc_sum<LP, RT>((char*)S.spc, (ROWS == 1 ? t.rspos : t.spos[r]) * sizeof(RT)) : 0.0;
    w[s] = wk;
    f[s] = (ROWS == 1 ? t.rW : t.W[r]) * wk * invrho;
    const double hk = (ROWS == 1 ? t.rhf : t.hf[r]) + (ROWS == 1 ? t.rcp : t.cp[r]) * (T - kTref);
    ph[s] = hk * (ROWS == 1 ? t.rW : t.W[r]) * wk;
  }
  const double hsum = seg_sum<L, ROWS>(ph);
  const double invD = rcp(rho * cpbar);
  const double fT = -hsum * invD;
#pragma unroll
  for (int s = 0; s < ROWS; ++s)
    if (s == sT && lane == lT) f[s] = fT;
  if constexpr (SAVE) *base = RhsBase{T, invT, invRT, sigma, cpbar, rho, invrho, invD, hsum};
  lds_sync();   // the LDS scratch is reused by the next evaluation
}

// df = f(u + du) - f(u) in difference form, given the base evaluation at u (base, w, and
// the concentrations and rate constants it left in LDS): every intermediate quantity is carried with
// its increment, formed from increments only, so the result has the relative accuracy of
// the compute type instead of the absolute accuracy eps |f| of a difference of two
// evaluations.  The increments of the scalar state functions (rho, ln T, 1/(Ru T)) are
// FP64.
// Base-state concentrations of the reactions one lane evaluates (NIT iterations of L
// reactions, four species slots each), gathered once per basis so that each of the M
// Jacobian-vector products reads only the increments from LDS.  At three waves per SIMD
// the compiler keeps this array in the lane's private (scratch) memory, so the reads go
// through the vector-memory path, which has spare bandwidth, instead of the LDS, which
// bounds the products.
template <int NIT, class RT>
struct ConcCache {
  RT c[NIT > 0 ? NIT : 1][4];
};

// Iterations cached for a layout (0: the products read the base concentrations from LDS):
// with GATHER, six for the one-row, M <= 8 layout (up to 384 reactions at 64 lanes).
// Whether the gather pays depends on the register pressure of the rest of the kernel, so
// both forms are compiled and the launch tuner chooses.
template <int L, int ROWS, int MMAX, int GATHER>
constexpr int jvp_cache_iters() { return (GATHER && L == 64 && ROWS == 1 && MMAX == 8) ? 6 : 0; }
template <int L, int ROWS, int MMAX>
constexpr bool has_gather() { return jvp_cache_iters<L, ROWS, MMAX, 1>() > 0; }

template <int L, int ROWS, class RT, int NIT = 0>
__device__ __forceinline__ void rhs_diff(const DevMech& m, const MechLds& t, const RhsBase& B,
                                         const double (&w)[ROWS], const double (&u)[ROWS],
                                         const double (&du)[ROWS], double (&df)[ROWS],
                                         const RhsLds<RT>& S, int lane,
                                         const ConcCache<NIT, RT>* cc = nullptr) {
  constexpr int LP = L * ROWS;
  const int ns = m.ns;
  const int sT = ns / L, lT = ns % L;
  const double T = B.T;
  const double dT = seg_bcast<L>(row_value<L, ROWS>(du, sT), lT);
  const double T1 = T + dT;
  double sc2[ROWS][2], sums[2];
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = s * L + lane;
    sc2[s][0] = (r < ns ? du[s] : 0.0) * (ROWS == 1 ? t.rinvW : t.invW[r]);
    sc2[s][1] = (r < ns ? du[s] : 0.0) * (ROWS == 1 ? t.rcp : t.cp[r]);
  }
  seg_sum_rows_k<L, ROWS, 2>(sc2, sums);
  const double dsigma = sums[0], dcp = sums[1];
  const double sigma1 = B.sigma + dsigma, cp1 = B.cpbar + dcp;
  const double rho = B.rho;
  const double invT1 = rcp(T1);
  const double drho = -rho * (dT * sigma1 + T * dsigma) * (invT1 * rcp(sigma1));
  const double rho1 = rho + drho;
  const double invrho1 = rcp(rho1);
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = s * L + lane;
    if (r < ns) {
      const int q = (ROWS == 1 ? t.rspos : t.spos[r]);
      *inc_at<LP, RT>((char*)S.spc, q * sizeof(RT)) = 1e-6 * (rho1 * du[s] + drho * u[s]) * (ROWS == 1 ? t.rinvW : t.invW[r]);
      acc_clear<LP, RT>((char*)S.spc, q * sizeof(RT));
    }
  }
  const double dlnT = log1p_small(dT * B.invT);
  const double dinvRT = -dT * (B.invRT * invT1);
  char* rb = (char*)S.spc;
  char* ab = acc_base<LP, RT>(rb, lane);
  lds_sync();
  // one reaction: rate-constant increments, concentration products with increments,
  // d q, scattered.  The increments and everything formed from them are FP64 in both
  // forms (the perturbation and difference of the finite-difference product); the
  // mixed form's base rate constants and concentrations are its FP32 values, exact in
  // FP64.
  auto diff_rx = [&](int j, const uint2 o, RT ca_, RT cb_, RT cc_, RT cd_) {
    const double2 bEf = t.bEf[j], bEr = t.bEr[j];
    const double dlf = bEf.x * dlnT - bEf.y * dinvRT;
    const double dlr = bEr.x * dlnT - bEr.y * dinvRT;
    const auto kj = S.k[j];
    const double kf = (double)kj.x, kr = (double)kj.y;
    const double dkf = kf * expm1_small(dlf);
    const double dkr = kr * expm1_small(dlr);
    const double ca = (double)ca_, cb = (double)cb_, cc = (double)cc_, cd = (double)cd_;
    const double dca = inc_read<LP, RT>(rb, o.x & 0xFFFFu);
    const double dcb = inc_read<LP, RT>(rb, o.x >> 16);
    const double dcc = inc_read<LP, RT>(rb, o.y & 0xFFFFu);
    const double dcd = inc_read<LP, RT>(rb, o.y >> 16);
    // products of concentrations with increments: d(ab) = (a + da) db + da b
    const double pf = ca * cb, dpf = (ca + dca) * dcb + dca * cb;
    const double pr = cc * cd, dpr = (cc + dcc) * dcd + dcc * cd;
    const double dq = ((kf + dkf) * dpf + dkf * pf) - ((kr + dkr) * dpr + dkr * pr);
    scatter_rate<LP, RT>(ab, o, dq);
  };
  if constexpr (NIT > 0) {
    if (cc) {
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int j = lane + it * L;
        if (j < m.nr) diff_rx(j, t.rxo[j], cc->c[it][0], cc->c[it][1], cc->c[it][2], cc->c[it][3]);
      }
    }
  }
  if (NIT == 0 || !cc) {
    // the next reaction's species offsets are loaded one iteration ahead in the layouts
    // with room for the two registers (measured 1-2 % faster there; the one-slot 64-lane
    // layouts spill them)
    constexpr bool kPrefetch = !(L == 64 && ROWS == 1);
    uint2 on = t.rxo[lane < m.nr ? lane : 0];
#pragma unroll ROK4E_RX_UNROLL
    for (int j = lane; j < m.nr; j += L) {
      uint2 o;
      if constexpr (kPrefetch) {
        o = on;
        on = t.rxo[min(j + L, m.nr - 1)];
      } else {
        o = t.rxo[j];
      }
      diff_rx(j, o, *(const RT*)(rb + (o.x & 0xFFFFu)), *(const RT*)(rb + (o.x >> 16)),
              *(const RT*)(rb + (o.y & 0xFFFFu)), *(const RT*)(rb + (o.y >> 16)));
    }
  }
  lds_sync();
  double ph[ROWS];
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = s * L + lane;
    const double dw = r < ns ? 1e6 * acc_sum<LP, RT>((char*)S.spc, (ROWS == 1 ? t.rspos : t.spos[r]) * sizeof(RT)) : 0.0;
    const double wk = w[s];
    df[s] = (ROWS == 1 ? t.rW : t.W[r]) * (dw * invrho1 - wk * drho * B.invrho * invrho1);
    const double hk = (ROWS == 1 ? t.rhf : t.hf[r]) + (ROWS == 1 ? t.rcp : t.cp[r]) * (T - kTref), dhk = (ROWS == 1 ? t.rcp : t.cp[r]) * dT;
    ph[s] = (ROWS == 1 ? t.rW : t.W[r]) * ((hk + dhk) * dw + dhk * wk);
  }
  const double dhsum = seg_sum<L, ROWS>(ph);
  const double D = rho * B.cpbar, dD = drho * cp1 + rho * dcp;
  // f_T = -hsum / D: the increment is -(dhsum - hsum dD / D) / (D + dD)
  const double dfT = -(dhsum - B.hsum * dD * B.invD) * rcp(D + dD);
#pragma unroll
  for (int s = 0; s < ROWS; ++s)
    if (s == sT && lane == lT) df[s] = dfT;
  lds_sync();
}

}  // namespace rok4e
