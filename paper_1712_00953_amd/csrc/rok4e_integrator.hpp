// Per-cell ROK4E integration on one segment of lanes (Algorithm a:ROK4E).
#pragma once

#include "rok4e_cons.hpp"
#include "rok4e_device.hpp"

namespace rok4e {

// Segment-local LDS views: right-hand-side scratch in the rate type RT, the projected
// M x M matrices in FP64.
template <class RT>
struct SegLds {
  RhsLds<RT> r;
  double* H;      // [MMAX * MMAX] Hessenberg matrix of the Arnoldi process
  double* LU;     // [MMAX * MMAX] factors of I - h gamma H
  double* rdiag;  // [MMAX] reciprocals of the diagonal of U
};

template <class RT>
__device__ __forceinline__ SegLds<RT> seg_lds(char* seg, const Launch& P) {
  SegLds<RT> S;
  S.r = RhsLds<RT>{(RT*)seg, (typename Pair2<RT>::type*)(seg + P.off_k)};
  S.H = (double*)(seg + P.off_H);
  S.LU = (double*)(seg + P.off_LU);
  S.rdiag = (double*)(seg + P.off_rdiag);
  return S;
}

// Constant entries of the segment's scratch: the absent reaction slot (concentration 1,
// FP64 increment 0).
template <class RT>
__device__ __forceinline__ void init_seg(const DevMech& m, const SegLds<RT>& S) {
  S.r.spc[m.ns] = (RT)1;
  ((double*)((char*)S.r.spc + m.lp * sizeof(RT)))[m.ns] = 0.0;
  lds_sync();
}

// State forms: the 0-D reactor (Y_k, T) at constant pressure, or the conservative
// variables of a compressible solver with the auxiliary temperature (ns + 6 rows).
constexpr int kFormReactor = 0, kFormConservative = 1;

template <int FORM> struct BaseOf { using type = RhsBase; };
template <> struct BaseOf<kFormConservative> { using type = RhsBaseCons; };

template <int FORM>
__device__ __forceinline__ int state_rows(const DevMech& m) {
  return FORM == kFormConservative ? m.ns + 6 : m.ns + 1;
}

// f(u) + s for the rows this lane holds (SAVE keeps the base quantities for rhs_diff).
template <int L, int ROWS, class RT, bool SAVE, int FORM = kFormReactor>
__device__ __forceinline__ void rhs_forced(const DevMech& m, const MechLds& t, const double (&u)[ROWS],
                                           double p, const double (&s)[ROWS], double (&f)[ROWS],
                                           const SegLds<RT>& S, int lane,
                                           typename BaseOf<FORM>::type* base, double (&w)[ROWS]) {
  if constexpr (FORM == kFormConservative) {
    static_assert(sizeof(RT) == 8, "the conservative form is FP64 only");
    rhs_cons<L, ROWS, SAVE>(m, t, u, s, f, S.r, lane, base, w);
  } else {
    rhs<L, ROWS, RT, SAVE>(m, t, u, p, f, S.r, lane, base, w);
#pragma unroll
    for (int i = 0; i < ROWS; ++i) f[i] = f[i] + s[i];
  }
}

// Arnoldi process with modified Gram-Schmidt and one classical re-orthogonalisation pass
// (Sec. 4.1, e:jac_proj) on finite-difference
// Jacobian-vector products (Sec. 4.3), J v = (f(u + delta v) - f(u)) / delta with the
// numerator in difference form.  Q holds this lane's rows of the orthonormal basis, H
// (LDS) the M x M Hessenberg matrix; both FP64.  Returns M_eff.  Needs the base
// evaluation of f at u (rhs with SAVE) just before.
template <int L, int ROWS, int MMAX, class RT, int FORM = kFormReactor, int GATHER = 0>
__device__ __forceinline__ int arnoldi(const DevMech& m, const MechLds& t, const Launch& P,
                                       const double (&u)[ROWS],
                                       const double (&fn)[ROWS], const typename BaseOf<FORM>::type& B,
                                       const double (&w)[ROWS], double (&Q)[ROWS][MMAX],
                                       const SegLds<RT>& S, int lane) {
  const int N = state_rows<FORM>(m);
  int Meff = P.M < N ? P.M : N;
#pragma unroll
  for (int i = 0; i < ROWS; ++i)
#pragma unroll
    for (int j = 0; j < MMAX; ++j) Q[i][j] = 0.0;
  // H is zero wherever the process does not reach (past M_eff, or all of it when
  // f_n = 0): the Hessenberg part is cleared first (every lane stores the same zeros).
#pragma unroll
  for (int j = 0; j < MMAX; ++j)
#pragma unroll
    for (int i = 0; i <= j + 1 && i < MMAX; ++i) S.H[i * MMAX + j] = 0.0;
  double sq[ROWS];
#pragma unroll
  for (int i = 0; i < ROWS; ++i) sq[i] = fn[i] * fn[i];
  const double beta2 = seg_sum<L, ROWS>(sq);
  if (beta2 == 0.0) return 0;
  double beta, rbeta;
  sqrt_rsqrt(beta2, beta, rbeta);
#pragma unroll
  for (int i = 0; i < ROWS; ++i) Q[i][0] = fn[i] * rbeta;
#pragma unroll
  for (int i = 0; i < ROWS; ++i) sq[i] = u[i] * u[i];
  const double delta = sqrt(P.eps_fd * (1.0 + sqrt(seg_sum<L, ROWS>(sq))));
  const double rdelta = 1.0 / delta;
  // base concentrations of this lane's reactions, left in LDS by the base evaluation
  constexpr int NIT = jvp_cache_iters<L, ROWS, MMAX, GATHER>();
  ConcCache<NIT, RT> cache;
  const bool cached = NIT > 0 && m.nr <= NIT * L;
  if constexpr (NIT > 0) {
    const char* rb = (const char*)S.r.spc;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int j = lane + it * L;
      const uint2 o = j < m.nr ? t.rxo[j] : make_uint2(0u, 0u);
      cache.c[it][0] = *(const RT*)(rb + (o.x & 0xFFFFu));
      cache.c[it][1] = *(const RT*)(rb + (o.x >> 16));
      cache.c[it][2] = *(const RT*)(rb + (o.y & 0xFFFFu));
      cache.c[it][3] = *(const RT*)(rb + (o.y >> 16));
    }
  }
#pragma unroll
  for (int j = 0; j < MMAX; ++j) {
    if (j >= Meff) break;
    double du[ROWS], d[ROWS], wv[ROWS];
#pragma unroll
    for (int i = 0; i < ROWS; ++i) du[i] = delta * Q[i][j];
    if constexpr (FORM == kFormConservative)
      rhs_diff_cons<L, ROWS, NIT>(m, t, B, w, u, du, d, S.r, lane, cached ? &cache : nullptr);
    else
      rhs_diff<L, ROWS, RT, NIT>(m, t, B, w, u, du, d, S.r, lane, cached ? &cache : nullptr);
#pragma unroll
    for (int i = 0; i < ROWS; ++i) wv[i] = d[i] * rdelta;
    double hj[MMAX];
#pragma unroll
    for (int i2 = 0; i2 < MMAX; ++i2) {
      hj[i2] = 0.0;
      if (i2 > j) continue;
      double pr[ROWS];
#pragma unroll
      for (int i = 0; i < ROWS; ++i) pr[i] = Q[i][i2] * wv[i];
      const double hij = seg_sum<L, ROWS>(pr);
      hj[i2] = hij;
#pragma unroll
      for (int i = 0; i < ROWS; ++i) wv[i] = wv[i] - hij * Q[i][i2];
    }
    // One classical re-orthogonalisation pass: all projections of the once-orthogonalised
    // w at once (one batched reduction; the columns not built yet are zero), removed and
    // added to H.  The Woodbury form of the stage solve (e:solve_kry_jac) holds for an
    // orthonormal basis, which plain modified Gram-Schmidt does not keep on stiff cells.
    double cpr[MMAX];
    constexpr int KG = MMAX % 8 == 0 ? 8 : 4;
#pragma unroll
    for (int g = 0; g < MMAX; g += KG) {
      double pr[ROWS][KG], cg[KG];
#pragma unroll
      for (int i = 0; i < ROWS; ++i)
#pragma unroll
        for (int k = 0; k < KG; ++k) pr[i][k] = Q[i][g + k] * wv[i];
      seg_sum_rows_k<L, ROWS, KG>(pr, cg);
#pragma unroll
      for (int k = 0; k < KG; ++k) cpr[g + k] = cg[k];
    }
    double hsq = 0.0;
#pragma unroll
    for (int i2 = 0; i2 < MMAX; ++i2) {
      if (i2 > j) continue;
      const double hfin = hj[i2] + cpr[i2];
      S.H[i2 * MMAX + j] = hfin;
      hsq = hsq + hfin * hfin;
#pragma unroll
      for (int i = 0; i < ROWS; ++i) wv[i] = wv[i] - cpr[i2] * Q[i][i2];
    }
    if (j + 1 < Meff) {
#pragma unroll
      for (int i = 0; i < ROWS; ++i) sq[i] = wv[i] * wv[i];
      const double hn2 = seg_sum<L, ROWS>(sq);
      // |J q_j| before the orthogonalization from the orthogonal decomposition
      // |w|^2 = sum_i h_ij^2 + h_{j+1,j}^2 (no separate reduction); the breakdown test
      // |w_new| <= 1e-12 |w| compares the squares
      if (!(hn2 > 1e-24 * (hsq + hn2))) {
        Meff = j + 1;
        break;
      }
      double hn, rhn;
      sqrt_rsqrt(hn2, hn, rhn);
      S.H[(j + 1) * MMAX + j] = hn;
#pragma unroll
      for (int i = 0; i < ROWS; ++i) Q[i][j + 1] = wv[i] * rhn;
    }
  }
  lds_sync();
  return Meff;
}

// LU with partial pivoting of the upper-Hessenberg A = I - hg H, hg = h gamma, over the
// full MMAX x MMAX: H is zero past M_eff (the Arnoldi process clears it), so A is the
// identity there and the padding neither pivots nor changes the leading block.  Only
// rows k and k+1 are pivot candidates in column k.  The row interchanges are recorded
// as bits of piv and the multipliers l_k kept at LU[(k+1) MMAX + k] without being moved
// by later interchanges, so a solve applies interchange k and elimination k in turn
// (the same operations on the same values as interchanging all rows first and
// substituting with the permuted unit-lower factor).  Every lane of the segment
// computes the same values in registers, two rows at a time: r is the pivot row k, s
// row k + 1 (one step per scheduling region, which keeps the register demand at two
// rows).  U goes to LU (upper part), the reciprocals of its diagonal to rdiag.  False
// when a pivot is zero.
template <int MMAX>
__device__ __forceinline__ bool lu_factor(const double* __restrict__ H, double hg, double* __restrict__ LU,
                                          double* __restrict__ rdiag, unsigned& piv) {
  double r[MMAX];
#pragma unroll
  for (int j = 0; j < MMAX; ++j) r[j] = (j == 0 ? 1.0 : 0.0) - hg * H[j];
  piv = 0u;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < MMAX; ++k) {
    __builtin_amdgcn_sched_barrier(0);
    double s[MMAX];
    if (k + 1 < MMAX) {
#pragma unroll
      for (int j = k; j < MMAX; ++j) s[j] = (j == k + 1 ? 1.0 : 0.0) - hg * H[(k + 1) * MMAX + j];
      const bool pv = fabs(s[k]) > fabs(r[k]);
      piv |= pv ? (1u << k) : 0u;
#pragma unroll
      for (int j = k; j < MMAX; ++j) {
        const double a = r[j], b = s[j];
        r[j] = pv ? b : a;
        s[j] = pv ? a : b;
      }
    }
    const double akk = r[k];
    ok = ok && akk != 0.0;
    const double rk = rcp(akk);
    rdiag[k] = rk;
#pragma unroll
    for (int j = k + 1; j < MMAX; ++j) LU[k * MMAX + j] = r[j];
    if (k + 1 < MMAX) {
      const double l = s[k] * rk;
      LU[(k + 1) * MMAX + k] = l;
#pragma unroll
      for (int j = k + 1; j < MMAX; ++j) r[j] = s[j] - l * r[j];
    }
  }
  return ok;
}

// x <- A^{-1} x for a segment-uniform vector x with the factors of lu_factor.  The rows
// of U are loaded one back-substitution step at a time (a scheduling barrier per row):
// hoisting all of them at once costs more registers than the kernel has at three waves
// per SIMD, and the spills cost more than the exposed load latency.
template <int MMAX>
__device__ __forceinline__ void lu_solve(const double* LU, const double* rdiag, unsigned piv,
                                         double (&x)[MMAX]) {
#pragma unroll
  for (int k = 0; k + 1 < MMAX; ++k) {
    const bool pv = ((piv >> k) & 1u) != 0u;
    const double a = x[k], b = x[k + 1];
    x[k] = pv ? b : a;
    x[k + 1] = (pv ? a : b) - LU[(k + 1) * MMAX + k] * x[k];
  }
#pragma unroll
  for (int i = MMAX - 1; i >= 0; --i) {
    __builtin_amdgcn_sched_barrier(0);
    double sacc = x[i];
#pragma unroll
    for (int j = i + 1; j < MMAX; ++j) sacc = sacc - LU[i * MMAX + j] * x[j];
    x[i] = sacc * rdiag[i];
  }
}

// k = F - Q (z - y) - corr with z = Q^T F and y = (I - h gamma H)^{-1} z
// (Algorithm a:ROK4E, stage update; Woodbury form e:solve_kry_jac).
template <int L, int ROWS, int MMAX>
__device__ __forceinline__ void stage_solve(const double (&F)[ROWS], const double (&corr)[ROWS],
                                            double (&k)[ROWS], const double (&Q)[ROWS][MMAX],
                                            const double* LU, const double* rdiag, unsigned piv) {
  // All MMAX projections are formed (columns past M_eff are zero) and reduced together,
  // in groups of up to eight.
  double z[MMAX], y[MMAX];
  constexpr int KG = MMAX % 8 == 0 ? 8 : 4;
  static_assert(MMAX % KG == 0, "MMAX must be a multiple of 4");
#pragma unroll
  for (int g = 0; g < MMAX; g += KG) {
    double pr[ROWS][KG], zg[KG];
#pragma unroll
    for (int i = 0; i < ROWS; ++i)
#pragma unroll
      for (int k = 0; k < KG; ++k) pr[i][k] = Q[i][g + k] * F[i];
    seg_sum_rows_k<L, ROWS, KG>(pr, zg);
#pragma unroll
    for (int k = 0; k < KG; ++k) {
      z[g + k] = zg[k];
      y[g + k] = zg[k];
    }
  }
  // past M_eff the columns of Q, z and y are zero, so the padded solve and sum add
  // exact zeros
  lu_solve<MMAX>(LU, rdiag, piv, y);
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    double qw = 0.0;
#pragma unroll
    for (int i2 = 0; i2 < MMAX; ++i2) qw = qw + Q[i][i2] * (z[i2] - y[i2]);
    k[i] = F[i] - qw - corr[i];
  }
}

// Integrator state of one cell between attempts (segment-uniform).  status: 0 running
// or done, 1 attempt limit, 2 step size underflow, 3 invalid input.
struct CellState {
  double t, h, lerr_prev;   // time, step, ln of the last accepted error (0: err_prev = 1)
  double hnext;             // step for a following call: the last proposal, or the larger
                            // of it and the proposal made before the last accepted step
                            // was shortened to end at dt
  int attempts, accepted, rejected, steps_done, status, Meff, basis_valid, pad;
};

// h0c > 0 (finite): the cell's own first trial step (the h_0 input of the algorithm).
__device__ __forceinline__ void cell_start(const Launch& P, CellState& c, double h0c = 0.0) {
  c.t = 0.0;
  c.h = P.fixed_steps > 0 ? P.dt / P.fixed_steps
                          : (h0c > 0.0 && __builtin_isfinite(h0c) ? h0c : (P.h0 > 0.0 ? P.h0 : P.dt));
  c.hnext = c.h;
  c.lerr_prev = 0.0;
  c.attempts = c.accepted = c.rejected = c.steps_done = c.status = c.Meff = c.basis_valid = c.pad = 0;
}

// True while the cell needs another attempt; reaching the attempt limit sets status 1.
// Called once before every attempt and once after the last.
__device__ __forceinline__ bool cell_running(const Launch& P, CellState& c) {
  if (c.status != 0) return false;
  const bool more = P.fixed_steps > 0 ? c.steps_done < P.fixed_steps : c.t < P.dt;
  if (!more) return false;
  const int max_att = P.max_attempts > 0 ? P.max_attempts : 1000000;
  if (c.attempts >= max_att) {
    c.status = 1;
    return false;
  }
  return true;
}

// One attempt of Algorithm a:ROK4E on the segment's cell, in place in u and c, with the
// readings: clipped last step, err_n = 1 before the first acceptance and updated on
// acceptance, basis (fn, Q, the LDS copy of H, M_eff) reused after a rejection,
// non-finite u* or err rejected.
template <int L, int ROWS, int MMAX, class RT, int FORM = kFormReactor, int GATHER = 0>
__device__ __forceinline__ void cell_attempt(const DevMech& m, const MechLds& tab, const Launch& P,
                                             double (&u)[ROWS], double p, const double (&s)[ROWS],
                                             const SegLds<RT>& S, int lane, CellState& c,
                                             double (&fn)[ROWS], double (&Q)[ROWS][MMAX]) {
  const int N = state_rows<FORM>(m);
  const double dt = P.dt;
  const double tiny = 16.0 * 2.220446049250313e-16 * dt;
  const bool fixed = P.fixed_steps > 0;
  double h = c.h;
  bool last = false;
  if (!fixed && h >= (dt - c.t) * (1.0 - 1e-12)) {
    h = dt - c.t;
    last = true;
  }
  const double hprop = c.h;
  if (!c.basis_valid) {
    double wbase[ROWS];
    typename BaseOf<FORM>::type base;
    rhs_forced<L, ROWS, RT, true, FORM>(m, tab, u, p, s, fn, S, lane, &base, wbase);
    c.Meff = arnoldi<L, ROWS, MMAX, RT, FORM, GATHER>(m, tab, P, u, fn, base, wbase, Q, S, lane);
    c.basis_valid = 1;
  }
  unsigned piv;
  if (!lu_factor<MMAX>(S.H, h * G, S.LU, S.rdiag, piv)) {
    ++c.attempts;
    ++c.rejected;
    c.h = h * 0.2;
    c.hnext = c.h;
    if (c.h < tiny) c.status = 2;
    return;
  }
  double k1[ROWS], k2[ROWS], k3[ROWS], k4[ROWS];
  double corr[ROWS], F[ROWS], arg[ROWS], fs[ROWS];
  double wtmp[ROWS];
  // Stage 1: F1 = f_n.
#pragma unroll
  for (int i = 0; i < ROWS; ++i) corr[i] = 0.0;
  stage_solve<L, ROWS, MMAX>(fn, corr, k1, Q, S.LU, S.rdiag, piv);
  // Stage 2: F2 = f(u + h a21 k1) + (g21/g) k1.
#pragma unroll
  for (int i = 0; i < ROWS; ++i) arg[i] = u[i] + h * (A21 * k1[i]);
  rhs_forced<L, ROWS, RT, false, FORM>(m, tab, arg, p, s, fs, S, lane, nullptr, wtmp);
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    corr[i] = (G21 / G) * k1[i];
    F[i] = fs[i] + corr[i];
  }
  stage_solve<L, ROWS, MMAX>(F, corr, k2, Q, S.LU, S.rdiag, piv);
  // Stage 3: F3 = f(u + h(a31 k1 + a32 k2)) + (g31 k1 + g32 k2)/g.
#pragma unroll
  for (int i = 0; i < ROWS; ++i) arg[i] = u[i] + h * (A31 * k1[i] + A32 * k2[i]);
  rhs_forced<L, ROWS, RT, false, FORM>(m, tab, arg, p, s, fs, S, lane, nullptr, wtmp);
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    corr[i] = (G31 * k1[i] + G32 * k2[i]) * (1.0 / G);
    F[i] = fs[i] + corr[i];
  }
  stage_solve<L, ROWS, MMAX>(F, corr, k3, Q, S.LU, S.rdiag, piv);
  // Stage 4 reuses f of stage 3 (a41 = a31, a42 = a32, a43 = 0).
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    corr[i] = (G41 * k1[i] + G42 * k2[i] + G43 * k3[i]) * (1.0 / G);
    F[i] = fs[i] + corr[i];
  }
  stage_solve<L, ROWS, MMAX>(F, corr, k4, Q, S.LU, S.rdiag, piv);

  double us[ROWS];
#pragma unroll
  for (int i = 0; i < ROWS; ++i) us[i] = u[i] + h * (B1 * k1[i] + B2 * k2[i] + B4 * k4[i]);
  ++c.attempts;
  if (fixed) {
#pragma unroll
    for (int i = 0; i < ROWS; ++i) u[i] = us[i];
    ++c.accepted;
    ++c.steps_done;
    c.basis_valid = 0;
    return;
  }
  // Embedded error e = h sum (bh_j - b_j) k_j, weighted RMS over the N rows.
  double en[ROWS][2], sums[2];
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const int r = (int)(i * L + lane);
    en[i][0] = 0.0;
    en[i][1] = 0.0;
    if (r < N) {
      const double e = h * (E1 * k1[i] + E2 * k2[i] + E3 * k3[i] + E4 * k4[i]);
      const double sc = P.atol + P.rtol * fabs(us[i]);
      const double ratio = e * rcp(sc);
      en[i][0] = ratio * ratio;
      en[i][1] = finite_(us[i]) ? 0.0 : 1.0;
    }
  }
  seg_sum_rows_k<L, ROWS, 2>(en, sums);
  double err = sqrt(sums[0] * (1.0 / N));
  const double nbad = sums[1];
  if (!finite_(err) || nbad != 0.0) err = __builtin_huge_val();
  // PI controller, alpha = 0.7/4, beta = 0.4/4:
  // 0.8 err_prev^0.1 / err^0.175 = 0.8 exp(0.1 ln err_prev - 0.175 ln err).
  const double lerr = log(fmax(err, 1e-10));
  const double fac = fmin(5.0, fmax(0.2, 0.8 * exp(0.1 * c.lerr_prev - 0.175 * lerr)));
  const double hstar = h * fac;
  if (err <= 1.0) {
#pragma unroll
    for (int i = 0; i < ROWS; ++i) u[i] = us[i];
    c.t = last ? dt : c.t + h;
    c.lerr_prev = lerr;
    ++c.accepted;
    c.basis_valid = 0;
    c.hnext = last ? fmax(hstar, hprop) : hstar;
  } else {
    ++c.rejected;
    c.hnext = hstar;
  }
  c.h = hstar;
  if (c.t < dt && c.h < tiny) c.status = 2;
}

// Integrates the segment's cell over [0, dt] in place in u (all attempts).
template <int L, int ROWS, int MMAX, class RT, int FORM = kFormReactor, int GATHER = 0>
__device__ __forceinline__ CellState integrate_cell(const DevMech& m, const MechLds& tab,
                                                    const Launch& P, double (&u)[ROWS], double p,
                                                    const double (&s)[ROWS], const SegLds<RT>& S,
                                                    int lane, double h0c = 0.0) {
  CellState c;
  cell_start(P, c, h0c);
  double fn[ROWS], Q[ROWS][MMAX];
  while (cell_running(P, c)) cell_attempt<L, ROWS, MMAX, RT, FORM, GATHER>(m, tab, P, u, p, s, S, lane, c, fn, Q);
  return c;
}

// Explicit Dormand-Prince 5(4) pair (the explicit reference integrator of the efficiency
// study, Sec. 5): published tableau, first-same-as-last, the ROK4E error norm, elementary
// controller h* = h min(5, max(0.2, 0.9 err^(-1/5))), h0 = dt, clipped last step.
namespace dp {
constexpr double a21 = 1.0 / 5;
constexpr double a31 = 3.0 / 40, a32 = 9.0 / 40;
constexpr double a41 = 44.0 / 45, a42 = -56.0 / 15, a43 = 32.0 / 9;
constexpr double a51 = 19372.0 / 6561, a52 = -25360.0 / 2187, a53 = 64448.0 / 6561, a54 = -212.0 / 729;
constexpr double a61 = 9017.0 / 3168, a62 = -355.0 / 33, a63 = 46732.0 / 5247, a64 = 49.0 / 176,
                 a65 = -5103.0 / 18656;
constexpr double b1 = 35.0 / 384, b3 = 500.0 / 1113, b4 = 125.0 / 192, b5 = -2187.0 / 6784, b6 = 11.0 / 84;
// b - b_hat (b2 = bh2 = b7 = 0)
constexpr double e1 = b1 - 5179.0 / 57600, e3 = b3 - 7571.0 / 16695, e4 = b4 - 393.0 / 640,
                 e5 = b5 - (-92097.0 / 339200), e6 = b6 - 187.0 / 2100, e7 = -1.0 / 40;
}  // namespace dp

template <int L, int ROWS, class RT>
__device__ __forceinline__ CellState rkdp_cell(const DevMech& m, const MechLds& tab, const Launch& P,
                                               double (&u)[ROWS], double p, const double (&s)[ROWS],
                                               const SegLds<RT>& S, int lane) {
  const int N = m.ns + 1;
  const double dt = P.dt;
  const double tiny = 16.0 * 2.220446049250313e-16 * dt;
  const bool fixed = P.fixed_steps > 0;
  CellState c;
  cell_start(P, c);
  double k1[ROWS], k2[ROWS], k3[ROWS], k4[ROWS], k5[ROWS], k6[ROWS], k7[ROWS], arg[ROWS];
  double wt[ROWS];
  rhs_forced<L, ROWS, RT, false>(m, tab, u, p, s, k1, S, lane, nullptr, wt);
  while (cell_running(P, c)) {
    double h = c.h;
    bool last = false;
    if (!fixed && h >= (dt - c.t) * (1.0 - 1e-12)) {
      h = dt - c.t;
      last = true;
    }
#pragma unroll
    for (int i = 0; i < ROWS; ++i) arg[i] = u[i] + h * (dp::a21 * k1[i]);
    rhs_forced<L, ROWS, RT, false>(m, tab, arg, p, s, k2, S, lane, nullptr, wt);
#pragma unroll
    for (int i = 0; i < ROWS; ++i) arg[i] = u[i] + h * (dp::a31 * k1[i] + dp::a32 * k2[i]);
    rhs_forced<L, ROWS, RT, false>(m, tab, arg, p, s, k3, S, lane, nullptr, wt);
#pragma unroll
    for (int i = 0; i < ROWS; ++i) arg[i] = u[i] + h * (dp::a41 * k1[i] + dp::a42 * k2[i] + dp::a43 * k3[i]);
    rhs_forced<L, ROWS, RT, false>(m, tab, arg, p, s, k4, S, lane, nullptr, wt);
#pragma unroll
    for (int i = 0; i < ROWS; ++i)
      arg[i] = u[i] + h * (dp::a51 * k1[i] + dp::a52 * k2[i] + dp::a53 * k3[i] + dp::a54 * k4[i]);
    rhs_forced<L, ROWS, RT, false>(m, tab, arg, p, s, k5, S, lane, nullptr, wt);
#pragma unroll
    for (int i = 0; i < ROWS; ++i)
      arg[i] = u[i] + h * (dp::a61 * k1[i] + dp::a62 * k2[i] + dp::a63 * k3[i] + dp::a64 * k4[i] +
                           dp::a65 * k5[i]);
    rhs_forced<L, ROWS, RT, false>(m, tab, arg, p, s, k6, S, lane, nullptr, wt);
#pragma unroll
    for (int i = 0; i < ROWS; ++i)
      arg[i] = u[i] + h * (dp::b1 * k1[i] + dp::b3 * k3[i] + dp::b4 * k4[i] + dp::b5 * k5[i] + dp::b6 * k6[i]);
    rhs_forced<L, ROWS, RT, false>(m, tab, arg, p, s, k7, S, lane, nullptr, wt);
    ++c.attempts;
    if (fixed) {
#pragma unroll
      for (int i = 0; i < ROWS; ++i) {
        u[i] = arg[i];
        k1[i] = k7[i];
      }
      ++c.accepted;
      ++c.steps_done;
      continue;
    }
    double en[ROWS][2], sums[2];
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const int r = (int)(i * L + lane);
      en[i][0] = 0.0;
      en[i][1] = 0.0;
      if (r < N) {
        const double e = h * (dp::e1 * k1[i] + dp::e3 * k3[i] + dp::e4 * k4[i] + dp::e5 * k5[i] +
                              dp::e6 * k6[i] + dp::e7 * k7[i]);
        const double ratio = e * rcp(P.atol + P.rtol * fabs(arg[i]));
        en[i][0] = ratio * ratio;
        en[i][1] = finite_(arg[i]) ? 0.0 : 1.0;
      }
    }
    seg_sum_rows_k<L, ROWS, 2>(en, sums);
    double err = sqrt(sums[0] * (1.0 / N));
    if (!finite_(err) || sums[1] != 0.0) err = __builtin_huge_val();
    const double fac = fmin(5.0, fmax(0.2, 0.9 * exp(-0.2 * log(fmax(err, 1e-10)))));
    if (err <= 1.0) {
#pragma unroll
      for (int i = 0; i < ROWS; ++i) {
        u[i] = arg[i];
        k1[i] = k7[i];
      }
      c.t = last ? dt : c.t + h;
      ++c.accepted;
    } else {
      ++c.rejected;
    }
    c.h = h * fac;
    if (c.t < dt && c.h < tiny) c.status = 2;
  }
  return c;
}

// Loads a cell's rows (Y, T, forcing) for this lane; returns false if the input is not a
// valid state (non-finite values, T <= 0, p <= 0).
template <int L, int ROWS>
__device__ __forceinline__ bool load_cell(const DevMech& m, const Launch& P, int64_t cell, int lane,
                                          double (&u)[ROWS], double (&s)[ROWS], double& p) {
  const int ns = m.ns, N = ns + 1;
  const int64_t n = P.n_cells;
  double bad[ROWS];
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const int r = i * L + lane;
    u[i] = 0.0;
    s[i] = 0.0;
    bad[i] = 0.0;
    if (r < ns) u[i] = P.Y[(int64_t)r * n + cell];
    else if (r == ns) u[i] = P.T[cell];
    if (P.S != nullptr && r < N) s[i] = P.S[(int64_t)r * n + cell];
    if (r < N && !finite_(u[i])) bad[i] = 1.0;
    if (r == ns && !(u[i] > 0.0)) bad[i] = 1.0;
  }
  p = P.p[cell];
  const double nbad = seg_sum<L, ROWS>(bad);
  return nbad == 0.0 && finite_(p) && p > 0.0;
}

template <int L, int ROWS>
__device__ __forceinline__ void store_cell(const DevMech& m, const Launch& P, int64_t cell, int lane,
                                           const double (&u)[ROWS]) {
  const int ns = m.ns;
  const int64_t n = P.n_cells;
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const int r = i * L + lane;
    if (r < ns) P.Y[(int64_t)r * n + cell] = u[i];
    else if (r == ns) P.T[cell] = u[i];
  }
}

}  // namespace rok4e
