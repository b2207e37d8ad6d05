// Reaction substep in the conservative variables of a compressible flow solver with the
// auxiliary temperature equation (Sec. 5, e:chemical_source_balanced, e:aux_t_equation).
//
// State rows of a cell (n = ns + 6):
//   rho Y_1 .. rho Y_ns, T, rho, rho u_x, rho u_y, rho u_z, rho E.
// The chemistry changes only the rho Y_k (constant-volume reactor, c_k = rho Y_k / W_k);
// every conservative row also receives its balancing constant s.  The temperature source
// is
//   dT/dt = ( -sum_k e_k F_k + |v|^2/2 F_rho - v . F_m + F_E ) / (rho c_v),
// F the forced derivatives of the conservative rows, v = (rho u) / rho, with the species
// energy read as the internal energy e_k = h_f,k + c_p,k (T - T_ref) - Ru T / W_k and
// rho c_v = sum_k rho Y_k (c_p,k - Ru / W_k): under this reading the auxiliary
// temperature equals the temperature of the conservative variables along the exact
// solution, which the paper states of the method.
//
// FP64 only; the reciprocals of the cell-uniform quantities (T, rho, rho c_v and their
// perturbed values, all positive) use the refined hardware reciprocal.  The reaction
// loops are those of rhs / rhs_diff with the constant-volume concentrations; the tables,
// the LDS scratch layout and the base-concentration cache of the Arnoldi process are
// shared with them.
#pragma once

#include "rok4e_device.hpp"

namespace rok4e {

// Cell-uniform quantities of a base evaluation in conservative variables.
struct RhsBaseCons {
  double T, invT, invRT, rho, D, N, vx, vy, vz, Frho, Fmx, Fmy, Fmz;
};

// Value of state row r of the segment's cell, in every lane.
template <int L, int ROWS>
__device__ __forceinline__ double row_of(const double (&x)[ROWS], int r) {
  return seg_bcast<L>(row_value<L, ROWS>(x, r / L), r % L);
}

// f(u) of one cell in conservative variables with the auxiliary temperature, balancing
// constants s included.  With SAVE the base quantities go to *base and the forced species
// derivatives F_k to w for rhs_diff_cons (the rate constants and concentrations stay in
// LDS as for rhs).
template <int L, int ROWS, bool SAVE>
__device__ __forceinline__ void rhs_cons(const DevMech& m, const MechLds& t, const double (&u)[ROWS],
                                         const double (&s)[ROWS], double (&f)[ROWS],
                                         const RhsLds<double>& S, int lane, RhsBaseCons* base,
                                         double (&w)[ROWS]) {
  constexpr int LP = L * ROWS;
  const int ns = m.ns;
  const double T = row_of<L, ROWS>(u, ns);
  const double rho = row_of<L, ROWS>(u, ns + 1);
  const double mx = row_of<L, ROWS>(u, ns + 2), my = row_of<L, ROWS>(u, ns + 3),
               mz = row_of<L, ROWS>(u, ns + 4);
  const double Frho = row_of<L, ROWS>(s, ns + 1);
  const double Fmx = row_of<L, ROWS>(s, ns + 2), Fmy = row_of<L, ROWS>(s, ns + 3),
               Fmz = row_of<L, ROWS>(s, ns + 4);
  const double FE = row_of<L, ROWS>(s, ns + 5);
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const int r = i * L + lane;
    if (r < ns) {
      const int q = (ROWS == 1 ? t.rspos : t.spos[r]);
      S.spc[q] = 1e-6 * u[i] * (ROWS == 1 ? t.rinvW : t.invW[r]);
      acc_clear<LP, double>((char*)S.spc, q * sizeof(double));
    }
  }
  const double lnT = log(T);
  const double invT = rcp(T);
  const double invRT = invT * (1.0 / kRu);
  char* rb = (char*)S.spc;
  char* ab = acc_base<LP, double>(rb, lane);
  lds_sync();
  for (int j = lane; j < m.nr; j += L) {
    const double2 lnA = t.lnA[j], bEf = t.bEf[j], bEr = t.bEr[j];
    const double kf = arrhenius(lnA.x, bEf.x, bEf.y, lnT, invRT, 0.0);
    const double kr = arrhenius(lnA.y, bEr.x, bEr.y, lnT, invRT, 0.0);
    if constexpr (SAVE) S.k[j] = {kf, kr};
    const uint2 o = t.rxo[j];
    const double pf = *(const double*)(rb + (o.x & 0xFFFFu)) * *(const double*)(rb + (o.x >> 16));
    const double pr = *(const double*)(rb + (o.y & 0xFFFFu)) * *(const double*)(rb + (o.y >> 16));
    scatter_rate<LP, double>(ab, o, kf * pf - kr * pr);
  }
  lds_sync();
  double es[ROWS][2], sums[2];
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const int r = i * L + lane;
    es[i][0] = 0.0;
    es[i][1] = 0.0;
    f[i] = s[i];   // flow rows: their constants; rows past the state: zero
    if (r < ns) {
      const double Wr = ROWS == 1 ? t.rW : t.W[r], iW = ROWS == 1 ? t.rinvW : t.invW[r];
      const double cp = ROWS == 1 ? t.rcp : t.cp[r], hf = ROWS == 1 ? t.rhf : t.hf[r];
      const double F = Wr * (1e6 * acc_sum<LP, double>(rb, (ROWS == 1 ? t.rspos : t.spos[r]) * sizeof(double))) + s[i];
      f[i] = F;
      if constexpr (SAVE) w[i] = F;
      const double ek = hf + cp * (T - kTref) - kRu * T * iW;
      es[i][0] = ek * F;
      es[i][1] = u[i] * (cp - kRu * iW);
    }
  }
  seg_sum_rows_k<L, ROWS, 2>(es, sums);
  const double D = sums[1];
  const double irho = rcp(rho);
  const double vx = mx * irho, vy = my * irho, vz = mz * irho;
  const double ke = vx * vx + vy * vy + vz * vz;
  const double vF = vx * Fmx + vy * Fmy + vz * Fmz;
  const double N = -sums[0] + 0.5 * ke * Frho - vF + FE;
  const double fT = N * rcp(D);
#pragma unroll
  for (int i = 0; i < ROWS; ++i)
    if (i * L + lane == ns) f[i] = fT;
  if constexpr (SAVE) *base = RhsBaseCons{T, invT, invRT, rho, D, N, vx, vy, vz, Frho, Fmx, Fmy, Fmz};
  lds_sync();
}

// df = f(u + du) - f(u) in conservative variables, in difference form (as rhs_diff):
// the concentration increments are 1e-6 d(rho Y_k) / W_k, the rate-constant, product and
// rate increments as there, and the temperature row carries the increments of the
// species energies, of rho c_v and of the velocities.  The balancing constants cancel in
// every row except through F_k and the flow constants inside the temperature source.
template <int L, int ROWS, int NIT = 0>
__device__ __forceinline__ void rhs_diff_cons(const DevMech& m, const MechLds& t, const RhsBaseCons& B,
                                              const double (&w)[ROWS], const double (&u)[ROWS],
                                              const double (&du)[ROWS], double (&df)[ROWS],
                                              const RhsLds<double>& S, int lane,
                                              const ConcCache<NIT, double>* cc = nullptr) {
  constexpr int LP = L * ROWS;
  const int ns = m.ns;
  const double T = B.T;
  const double dT = row_of<L, ROWS>(du, ns);
  const double drho = row_of<L, ROWS>(du, ns + 1);
  const double dmx = row_of<L, ROWS>(du, ns + 2), dmy = row_of<L, ROWS>(du, ns + 3),
               dmz = row_of<L, ROWS>(du, ns + 4);
  const double T1 = T + dT;
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const int r = i * L + lane;
    if (r < ns) {
      const int q = (ROWS == 1 ? t.rspos : t.spos[r]);
      *inc_at<LP, double>((char*)S.spc, q * sizeof(double)) = 1e-6 * du[i] * (ROWS == 1 ? t.rinvW : t.invW[r]);
      acc_clear<LP, double>((char*)S.spc, q * sizeof(double));
    }
  }
  const double dlnT = log1p_small(dT * B.invT);
  const double dinvRT = -dT * (B.invRT * rcp(T1));
  char* rb = (char*)S.spc;
  char* ab = acc_base<LP, double>(rb, lane);
  lds_sync();
  auto diff_rx = [&](int j, const uint2 o, double ca, double cb, double cc_, double cd) {
    const double2 bEf = t.bEf[j], bEr = t.bEr[j];
    const double dlf = bEf.x * dlnT - bEf.y * dinvRT;
    const double dlr = bEr.x * dlnT - bEr.y * dinvRT;
    const double2 kj = S.k[j];
    const double dkf = kj.x * expm1_small(dlf);
    const double dkr = kj.y * expm1_small(dlr);
    const double dca = *(const double*)(rb + (o.x & 0xFFFFu) + LP * sizeof(double));
    const double dcb = *(const double*)(rb + (o.x >> 16) + LP * sizeof(double));
    const double dcc = *(const double*)(rb + (o.y & 0xFFFFu) + LP * sizeof(double));
    const double dcd = *(const double*)(rb + (o.y >> 16) + LP * sizeof(double));
    const double pf = ca * cb, dpf = (ca + dca) * dcb + dca * cb;
    const double pr = cc_ * cd, dpr = (cc_ + dcc) * dcd + dcc * cd;
    const double dq = ((kj.x + dkf) * dpf + dkf * pf) - ((kj.y + dkr) * dpr + dkr * pr);
    scatter_rate<LP, double>(ab, o, dq);
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
    for (int j = lane; j < m.nr; j += L) {
      const uint2 o = t.rxo[j];
      diff_rx(j, o, *(const double*)(rb + (o.x & 0xFFFFu)), *(const double*)(rb + (o.x >> 16)),
              *(const double*)(rb + (o.y & 0xFFFFu)), *(const double*)(rb + (o.y >> 16)));
    }
  }
  lds_sync();
  double es[ROWS][2], sums[2];
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const int r = i * L + lane;
    es[i][0] = 0.0;
    es[i][1] = 0.0;
    df[i] = 0.0;
    if (r < ns) {
      const double Wr = ROWS == 1 ? t.rW : t.W[r], iW = ROWS == 1 ? t.rinvW : t.invW[r];
      const double cp = ROWS == 1 ? t.rcp : t.cp[r], hf = ROWS == 1 ? t.rhf : t.hf[r];
      const double dF = Wr * (1e6 * acc_sum<LP, double>(rb, (ROWS == 1 ? t.rspos : t.spos[r]) * sizeof(double)));
      df[i] = dF;
      const double cv = cp - kRu * iW;
      const double ek = hf + cp * (T - kTref) - kRu * T * iW, dek = cv * dT;
      es[i][0] = (ek + dek) * dF + dek * w[i];
      es[i][1] = du[i] * cv;
    }
  }
  seg_sum_rows_k<L, ROWS, 2>(es, sums);
  const double dD = sums[1];
  // v = m / rho: dv = (dm - v drho) / (rho + drho); d(|v|^2 / 2) = dv . (v + dv / 2)
  const double irho1 = rcp(B.rho + drho);
  const double dvx = (dmx - B.vx * drho) * irho1, dvy = (dmy - B.vy * drho) * irho1,
               dvz = (dmz - B.vz * drho) * irho1;
  const double dke = dvx * (B.vx + 0.5 * dvx) + dvy * (B.vy + 0.5 * dvy) + dvz * (B.vz + 0.5 * dvz);
  const double dvF = dvx * B.Fmx + dvy * B.Fmy + dvz * B.Fmz;
  const double dN = -sums[0] + dke * B.Frho - dvF;
  const double iD1 = rcp(B.D + dD);
  const double dfT = (dN - B.N * dD * rcp(B.D)) * iD1;
#pragma unroll
  for (int i = 0; i < ROWS; ++i)
    if (i * L + lane == ns) df[i] = dfT;
  lds_sync();
}

// Loads a cell's conservative rows (U: [(ns+5) x n], rows rho Y_1..rho Y_ns, rho, rho u
// (3), rho E) and balancing constants into the auxiliary-temperature state and sets its
// temperature from U (rho e = rho E - |rho u|^2 / (2 rho) = sum_k rho Y_k e_k(T), linear
// in T).  Returns false for non-finite input, rho <= 0, rho c_v <= 0 or T <= 0.
template <int L, int ROWS>
__device__ __forceinline__ bool load_cell_cons(const DevMech& m, const MechLds& t, const Launch& P,
                                               int64_t cell, int lane, double (&u)[ROWS],
                                               double (&s)[ROWS]) {
  const int ns = m.ns;
  const int64_t n = P.n_cells;
  double x[ROWS][4], sums[4];
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const int r = i * L + lane;
    u[i] = 0.0;
    s[i] = 0.0;
    x[i][0] = x[i][1] = x[i][2] = x[i][3] = 0.0;
    const int src = r < ns ? r : (r > ns && r <= ns + 5 ? r - 1 : -1);
    if (src >= 0) {
      u[i] = P.Y[(int64_t)src * n + cell];
      if (P.S != nullptr) s[i] = P.S[(int64_t)src * n + cell];
      if (!finite_(u[i])) x[i][2] = 1.0;
    }
    if (r < ns) {
      const double iW = ROWS == 1 ? t.rinvW : t.invW[r];
      const double cp = ROWS == 1 ? t.rcp : t.cp[r], hf = ROWS == 1 ? t.rhf : t.hf[r];
      x[i][0] = u[i] * (hf - cp * kTref);
      x[i][1] = u[i] * (cp - kRu * iW);
    }
  }
  seg_sum_rows_k<L, ROWS, 4>(x, sums);
  const double rho = row_of<L, ROWS>(u, ns + 1);
  const double mx = row_of<L, ROWS>(u, ns + 2), my = row_of<L, ROWS>(u, ns + 3),
               mz = row_of<L, ROWS>(u, ns + 4), E = row_of<L, ROWS>(u, ns + 5);
  const double D = sums[1];
  const double T = (E - 0.5 * (mx * mx + my * my + mz * mz) / rho - sums[0]) / D;
  const bool ok = sums[2] == 0.0 && rho > 0.0 && D > 0.0 && finite_(T) && T > 0.0;
#pragma unroll
  for (int i = 0; i < ROWS; ++i)
    if (i * L + lane == ns) u[i] = T;
  return ok;
}

// Stores the conservative rows of the state to U and its temperature to P.T (if given).
template <int L, int ROWS>
__device__ __forceinline__ void store_cell_cons(const DevMech& m, const Launch& P, int64_t cell, int lane,
                                                const double (&u)[ROWS]) {
  const int ns = m.ns;
  const int64_t n = P.n_cells;
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const int r = i * L + lane;
    if (r < ns) P.Y[(int64_t)r * n + cell] = u[i];
    else if (r == ns && P.T != nullptr) P.T[cell] = u[i];
    else if (r > ns && r <= ns + 5) P.Y[(int64_t)(r - 1) * n + cell] = u[i];
  }
}

}  // namespace rok4e
