// FP64 CPU oracle for the batched ROK4E reaction substep.
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, scalar reference that the
// HIP path is checked against.  Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark may load it.  It shares no code, header, table or
// helper with the HIP library; both sides get their inputs from the seeded generator.
//
// What is computed (paper: Wu, Ma & Ihme, "Efficient time stepping for reactive
// turbulent simulations with stiff chemistry"):
//   * the right-hand side of the adiabatic 0-D reactor, Sec. 4.4 eq. e:cv_reactor,
//     read as a constant-pressure reactor (c_p with h_k) with mass-action rates;
//   * the matrix-free finite-difference Jacobian-vector product, Sec. 4.3;
//   * the Arnoldi process giving Q_n and the Hessenberg H_n = Q_n^T J_n Q_n,
//     Sec. 4.1 eq. e:jac_proj (modified Gram-Schmidt with one classical
//     re-orthogonalisation pass);
//   * the four stages in the transformed form, Sec. 4.3 eq. e:s_stage_row_transformed,
//     with (I - h gamma A_n)^{-1} applied through the twice-used Woodbury identity,
//     eq. e:solve_kry_jac;
//   * the embedded error estimate and the PI step-size controller, Sec. 4.3;
//   * the integration loop of Algorithm a:ROK4E.
// Where the paper is silent or garbled the readings are:
//   - coefficient table t:coeff_rok4e: the b row reads (b1, b2, b3, b4) =
//     (0.1943.., 0.4831.., 0, 0.3224..) and the b-hat row (.., .., 0.1865.., 0);
//   - the ROW form e:s_stage_row carries h in front of A_n sum gamma_ij k_j;
//   - error norm: weighted RMS over all N components with scale atol + rtol |u*_i|;
//   - err_n = 1 before the first accepted step; err_n is updated on accept only;
//   - the last step is clipped to the interval end;
//   - FD increment delta = sqrt(eps (1 + ||u_n||_2)) for unit-norm Arnoldi vectors, with
//     eps = 2^-52; the difference f(u + du) - f(u) (du = delta v) is evaluated in
//     difference form: every quantity of f is carried with its exact-arithmetic increment
//     (d rho, d c_k, d k_f = k_f expm1(d x), d q_j, ...), which is algebraically the same
//     number as the literal difference without its subtractive cancellation (the literal
//     form, JVP mode 3, leaves rounding noise ~eps |f| / delta in every product);
//   - Arnoldi: M_eff = min(M, N); stop early when the new vector's norm falls below
//     1e-12 of the norm before orthogonalisation; ||f_n|| = 0 gives M_eff = 0;
//   - after a rejected step the basis of the same u_n is reused (identical result);
//   - non-finite u* or err counts as a rejection with err = +inf;
//   - h_0 = dt unless given (per cell in orc_integrate_h, which also returns the step to
//     start the next call from: the controller's last proposal, or the larger of it and
//     the proposal made before the last step was shortened to end at dt).
// Also here, for the efficiency study of Sec. 5: the explicit Dormand-Prince 5(4) pair
// (published tableau, first-same-as-last, the same error norm, elementary controller).
// And the reaction substep in the conservative variables of a compressible solver with
// the auxiliary temperature equation (Sec. 5, e:chemical_source_balanced and
// e:aux_t_equation; ConsProblem), reading the species energy there as the internal
// energy e_k = h_k - Ru T / W_k.
//
// Built with -O2 -fno-fast-math -ffp-contract=off so each operation rounds once.

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <limits>
#include <type_traits>
#include <vector>
#include <omp.h>
#include <quadmath.h>

namespace {

using cplx = std::complex<double>;
using quad = __float128;

// exp and log for the three scalar types of the right-hand side.
inline double exp_(double x) { return std::exp(x); }
inline cplx exp_(const cplx& x) { return std::exp(x); }
inline quad exp_(quad x) { return expq(x); }
inline double log_(double x) { return std::log(x); }
inline cplx log_(const cplx& x) { return std::log(x); }
inline quad log_(quad x) { return logq(x); }

constexpr double kRu = 8.314462618;      // J/(mol K)
constexpr double kTref = 298.15;         // K

// ROK4E coefficients, table t:coeff_rok4e (row labels read as stated above).
constexpr double G = 0.572816062482135;
constexpr double G21 = -0.602765307997356;
constexpr double G31 = -1.389195789724843, G32 = 1.072950969011413;
constexpr double G41 = 0.992356412977094, G42 = -1.390032613873701, G43 = -0.440875890223325;
constexpr double A21 = 0.432364435748567;
constexpr double A31 = -0.514211316876170, A32 = 1.382271144617360;
constexpr double A41 = -0.514211316876170, A42 = 1.382271144617360, A43 = 0.0;
constexpr double B1 = 0.194335256262729, B2 = 0.483167813989227, B3 = 0.0, B4 = 0.322496929748044;
constexpr double BH1 = -0.217819895945721, BH2 = 1.03130847478467, BH3 = 0.186511421161047, BH4 = 0.0;

}  // namespace

extern "C" {

typedef struct {
  int32_t n_species, n_reactions;
  const double *W, *cp, *hf;              // [ns]: kg/mol, J/(kg K), J/kg
  const int32_t *reac, *prod;             // [nr*2], -1 where absent
  const double *lnAf, *bf, *Ef, *lnAr, *br, *Er;   // [nr]; A in cm-mol-s, E in J/mol
} orc_mech;

typedef struct {
  int32_t M;             // Krylov dimension
  int32_t jvp;           // 0 finite difference (difference form), 1 complex step,
                         // 2 exact (linear problems), 3 finite difference (literal form)
  int32_t fixed_steps;   // 0 adaptive, n > 0: n equal steps without error control
  int32_t max_attempts;  // attempts allowed per cell (<= 0: 1000000)
  double eps_fd;         // unit roundoff used in the FD increment (<= 0: 2^-52)
  double h0;             // first trial step (<= 0: dt)
} orc_opts;

}  // extern "C"

namespace {

// ---------------------------------------------------------------- problems ----

// One 0-D reactor cell: u = (Y_1..Y_ns, T), constant pressure p, optional constant
// forcing s (length ns+1) added to f.
struct CellProblem {
  static constexpr bool kComplex = true;
  static constexpr bool kDiff = true;
  const orc_mech* m;
  double p;
  const double* s;   // may be null
  int n() const { return m->n_species + 1; }

  template <class S>
  void f(const S* u, S* out) const {
    const int ns = m->n_species, nr = m->n_reactions;
    const S T = u[ns];
    S sigma = 0.0, cpbar = 0.0;
    for (int k = 0; k < ns; ++k) sigma += u[k] / S(m->W[k]);
    for (int k = 0; k < ns; ++k) cpbar += u[k] * S(m->cp[k]);
    const S rho = S(p) / (S(kRu) * T * sigma);                 // kg/m^3
    std::vector<S> c(ns), wdot(ns, S(0.0));
    for (int k = 0; k < ns; ++k) c[k] = S(1e-6) * rho * u[k] / S(m->W[k]);   // mol/cm^3
    const S lnT = log_(T);
    const S invRT = S(1.0) / (S(kRu) * T);
    for (int j = 0; j < nr; ++j) {
      const S kf = exp_(S(m->lnAf[j]) + S(m->bf[j]) * lnT - S(m->Ef[j]) * invRT);
      const S kr = exp_(S(m->lnAr[j]) + S(m->br[j]) * lnT - S(m->Er[j]) * invRT);
      S pf = 1.0, pr = 1.0;
      for (int a = 0; a < 2; ++a) {
        if (m->reac[2 * j + a] >= 0) pf = pf * c[m->reac[2 * j + a]];
        if (m->prod[2 * j + a] >= 0) pr = pr * c[m->prod[2 * j + a]];
      }
      const S q = kf * pf - kr * pr;                            // mol/(cm^3 s)
      // omega_k += nu_kj q_j with the net coefficient nu_kj (products - reactants),
      // added once per distinct species of reaction j, reactions in index order.
      int sp[4], nu[4], nsp = 0;
      for (int a = 0; a < 2; ++a) {
        const int r = m->reac[2 * j + a];
        if (r < 0) continue;
        int i = 0;
        while (i < nsp && sp[i] != r) ++i;
        if (i == nsp) { sp[nsp] = r; nu[nsp] = 0; ++nsp; }
        nu[i] -= 1;
      }
      for (int a = 0; a < 2; ++a) {
        const int r = m->prod[2 * j + a];
        if (r < 0) continue;
        int i = 0;
        while (i < nsp && sp[i] != r) ++i;
        if (i == nsp) { sp[nsp] = r; nu[nsp] = 0; ++nsp; }
        nu[i] += 1;
      }
      for (int i = 0; i < nsp; ++i) wdot[sp[i]] += S(static_cast<double>(nu[i])) * q;
    }
    S hsum = 0.0;
    for (int k = 0; k < ns; ++k) {
      const S w = S(1e6) * wdot[k];                             // mol/(m^3 s)
      out[k] = S(m->W[k]) * w / rho;
      const S hk = S(m->hf[k]) + S(m->cp[k]) * (T - S(kTref));
      hsum += hk * S(m->W[k]) * w;
    }
    out[ns] = -hsum / (rho * cpbar);
    if (s)
      for (int k = 0; k <= ns; ++k) out[k] += S(s[k]);
  }

  // Net stoichiometric coefficients of reaction j (species, coefficient), in the order
  // reactants then products, each species once.
  int stoich(int j, int* sp, int* nu) const {
    int nsp = 0;
    for (int side = 0; side < 2; ++side)
      for (int a = 0; a < 2; ++a) {
        const int r = side == 0 ? m->reac[2 * j + a] : m->prod[2 * j + a];
        if (r < 0) continue;
        int i = 0;
        while (i < nsp && sp[i] != r) ++i;
        if (i == nsp) { sp[nsp] = r; nu[nsp] = 0; ++nsp; }
        nu[i] += side == 0 ? -1 : 1;
      }
    return nsp;
  }

  // out = f(u + du) - f(u), evaluated in difference form: each intermediate quantity x
  // of f is carried with its increment dx = x(u + du) - x(u), formed from increments
  // only (no difference of two nearly equal values).  The forcing cancels.
  void fdiff(const double* u, const double* du, double* out) const {
    const int ns = m->n_species, nr = m->n_reactions;
    const double T = u[ns], dT = du[ns], T1 = T + dT;
    double sigma = 0.0, dsigma = 0.0, cpbar = 0.0, dcp = 0.0;
    for (int k = 0; k < ns; ++k) {
      sigma += u[k] / m->W[k];
      dsigma += du[k] / m->W[k];
      cpbar += u[k] * m->cp[k];
      dcp += du[k] * m->cp[k];
    }
    const double sigma1 = sigma + dsigma, cp1 = cpbar + dcp;
    const double rho = p / (kRu * T * sigma);
    // rho(u + du) - rho(u) = -rho (dT sigma1 + T dsigma) / (T1 sigma1)
    const double drho = -rho * (dT * sigma1 + T * dsigma) / (T1 * sigma1);
    const double rho1 = rho + drho;
    std::vector<double> c(ns), dc(ns), wdot(ns, 0.0), dwdot(ns, 0.0);
    for (int k = 0; k < ns; ++k) {
      c[k] = 1e-6 * rho * u[k] / m->W[k];
      dc[k] = 1e-6 * (rho1 * du[k] + drho * u[k]) / m->W[k];
    }
    const double lnT = std::log(T), dlnT = std::log1p(dT / T);
    const double invRT = 1.0 / (kRu * T), dinvRT = -dT / (kRu * T * T1);
    for (int j = 0; j < nr; ++j) {
      const double kf = std::exp(m->lnAf[j] + m->bf[j] * lnT - m->Ef[j] * invRT);
      const double kr = std::exp(m->lnAr[j] + m->br[j] * lnT - m->Er[j] * invRT);
      const double dkf = kf * std::expm1(m->bf[j] * dlnT - m->Ef[j] * dinvRT);
      const double dkr = kr * std::expm1(m->br[j] * dlnT - m->Er[j] * dinvRT);
      // product of concentrations and its increment: d(ab) = a1 db + da b
      double pf = 1.0, dpf = 0.0, pr = 1.0, dpr = 0.0;
      for (int a = 0; a < 2; ++a) {
        const int r = m->reac[2 * j + a];
        if (r >= 0) { dpf = (pf + dpf) * dc[r] + dpf * c[r]; pf = pf * c[r]; }
        const int q = m->prod[2 * j + a];
        if (q >= 0) { dpr = (pr + dpr) * dc[q] + dpr * c[q]; pr = pr * c[q]; }
      }
      const double q = kf * pf - kr * pr;
      const double dq = ((kf + dkf) * dpf + dkf * pf) - ((kr + dkr) * dpr + dkr * pr);
      int sp[4], nu[4];
      const int nsp = stoich(j, sp, nu);
      for (int i = 0; i < nsp; ++i) {
        wdot[sp[i]] += static_cast<double>(nu[i]) * q;
        dwdot[sp[i]] += static_cast<double>(nu[i]) * dq;
      }
    }
    double hsum = 0.0, dhsum = 0.0;
    for (int k = 0; k < ns; ++k) {
      const double w = 1e6 * wdot[k], dw = 1e6 * dwdot[k];
      // W (w1/rho1 - w/rho) = W (dw/rho1 - w drho/(rho rho1))
      out[k] = m->W[k] * (dw / rho1 - w * drho / (rho * rho1));
      const double hk = m->hf[k] + m->cp[k] * (T - kTref), dhk = m->cp[k] * dT;
      hsum += hk * m->W[k] * w;
      dhsum += m->W[k] * ((hk + dhk) * dw + dhk * w);
    }
    // f_T = -hsum / D with D = rho cp_mix
    const double D = rho * cpbar, dD = drho * cp1 + rho * dcp;
    out[ns] = -(dhsum / (D + dD) - hsum * dD / (D * (D + dD)));
  }
};

// Net production rates wdot_k = sum_j nu_kj q_j (mol/(cm^3 s)) of the mass-action
// mechanism at concentrations c (mol/cm^3) and temperature T, reactions in index order.
template <class S>
void net_rates(const orc_mech* m, const S* c, S T, S* wdot) {
  const int ns = m->n_species, nr = m->n_reactions;
  for (int k = 0; k < ns; ++k) wdot[k] = S(0.0);
  const S lnT = log_(T);
  const S invRT = S(1.0) / (S(kRu) * T);
  for (int j = 0; j < nr; ++j) {
    const S kf = exp_(S(m->lnAf[j]) + S(m->bf[j]) * lnT - S(m->Ef[j]) * invRT);
    const S kr = exp_(S(m->lnAr[j]) + S(m->br[j]) * lnT - S(m->Er[j]) * invRT);
    S pf = 1.0, pr = 1.0;
    for (int a = 0; a < 2; ++a) {
      if (m->reac[2 * j + a] >= 0) pf = pf * c[m->reac[2 * j + a]];
      if (m->prod[2 * j + a] >= 0) pr = pr * c[m->prod[2 * j + a]];
    }
    const S q = kf * pf - kr * pr;
    for (int a = 0; a < 2; ++a) {
      if (m->reac[2 * j + a] >= 0) wdot[m->reac[2 * j + a]] -= q;
      if (m->prod[2 * j + a] >= 0) wdot[m->prod[2 * j + a]] += q;
    }
  }
}

// One cell in the conservative variables of a compressible flow solver, with the
// auxiliary temperature of Sec. 5 (e:chemical_source_balanced, e:aux_t_equation):
//   u = (rho Y_1 .. rho Y_ns, T, rho, rho u_x, rho u_y, rho u_z, rho E),  n = ns + 6.
// The chemistry changes only the rho Y_k (constant-volume reactor: c_k = rho Y_k / W_k);
// every conservative row also receives its balancing constant s (the transport term of
// the previous step; s may be null, its T entry is not used).  The temperature source is
//   dT/dt = ( -sum_k e_k F_k + |v|^2/2 F_rho - v . F_m + F_E ) / (rho c_v),
// F the forced derivatives of the conservative rows, v = (rho u) / rho.
// Reading: the species energy of e:aux_t_equation is the mass-specific internal energy
// e_k = h_k - Ru T / W_k (h_k = h_f,k + c_p,k (T - T_ref)), and rho c_v = sum_k rho Y_k
// (c_p,k - Ru / W_k).  With it the auxiliary temperature equals the temperature of the
// conservative variables along the exact solution, the property Sec. 5 states; with
// the enthalpy it would not.
struct ConsProblem {
  static constexpr bool kComplex = true;
  static constexpr bool kDiff = true;
  const orc_mech* m;
  const double* s;   // may be null
  int n() const { return m->n_species + 6; }

  double srow(int i) const { return s ? s[i] : 0.0; }

  template <class S>
  void f(const S* u, S* out) const {
    const int ns = m->n_species;
    const S T = u[ns], rho = u[ns + 1];
    std::vector<S> c(ns), wdot(ns);
    for (int k = 0; k < ns; ++k) c[k] = S(1e-6) * u[k] / S(m->W[k]);   // mol/cm^3
    net_rates<S>(m, c.data(), T, wdot.data());
    S esum = 0.0, D = 0.0;
    for (int k = 0; k < ns; ++k) {
      out[k] = S(m->W[k]) * (S(1e6) * wdot[k]) + S(srow(k));           // kg/(m^3 s)
      const S ek = S(m->hf[k]) + S(m->cp[k]) * (T - S(kTref)) - S(kRu) * T / S(m->W[k]);
      esum += ek * out[k];
      D += u[k] * (S(m->cp[k]) - S(kRu) / S(m->W[k]));
    }
    for (int i = 1; i <= 5; ++i) out[ns + i] = S(srow(ns + i));
    S ke = 0.0, vF = 0.0;
    for (int d = 0; d < 3; ++d) {
      const S v = u[ns + 2 + d] / rho;
      ke += v * v;
      vF += v * out[ns + 2 + d];
    }
    out[ns] = (-esum + S(0.5) * ke * out[ns + 1] - vF + out[ns + 5]) / D;
  }

  // out = f(u + du) - f(u) in difference form (every quantity carried with its
  // increment, as CellProblem::fdiff); the balancing constants cancel except inside the
  // temperature row, which uses the forced derivatives.
  void fdiff(const double* u, const double* du, double* out) const {
    const int ns = m->n_species, nr = m->n_reactions;
    const double T = u[ns], dT = du[ns], T1 = T + dT;
    const double rho = u[ns + 1], drho = du[ns + 1];
    std::vector<double> c(ns), dc(ns), wdot(ns, 0.0), dwdot(ns, 0.0);
    for (int k = 0; k < ns; ++k) {
      c[k] = 1e-6 * u[k] / m->W[k];
      dc[k] = 1e-6 * du[k] / m->W[k];
    }
    const double lnT = std::log(T), dlnT = std::log1p(dT / T);
    const double invRT = 1.0 / (kRu * T), dinvRT = -dT / (kRu * T * T1);
    for (int j = 0; j < nr; ++j) {
      const double kf = std::exp(m->lnAf[j] + m->bf[j] * lnT - m->Ef[j] * invRT);
      const double kr = std::exp(m->lnAr[j] + m->br[j] * lnT - m->Er[j] * invRT);
      const double dkf = kf * std::expm1(m->bf[j] * dlnT - m->Ef[j] * dinvRT);
      const double dkr = kr * std::expm1(m->br[j] * dlnT - m->Er[j] * dinvRT);
      double pf = 1.0, dpf = 0.0, pr = 1.0, dpr = 0.0;
      for (int a = 0; a < 2; ++a) {
        const int r = m->reac[2 * j + a];
        if (r >= 0) { dpf = (pf + dpf) * dc[r] + dpf * c[r]; pf = pf * c[r]; }
        const int q = m->prod[2 * j + a];
        if (q >= 0) { dpr = (pr + dpr) * dc[q] + dpr * c[q]; pr = pr * c[q]; }
      }
      const double q = kf * pf - kr * pr;
      const double dq = ((kf + dkf) * dpf + dkf * pf) - ((kr + dkr) * dpr + dkr * pr);
      for (int a = 0; a < 2; ++a) {
        const int r = m->reac[2 * j + a];
        if (r >= 0) { wdot[r] -= q; dwdot[r] -= dq; }
        const int p = m->prod[2 * j + a];
        if (p >= 0) { wdot[p] += q; dwdot[p] += dq; }
      }
    }
    double esum = 0.0, desum = 0.0, D = 0.0, dD = 0.0;
    for (int k = 0; k < ns; ++k) {
      const double F = m->W[k] * (1e6 * wdot[k]) + srow(k);
      const double dF = m->W[k] * (1e6 * dwdot[k]);
      out[k] = dF;
      const double cv = m->cp[k] - kRu / m->W[k];
      const double ek = m->hf[k] + m->cp[k] * (T - kTref) - kRu * T / m->W[k], dek = cv * dT;
      esum += ek * F;
      desum += (ek + dek) * dF + dek * F;
      D += u[k] * cv;
      dD += du[k] * cv;
    }
    for (int i = 1; i <= 5; ++i) out[ns + i] = 0.0;
    // v = m / rho: dv = (dm rho - m drho) / (rho (rho + drho)); d(|v|^2/2) = dv . (v + dv/2)
    double ke = 0.0, vF = 0.0, dke = 0.0, dvF = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double mv = u[ns + 2 + d], dmv = du[ns + 2 + d];
      const double v = mv / rho, dv = (dmv * rho - mv * drho) / (rho * (rho + drho));
      const double Fm = srow(ns + 2 + d);
      ke += v * v;
      vF += v * Fm;
      dke += dv * (v + 0.5 * dv);
      dvF += dv * Fm;
    }
    const double Frho = srow(ns + 1), FE = srow(ns + 5);
    const double N = -esum + 0.5 * ke * Frho - vF + FE;
    const double dN = -desum + dke * Frho - dvF;
    // f_T = N / D: the increment is dN / (D + dD) - N dD / (D (D + dD))
    out[ns] = dN / (D + dD) - N * dD / (D * (D + dD));
  }
};

// Temperature of the conservative variables U = (rho Y_1..rho Y_ns, rho, rho u (3),
// rho E) of one cell: rho e = rho E - |rho u|^2 / (2 rho) = sum_k rho Y_k e_k(T), which
// is linear in T for constant c_p,k.  Returns NaN where rho c_v <= 0.
double cons_temperature(const orc_mech* m, const double* U) {
  const int ns = m->n_species;
  const double rho = U[ns];
  double e0 = 0.0, D = 0.0, m2 = 0.0;
  for (int k = 0; k < ns; ++k) {
    e0 += U[k] * (m->hf[k] - m->cp[k] * kTref);
    D += U[k] * (m->cp[k] - kRu / m->W[k]);
  }
  for (int d = 0; d < 3; ++d) m2 += U[ns + 1 + d] * U[ns + 1 + d];
  if (!(D > 0.0)) return std::numeric_limits<double>::quiet_NaN();
  return (U[ns + 4] - 0.5 * m2 / rho - e0) / D;
}

// Linear test problem f(u) = A u + c (A row-major n x n).
struct LinearProblem {
  static constexpr bool kComplex = true;
  static constexpr bool kDiff = true;
  int nn;
  const double* A;
  const double* c;
  int n() const { return nn; }
  template <class S>
  void f(const S* u, S* out) const {
    for (int i = 0; i < nn; ++i) {
      S acc = c ? S(c[i]) : S(0.0);
      for (int j = 0; j < nn; ++j) acc += A[i * nn + j] * u[j];
      out[i] = acc;
    }
  }
  // A du is exactly f(u + du) - f(u) for an affine f.
  void fdiff(const double*, const double* du, double* out) const { exact_jvp(du, out); }
  void exact_jvp(const double* v, double* out) const {
    for (int i = 0; i < nn; ++i) {
      double acc = 0.0;
      for (int j = 0; j < nn; ++j) acc += A[i * nn + j] * v[j];
      out[i] = acc;
    }
  }
};

}  // namespace

extern "C" {
// Right-hand side supplied by the caller: out = f(u), u and out of length n.
typedef void (*orc_rhs_fn)(int n, const double* u, double* out, void* ctx);
}

namespace {

// A caller-supplied f (finite-difference Jacobian-vector products only).
struct CallbackProblem {
  static constexpr bool kComplex = false;
  static constexpr bool kDiff = false;
  int nn;
  orc_rhs_fn fn;
  void* ctx;
  int n() const { return nn; }
  template <class S>
  void f(const S* u, S* out) const {
    if constexpr (std::is_same<S, double>::value) fn(nn, u, out, ctx);
  }
};

double norm2(const std::vector<double>& x) {
  double s = 0.0;
  for (double v : x) s += v * v;
  return std::sqrt(s);
}

double dot(const double* a, const double* b, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

// Jacobian-vector product J(u) v in the selected mode.  fu = f(u).
template <class P>
bool jvp(const P& prob, int mode, double eps_fd, const std::vector<double>& u,
         const std::vector<double>& fu, const double* v, double* out) {
  const int n = prob.n();
  if (mode == 0 || mode == 3) {
    // Finite difference, Sec. 4.3: (f(u + delta v) - f(u)) / delta.
    const double delta = std::sqrt(eps_fd * (1.0 + norm2(u)));
    std::vector<double> du(n), d(n);
    for (int i = 0; i < n; ++i) du[i] = delta * v[i];
    if constexpr (P::kDiff) {
      if (mode == 0) {
        prob.fdiff(u.data(), du.data(), d.data());
        for (int i = 0; i < n; ++i) out[i] = d[i] / delta;
        return true;
      }
    }
    // literal form: difference of two separately rounded evaluations
    std::vector<double> up(n), fp(n);
    for (int i = 0; i < n; ++i) up[i] = u[i] + du[i];
    prob.template f<double>(up.data(), fp.data());
    for (int i = 0; i < n; ++i) out[i] = (fp[i] - fu[i]) / delta;
    return true;
  }
  if (mode == 1 && P::kComplex) {
    // Complex step: Im f(u + i eps v) / eps, exact to roundoff for analytic f.
    const double eps = 1e-30;
    std::vector<cplx> uc(n), fc(n);
    for (int i = 0; i < n; ++i) uc[i] = cplx(u[i], eps * v[i]);
    prob.template f<cplx>(uc.data(), fc.data());
    for (int i = 0; i < n; ++i) out[i] = fc[i].imag() / eps;
    return true;
  }
  if constexpr (std::is_same<P, LinearProblem>::value) {
    if (mode == 2) {
      prob.exact_jvp(v, out);
      return true;
    }
  }
  return false;
}

// Arnoldi with modified Gram-Schmidt and one classical re-orthogonalisation pass,
// Sec. 4.1 (Q: n x M column-major, H: M x M
// row-major).  Returns M_eff.
template <class P>
int arnoldi(const P& prob, int mode, double eps_fd, int M, const std::vector<double>& u,
            const std::vector<double>& fu, std::vector<double>& Q, std::vector<double>& H) {
  const int n = prob.n();
  std::fill(Q.begin(), Q.end(), 0.0);
  std::fill(H.begin(), H.end(), 0.0);
  int Meff = M < n ? M : n;
  const double beta = norm2(fu);
  if (beta == 0.0) return 0;
  for (int i = 0; i < n; ++i) Q[i] = fu[i] / beta;
  std::vector<double> w(n);
  for (int j = 0; j < Meff; ++j) {
    if (!jvp(prob, mode, eps_fd, u, fu, &Q[j * n], w.data())) return -1;
    const double wnorm0 = norm2(w);
    for (int i = 0; i <= j; ++i) {
      const double hij = dot(&Q[i * n], w.data(), n);
      H[i * M + j] = hij;
      for (int r = 0; r < n; ++r) w[r] -= hij * Q[i * n + r];
    }
    // One classical re-orthogonalisation pass: all projections of the once-orthogonalised
    // w are taken at once and removed, and added to H.  The Woodbury form of the stage
    // solve (e:solve_kry_jac) holds for an orthonormal basis; without this pass the basis
    // of a stiff cell loses orthogonality to ~1e-2 at M = 8.
    {
      std::vector<double> cpr(j + 1);
      for (int i = 0; i <= j; ++i) cpr[i] = dot(&Q[i * n], w.data(), n);
      for (int i = 0; i <= j; ++i) {
        H[i * M + j] += cpr[i];
        for (int r = 0; r < n; ++r) w[r] -= cpr[i] * Q[i * n + r];
      }
    }
    if (j + 1 < Meff) {
      const double hn = norm2(w);
      if (!(hn > 1e-12 * wnorm0)) return j + 1;     // breakdown: invariant subspace
      H[(j + 1) * M + j] = hn;
      for (int r = 0; r < n; ++r) Q[(j + 1) * n + r] = w[r] / hn;
    }
  }
  return Meff;
}

// Dense LU with partial pivoting of an m x m row-major matrix (in place).
bool lu_factor(std::vector<double>& a, int m, std::vector<int>& piv) {
  piv.resize(m);
  for (int k = 0; k < m; ++k) {
    int p = k;
    for (int i = k + 1; i < m; ++i)
      if (std::fabs(a[i * m + k]) > std::fabs(a[p * m + k])) p = i;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < m; ++j) std::swap(a[k * m + j], a[p * m + j]);
    if (a[k * m + k] == 0.0) return false;
    for (int i = k + 1; i < m; ++i) {
      const double l = a[i * m + k] / a[k * m + k];
      a[i * m + k] = l;
      for (int j = k + 1; j < m; ++j) a[i * m + j] -= l * a[k * m + j];
    }
  }
  return true;
}

// Solves (P A) x = P b with the factors of lu_factor: whole rows were swapped there, so
// all row interchanges are applied to b first, then unit-lower and upper substitution.
void lu_solve(const std::vector<double>& a, int m, const std::vector<int>& piv, double* x) {
  for (int k = 0; k < m; ++k)
    if (piv[k] != k) std::swap(x[k], x[piv[k]]);
  for (int k = 0; k < m; ++k)
    for (int i = k + 1; i < m; ++i) x[i] -= a[i * m + k] * x[k];
  for (int i = m - 1; i >= 0; --i) {
    double s = x[i];
    for (int j = i + 1; j < m; ++j) s -= a[i * m + j] * x[j];
    x[i] = s / a[i * m + i];
  }
}

struct Result {
  int status = 0;       // 0 ok, 1 attempt limit, 2 step underflow, 3 bad input, 4 bad mode
  int accepted = 0;
  int rejected = 0;
  double h_next = 0.0;  // first trial step for a following call (see rok4e_one)
};

// Optional per-attempt record: (t at the start of the attempt, h, err, accepted).
struct Trace {
  double* buf = nullptr;
  int cap = 0;
  int n = 0;
  void add(double t, double h, double err, bool acc) {
    if (n < cap) {
      buf[4 * n + 0] = t; buf[4 * n + 1] = h; buf[4 * n + 2] = err; buf[4 * n + 3] = acc ? 1.0 : 0.0;
    }
    ++n;
  }
};

bool all_finite(const std::vector<double>& x) {
  for (double v : x)
    if (!std::isfinite(v)) return false;
  return true;
}

// One cell: Algorithm a:ROK4E over [0, dt].  u is overwritten with the state at dt
// (or at the last accepted time on failure).
template <class P>
// h0_cell > 0 (finite) replaces the first trial step h_0 of Algorithm a:ROK4E for this
// call.  res.h_next is the step to start a following call from: the controller's
// proposal after the last attempt, or, when the last accepted step had been shortened
// to end at dt, the larger of that proposal and the one made before the shortening.
Result rok4e_one(const P& prob, std::vector<double>& u, double dt, double rtol, double atol,
                 const orc_opts& o, Trace* trace = nullptr, double h0_cell = 0.0) {
  Result res;
  const int n = prob.n();
  const int M = o.M;
  const double eps_fd = o.eps_fd > 0.0 ? o.eps_fd : std::ldexp(1.0, -52);
  const int max_att = o.max_attempts > 0 ? o.max_attempts : 1000000;
  std::vector<double> fn(n), Q(static_cast<size_t>(n) * M), H(static_cast<size_t>(M) * M);
  std::vector<double> k1(n), k2(n), k3(n), k4(n), F(n), arg(n), fs(n), ustar(n), e(n);
  std::vector<double> L, z(M), y(M);
  std::vector<int> piv;
  int Meff = 0;
  bool basis_valid = false;

  double t = 0.0;
  double h = o.h0 > 0.0 ? o.h0 : dt;
  if (h0_cell > 0.0 && std::isfinite(h0_cell)) h = h0_cell;
  double err_prev = 1.0;
  int attempts = 0;
  const bool fixed = o.fixed_steps > 0;
  if (fixed) h = dt / o.fixed_steps;
  int steps_done = 0;
  res.h_next = h;

  // Applies k = F - Q (z - y) - sum_j (gamma_ij / gamma) k_j with y = (I - h gamma H)^{-1} z,
  // z = Q^T F (Algorithm a:ROK4E, stage update).
  auto stage_solve = [&](const std::vector<double>& Fi, std::vector<double>& ki,
                         const std::vector<double>& corr) {
    for (int i = 0; i < Meff; ++i) z[i] = dot(&Q[i * n], Fi.data(), n);
    for (int i = 0; i < Meff; ++i) y[i] = z[i];
    if (Meff > 0) lu_solve(L, Meff, piv, y.data());
    for (int r = 0; r < n; ++r) {
      double qw = 0.0;
      for (int i = 0; i < Meff; ++i) qw += Q[i * n + r] * (z[i] - y[i]);
      ki[r] = Fi[r] - qw - corr[r];
    }
  };

  std::vector<double> corr(n);
  while (fixed ? steps_done < o.fixed_steps : t < dt) {
    if (attempts >= max_att) { res.status = 1; break; }
    const double hprop = h;   // the controller's proposal, before any shortening
    bool last = false;
    if (!fixed && h >= (dt - t) * (1.0 - 1e-12)) { h = dt - t; last = true; }

    if (!basis_valid) {
      prob.template f<double>(u.data(), fn.data());
      Meff = arnoldi(prob, o.jvp, eps_fd, M, u, fn, Q, H);
      if (Meff < 0) { res.status = 4; return res; }
      basis_valid = true;
    }
    // L = I - h gamma H (M_eff x M_eff), factored once per attempt.
    L.assign(static_cast<size_t>(Meff) * Meff, 0.0);
    for (int i = 0; i < Meff; ++i)
      for (int j = 0; j < Meff; ++j)
        L[i * Meff + j] = (i == j ? 1.0 : 0.0) - h * G * H[i * M + j];
    if (Meff > 0 && !lu_factor(L, Meff, piv)) {
      // Singular projected matrix: treat as a failed (rejected) attempt.
      ++attempts; ++res.rejected;
      h *= 0.2;
      res.h_next = h;
      if (h < 16.0 * std::numeric_limits<double>::epsilon() * dt) { res.status = 2; break; }
      continue;
    }
    // Stage 1: F1 = f_n.
    std::fill(corr.begin(), corr.end(), 0.0);
    stage_solve(fn, k1, corr);
    // Stage 2: F2 = f(u + h a21 k1) + (g21/g) k1.
    for (int r = 0; r < n; ++r) arg[r] = u[r] + h * (A21 * k1[r]);
    prob.template f<double>(arg.data(), fs.data());
    for (int r = 0; r < n; ++r) corr[r] = (G21 / G) * k1[r];
    for (int r = 0; r < n; ++r) F[r] = fs[r] + corr[r];
    stage_solve(F, k2, corr);
    // Stage 3: F3 = f(u + h(a31 k1 + a32 k2)) + (g31 k1 + g32 k2)/g.
    for (int r = 0; r < n; ++r) arg[r] = u[r] + h * (A31 * k1[r] + A32 * k2[r]);
    prob.template f<double>(arg.data(), fs.data());
    for (int r = 0; r < n; ++r) corr[r] = (G31 * k1[r] + G32 * k2[r]) / G;
    for (int r = 0; r < n; ++r) F[r] = fs[r] + corr[r];
    stage_solve(F, k3, corr);
    // Stage 4 reuses f of stage 3: a41 = a31, a42 = a32, a43 = 0.
    for (int r = 0; r < n; ++r) corr[r] = (G41 * k1[r] + G42 * k2[r] + G43 * k3[r]) / G;
    for (int r = 0; r < n; ++r) F[r] = fs[r] + corr[r];
    stage_solve(F, k4, corr);

    for (int r = 0; r < n; ++r)
      ustar[r] = u[r] + h * (B1 * k1[r] + B2 * k2[r] + B3 * k3[r] + B4 * k4[r]);
    ++attempts;
    if (fixed) {
      u = ustar;
      ++res.accepted;
      ++steps_done;
      basis_valid = false;
      continue;
    }
    // Embedded error e = u_hat - u* = h sum_j (bh_j - b_j) k_j, weighted RMS norm.
    double ss = 0.0;
    for (int r = 0; r < n; ++r) {
      e[r] = h * ((BH1 - B1) * k1[r] + (BH2 - B2) * k2[r] + (BH3 - B3) * k3[r] + (BH4 - B4) * k4[r]);
      const double sc = atol + rtol * std::fabs(ustar[r]);
      const double ratio = e[r] / sc;
      ss += ratio * ratio;
    }
    double err = std::sqrt(ss / n);
    if (!std::isfinite(err) || !all_finite(ustar)) err = std::numeric_limits<double>::infinity();
    // PI controller: alpha = 0.7/4, beta = 0.4/4.
    const double fac = std::fmin(5.0, std::fmax(0.2, 0.8 * std::pow(std::fmax(err_prev, 1e-10), 0.1) /
                                                     std::pow(std::fmax(err, 1e-10), 0.175)));
    const double hstar = h * fac;
    if (trace) trace->add(t, h, err, err <= 1.0);
    if (err <= 1.0) {
      u = ustar;
      t = last ? dt : t + h;
      err_prev = err;
      h = hstar;
      ++res.accepted;
      basis_valid = false;
      res.h_next = last ? std::fmax(hstar, hprop) : hstar;
    } else {
      h = hstar;
      ++res.rejected;
      res.h_next = hstar;
    }
    if (t < dt && h < 16.0 * std::numeric_limits<double>::epsilon() * dt) { res.status = 2; break; }
  }
  return res;
}

// Dense Rosenbrock (ROW) step with the full Jacobian assembled column by column from
// the same JVP mode: the classical ROW method e:s_stage_row with A_n = J_n,
// fixed steps, used to check that M = N reduces ROK4E to it.
template <class P>
int row_dense(const P& prob, std::vector<double>& u, double dt, int nsteps, int mode, double eps_fd) {
  const int n = prob.n();
  const double h = dt / nsteps;
  std::vector<double> fn(n), J(static_cast<size_t>(n) * n), col(n), ev(n), L;
  std::vector<double> k[4] = {std::vector<double>(n), std::vector<double>(n), std::vector<double>(n),
                              std::vector<double>(n)};
  std::vector<double> arg(n), fs(n), F(n), corr(n);
  std::vector<int> piv;
  const double gam[4][4] = {{0, 0, 0, 0}, {G21, 0, 0, 0}, {G31, G32, 0, 0}, {G41, G42, G43, 0}};
  for (int step = 0; step < nsteps; ++step) {
    prob.template f<double>(u.data(), fn.data());
    for (int c = 0; c < n; ++c) {
      std::fill(ev.begin(), ev.end(), 0.0);
      ev[c] = 1.0;
      if (!jvp(prob, mode, eps_fd, u, fn, ev.data(), col.data())) return -1;
      for (int r = 0; r < n; ++r) J[r * n + c] = col[r];
    }
    L.assign(static_cast<size_t>(n) * n, 0.0);
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) L[r * n + c] = (r == c ? 1.0 : 0.0) - h * G * J[r * n + c];
    if (!lu_factor(L, n, piv)) return -2;
    for (int i = 0; i < 4; ++i) {
      if (i == 0) {
        fs = fn;
      } else if (i == 1) {
        for (int r = 0; r < n; ++r) arg[r] = u[r] + h * (A21 * k[0][r]);
        prob.template f<double>(arg.data(), fs.data());
      } else if (i == 2) {
        for (int r = 0; r < n; ++r) arg[r] = u[r] + h * (A31 * k[0][r] + A32 * k[1][r]);
        prob.template f<double>(arg.data(), fs.data());
      }  // i == 3 reuses fs of stage 3
      for (int r = 0; r < n; ++r) {
        double cr = 0.0;
        for (int j = 0; j < i; ++j) cr += gam[i][j] * k[j][r];
        corr[r] = cr / G;
        F[r] = fs[r] + corr[r];
      }
      lu_solve(L, n, piv, F.data());
      for (int r = 0; r < n; ++r) k[i][r] = F[r] - corr[r];
    }
    for (int r = 0; r < n; ++r)
      u[r] = u[r] + h * (B1 * k[0][r] + B2 * k[1][r] + B3 * k[2][r] + B4 * k[3][r]);
  }
  return 0;
}

// Explicit Dormand-Prince 5(4) Runge-Kutta pair (the paper's explicit reference
// integrator, Sec. 5 efficiency study), from the published tableau: seven stages with the
// last one evaluated at the new solution (first-same-as-last), the fifth-order solution
// propagated and the fourth-order one used for the error estimate.
namespace dp {
constexpr double c2 = 1.0 / 5, c3 = 3.0 / 10, c4 = 4.0 / 5, c5 = 8.0 / 9;
constexpr double a21 = 1.0 / 5;
constexpr double a31 = 3.0 / 40, a32 = 9.0 / 40;
constexpr double a41 = 44.0 / 45, a42 = -56.0 / 15, a43 = 32.0 / 9;
constexpr double a51 = 19372.0 / 6561, a52 = -25360.0 / 2187, a53 = 64448.0 / 6561, a54 = -212.0 / 729;
constexpr double a61 = 9017.0 / 3168, a62 = -355.0 / 33, a63 = 46732.0 / 5247, a64 = 49.0 / 176,
                 a65 = -5103.0 / 18656;
constexpr double b1 = 35.0 / 384, b3 = 500.0 / 1113, b4 = 125.0 / 192, b5 = -2187.0 / 6784, b6 = 11.0 / 84;
constexpr double bh1 = 5179.0 / 57600, bh3 = 7571.0 / 16695, bh4 = 393.0 / 640, bh5 = -92097.0 / 339200,
                 bh6 = 187.0 / 2100, bh7 = 1.0 / 40;
}  // namespace dp

// One cell over [0, dt] with RKDP 5(4): the same error norm as ROK4E (weighted RMS of the
// embedded difference, scale atol + rtol |u_{n+1}|), the elementary controller
// h* = h min(5, max(0.2, 0.9 err^(-1/5))), h0 = dt, clipped last step.
template <class P>
Result rkdp_one(const P& prob, std::vector<double>& u, double dt, double rtol, double atol, const orc_opts& o) {
  Result res;
  const int n = prob.n();
  const int max_att = o.max_attempts > 0 ? o.max_attempts : 1000000;
  const bool fixed = o.fixed_steps > 0;
  std::vector<double> k1(n), k2(n), k3(n), k4(n), k5(n), k6(n), k7(n), arg(n), u5(n);
  double t = 0.0, h = fixed ? dt / o.fixed_steps : (o.h0 > 0.0 ? o.h0 : dt);
  int attempts = 0, steps_done = 0;
  prob.template f<double>(u.data(), k1.data());
  while (fixed ? steps_done < o.fixed_steps : t < dt) {
    if (attempts >= max_att) { res.status = 1; break; }
    bool last = false;
    if (!fixed && h >= (dt - t) * (1.0 - 1e-12)) { h = dt - t; last = true; }
    for (int r = 0; r < n; ++r) arg[r] = u[r] + h * (dp::a21 * k1[r]);
    prob.template f<double>(arg.data(), k2.data());
    for (int r = 0; r < n; ++r) arg[r] = u[r] + h * (dp::a31 * k1[r] + dp::a32 * k2[r]);
    prob.template f<double>(arg.data(), k3.data());
    for (int r = 0; r < n; ++r) arg[r] = u[r] + h * (dp::a41 * k1[r] + dp::a42 * k2[r] + dp::a43 * k3[r]);
    prob.template f<double>(arg.data(), k4.data());
    for (int r = 0; r < n; ++r)
      arg[r] = u[r] + h * (dp::a51 * k1[r] + dp::a52 * k2[r] + dp::a53 * k3[r] + dp::a54 * k4[r]);
    prob.template f<double>(arg.data(), k5.data());
    for (int r = 0; r < n; ++r)
      arg[r] = u[r] + h * (dp::a61 * k1[r] + dp::a62 * k2[r] + dp::a63 * k3[r] + dp::a64 * k4[r] +
                           dp::a65 * k5[r]);
    prob.template f<double>(arg.data(), k6.data());
    for (int r = 0; r < n; ++r)
      u5[r] = u[r] + h * (dp::b1 * k1[r] + dp::b3 * k3[r] + dp::b4 * k4[r] + dp::b5 * k5[r] + dp::b6 * k6[r]);
    prob.template f<double>(u5.data(), k7.data());
    ++attempts;
    if (fixed) {
      u = u5;
      k1 = k7;
      ++res.accepted;
      ++steps_done;
      continue;
    }
    double ss = 0.0;
    for (int r = 0; r < n; ++r) {
      const double e = h * ((dp::b1 - dp::bh1) * k1[r] + (dp::b3 - dp::bh3) * k3[r] + (dp::b4 - dp::bh4) * k4[r] +
                            (dp::b5 - dp::bh5) * k5[r] + (dp::b6 - dp::bh6) * k6[r] - dp::bh7 * k7[r]);
      const double ratio = e / (atol + rtol * std::fabs(u5[r]));
      ss += ratio * ratio;
    }
    double err = std::sqrt(ss / n);
    if (!std::isfinite(err) || !all_finite(u5)) err = std::numeric_limits<double>::infinity();
    const double fac = std::fmin(5.0, std::fmax(0.2, 0.9 * std::pow(std::fmax(err, 1e-10), -0.2)));
    if (err <= 1.0) {
      u = u5;
      k1 = k7;
      t = last ? dt : t + h;
      ++res.accepted;
    } else {
      ++res.rejected;
    }
    h *= fac;
    if (t < dt && h < 16.0 * std::numeric_limits<double>::epsilon() * dt) { res.status = 2; break; }
  }
  return res;
}

bool cell_input_ok(const orc_mech* m, const double* Y, const double* T, const double* p,
                   int64_t n, int64_t c) {
  for (int k = 0; k < m->n_species; ++k)
    if (!std::isfinite(Y[k * n + c])) return false;
  return std::isfinite(T[c]) && T[c] > 0.0 && std::isfinite(p[c]) && p[c] > 0.0;
}

}  // namespace

extern "C" {

// Coefficients in the order gamma, g21, g31, g32, g41, g42, g43, a21, a31, a32, a41,
// a42, a43, b1..b4, bh1..bh4 (21 values).
int orc_coefficients(double* out, int n) {
  const double c[21] = {G, G21, G31, G32, G41, G42, G43, A21, A31, A32, A41, A42, A43,
                        B1, B2, B3, B4, BH1, BH2, BH3, BH4};
  if (n < 21) return -1;
  std::memcpy(out, c, sizeof c);
  return 21;
}

// Right-hand side for n cells in the structure-of-arrays layout (Y[k*n + c]).
// S (optional) is the forcing [(ns+1) * n], same layout with T last.
int orc_rhs(const orc_mech* m, int64_t n, const double* Y, const double* T, const double* p,
            const double* S, double* dY, double* dT) {
  const int ns = m->n_species;
  for (int64_t c = 0; c < n; ++c) {
    std::vector<double> u(ns + 1), f(ns + 1), s;
    for (int k = 0; k < ns; ++k) u[k] = Y[k * n + c];
    u[ns] = T[c];
    if (S) {
      s.resize(ns + 1);
      for (int k = 0; k <= ns; ++k) s[k] = S[k * n + c];
    }
    CellProblem prob{m, p[c], S ? s.data() : nullptr};
    prob.f<double>(u.data(), f.data());
    for (int k = 0; k < ns; ++k) dY[k * n + c] = f[k];
    dT[c] = f[ns];
  }
  return 0;
}

// Jacobian-vector product of one cell: out = J(u) v in the given mode (u and v of
// length ns+1).
int orc_cell_jvp(const orc_mech* m, const double* u, double p, const double* v, int mode,
                 double eps_fd, double* out) {
  const int n = m->n_species + 1;
  CellProblem prob{m, p, nullptr};
  std::vector<double> uu(u, u + n), fu(n);
  prob.f<double>(uu.data(), fu.data());
  return jvp(prob, mode, eps_fd > 0 ? eps_fd : std::ldexp(1.0, -52), uu, fu, v, out) ? 0 : -1;
}

// f(u + du) - f(u) of one cell, evaluated in quadruple precision (113-bit significand)
// and rounded to double: the reference for the difference-form evaluation.
int orc_cell_fdiff_quad(const orc_mech* m, const double* u, double p, const double* du, double* out) {
  const int n = m->n_species + 1;
  CellProblem prob{m, p, nullptr};
  std::vector<quad> a(n), b(n), fa(n), fb(n);
  for (int i = 0; i < n; ++i) {
    a[i] = (quad)u[i];
    b[i] = (quad)u[i] + (quad)du[i];
  }
  prob.f<quad>(a.data(), fa.data());
  prob.f<quad>(b.data(), fb.data());
  for (int i = 0; i < n; ++i) out[i] = (double)(fb[i] - fa[i]);
  return 0;
}

// f(u + du) - f(u) of one cell in difference form (the FD numerator of JVP mode 0).
int orc_cell_fdiff(const orc_mech* m, const double* u, double p, const double* du, double* out) {
  CellProblem prob{m, p, nullptr};
  prob.fdiff(u, du, out);
  return 0;
}

// Arnoldi basis of one cell.  Q is n x M (column j at Q[j*n]), H is M x M row-major.
int orc_cell_arnoldi(const orc_mech* m, const double* u, double p, int M, int mode,
                     double eps_fd, double* Q, double* H) {
  const int n = m->n_species + 1;
  CellProblem prob{m, p, nullptr};
  std::vector<double> uu(u, u + n), fu(n), QQ(static_cast<size_t>(n) * M), HH(static_cast<size_t>(M) * M);
  prob.f<double>(uu.data(), fu.data());
  const int Meff = arnoldi(prob, mode, eps_fd > 0 ? eps_fd : std::ldexp(1.0, -52), M, uu, fu, QQ, HH);
  std::memcpy(Q, QQ.data(), QQ.size() * sizeof(double));
  std::memcpy(H, HH.data(), HH.size() * sizeof(double));
  return Meff;
}

// Integrates n cells over [0, dt] in place.  acc/rej/status may be null.
// As orc_integrate with per-cell first trial steps: h_io[c] > 0 (finite) is cell c's
// h_0; on return h_io[c] holds the step to start the next call from (Result::h_next),
// for cells with valid input.  h_io may be null.
int orc_integrate_h(const orc_mech* m, const orc_opts* o, int64_t n, double* Y, double* T,
                    const double* p, const double* S, double dt, double rtol, double atol,
                    double* h_io, int32_t* acc, int32_t* rej, int32_t* status, int nthreads) {
  const int ns = m->n_species;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t c = 0; c < n; ++c) {
    Result r;
    if (!cell_input_ok(m, Y, T, p, n, c)) {
      r.status = 3;
    } else {
      std::vector<double> u(ns + 1), s;
      for (int k = 0; k < ns; ++k) u[k] = Y[k * n + c];
      u[ns] = T[c];
      if (S) {
        s.resize(ns + 1);
        for (int k = 0; k <= ns; ++k) s[k] = S[k * n + c];
      }
      CellProblem prob{m, p[c], S ? s.data() : nullptr};
      r = rok4e_one(prob, u, dt, rtol, atol, *o, nullptr, h_io ? h_io[c] : 0.0);
      for (int k = 0; k < ns; ++k) Y[k * n + c] = u[k];
      T[c] = u[ns];
      if (h_io) h_io[c] = r.h_next;
    }
    if (acc) acc[c] = r.accepted;
    if (rej) rej[c] = r.rejected;
    if (status) status[c] = r.status;
  }
  return 0;
}

int orc_integrate(const orc_mech* m, const orc_opts* o, int64_t n, double* Y, double* T,
                  const double* p, const double* S, double dt, double rtol, double atol,
                  int32_t* acc, int32_t* rej, int32_t* status, int nthreads) {
  return orc_integrate_h(m, o, n, Y, T, p, S, dt, rtol, atol, nullptr, acc, rej, status, nthreads);
}

// ---------------------------------------------- conservative variables (Sec. 5) ----
// U: [(ns+5) * n] structure of arrays, rows rho Y_1..rho Y_ns, rho, rho u_x, rho u_y,
// rho u_z, rho E (SI units); S: the balancing constants, same layout, may be null.

// Temperature of every cell's conservative variables (NaN where rho c_v <= 0).
int orc_cons_temperature(const orc_mech* m, int64_t n, const double* U, double* T) {
  const int ns = m->n_species;
  std::vector<double> col(ns + 5);
  for (int64_t c = 0; c < n; ++c) {
    for (int r = 0; r < ns + 5; ++r) col[r] = U[r * n + c];
    T[c] = cons_temperature(m, col.data());
  }
  return 0;
}

// f of one cell in the auxiliary-temperature state u (length ns+6); s may be null.
int orc_cons_f(const orc_mech* m, const double* u, const double* s, double* out) {
  ConsProblem prob{m, s};
  prob.f<double>(u, out);
  return 0;
}

// f(u + du) - f(u) of one cell: difference form, or (quad != 0) both evaluations in
// quadruple precision, rounded to double after the subtraction.
int orc_cons_fdiff(const orc_mech* m, const double* u, const double* s, const double* du, int quad_,
                   double* out) {
  ConsProblem prob{m, s};
  const int n = prob.n();
  if (!quad_) {
    prob.fdiff(u, du, out);
    return 0;
  }
  std::vector<quad> a(n), b(n), fa(n), fb(n);
  for (int i = 0; i < n; ++i) {
    a[i] = (quad)u[i];
    b[i] = (quad)u[i] + (quad)du[i];
  }
  prob.f<quad>(a.data(), fa.data());
  prob.f<quad>(b.data(), fb.data());
  for (int i = 0; i < n; ++i) out[i] = (double)(fb[i] - fa[i]);
  return 0;
}

// J(u) v of one auxiliary-temperature cell in the given JVP mode (0 FD, 1 complex step).
int orc_cons_jvp(const orc_mech* m, const double* u, const double* s, const double* v, int mode,
                 double* out) {
  ConsProblem prob{m, s};
  const int n = prob.n();
  std::vector<double> uu(u, u + n), fu(n);
  prob.f<double>(uu.data(), fu.data());
  return jvp(prob, mode, std::ldexp(1.0, -52), uu, fu, v, out) ? 0 : -1;
}

// Integrates n cells of conservative variables over [0, dt] in place: the auxiliary
// temperature starts from the temperature of U, the state (rho Y, T, rho, rho u, rho E)
// is integrated by ROK4E, U receives the conservative rows at dt and T_aux (optional)
// the auxiliary temperature at dt.  A cell with non-finite input, rho <= 0,
// rho c_v <= 0 or T <= 0 keeps its state and reports status 3.
int orc_integrate_cons(const orc_mech* m, const orc_opts* o, int64_t n, double* U, const double* S,
                       double dt, double rtol, double atol, double* T_aux, int32_t* acc, int32_t* rej,
                       int32_t* status, int nthreads) {
  const int ns = m->n_species;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t c = 0; c < n; ++c) {
    Result r;
    std::vector<double> col(ns + 5), u(ns + 6), s;
    bool ok = true;
    for (int i = 0; i < ns + 5; ++i) {
      col[i] = U[i * n + c];
      ok = ok && std::isfinite(col[i]);
    }
    const double T0 = ok ? cons_temperature(m, col.data()) : 0.0;
    ok = ok && col[ns] > 0.0 && std::isfinite(T0) && T0 > 0.0;
    if (!ok) {
      r.status = 3;
    } else {
      for (int k = 0; k < ns; ++k) u[k] = col[k];
      u[ns] = T0;
      for (int i = 0; i < 5; ++i) u[ns + 1 + i] = col[ns + i];
      if (S) {
        s.assign(ns + 6, 0.0);
        for (int k = 0; k < ns; ++k) s[k] = S[k * n + c];
        for (int i = 0; i < 5; ++i) s[ns + 1 + i] = S[(ns + i) * n + c];
      }
      ConsProblem prob{m, S ? s.data() : nullptr};
      r = rok4e_one(prob, u, dt, rtol, atol, *o);
      for (int k = 0; k < ns; ++k) U[k * n + c] = u[k];
      for (int i = 0; i < 5; ++i) U[(ns + i) * n + c] = u[ns + 1 + i];
      if (T_aux) T_aux[c] = u[ns];
    }
    if (acc) acc[c] = r.accepted;
    if (rej) rej[c] = r.rejected;
    if (status) status[c] = r.status;
  }
  return 0;
}

// ROK4E on the linear problem u' = A u + c (A row-major n x n), u in place.
// trace (optional, 4 doubles per attempt, up to trace_cap attempts) records t, h, err
// and the accept flag of each adaptive attempt; *n_trace receives the attempt count.
int orc_integrate_linear(int n, const double* A, const double* c, const orc_opts* o, double* u,
                         double dt, double rtol, double atol, int32_t* acc, int32_t* rej,
                         int32_t* status, double* trace, int trace_cap, int32_t* n_trace) {
  LinearProblem prob{n, A, c};
  std::vector<double> uu(u, u + n);
  Trace tr;
  tr.buf = trace;
  tr.cap = trace ? trace_cap : 0;
  Result r = rok4e_one(prob, uu, dt, rtol, atol, *o, &tr);
  if (n_trace) *n_trace = tr.n;
  std::memcpy(u, uu.data(), n * sizeof(double));
  if (acc) *acc = r.accepted;
  if (rej) *rej = r.rejected;
  if (status) *status = r.status;
  return 0;
}

// RKDP 5(4) on n cells over [0, dt] in place (the explicit reference integrator).
int orc_integrate_rkdp(const orc_mech* m, const orc_opts* o, int64_t n, double* Y, double* T,
                       const double* p, const double* S, double dt, double rtol, double atol,
                       int32_t* acc, int32_t* rej, int32_t* status, int nthreads) {
  const int ns = m->n_species;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t c = 0; c < n; ++c) {
    Result r;
    if (!cell_input_ok(m, Y, T, p, n, c)) {
      r.status = 3;
    } else {
      std::vector<double> u(ns + 1), s;
      for (int k = 0; k < ns; ++k) u[k] = Y[k * n + c];
      u[ns] = T[c];
      if (S) {
        s.resize(ns + 1);
        for (int k = 0; k <= ns; ++k) s[k] = S[k * n + c];
      }
      CellProblem prob{m, p[c], S ? s.data() : nullptr};
      r = rkdp_one(prob, u, dt, rtol, atol, *o);
      for (int k = 0; k < ns; ++k) Y[k * n + c] = u[k];
      T[c] = u[ns];
    }
    if (acc) acc[c] = r.accepted;
    if (rej) rej[c] = r.rejected;
    if (status) status[c] = r.status;
  }
  return 0;
}

// RKDP 5(4) on the linear problem u' = A u + c (for the order pins).
int orc_rkdp_linear(int n, const double* A, const double* c, const orc_opts* o, double* u, double dt,
                    double rtol, double atol, int32_t* acc, int32_t* rej, int32_t* status) {
  LinearProblem prob{n, A, c};
  std::vector<double> uu(u, u + n);
  Result r = rkdp_one(prob, uu, dt, rtol, atol, *o);
  std::memcpy(u, uu.data(), n * sizeof(double));
  if (acc) *acc = r.accepted;
  if (rej) *rej = r.rejected;
  if (status) *status = r.status;
  return 0;
}

// x = A^{-1} b through lu_factor / lu_solve (the projected solve of the stages), for
// the pins; piv (m entries, may be null) receives the row chosen at each step.
// Returns 0, or -1 for a zero pivot.
int orc_lu_solve(int m, const double* A, const double* b, double* x, int* piv) {
  std::vector<double> a(A, A + (size_t)m * m);
  std::vector<int> pv;
  if (!lu_factor(a, m, pv)) return -1;
  for (int i = 0; i < m; ++i) x[i] = b[i];
  lu_solve(a, m, pv, x);
  if (piv)
    for (int i = 0; i < m; ++i) piv[i] = pv[i];
  return 0;
}

// Dormand-Prince tableau in the order c2..c5, a21, a31, a32, a41..a43, a51..a54,
// a61..a65, b1, b3..b6, bh1, bh3..bh7 (30 values; b2 = bh2 = b7 = 0), for the pins.
void orc_rkdp_coefficients(double* out) {
  const double v[30] = {dp::c2,  dp::c3,  dp::c4,  dp::c5,  dp::a21, dp::a31, dp::a32, dp::a41,
                        dp::a42, dp::a43, dp::a51, dp::a52, dp::a53, dp::a54, dp::a61, dp::a62,
                        dp::a63, dp::a64, dp::a65, dp::b1,  dp::b3,  dp::b4,  dp::b5,  dp::b6,
                        dp::bh1, dp::bh3, dp::bh4, dp::bh5, dp::bh6, dp::bh7};
  std::memcpy(out, v, sizeof(v));
}

// ROK4E on a caller-supplied autonomous system u' = f(u) (finite-difference JVPs).
int orc_integrate_callback(int n, orc_rhs_fn fn, void* ctx, const orc_opts* o, double* u,
                           double dt, double rtol, double atol, int32_t* acc, int32_t* rej,
                           int32_t* status) {
  CallbackProblem prob{n, fn, ctx};
  std::vector<double> uu(u, u + n);
  Result r = rok4e_one(prob, uu, dt, rtol, atol, *o);
  std::memcpy(u, uu.data(), n * sizeof(double));
  if (acc) *acc = r.accepted;
  if (rej) *rej = r.rejected;
  if (status) *status = r.status;
  return 0;
}

// Dense ROW with the full Jacobian, fixed steps, on the linear problem.
int orc_row_dense_linear(int n, const double* A, const double* c, double* u, double dt, int nsteps,
                         int mode) {
  LinearProblem prob{n, A, c};
  std::vector<double> uu(u, u + n);
  const int rc = row_dense(prob, uu, dt, nsteps, mode, std::ldexp(1.0, -52));
  std::memcpy(u, uu.data(), n * sizeof(double));
  return rc;
}

// Dense ROW with the full Jacobian, fixed steps, on one reactor cell (u of length ns+1).
int orc_row_dense_cell(const orc_mech* m, double* u, double p, double dt, int nsteps, int mode) {
  CellProblem prob{m, p, nullptr};
  const int n = m->n_species + 1;
  std::vector<double> uu(u, u + n);
  const int rc = row_dense(prob, uu, dt, nsteps, mode, std::ldexp(1.0, -52));
  std::memcpy(u, uu.data(), n * sizeof(double));
  return rc;
}

}  // extern "C"
