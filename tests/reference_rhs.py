"""An independent NumPy right-hand side of the constant-pressure adiabatic reactor
(test helper for the SciPy cross-check).

It takes a different route from the oracle: a dense stoichiometric matrix, molar
production rates from a matrix product, and the energy equation written with molar
enthalpies.
"""
import numpy as np

RU = 8.314462618


class DenseReactor:
    def __init__(self, mech, p):
        self.m = mech
        self.p = p
        ns, nr = mech.n_species, mech.n_reactions
        self.nu = np.zeros((ns, nr))
        self.Rf = np.zeros((ns, nr))       # reactant multiplicities (exponents)
        self.Rr = np.zeros((ns, nr))       # product multiplicities
        for j in range(nr):
            for s in mech.reac[j]:
                if s >= 0:
                    self.nu[s, j] -= 1
                    self.Rf[s, j] += 1
            for s in mech.prod[j]:
                if s >= 0:
                    self.nu[s, j] += 1
                    self.Rr[s, j] += 1

    def __call__(self, t, u):
        m = self.m
        Y, T = u[:-1], u[-1]
        conc_si = self.p / (RU * T) * (Y / m.W) / np.sum(Y / m.W)       # mol/m^3
        c = conc_si * 1e-6                                             # mol/cm^3
        kf = np.exp(m.lnAf + m.bf * np.log(T) - m.Ef / (RU * T))
        kr = np.exp(m.lnAr + m.br * np.log(T) - m.Er / (RU * T))
        # products of concentrations as exp(R^T ln c) would fail for c <= 0; use powers
        pf = np.prod(np.where(self.Rf > 0, c[:, None] ** self.Rf, 1.0), axis=0)
        pr = np.prod(np.where(self.Rr > 0, c[:, None] ** self.Rr, 1.0), axis=0)
        wdot = 1e6 * (self.nu @ (kf * pf - kr * pr))                   # mol/(m^3 s)
        rho = np.sum(conc_si * m.W)                                    # kg/m^3
        Hmol = (m.hf + m.cp * (T - 298.15)) * m.W                      # J/mol
        cp_mass = np.sum(Y * m.cp)
        dY = wdot * m.W / rho
        dT = -np.sum(Hmol * wdot) / (rho * cp_mass)
        return np.concatenate([dY, [dT]])
