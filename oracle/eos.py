"""Bulk free energies, chemical potentials, pressures and the Maxwell construction
(oracle; test infrastructure only).

Definitions (Sec. II A):
    chemical potential   mu = E_f'(rho) - kappa lap(rho)                   (Eq. 2)
    non-ideal EOS        p_EOS = rho E_f'(rho) - E_f(rho)                  (below Eq. 4)

van der Waals (Sec. IV A, Eq. 30):
    E_f = rho R T ln[rho / (1 - b rho)] - a rho^2
    mu_EOS = R T [ln(rho / (1 - b rho)) + 1 / (1 - b rho)] - 2 a rho
    T_c = 8 a / (27 R b),  rho_c = 1 / (3 b)

Carnahan-Starling: not in the paper.  Reading used here, with eta = b rho / 4 and
the same ideal-gas convention as the paper's vdW free energy (rho R T ln rho):
    E_f = rho R T [ln rho + (4 eta - 3 eta^2) / (1 - eta)^2] - a rho^2
    mu_EOS = R T [ln rho + 1 + (8 eta - 9 eta^2 + 3 eta^3) / (1 - eta)^3] - 2 a rho
    p_EOS = rho R T (1 + eta + eta^2 - eta^3) / (1 - eta)^3 - a rho^2
The critical point of this EOS has no closed form; it is found numerically from
dp/drho = d2p/drho2 = 0.

All functions accept Python floats or float64 tensors.
"""

import math

import numpy as np
import torch
from scipy.optimize import brentq


def _log(x):
    if torch.is_tensor(x):
        return torch.log(x)
    if isinstance(x, np.ndarray):
        return np.log(x)
    return math.log(x)


class VanDerWaals:
    """van der Waals bulk free energy of Eq. 30 (parity pinned: Table II, mu^an)."""

    name = "vdW"

    def __init__(self, a=9.0 / 392.0, b=2.0 / 21.0, R=1.0):
        self.a, self.b, self.R = float(a), float(b), float(R)

    @property
    def Tc(self):
        return 8.0 * self.a / (27.0 * self.R * self.b)

    @property
    def rhoc(self):
        return 1.0 / (3.0 * self.b)

    @property
    def rho_max(self):
        return 1.0 / self.b

    def free_energy(self, rho, T):
        return rho * self.R * T * _log(rho / (1.0 - self.b * rho)) - self.a * rho * rho

    def mu(self, rho, T):
        """E_f'(rho); Eq. 30 without the -kappa lap(rho) term."""
        br = 1.0 - self.b * rho
        return self.R * T * (_log(rho / br) + 1.0 / br) - 2.0 * self.a * rho

    def p(self, rho, T):
        """p_EOS = rho E_f' - E_f = rho R T / (1 - b rho) - a rho^2."""
        return rho * self.R * T / (1.0 - self.b * rho) - self.a * rho * rho

    def dp(self, rho, T):
        br = 1.0 - self.b * rho
        return self.R * T / (br * br) - 2.0 * self.a * rho


class CarnahanStarling:
    """Carnahan-Starling bulk free energy (reading; not in the paper).

    Parity: pinned to the paper's definitions Eq. 2-4 (mu = E_f', p = rho mu - E_f)
    and to the hard-sphere compressibility factor at a = 0; the coexistence values
    themselves are fixed only by this reading.
    """

    name = "CS"

    def __init__(self, a=0.0282217394824, b=0.149078724791, R=1.0):
        self.a, self.b, self.R = float(a), float(b), float(R)
        self._crit = None

    def free_energy(self, rho, T):
        eta = self.b * rho / 4.0
        return rho * self.R * T * (_log(rho) + (4 * eta - 3 * eta * eta) / (1 - eta) ** 2) \
            - self.a * rho * rho

    def mu(self, rho, T):
        eta = self.b * rho / 4.0
        return self.R * T * (_log(rho) + 1.0 + (8 * eta - 9 * eta ** 2 + 3 * eta ** 3) / (1 - eta) ** 3) \
            - 2.0 * self.a * rho

    def p(self, rho, T):
        eta = self.b * rho / 4.0
        return rho * self.R * T * (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3 - self.a * rho * rho

    def dp(self, rho, T, h=None):
        # derivative of the hard-sphere part g(eta) = eta Z(eta) written out by hand
        eta = self.b * rho / 4.0
        num = 1 + 4 * eta + 4 * eta ** 2 - 4 * eta ** 3 + eta ** 4
        return self.R * T * num / (1 - eta) ** 4 - 2.0 * self.a * rho

    @property
    def rho_max(self):
        return 4.0 / self.b

    def _critical(self):
        if self._crit is None:
            # p = (4 R T / b) g(eta) - a (4/b)^2 eta^2 with g = eta Z(eta).
            # dp/deta = 0 and d2p/deta2 = 0  =>  g'(eta) = eta g''(eta).
            def g1(e):
                return (1 + 4 * e + 4 * e ** 2 - 4 * e ** 3 + e ** 4) / (1 - e) ** 4

            def g2(e):
                n = 1 + 4 * e + 4 * e ** 2 - 4 * e ** 3 + e ** 4
                dn = 4 + 8 * e - 12 * e ** 2 + 4 * e ** 3
                return (dn * (1 - e) + 4 * n) / (1 - e) ** 5

            eta_c = brentq(lambda e: g1(e) - e * g2(e), 0.05, 0.3, xtol=1e-15)
            # T from dp/deta = 0:  (4 R T / b) g'(eta) = 2 a (4/b)^2 eta
            Tc = 2.0 * self.a * (4.0 / self.b) ** 2 * eta_c / ((4.0 * self.R / self.b) * g1(eta_c))
            self._crit = (4.0 * eta_c / self.b, Tc)
        return self._crit

    @property
    def Tc(self):
        return self._critical()[1]

    @property
    def rhoc(self):
        return self._critical()[0]


def make_eos(name, a=None, b=None, R=1.0):
    if name in ("vdW", "vdw", 0):
        return VanDerWaals(a if a is not None else 9.0 / 392.0, b if b is not None else 2.0 / 21.0, R)
    if name in ("CS", "cs", 1):
        return CarnahanStarling(a if a is not None else 0.0282217394824,
                                b if b is not None else 0.149078724791, R)
    raise ValueError(name)


def spinodals(eos, T):
    """Densities where dp/drho = 0 (gas-side maximum, liquid-side minimum)."""
    grid = [eos.rho_max * (i + 0.5) / 4000 for i in range(4000)]
    vals = [eos.dp(r, T) for r in grid]
    roots = []
    for i in range(len(grid) - 1):
        if vals[i] == 0 or vals[i] * vals[i + 1] < 0:
            roots.append(brentq(lambda r: eos.dp(r, T), grid[i], grid[i + 1], xtol=1e-15, rtol=1e-15))
    if len(roots) != 2:
        raise ValueError(f"no liquid-gas coexistence at T={T} (T >= T_c?)")
    return roots[0], roots[1]


def maxwell(eos, T_over_Tc):
    """Maxwell (equal-area) construction: rho_g < rho_l with equal mu_EOS and p_EOS.

    Bracketed: the pressure P is bisected between the two spinodal pressures; at
    each P the gas and liquid roots of p_EOS(rho) = P are bracketed on their own
    branches.  Returns dict(rho_g, rho_l, mu, p).
    Parity pinned: Table II analytical columns and mu^an (Appendix A).
    """
    T = T_over_Tc * eos.Tc
    s1, s2 = spinodals(eos, T)
    p_hi = eos.p(s1, T)
    p_lo = max(eos.p(s2, T), 0.0)
    tiny = 1e-300

    def branches(P):
        rg = brentq(lambda r: eos.p(r, T) - P, tiny if P > 0 else s1 * 1e-12, s1, xtol=1e-200, rtol=1e-15,
                    maxiter=500)
        rl = brentq(lambda r: eos.p(r, T) - P, s2, eos.rho_max * (1 - 1e-15), xtol=1e-200, rtol=1e-15,
                    maxiter=500)
        return rg, rl

    def dmu(P):
        rg, rl = branches(P)
        return eos.mu(rl, T) - eos.mu(rg, T)

    eps = (p_hi - p_lo) * 1e-12
    P = brentq(dmu, p_lo + eps, p_hi - eps, xtol=1e-200, rtol=1e-15, maxiter=500)
    rg, rl = branches(P)
    return {"rho_g": rg, "rho_l": rl, "mu": eos.mu(rg, T), "p": P, "T": T}
