"""Sec. IV B on the GPU: droplets of radius 20, 25, 30 and 40 on a 120 x 120 periodic
lattice (vdW a = 9/392, b = 2/21, kappa = 0.02, T = 0.8 Tc, MRT at constant nu = 0.15,
float64, 5e4 steps) against the Young-Laplace law (Eq. 32): the liquid and gas
densities follow from p_l, p_g = p_sat + rho_{l,g} / (rho_l - rho_g) theta / R, with
the surface tension theta of the discrete flat profile (R13, from the oracle's Newton
solution) and the equimolar radius R.  The improved scheme stays within the paper's
0.23 % (measured: 0.017 %); the standard scheme's gas density misses by tens of
percent (measured 35.0-37.6 %, the paper: up to 35.3 %, with MRT rates it does not
give)."""

import math

import numpy as np
import pytest
import torch
from scipy.optimize import brentq

from oracle import discrete_equilibrium as de
from oracle import eos
from oracle.lattice import D2Q9
from paper_2008_01473_amd import inputs

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2008_01473_amd import runtime  # noqa: E402  (raises if liblbm.so is missing)

VDW = eos.VanDerWaals()


@pytest.mark.parametrize("scheme", ["improved", "standard"])
def test_droplets_against_young_laplace(scheme):
    t = 0.8
    T = t * VDW.Tc
    mx = eos.maxwell(VDW, t)
    flat, _, _ = de.solve(inputs.slab((1, 100), mx["rho_g"], mx["rho_l"], 4.0), VDW, T, 0.02, D2Q9)
    theta = 0.02 * float(np.sum((np.roll(flat[0], -1) - flat[0]) ** 2)) / 2
    s1, s2 = eos.spinodals(VDW, T)
    n, worst = 120, 0.0
    for r in (20, 25, 30, 40):
        p = runtime.params("D2Q9", n, n, 1, eos="vdW", T_over_Tc=t, kappa=0.02, tau=1.0, scheme=scheme,
                           collision="mrt", tau_e=1.0, tau_s=1.0, tau_q=1.0, nu=0.15)
        rho0 = inputs.droplet((n, n), mx["rho_g"], mx["rho_l"], float(r), 5.0, noise=0.0)
        print(f"case {scheme} droplet r={r}, 5e4 steps", flush=True)
        sim = runtime.LBM(p)
        sim.init(rho0)
        sim.step(50000)
        rho, _, _ = sim.moments()
        assert sim.diagnostics()[0]["status"] == 0
        sim.close()
        rho = rho.view(n, n).cpu().numpy()
        rl, rg = rho[n // 2, n // 2], rho[0, 0]
        R = math.sqrt((rho.sum() - n * n * rg) / (rl - rg) / math.pi)
        dr = mx["rho_l"] - mx["rho_g"]
        rl_th = brentq(lambda x: VDW.p(x, T) - (mx["p"] + mx["rho_l"] / dr * theta / R), s2, 0.999 / VDW.b)
        rg_th = brentq(lambda x: VDW.p(x, T) - (mx["p"] + mx["rho_g"] / dr * theta / R), 1e-9, s1)
        errs = (abs(rl / rl_th - 1), abs(rg / rg_th - 1))
        worst = max(worst, *errs)
        print(f"  R {R:.3f}: rho_l {rl:.6f} (Young-Laplace {rl_th:.6f}), rho_g {rg:.6f} ({rg_th:.6f}), "
              f"rel err {errs[0]:.2e} {errs[1]:.2e}", flush=True)
    print(f"{scheme}: max rel err {worst:.3e}", flush=True)
    if scheme == "improved":
        assert worst < 2.3e-3
    else:
        assert 0.30 < worst < 0.40
