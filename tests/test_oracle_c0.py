"""Pins of the oracle's p_m offset, p_m = (c0 + mu)/3 (an extension, not the
paper's method, whose c0 is 1): an independently written scalar step, the force
of Eq. 24 unchanged, the discrete equilibrium at rest still an exact fixed point,
and c0 = 1 giving back the paper's scheme."""

import pytest
import torch

import brute_force
from oracle import discrete_equilibrium as de
from oracle import eos, model
from oracle.lattice import D2Q9, D3Q19
from paper_2008_01473_amd import inputs

from test_oracle_step import _random_f, _to_dict

DT = torch.float64
VDW = eos.VanDerWaals()


@pytest.mark.parametrize("lat,shape", [(D2Q9, (4, 5)), (D3Q19, (3, 4, 5))])
@pytest.mark.parametrize("E", [VDW, eos.CarnahanStarling()])
def test_c0_matches_brute_force(lat, shape, E):
    prm = model.Params(lattice=lat, eos=E, T_over_Tc=0.8, kappa=0.03, tau=0.7, c0=0.6)
    f = _random_f(prm, shape, 19)
    ref, _ = brute_force.step(_to_dict(f, lat), tuple(reversed(shape)), lambda r: E.mu(r, prm.T),
                              lambda r: E.p(r, prm.T), prm.kappa, prm.tau, "improved", c0=0.6)
    got = _to_dict(model.step(f, prm), lat)
    assert max(abs(got[k] - ref[k]) for k in ref) < 1e-13


def test_c0_with_plates_and_mrt_matches_brute_force():
    mrt = dict(s_e=1 / 1.1, s_eps=1 / 1.3, s_q=1 / 0.9, nu=0.07)
    prm = model.Params(lattice=D2Q9, eos=VDW, T_over_Tc=0.8, kappa=0.03, tau=0.7, c0=0.6, walls=(0.02, -0.04),
                       relaxation=[1.0, mrt["s_e"], mrt["s_eps"], 1.0, mrt["s_q"], 1.0, mrt["s_q"], 1 / 0.7, 1 / 0.7],
                       nu=mrt["nu"])
    f = _random_f(prm, (5, 4), 23)
    ref, _ = brute_force.step(_to_dict(f, D2Q9), (4, 5), lambda r: VDW.mu(r, prm.T), lambda r: VDW.p(r, prm.T),
                              prm.kappa, prm.tau, "improved", mrt=mrt, walls=(0.02, -0.04), c0=0.6)
    got = _to_dict(model.step(f, prm), D2Q9)
    assert max(abs(got[k] - ref[k]) for k in ref) < 1e-13


def test_c0_leaves_the_force_and_gives_back_the_paper_at_one():
    base = model.Params(lattice=D2Q9, eos=VDW, T_over_Tc=0.8, kappa=0.03, tau=0.8)
    f = _random_f(base, (10, 12), 29)
    shifted = model.Params(lattice=D2Q9, eos=VDW, T_over_Tc=0.8, kappa=0.03, tau=0.8, c0=0.55)
    a, b = model.fields(f, base), model.fields(f, shifted)
    assert torch.equal(a["F"], b["F"])                       # Eq. 24: F = (1/3 - rho) grad mu
    assert torch.allclose(b["pm"] - a["pm"], torch.full_like(a["pm"], (0.55 - 1.0) / 3), atol=1e-15)
    one = model.Params(lattice=D2Q9, eos=VDW, T_over_Tc=0.8, kappa=0.03, tau=0.8, c0=1.0)
    assert torch.equal(model.step(f, one), model.step(f, base))
    assert not torch.allclose(model.step(f, shifted), model.step(f, base))


def test_rest_state_is_a_fixed_point_for_any_c0():
    t = 0.7
    mx = eos.maxwell(VDW, t)
    r0 = inputs.droplet((24, 24), mx["rho_g"], mx["rho_l"], 6.0)
    rho, _, res = de.solve(r0, VDW, t * VDW.Tc, 0.02, D2Q9)
    assert res < 1e-12
    for c0 in (0.6, 0.8):
        prm = model.Params(lattice=D2Q9, eos=VDW, T_over_Tc=t, kappa=0.02, tau=1.0, c0=c0)
        f = model.init(torch.tensor(rho), prm)
        f1 = model.run(f, prm, 2)
        assert (f1 - f).abs().max() < 1e-13
        assert model.fields(f1, prm)["u"].abs().max() < 2.2e-14
        # with c0 = 0.6 the gas rest population rho - 5 p_m / 3 of Eq. 27 is positive
        if c0 == 0.6:
            assert float(f[0].min()) > 0
