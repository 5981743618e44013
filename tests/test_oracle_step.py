"""Pins of the oracle's time step: brute force on tiny lattices, exact mass
conservation, streaming as a permutation."""

import pytest
import torch

import brute_force
from oracle import eos, model
from oracle.lattice import D2Q9, D3Q19

DT = torch.float64

VARIANTS = [("improved", "chempot"), ("standard", "chempot"), ("standard", "ptensor")]


def _random_f(prm, shape, seed, amp=0.02):
    g = torch.Generator().manual_seed(seed)
    rho = 1.0 + 5.0 * torch.rand(shape, generator=g, dtype=DT)
    u = 0.05 * torch.randn((prm.lattice.D,) + shape, generator=g, dtype=DT)
    f = model.init(rho, prm, u)
    return f + amp * torch.rand(f.shape, generator=g, dtype=DT) * f.abs().mean()


def _to_dict(f, lat):
    out = {}
    shape = f.shape[1:]
    D = lat.D
    for a in range(lat.Q):
        for idx in torch.cartesian_prod(*[torch.arange(n) for n in shape]).tolist():
            idx = idx if isinstance(idx, list) else [idx]
            node = tuple(idx[D - 1 - d] for d in range(D))      # (x, y[, z])
            out[(a, node)] = float(f[(a,) + tuple(idx)])
    return out


@pytest.mark.parametrize("scheme,form", VARIANTS)
@pytest.mark.parametrize("lat,shape", [(D2Q9, (3, 3)), (D2Q9, (4, 5)), (D3Q19, (3, 3, 3)), (D3Q19, (3, 4, 5))])
@pytest.mark.parametrize("E", [eos.VanDerWaals(), eos.CarnahanStarling()])
def test_oracle_matches_brute_force(scheme, form, lat, shape, E):
    prm = model.Params(lattice=lat, eos=E, T_over_Tc=0.8, kappa=0.03, tau=0.7, scheme=scheme, force_form=form)
    f = _random_f(prm, shape, 11)
    ref, flds = brute_force.step(_to_dict(f, lat), tuple(reversed(shape)), lambda r: E.mu(r, prm.T),
                                 lambda r: E.p(r, prm.T), prm.kappa, prm.tau, scheme, form)
    got = _to_dict(model.step(f, prm), lat)
    err = max(abs(got[k] - ref[k]) for k in ref)
    assert err < 1e-13, err
    fl = model.fields(f, prm)
    D = lat.D
    for node, val in flds["u"].items():
        idx = tuple(node[D - 1 - k] for k in range(D))
        for d in range(D):
            assert abs(fl["u"][(d,) + idx] - val[d]) < 1e-14


@pytest.mark.parametrize("scheme,form", VARIANTS)
@pytest.mark.parametrize("lat,shape", [(D2Q9, (16, 18)), (D3Q19, (6, 7, 8))])
def test_mass_conserved_each_step(scheme, form, lat, shape):
    prm = model.Params(lattice=lat, eos=eos.VanDerWaals(), T_over_Tc=0.85, kappa=0.02, tau=0.9,
                       scheme=scheme, force_form=form)
    f = _random_f(prm, shape, 3)
    m0 = float(f.sum())
    for _ in range(5):
        f = model.step(f, prm)
        assert abs(float(f.sum()) - m0) <= 1e-13 * abs(m0)


@pytest.mark.parametrize("lat,shape", [(D2Q9, (4, 5)), (D3Q19, (3, 4, 5))])
def test_streaming_is_the_eq10_permutation(lat, shape):
    N = int(torch.tensor(shape).prod())
    for a in range(lat.Q):
        for k in (0, N // 2, N - 1):
            fs = torch.zeros((lat.Q,) + shape, dtype=DT)
            idx = list(torch.unravel_index(torch.tensor(k), shape))
            fs[(a,) + tuple(int(i) for i in idx)] = 1.0
            out = model.stream(fs, lat)
            assert float(out.sum()) == 1.0 and float(out[a].sum()) == 1.0
            # the single population moved to x + e_a (periodic)
            D = lat.D
            tgt = [int(idx[i]) for i in range(D)]
            for d in range(D):
                ax = D - 1 - d
                tgt[ax] = (tgt[ax] + int(lat.e[a, d])) % shape[ax]
            assert float(out[(a,) + tuple(tgt)]) == 1.0


@pytest.mark.parametrize("lat,shape", [(D2Q9, (8, 9)), (D3Q19, (4, 5, 6))])
def test_uniform_state_is_stationary(lat, shape):
    # uniform density at rest: no force, no correction, equilibrium streams onto itself
    for scheme in ("improved", "standard"):
        prm = model.Params(lattice=lat, eos=eos.VanDerWaals(), T_over_Tc=0.9, kappa=0.02, tau=0.8, scheme=scheme)
        f = model.init(torch.full(shape, 2.3, dtype=DT), prm)
        f1 = model.run(f, prm, 3)
        assert torch.allclose(f1, f, atol=2e-14, rtol=0)


def test_relaxation_rate_of_conserved_moments_is_irrelevant():
    # Sec. II A: the rates of the conserved moments (tau_c) do not change the result
    prm1 = model.Params(lattice=D2Q9, eos=eos.VanDerWaals(), T_over_Tc=0.8, kappa=0.02, tau=0.8)
    s = [1 / 0.8] * 9
    s[0] = s[3] = s[5] = 1.0
    prm2 = model.Params(lattice=D2Q9, eos=eos.VanDerWaals(), T_over_Tc=0.8, kappa=0.02, tau=0.8, relaxation=s)
    s3 = list(s)
    s3[0] = s3[3] = s3[5] = 0.37
    prm3 = model.Params(lattice=D2Q9, eos=eos.VanDerWaals(), T_over_Tc=0.8, kappa=0.02, tau=0.8, relaxation=s3)
    f = _random_f(prm1, (6, 7), 5)
    a, b, c = model.step(f, prm1), model.step(f, prm2), model.step(f, prm3)
    assert torch.allclose(a, b, atol=1e-14)
    assert torch.allclose(b, c, atol=1e-14)
