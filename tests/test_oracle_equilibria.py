"""Pins of the oracle's equilibria, forcing and correction terms (Eqs. 11, 14, 25-29)."""

import pytest
import torch

from oracle import eos, model
from oracle.lattice import (CS2, D2Q9, D3Q19, d2q9_inverse_transformation_matrix,
                            d2q9_transformation_matrix)

DT = torch.float64


def _state(lat, seed=0, shape=None):
    g = torch.Generator().manual_seed(seed)
    shape = shape or ((3, 4) if lat.D == 2 else (2, 3, 4))
    rho = 0.3 + 7.0 * torch.rand(shape, generator=g, dtype=DT)
    u = 0.1 * torch.randn((lat.D,) + shape, generator=g, dtype=DT)
    pm = 0.3 + 0.1 * torch.rand(shape, generator=g, dtype=DT)
    F = 0.01 * torch.randn((lat.D,) + shape, generator=g, dtype=DT)
    d = 0.01 * torch.randn((lat.D,) + shape, generator=g, dtype=DT)
    return rho, u, pm, F, d


def _moment(f, lat, powers):
    w = torch.ones(lat.Q, dtype=DT)
    for dd, n in enumerate(powers):
        w = w * lat.ef[:, dd] ** n
    return torch.einsum("a,a...->...", w, f)


def test_transformation_matrix_orthogonal_and_matches_eq11():
    M = d2q9_transformation_matrix()
    G = M @ M.T
    assert torch.allclose(G, torch.diag(torch.diag(G)), atol=0)
    assert torch.allclose(d2q9_inverse_transformation_matrix() @ M, torch.eye(9, dtype=DT), atol=1e-15)
    # M^-1 m_eq(Eq. 11) is the textbook second-order equilibrium
    rho, u, pm, _, _ = _state(D2Q9)
    prm = model.Params(lattice=D2Q9, eos=eos.VanDerWaals(), scheme="standard")
    f1 = model.equilibrium(rho, u, rho / 3, prm)
    f2 = model.textbook_equilibrium(rho, u, D2Q9)
    assert torch.allclose(f1, f2, atol=1e-14, rtol=0)


@pytest.mark.parametrize("lat", [D2Q9, D3Q19])
def test_improved_equilibrium_moments_eq25_eq26(lat):
    rho, u, pm, _, _ = _state(lat, 1)
    prm = model.Params(lattice=lat, eos=eos.VanDerWaals(), scheme="improved")
    f = model.equilibrium(rho, u, pm, prm)
    D = lat.D

    def mom(*idx):
        powers = [0] * D
        for i in idx:
            powers[i] += 1
        return _moment(f, lat, powers)

    assert torch.allclose(mom(), rho, atol=1e-13)
    for i in range(D):
        assert torch.allclose(mom(i), rho * u[i], atol=1e-13)
        for j in range(D):
            want = rho * u[i] * u[j] + (pm if i == j else 0.0)            # Eq. 25
            assert torch.allclose(mom(i, j), want, atol=1e-13)
            for k in range(D):
                idx = (i, j, k)
                if lat.D == 3 and len(set(idx)) == 3:
                    continue                                               # e_x e_y e_z == 0 on D3Q19
                pref = rho * CS2 if (i == j == k) else pm                  # Eq. 26
                want = pref * (u[i] * (j == k) + u[j] * (i == k) + u[k] * (i == j))
                assert torch.allclose(mom(i, j, k), want, atol=1e-13), idx


@pytest.mark.parametrize("lat", [D2Q9, D3Q19])
def test_improved_reduces_to_standard_at_gamma_one(lat):
    rho, u, _, _, _ = _state(lat, 2)
    imp = model.Params(lattice=lat, eos=eos.VanDerWaals(), scheme="improved")
    std = model.Params(lattice=lat, eos=eos.VanDerWaals(), scheme="standard")
    f1 = model.equilibrium(rho, u, rho * CS2, imp)
    f2 = model.equilibrium(rho, u, rho * CS2, std)
    assert torch.allclose(f1, f2, atol=1e-14)
    assert torch.allclose(f2, model.textbook_equilibrium(rho, u, lat), atol=1e-14)


def test_d2q9_moment_rule_reproduces_eq27():
    """The moment-prescription rule used to extend Eq. 27 to D3Q19, applied to D2Q9,
    gives M^-1 of Eq. 27."""
    rho, u, pm, _, _ = _state(D2Q9, 3)
    prm = model.Params(lattice=D2Q9, eos=eos.VanDerWaals(), scheme="improved")
    assert torch.allclose(model.moment_equilibrium(rho, u, pm, D2Q9), model.equilibrium(rho, u, pm, prm),
                          atol=1e-13)


def test_d2q9_improved_rest_state_populations():
    # at u = 0: rest rho - 5 p_m / 3, axis p_m / 3, diagonal p_m / 12
    rho = torch.tensor([[2.0, 5.0]], dtype=DT)
    pm = torch.tensor([[0.34, 0.31]], dtype=DT)
    u = torch.zeros((2, 1, 2), dtype=DT)
    f = model.equilibrium(rho, u, pm, model.Params(lattice=D2Q9, eos=eos.VanDerWaals()))
    assert torch.allclose(f[0], rho - 5 * pm / 3, atol=1e-15)
    for a in range(1, 5):
        assert torch.allclose(f[a], pm / 3, atol=1e-15)
    for a in range(5, 9):
        assert torch.allclose(f[a], pm / 12, atol=1e-15)


@pytest.mark.parametrize("lat", [D2Q9, D3Q19])
def test_guo_forcing_moments(lat):
    _, u, _, F, _ = _state(lat, 4)
    G = model.guo_forcing(u, F, lat)
    D = lat.D
    assert G.sum(0).abs().max() < 1e-15
    for i in range(D):
        p = [0] * D
        p[i] = 1
        assert torch.allclose(_moment(G, lat, p), F[i], atol=1e-15)
        for j in range(D):
            p = [0] * D
            p[i] += 1
            p[j] += 1
            assert torch.allclose(_moment(G, lat, p), u[i] * F[j] + F[i] * u[j], atol=1e-15)


@pytest.mark.parametrize("lat", [D2Q9, D3Q19])
def test_correction_moments(lat):
    _, _, _, _, d = _state(lat, 5)
    C = model.min_norm_correction(d, lat)
    D = lat.D
    assert C.sum(0).abs().max() < 1e-15
    for i in range(D):
        p = [0] * D
        p[i] = 1
        assert _moment(C, lat, p).abs().max() < 1e-15
        for j in range(D):
            p = [0] * D
            p[i] += 1
            p[j] += 1
            want = 3 * d[i] if i == j else torch.zeros_like(d[i])
            assert torch.allclose(_moment(C, lat, p), want, atol=1e-15)


def test_d2q9_min_norm_correction_is_eq29():
    _, _, _, _, d = _state(D2Q9, 6)
    Cp = torch.einsum("ak,k...->a...", d2q9_inverse_transformation_matrix(), model.d2q9_correction_moments(d))
    assert torch.allclose(model.min_norm_correction(d, D2Q9), Cp, atol=1e-15)


def test_d2q9_moment_space_equals_population_space_bgk():
    """With Lambda = I / tau the moment-space collision (Eq. 28) equals the
    population-space BGK update with f_eq = M^-1 m_eq and C = M^-1 C."""
    g = torch.Generator().manual_seed(7)
    shape = (5, 6)
    rho, u, pm, F, d = _state(D2Q9, 7, shape)
    prm = model.Params(lattice=D2Q9, eos=eos.VanDerWaals(), T_over_Tc=0.8, kappa=0.02, tau=0.73)
    f = model.equilibrium(rho, u, pm, prm) + 0.01 * torch.rand((9,) + shape, generator=g, dtype=DT)
    fl = model.fields(f, prm)
    fs = model.collide(f, prm, fl)
    feq = model.equilibrium(fl["rho"], fl["u"], fl["pm"], prm)
    G = model.guo_forcing(fl["u"], fl["F"], D2Q9)
    C = model.min_norm_correction(model.correction_strengths(fl["rho"], fl["u"], fl["pm"], prm), D2Q9)
    om = 1 / prm.tau
    ref = f - om * (f - feq) + (1 - om / 2) * (G + C)
    assert torch.allclose(fs, ref, atol=1e-13)
