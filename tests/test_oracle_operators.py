"""Pins of the oracle's discrete operators (Eq. 17-19)."""

import itertools

import pytest
import torch

from oracle import operators as ops
from oracle.lattice import D2Q9, D3Q19


def _poly_field(shape, coeffs):
    """phi = sum c * x^i y^j (z^k) on a grid indexed [(z,) y, x]."""
    D = len(shape)
    grids = torch.meshgrid(*[torch.arange(n, dtype=torch.float64) for n in shape], indexing="ij")
    xyz = [grids[D - 1 - d] for d in range(D)]    # component d
    phi = torch.zeros(shape, dtype=torch.float64)
    for powers, c in coeffs.items():
        term = torch.full(shape, c, dtype=torch.float64)
        for d, n in enumerate(powers):
            term = term * xyz[d] ** n
        phi = phi + term
    return phi, xyz


def _random_cubic(D, seed):
    g = torch.Generator().manual_seed(seed)
    coeffs = {}
    for powers in itertools.product(range(4), repeat=D):
        if sum(powers) <= 3:
            coeffs[powers] = float(torch.randn(1, generator=g)) * 0.1
    return coeffs


def _analytic(coeffs, D, xyz, deriv):
    """Evaluate the derivative given as a tuple of orders per component."""
    out = torch.zeros_like(xyz[0])
    for powers, c in coeffs.items():
        cc = c
        term = torch.ones_like(xyz[0])
        ok = True
        for d in range(D):
            n, k = powers[d], deriv[d]
            if k > n:
                ok = False
                break
            for i in range(k):
                cc *= (n - i)
            term = term * xyz[d] ** (n - k)
        if ok:
            out = out + cc * term
    return out


@pytest.mark.parametrize("lat,shape", [(D2Q9, (12, 13)), (D3Q19, (9, 10, 11))])
def test_gradient_error_term_eq19_exact_on_cubics(lat, shape):
    """Eq. 19: grad_d(phi) = grad(phi) + (1/6) grad(lap phi), exact for cubic phi
    (delta_t = 1); checked away from the periodic wrap."""
    D = lat.D
    coeffs = _random_cubic(D, 1)
    phi, xyz = _poly_field(shape, coeffs)
    g = ops.grad(phi, lat)
    inner = tuple(slice(1, n - 1) for n in shape)
    for d in range(D):
        exact = _analytic(coeffs, D, xyz, tuple(1 if k == d else 0 for k in range(D)))
        third = torch.zeros_like(exact)
        for k in range(D):
            order = [0] * D
            order[d] += 1
            order[k] += 2
            third = third + _analytic(coeffs, D, xyz, tuple(order))
        assert torch.allclose(g[d][inner], (exact + third / 6.0)[inner], atol=1e-11, rtol=0)
        # the discrete gradient differs from the exact one by the Eq. 19 term, so
        # dropping it must fail somewhere
        assert (g[d][inner] - exact[inner]).abs().max() > 1e-6 or third[inner].abs().max() < 1e-12


@pytest.mark.parametrize("lat,shape", [(D2Q9, (12, 13)), (D3Q19, (9, 10, 11))])
def test_laplacian_exact_on_cubics(lat, shape):
    D = lat.D
    coeffs = _random_cubic(D, 2)
    phi, xyz = _poly_field(shape, coeffs)
    L = ops.laplacian(phi, lat)
    exact = sum(_analytic(coeffs, D, xyz, tuple(2 if k == d else 0 for k in range(D))) for d in range(D))
    inner = tuple(slice(1, n - 1) for n in shape)
    assert torch.allclose(L[inner], exact[inner], atol=1e-11, rtol=0)


def test_d2q9_stencils_written_out():
    # the D2Q9 isotropic stencils in their explicit 9-point form
    phi = torch.randn(7, 8, dtype=torch.float64)
    E, W = torch.roll(phi, -1, 1), torch.roll(phi, 1, 1)
    N, S = torch.roll(phi, -1, 0), torch.roll(phi, 1, 0)
    NE, NW = torch.roll(phi, (-1, -1), (0, 1)), torch.roll(phi, (-1, 1), (0, 1))
    SW, SE = torch.roll(phi, (1, 1), (0, 1)), torch.roll(phi, (1, -1), (0, 1))
    lap = (4 * (E + W + N + S) + (NE + NW + SW + SE) - 20 * phi) / 6
    gx = (4 * (E - W) + (NE - NW - SW + SE)) / 12
    gy = (4 * (N - S) + (NE + NW - SW - SE)) / 12
    assert torch.allclose(ops.laplacian(phi, D2Q9), lap, atol=1e-14)
    g = ops.grad(phi, D2Q9)
    assert torch.allclose(g[0], gx, atol=1e-14)
    assert torch.allclose(g[1], gy, atol=1e-14)


@pytest.mark.parametrize("lat,shape", [(D2Q9, (4, 5)), (D3Q19, (3, 4, 5))])
def test_operator_symmetries_on_periodic_lattice(lat, shape):
    """Dense matrices of the operators: lap is symmetric, each grad component is
    antisymmetric, and all annihilate constants."""
    N = int(torch.tensor(shape).prod())
    L = torch.zeros(N, N, dtype=torch.float64)
    G = torch.zeros(lat.D, N, N, dtype=torch.float64)
    for k in range(N):
        e = torch.zeros(N, dtype=torch.float64)
        e[k] = 1.0
        e = e.view(shape)
        L[:, k] = ops.laplacian(e, lat).reshape(-1)
        G[:, :, k] = ops.grad(e, lat).reshape(lat.D, -1)
    assert torch.allclose(L, L.T, atol=1e-15)
    for d in range(lat.D):
        assert torch.allclose(G[d], -G[d].T, atol=1e-15)
        assert torch.allclose(G[d].sum(1), torch.zeros(N, dtype=torch.float64), atol=1e-14)
    assert torch.allclose(L.sum(1), torch.zeros(N, dtype=torch.float64), atol=1e-14)


def test_shift_direction():
    phi = torch.arange(20, dtype=torch.float64).view(4, 5)   # value = 5 y + x
    s = ops.shifted(phi, [1, 0])
    assert s[2, 3] == phi[2, 4]
    s = ops.shifted(phi, [0, -1])
    assert s[2, 3] == phi[1, 3]
