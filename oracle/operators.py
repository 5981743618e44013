"""Isotropic finite-difference operators on periodic lattices (oracle; test
infrastructure only).

Gradient, Eq. 17 (delta_t = 1, c_s^2 = 1/3):
    grad(phi)(x) = (1 / c_s^2) sum_a w_a phi(x + e_a) e_a

Laplacian: the paper uses lap(rho) in Eq. 2 / Eq. 30 without printing its
discretisation.  Reading used here: the isotropic form built from the same
weights,
    lap(phi)(x) = (2 / c_s^2) sum_a w_a [phi(x + e_a) - phi(x)],
which for D2Q9 is [4(E + W + N + S) + (NE + NW + SW + SE) - 20 phi] / 6.

Divergence of a vector or tensor field applies Eq. 17 to each component.

Parity pinned (tests): Eq. 19 exactly on cubic polynomials (the discrete gradient
equals grad + (1/6) grad lap), the Laplacian is exact on cubics, and on a periodic
lattice grad^T = -grad and lap^T = lap.
"""

import torch

from .lattice import CS2


def shifted(phi, e):
    """phi(x + e) for a periodic field indexed [..., (z,) y, x]."""
    D = len(e)
    dims = tuple(range(phi.ndim - D, phi.ndim))          # (z, y, x) or (y, x)
    shifts = tuple(-int(e[D - 1 - k]) for k in range(D))  # axis k holds component D-1-k
    if all(s == 0 for s in shifts):
        return phi
    return torch.roll(phi, shifts=shifts, dims=dims)


def grad(phi, lat):
    """Eq. 17.  Returns a tensor of shape (D, *phi.shape); component 0 is x."""
    out = torch.zeros((lat.D,) + tuple(phi.shape), dtype=phi.dtype)
    for a in range(lat.Q):
        if lat.e[a].abs().sum() == 0:
            continue
        s = shifted(phi, lat.e[a].tolist())
        for d in range(lat.D):
            if lat.e[a, d] != 0:
                out[d] = out[d] + lat.w[a] * lat.e[a, d].item() * s
    return out / CS2


def partial(phi, lat, d):
    """Component d of Eq. 17 applied to the scalar field phi."""
    out = torch.zeros_like(phi)
    for a in range(lat.Q):
        if lat.e[a, d] != 0:
            out = out + lat.w[a] * lat.e[a, d].item() * shifted(phi, lat.e[a].tolist())
    return out / CS2


def laplacian(phi, lat):
    out = torch.zeros_like(phi)
    for a in range(lat.Q):
        if lat.e[a].abs().sum() == 0:
            continue
        out = out + lat.w[a] * (shifted(phi, lat.e[a].tolist()) - phi)
    return 2.0 * out / CS2


def divergence_tensor(P, lat):
    """(div P)_j = sum_i partial_i P_ij, each partial_i from Eq. 17.
    P has shape (D, D, *grid).  Returns (D, *grid)."""
    out = torch.zeros((lat.D,) + tuple(P.shape[2:]), dtype=P.dtype)
    for j in range(lat.D):
        for i in range(lat.D):
            out[j] = out[j] + partial(P[i, j], lat, i)
    return out
