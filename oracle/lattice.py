"""Discrete velocity sets (oracle; test infrastructure only).

D2Q9 follows Sec. II A of the paper: weights 4/9 (rest), 1/9 (axis), 1/36
(diagonal), lattice sound speed c_s^2 = 1/3, delta_x = delta_t = 1 (Sec. II B).
Velocity order: rest; E, N, W, S; NE, NW, SW, SE.  This order, together with the
transformation matrix below, is the one for which Eq. 11 is the standard
second-order equilibrium (checked in the tests against the textbook formula).

D3Q19 is not in the paper (it treats D2Q9 only); it is the standard 19-velocity
cube set with weights 1/3, 1/18, 1/36.  Order: rest; +x, -x, +y, -y, +z, -z; then
the twelve edge vectors in opposite pairs.

Arrays of lattice fields are indexed [..., z, y, x] (x fastest) in 3D and
[..., y, x] in 2D.  Velocity component d = 0, 1, 2 means x, y, z.
"""

from fractions import Fraction

import torch

DT = torch.float64
CS2 = 1.0 / 3.0  # c_s^2, Sec. II A below Eq. 13


class Lattice:
    def __init__(self, name, vectors, weights):
        self.name = name
        self.e = torch.tensor(vectors, dtype=torch.long)          # (Q, D)
        self.ef = self.e.to(DT)
        self.w = torch.tensor([float(Fraction(x)) for x in weights], dtype=DT)
        self.w_exact = [Fraction(x) for x in weights]
        self.Q, self.D = self.e.shape

    def opposite(self):
        """Index of -e_a for every a."""
        out = []
        for a in range(self.Q):
            m = (self.e == -self.e[a]).all(dim=1).nonzero()
            out.append(int(m[0, 0]))
        return out

    def __repr__(self):
        return f"Lattice({self.name})"


D2Q9 = Lattice(
    "D2Q9",
    [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)],
    ["4/9"] + ["1/9"] * 4 + ["1/36"] * 4,
)

D3Q19 = Lattice(
    "D3Q19",
    [(0, 0, 0),
     (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
     (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
     (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
     (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)],
    ["1/3"] + ["1/18"] * 6 + ["1/36"] * 12,
)

LATTICES = {"D2Q9": D2Q9, "D3Q19": D3Q19}


def d2q9_transformation_matrix():
    """Transformation matrix M of the D2Q9 moment-space collision (Eqs. 7-11).

    The paper does not print M.  Its equilibrium moments (Eq. 11) are those of
    the Lallemand-Luo basis, whose rows are the polynomials
        rho: 1,  e: -4 + 3|e|^2,  eps: 4 - (21/2)|e|^2 + (9/2)|e|^4,
        j_x: e_x,  q_x: (-5 + 3|e|^2) e_x,  j_y: e_y,  q_y: (-5 + 3|e|^2) e_y,
        p_xx: e_x^2 - e_y^2,  p_xy: e_x e_y,
    evaluated on the velocity set.  Returns a (9, 9) float64 tensor.
    Pinned in the tests: M^-1 applied to Eq. 11 gives the textbook equilibrium.
    """
    rows = []
    for ex, ey in D2Q9.e.tolist():
        c2 = ex * ex + ey * ey
        rows.append([
            1.0,
            -4.0 + 3.0 * c2,
            4.0 - 10.5 * c2 + 4.5 * c2 * c2,
            ex,
            (-5.0 + 3.0 * c2) * ex,
            ey,
            (-5.0 + 3.0 * c2) * ey,
            ex * ex - ey * ey,
            ex * ey,
        ])
    return torch.tensor(rows, dtype=DT).T.contiguous()


def d2q9_inverse_transformation_matrix():
    """M^-1.  The rows of M are mutually orthogonal, so M^-1 = M^T diag(1 / |row_k|^2),
    with the squared row norms (integers) computed exactly."""
    M = d2q9_transformation_matrix()
    norms = (M * M).sum(1)
    return (M.T / norms).contiguous()


def moment_monomials(lat):
    """Monomials in e that span the population space of `lat`, as a list of
    exponent tuples, ordered by total degree.

    D2Q9: 1, e_x, e_y, e_x^2, e_y^2, e_x e_y, e_x e_y^2, e_x^2 e_y, e_x^2 e_y^2.
    D3Q19: 1, e_i, e_i e_j, e_i e_j^2 (i != j), e_i^2 e_j^2 (i < j).
    """
    if lat.D == 2:
        return [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (1, 2), (2, 1), (2, 2)]
    return [(0, 0, 0),
            (1, 0, 0), (0, 1, 0), (0, 0, 1),
            (2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 1, 0), (1, 0, 1), (0, 1, 1),
            (1, 2, 0), (1, 0, 2), (2, 1, 0), (0, 1, 2), (2, 0, 1), (0, 2, 1),
            (2, 2, 0), (2, 0, 2), (0, 2, 2)]


def monomial_matrix(lat):
    """A[k, a] = prod_d e_{a,d}^{n_{k,d}} for the monomials of moment_monomials."""
    mons = moment_monomials(lat)
    A = torch.zeros(len(mons), lat.Q, dtype=DT)
    for k, n in enumerate(mons):
        col = torch.ones(lat.Q, dtype=DT)
        for d in range(lat.D):
            col = col * lat.ef[:, d] ** n[d]
        A[k] = col
    return A
