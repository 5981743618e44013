"""One time step of the forcing-based free-energy LB method, standard and improved
schemes (oracle; test infrastructure only).

Everything is float64 on the CPU, periodic in every direction, delta_x = delta_t = 1.
The order of operations in `step` follows the paper:

  1. rho = sum_a f_a,  j = sum_a e_a f_a                        (Eq. 12)
  2. mu = E_f'(rho) - kappa lap(rho)                            (Eq. 2, Eq. 30)
  3. force
       standard, chemical-potential form: F = grad(rho c_s^2) - rho grad(mu)   (Eq. 13 right)
       standard, pressure-tensor form:    F = grad(rho c_s^2) - div P          (Eq. 13 left,
                                          P from Eqs. 4-5)
       improved:                          F = (1/3 - rho) grad(mu)             (Eq. 24)
  4. u = (j + F/2) / rho                                        (Eq. 12)
  5. Guo forcing G_a (Eq. 14); in moment space S = M G
  6. equilibrium: Eq. 11 (standard) or Eq. 27 with gamma = 3 p_m / rho,
     p_m = (1 + mu) / 3 (improved, Sec. III)
  7. improved only: correction C = (0, 9 C1, 0, 0, 0, 0, 0, 3 C7, 0),
     C1 = d_x + d_y, C7 = d_x - d_y, d_i = partial_i(phi u_i), phi = rho c_s^2 - p_m (Eq. 29)
  8. collision in moment space, m* = m - Lambda (m - m_eq) + (I - Lambda/2)(S + C)   (Eq. 9, Eq. 28)
  9. streaming f_a(x + e_a, t + 1) = f*_a(x, t)                 (Eq. 10)

Readings where the paper is silent (each is listed with its reason in the design
notes of the repository):
  * lap is the isotropic stencil of operators.laplacian.
  * partial_i(phi u_i) is the i-th component of Eq. 17 applied to the field phi u_i.
  * Lambda = I / tau (BGK, "a special case" of MRT per Sec. II A); a full
    relaxation vector may be passed for D2Q9 (Eq. 8, in the order of M's rows).
  * with `walls` set (D2Q9), the lattice is bounded in y by two plates halfway
    between rows -1 / 0 and ny-1 / ny that move along x with the given speeds
    (Sec. IV B's channel): a population that would stream out of a plate comes back
    at the node it left, reversed, plus feq_b - feq_-b of the scheme's own
    equilibrium at the node's rho, p_m and the plate velocity U_w (halfway
    bounce-back with a moving-wall term; for the standard equilibrium this is the
    familiar 6 w_b rho (e_b . U_w); the paper cites its no-slip scheme without
    stating it, and the improved equilibrium's odd part carries p_m).  The
    stencils see beyond a plate the mirror image of the fluid: rho, mu and
    phi u_x even, phi u_y odd (an impermeable, neutrally wetting plate).
  * with `nu` set (D2Q9), the shear rates (rows p_xx, p_xy) are 1/tau_v with
    tau_v chosen so that the kinematic viscosity nu = eta / rho is the same at
    every node: eta = rho c_s^2 (tau_v - 1/2) in the standard scheme (Sec. II A)
    and eta = p_m (tau_v - 1/2) in the improved one (Sec. III).
  * the pressure-tensor divergence applies Eq. 17 to every component P_ij.
  * initial populations are the scheme's own equilibrium at (rho0, u0), with
    p_m evaluated from mu(rho0) including the -kappa lap(rho0) term.

D3Q19 (not in the paper) is an extension built by the same rules:
  * the standard equilibrium is the textbook second-order one (for D2Q9 it equals
    M^-1 of Eq. 11, checked in the tests);
  * the improved equilibrium is the unique population vector whose moments are
    the standard ones changed by (p_m - rho c_s^2) times: delta_ij in the second
    moments (Eq. 25), u_i in the off-diagonal third moments sum e_i e_j^2 f (Eq. 26),
    c_s^2 in the fourth moments sum e_i^2 e_j^2 f (the change Eq. 27 makes on D2Q9);
  * C is the minimum-norm population vector with zero mass and momentum and
    second moments diag(3 d_i) (on D2Q9 this is exactly M^-1 of Eq. 29's C).
  Applied to D2Q9, both constructions reproduce the paper's moment-space forms
  (checked in the tests), so the 3D scheme is the 2D one by the same rule.
"""

from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import torch

from .lattice import CS2, DT, D2Q9, LATTICES, d2q9_inverse_transformation_matrix, \
    d2q9_transformation_matrix, monomial_matrix, moment_monomials
from .operators import divergence_tensor, grad, laplacian, partial


@dataclass
class Params:
    lattice: object = D2Q9
    eos: object = None
    T_over_Tc: float = 0.8
    kappa: float = 0.02
    tau: float = 1.0
    scheme: str = "improved"          # "improved" | "standard"
    force_form: str = "chempot"       # "chempot" | "ptensor" (standard scheme only)
    relaxation: Optional[Sequence[float]] = None   # D2Q9 MRT rates; None => BGK 1/tau
    nu: Optional[float] = None        # D2Q9: constant kinematic viscosity -> per-node tau_v
    walls: Optional[Tuple[float, float]] = None   # D2Q9: plate speeds (bottom, top) along x
    c0: float = 1.0                   # improved scheme: p_m = (c0 + mu) / 3 (the paper: 1)
    extra: dict = field(default_factory=dict)

    def __post_init__(self):
        if isinstance(self.lattice, str):
            self.lattice = LATTICES[self.lattice]
        if self.scheme not in ("improved", "standard"):
            raise ValueError(self.scheme)
        if self.force_form not in ("chempot", "ptensor"):
            raise ValueError(self.force_form)
        if self.scheme == "improved" and self.force_form != "chempot":
            raise ValueError("the improved scheme is defined with the chemical-potential force (Eq. 24)")
        if self.walls is not None and (self.lattice.Q != 9 or self.force_form != "chempot"):
            raise ValueError("plates are implemented for D2Q9 with the chemical-potential force")

    @property
    def T(self):
        return self.T_over_Tc * self.eos.Tc


# ----------------------------------------------------------------------------- fields

def density_momentum(f, lat):
    """Eq. 12: rho = sum f, j = sum e f (j is the bare first moment, without F/2)."""
    rho = f.sum(0)
    j = torch.einsum("ad,a...->d...", lat.ef, f)
    return rho, j


def _stencil(op, phi, prm, parity=1.0, *args):
    """Apply a stencil; with plates, on phi extended by one mirror row beyond each
    plate (times `parity`, -1 for a wall-normal component), cropped back."""
    if prm.walls is None:
        return op(phi, prm.lattice, *args)
    ext = torch.cat([parity * phi[..., :1, :], phi, parity * phi[..., -1:, :]], dim=-2)
    return op(ext, prm.lattice, *args)[..., 1:-1, :]


def chemical_potential(rho, prm):
    """Eq. 2 with the bulk part of Eq. 30 (or the CS reading)."""
    return prm.eos.mu(rho, prm.T) - prm.kappa * _stencil(laplacian, rho, prm)


def modified_pressure(mu, c0=1.0):
    """p_m = (1 + mu) / 3, Sec. III.  c0 != 1 replaces the 1 (an extension, not the
    paper's method: F of Eq. 24 depends on grad p_m only)."""
    return (c0 + mu) / 3.0


def pressure_tensor(rho, prm):
    """Eqs. 4-5: P = (p_EOS - kappa rho lap rho - kappa/2 |grad rho|^2) I + kappa grad rho grad rho."""
    lat = prm.lattice
    g = grad(rho, lat)
    p = prm.eos.p(rho, prm.T) - prm.kappa * rho * laplacian(rho, lat) - 0.5 * prm.kappa * (g * g).sum(0)
    P = torch.zeros((lat.D, lat.D) + tuple(rho.shape), dtype=DT)
    for i in range(lat.D):
        for j in range(lat.D):
            P[i, j] = prm.kappa * g[i] * g[j]
        P[i, i] = P[i, i] + p
    return P


def force(rho, mu, prm):
    lat = prm.lattice
    if prm.scheme == "improved":
        return (1.0 / 3.0 - rho) * _stencil(grad, mu, prm)            # Eq. 24
    if prm.force_form == "chempot":
        return _stencil(grad, rho * CS2, prm) - rho * _stencil(grad, mu, prm)   # Eq. 13, right
    return grad(rho * CS2, lat) - divergence_tensor(pressure_tensor(rho, prm), lat)  # Eq. 13, left


def fields(f, prm):
    """Macroscopic fields at the time level of f: rho, j, mu, F, u, p_m."""
    lat = prm.lattice
    rho, j = density_momentum(f, lat)
    mu = chemical_potential(rho, prm)
    F = force(rho, mu, prm)
    u = (j + 0.5 * F) / rho                                          # Eq. 12
    pm = modified_pressure(mu, prm.c0) if prm.scheme == "improved" else rho * CS2
    return {"rho": rho, "j": j, "mu": mu, "F": F, "u": u, "pm": pm}


# ----------------------------------------------------------------------------- source terms

def guo_forcing(u, F, lat):
    """Eq. 14: G_a = w_a [(e_a - u) / c_s^2 + (e_a . u) e_a / c_s^4] . F."""
    G = torch.zeros((lat.Q,) + tuple(u.shape[1:]), dtype=DT)
    for a in range(lat.Q):
        ea = lat.ef[a].view((lat.D,) + (1,) * (u.ndim - 1))
        eu = (ea * u).sum(0)
        vec = (ea - u) / CS2 + eu * ea / (CS2 * CS2)
        G[a] = lat.w[a] * (vec * F).sum(0)
    return G


def correction_strengths(rho, u, pm, prm):
    """d_i = partial_i(phi u_i) with phi = rho c_s^2 - p_m (Eq. 29), each partial from Eq. 17."""
    phi = rho * CS2 - pm
    return torch.stack([_stencil(partial, phi * u[i], prm, -1.0 if i == 1 else 1.0, i)
                        for i in range(prm.lattice.D)])


def d2q9_correction_moments(d):
    """Eq. 28-29: C = (0, 9 C1, 0, 0, 0, 0, 0, 3 C7, 0)^T in the basis of M."""
    C1 = d[0] + d[1]
    C7 = d[0] - d[1]
    C = torch.zeros((9,) + tuple(d.shape[1:]), dtype=DT)
    C[1] = 9.0 * C1
    C[7] = 3.0 * C7
    return C


def min_norm_correction(d, lat):
    """Population-space correction with sum C = 0, sum e C = 0, sum e_i e_j C = diag(3 d_i),
    of minimum Euclidean norm (the D3Q19 extension; equals M^-1 of Eq. 29 on D2Q9)."""
    mons = [n for n in moment_monomials(lat) if sum(n) <= 2]
    A = torch.zeros(len(mons), lat.Q, dtype=DT)
    for k, n in enumerate(mons):
        col = torch.ones(lat.Q, dtype=DT)
        for dd in range(lat.D):
            col = col * lat.ef[:, dd] ** n[dd]
        A[k] = col
    pinv = A.T @ torch.linalg.inv(A @ A.T)                 # (Q, K)
    b = torch.zeros((len(mons),) + tuple(d.shape[1:]), dtype=DT)
    for k, n in enumerate(mons):
        if sum(n) == 2 and max(n) == 2:                     # e_i^2
            i = n.index(2)
            b[k] = 3.0 * d[i]
    return torch.einsum("ak,k...->a...", pinv, b)


# ----------------------------------------------------------------------------- equilibria

def d2q9_equilibrium_moments(rho, u, pm, scheme):
    """Eq. 11 (standard) or Eq. 27 (improved, gamma = 3 p_m / rho), basis of M."""
    ux, uy = u[0], u[1]
    u2 = ux * ux + uy * uy
    if scheme == "standard":
        comps = [torch.ones_like(rho), -2.0 + 3.0 * u2, 1.0 - 3.0 * u2, ux, -ux, uy, -uy,
                 ux * ux - uy * uy, ux * uy]
    else:
        g = 3.0 * pm / rho
        comps = [torch.ones_like(rho), -4.0 + 3.0 * u2 + 2.0 * g, 4.0 - 3.0 * u2 - 3.0 * g, ux,
                 (g - 2.0) * ux, uy, (g - 2.0) * uy, ux * ux - uy * uy, ux * uy]
    return torch.stack([rho * c for c in comps])


def textbook_equilibrium(rho, u, lat):
    """w_a rho [1 + e.u / c_s^2 + (e.u)^2 / (2 c_s^4) - u^2 / (2 c_s^2)]."""
    feq = torch.zeros((lat.Q,) + tuple(rho.shape), dtype=DT)
    u2 = (u * u).sum(0)
    for a in range(lat.Q):
        ea = lat.ef[a].view((lat.D,) + (1,) * rho.ndim)
        eu = (ea * u).sum(0)
        feq[a] = lat.w[a] * rho * (1.0 + eu / CS2 + eu * eu / (2 * CS2 * CS2) - u2 / (2 * CS2))
    return feq


def moment_equilibrium(rho, u, pm, lat):
    """Improved equilibrium from its moments (the rule stated in the module docstring)."""
    A = monomial_matrix(lat)
    mons = moment_monomials(lat)
    b = torch.einsum("ka,a...->k...", A, textbook_equilibrium(rho, u, lat))
    dp = pm - rho * CS2
    for k, n in enumerate(mons):
        deg = sum(n)
        if deg == 2 and max(n) == 2:                       # e_i^2 : Eq. 25
            b[k] = b[k] + dp
        elif deg == 3:                                     # e_i e_j^2, i != j : Eq. 26
            i = n.index(1)
            b[k] = b[k] + dp * u[i]
        elif deg == 4:                                     # e_i^2 e_j^2 : as Eq. 27 on D2Q9
            b[k] = b[k] + dp * CS2
    return torch.einsum("ak,k...->a...", torch.linalg.inv(A), b)


def equilibrium(rho, u, pm, prm):
    lat = prm.lattice
    if lat.D == 2 and lat.Q == 9:
        Minv = d2q9_inverse_transformation_matrix()
        return torch.einsum("ak,k...->a...", Minv, d2q9_equilibrium_moments(rho, u, pm, prm.scheme))
    if prm.scheme == "standard":
        return textbook_equilibrium(rho, u, lat)
    return moment_equilibrium(rho, u, pm, lat)


# ----------------------------------------------------------------------------- collision, streaming

def collide(f, prm, fl=None):
    """Post-collision populations f*, Eq. 9 (standard) / Eq. 28 (improved)."""
    lat = prm.lattice
    if fl is None:
        fl = fields(f, prm)
    rho, u, F, pm = fl["rho"], fl["u"], fl["F"], fl["pm"]
    G = guo_forcing(u, F, lat)
    improved = prm.scheme == "improved"
    if lat.D == 2 and lat.Q == 9:
        M = d2q9_transformation_matrix()
        Minv = d2q9_inverse_transformation_matrix()
        s = torch.full((9,), 1.0 / prm.tau, dtype=DT) if prm.relaxation is None \
            else torch.tensor(list(prm.relaxation), dtype=DT)
        s = s.view((9,) + (1,) * rho.ndim)
        if prm.nu is not None:
            s = s.expand((9,) + tuple(rho.shape)).clone()
            if improved:
                tau_v = prm.nu * rho / pm + 0.5          # eta = p_m (tau_v - 1/2), nu = eta / rho
            else:
                tau_v = torch.full_like(rho, prm.nu / CS2 + 0.5)   # eta = rho c_s^2 (tau_v - 1/2)
            s[7] = 1.0 / tau_v
            s[8] = 1.0 / tau_v
        m = torch.einsum("ka,a...->k...", M, f)
        meq = d2q9_equilibrium_moments(rho, u, pm, prm.scheme)
        S = torch.einsum("ka,a...->k...", M, G)
        if improved:
            S = S + d2q9_correction_moments(correction_strengths(rho, u, pm, prm))
        mstar = m - s * (m - meq) + (1.0 - 0.5 * s) * S
        return torch.einsum("ak,k...->a...", Minv, mstar)
    if prm.relaxation is not None or prm.nu is not None:
        raise ValueError("relaxation vectors and nu are defined for D2Q9 only")
    feq = equilibrium(rho, u, pm, prm)
    src = G
    if improved:
        src = src + min_norm_correction(correction_strengths(rho, u, pm, prm), lat)
    om = 1.0 / prm.tau
    return f - om * (f - feq) + (1.0 - 0.5 * om) * src


def stream(fstar, lat):
    """Eq. 10: f_a(x + e_a) = f*_a(x) on a periodic lattice."""
    out = torch.empty_like(fstar)
    D = lat.D
    dims = tuple(range(1, 1 + D))
    for a in range(lat.Q):
        shifts = tuple(int(lat.e[a, D - 1 - k]) for k in range(D))
        out[a] = torch.roll(fstar[a], shifts=shifts, dims=tuple(d - 1 for d in dims))
    return out


def bounce_back(out, fstar, fl, prm):
    """Plates (see the module notes): replace the populations that streamed in from
    beyond a plate by the reversed ones of the same node plus the moving-wall term,
    evaluated with the node's rho and p_m of the collision (fields `fl`)."""
    lat = prm.lattice
    e = lat.e.tolist()
    for row, U in ((0, prm.walls[0]), (-1, prm.walls[1])):
        rho, pm = fl["rho"][row:row + 1 if row == 0 else None, :], fl["pm"][row:row + 1 if row == 0 else None, :]
        uw = torch.zeros((2,) + tuple(rho.shape), dtype=DT)
        uw[0] = U
        feq = equilibrium(rho, uw, pm, prm)
        into = 1 if row == 0 else -1          # e_y of the populations coming back from this plate
        for a in range(lat.Q):
            if e[a][1] == into:
                opp = e.index([-e[a][0], -e[a][1]])
                out[a, row, :] = fstar[opp, row, :] + (feq[a] - feq[opp])[0]
    return out


def step(f, prm):
    """One time step: returns f at t + 1 (post-streaming, pre-collision)."""
    fl = fields(f, prm)
    fstar = collide(f, prm, fl)
    out = stream(fstar, prm.lattice)
    if prm.walls is not None:
        out = bounce_back(out, fstar, fl, prm)
    return out


def run(f, prm, n):
    for _ in range(n):
        f = step(f, prm)
    return f


def init(rho0, prm, u0=None):
    """f(x, 0) = f_eq(rho0, u0) with the scheme's equilibrium (reading: the paper
    does not state its initial populations)."""
    lat = prm.lattice
    rho0 = rho0.to(DT)
    if u0 is None:
        u0 = torch.zeros((lat.D,) + tuple(rho0.shape), dtype=DT)
    if prm.scheme == "improved":
        pm = modified_pressure(chemical_potential(rho0, prm), prm.c0)
    else:
        pm = rho0 * CS2
    return equilibrium(rho0, u0, pm, prm)


def diagnostics(f, prm):
    """Mass, momentum sum(j + F/2), max |u|, min/max mu at the time level of f."""
    fl = fields(f, prm)
    mom = (fl["j"] + 0.5 * fl["F"]).reshape(prm.lattice.D, -1).sum(1)
    speed = torch.sqrt((fl["u"] * fl["u"]).sum(0))
    return {"mass": float(fl["rho"].sum()), "mom": [float(x) for x in mom],
            "max_u": float(speed.max()), "mu_min": float(fl["mu"].min()), "mu_max": float(fl["mu"].max())}
