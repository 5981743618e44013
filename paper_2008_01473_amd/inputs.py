"""Seeded synthetic initial density fields.

These generators build the initial conditions of the paper's workloads and hold
none of the method's arithmetic: the coexistence densities, radius, widths and
seeds are all arguments.  Both the GPU path and its CPU checker receive the same
arrays from here.

* flat liquid slab (Sec. IV A): liquid between x = nx/4 and x = 3 nx/4, tanh
  edges of width W using the same 2(.)/W convention as Eq. 31;
* circular / spherical droplet (Sec. IV B, Eq. 31), centred at the middle of the
  domain, node coordinates x_i = i;
* optional i.i.d. uniform noise U(-amp, +amp) from numpy's default_rng(seed).

Arrays are float64, indexed [y, x] (2D) or [z, y, x] (3D), x fastest.
"""

import numpy as np


def _noise(shape, amplitude, seed):
    if amplitude == 0.0:
        return np.zeros(shape)
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, size=shape)


def slab(shape, rho_g, rho_l, width=4.0, noise=0.0, seed=0):
    """Flat interfaces normal to x at nx/4 and 3nx/4; `shape` = (ny, nx) or (nz, ny, nx)."""
    nx = shape[-1]
    x = np.arange(nx, dtype=np.float64)
    x1, x2 = 0.25 * nx, 0.75 * nx
    prof = rho_g + 0.5 * (rho_l - rho_g) * (np.tanh(2.0 * (x - x1) / width) - np.tanh(2.0 * (x - x2) / width))
    rho = np.broadcast_to(prof, shape).copy()
    return rho + _noise(shape, noise, seed)


def droplet(shape, rho_g, rho_l, radius, width=5.0, center=None, noise=0.0, seed=0):
    """Eq. 31 profile: (rho_l + rho_g)/2 - (rho_l - rho_g)/2 tanh(2 (r0 - r) / W) with r0 the
    distance to the centre (default: the middle of the domain, n_d / 2 per axis)."""
    D = len(shape)
    if center is None:
        center = tuple(0.5 * n for n in reversed(shape))   # (x0, y0[, z0])
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    r2 = np.zeros(shape)
    for k in range(D):                        # axis k holds component D-1-k
        r2 += (grids[k] - center[D - 1 - k]) ** 2
    r0 = np.sqrt(r2)
    rho = 0.5 * (rho_l + rho_g) - 0.5 * (rho_l - rho_g) * np.tanh(2.0 * (r0 - radius) / width)
    return rho + _noise(shape, noise, seed)


def uniform(shape, rho, noise=0.0, seed=0):
    return np.full(shape, float(rho)) + _noise(shape, noise, seed)


def batch_specs(count=96, seed=0, sizes=(64, 128, 256, 512), t_range=(0.5, 0.95),
                kappa_range=(0.005, 0.02)):
    """Seeded specification of a coexistence-curve sweep: square lattices with the
    side drawn uniformly from `sizes`, a flat slab or a droplet of radius 0.2 n with
    probability 1/2 each, T/Tc and kappa uniform in the given ranges."""
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(count):
        n = int(rng.choice(sizes))
        shape = "droplet" if rng.random() < 0.5 else "slab"
        specs.append({
            "n": n,
            "shape": shape,
            "T_over_Tc": float(rng.uniform(*t_range)),
            "kappa": float(rng.uniform(*kappa_range)),
            "seed": int(rng.integers(0, 2**31 - 1)),
        })
    return specs
