"""Helpers of the GPU-vs-oracle parity tests: build matching oracle parameters,
run the oracle, compare fields with the relative error of a field,
    err_X = max |X_gpu - X_oracle| / max(max |X_oracle|, floor_X).
Floors: u = 1e-2, mu = 1e-3, none for populations and rho.  The velocity is a
first moment of populations of size O(rho/9), so its rounding error follows the
populations' (absolute, in lattice units) whatever |u| is; once the improved
scheme has damped |u| a relative bar on u alone would tighten without limit.
With the floor, |u| < 1e-2 is held to 1e-14 absolute (lattice units).
"""

import numpy as np
import torch

from oracle import eos as oeos
from oracle import model

EOS_NAMES = {0: "vdW", 1: "CS"}


def oracle_params(p):
    """Oracle Params equivalent to a ctypes lbm_params record."""
    E = oeos.make_eos(EOS_NAMES[p.eos], p.a, p.b, p.R)
    relaxation, nu = None, None
    if p.collision == 1:            # MRT: Eq. 8 rates in the order of M's rows, tau_c = 1
        relaxation = [1.0, 1 / p.tau_e, 1 / p.tau_s, 1.0, 1 / p.tau_q, 1.0, 1 / p.tau_q, 1 / p.tau, 1 / p.tau]
        nu = p.nu if p.nu > 0 else None
    return model.Params(lattice="D2Q9" if p.lattice == 0 else "D3Q19", eos=E, T_over_Tc=p.T_over_Tc,
                        kappa=p.kappa, tau=p.tau, scheme="improved" if p.scheme == 1 else "standard",
                        force_form="ptensor" if p.force_form == 1 else "chempot", relaxation=relaxation, nu=nu,
                        walls=(p.wall_u_bottom, p.wall_u_top) if p.walls else None, c0=p.c0 if p.c0 > 0 else 1.0)


def shape_of(p):
    return (p.ny, p.nx) if p.lattice == 0 else (p.nz, p.ny, p.nx)


def rel_err(gpu, ref, floor=0.0):
    g = torch.as_tensor(gpu).detach().cpu().to(torch.float64)
    r = torch.as_tensor(ref).detach().cpu().to(torch.float64)
    scale = max(float(r.abs().max()), floor)
    return float((g - r).abs().max()) / scale if scale > 0 else float((g - r).abs().max())


def oracle_run(p, rho0, steps_list, u0=None):
    """Run the oracle from rho0 and return {steps: (f, fields)} at each requested step."""
    prm = oracle_params(p)
    shape = shape_of(p)
    r0 = torch.as_tensor(np.asarray(rho0, dtype=np.float64)).reshape(shape)
    u = None if u0 is None else torch.as_tensor(np.asarray(u0, dtype=np.float64)).reshape((-1,) + shape)
    f = model.init(r0, prm, u)
    out, t = {}, 0
    for s in sorted(steps_list):
        f = model.run(f, prm, s - t)
        t = s
        out[s] = (f.clone(), model.fields(f, prm))
    return out


def compare(sim, p, ref, lat_index=0, f_tol=1e-12, fields_tol=1e-12, u_floor=1e-2):
    """Compare populations and fields of lattice `lat_index` of `sim` against an
    oracle (f, fields) pair.  Returns the dict of relative errors."""
    f_ref, fl = ref
    shape = shape_of(p)
    n = int(np.prod(shape))
    off = sim.offsets()[lat_index]
    f = sim.get_f()[:, off:off + n].reshape((-1,) + shape)
    rho, u, mu = sim.moments()
    rho = rho[off:off + n].reshape(shape)
    u = u[:, off:off + n].reshape((-1,) + shape)
    mu = mu[off:off + n].reshape(shape)
    errs = {"f": rel_err(f, f_ref), "rho": rel_err(rho, fl["rho"]), "u": rel_err(u, fl["u"], u_floor),
            "mu": rel_err(mu, fl["mu"], 1e-3)}
    assert errs["f"] <= f_tol, errs
    for k in ("rho", "u", "mu"):
        assert errs[k] <= fields_tol, errs
    return errs
