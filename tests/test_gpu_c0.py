"""GPU step with the p_m offset p_m = (c0 + mu)/3 (c0 != 1 is an extension, not the
paper's method) against the oracle through the C ABI."""

import numpy as np
import pytest
import torch

from oracle import eos as oeos
from paper_2008_01473_amd import inputs
from parity_util import compare, oracle_run, rel_err

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2008_01473_amd import runtime  # noqa: E402  (raises if liblbm.so is missing)


def _droplet(shape, t, r):
    m = oeos.maxwell(oeos.make_eos("vdW"), t)
    return inputs.droplet(shape, m["rho_g"], m["rho_l"], r, 5.0, noise=1e-4, seed=3)


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_c0_fp64_droplet_at_low_temperature(lattice):
    shape = (45, 70) if lattice == "D2Q9" else (16, 18, 20)
    nx, ny = shape[-1], shape[-2]
    nz = 1 if lattice == "D2Q9" else shape[0]
    p = runtime.params(lattice, nx, ny, nz, T_over_Tc=0.7, kappa=0.02, tau=1.0, c0=0.6)
    rho0 = _droplet(shape, 0.7, 12.0 if lattice == "D2Q9" else 6.0)
    print(f"case {lattice} fp64 c0=0.6 T/Tc=0.7", flush=True)
    sim = runtime.LBM(p)
    sim.init(rho0)
    steps = (1, 10, 60) if lattice == "D2Q9" else (1, 8)
    refs = oracle_run(p, rho0, list(steps))
    t = 0
    for s in steps:
        sim.step(s - t)
        t = s
        compare(sim, p, refs[s])
    sim.close()


def test_c0_fp32_deviation_storage():
    shape = (45, 70)
    p = runtime.params("D2Q9", 70, 45, 1, T_over_Tc=0.7, kappa=0.02, tau=1.0, c0=0.6, precision="fp32")
    rho0 = _droplet(shape, 0.7, 12.0)
    sim = runtime.LBM(p)
    sim.init(rho0)
    sim.step(10)
    f_ref, fl = oracle_run(p, rho0, [10])[10]
    n = int(np.prod(shape))
    f = sim.get_f()[:, :n].reshape((-1,) + shape)
    rho, u, mu = sim.moments()
    errs = {"f": rel_err(f, f_ref), "rho": rel_err(rho.reshape(shape), fl["rho"]),
            "u_abs": float((u.reshape((-1,) + shape).cpu() - fl["u"]).abs().max())}
    print("fp32 c0 errors", errs, flush=True)
    assert errs["f"] < 2e-6 and errs["rho"] < 2e-6 and errs["u_abs"] < 2e-6
    sim.close()


def test_c0_zero_selects_the_paper():
    a = runtime.params("D2Q9", 24, 20, 1, c0=0.0)
    b = runtime.params("D2Q9", 24, 20, 1, c0=1.0)
    rho0 = _droplet((20, 24), 0.8, 5.0)
    out = []
    for p in (a, b):
        sim = runtime.LBM(p)
        sim.init(rho0)
        sim.step(5)
        out.append(sim.get_f().cpu())
        sim.close()
    assert torch.equal(out[0], out[1])
