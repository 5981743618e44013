"""GPU D2Q9 MRT collision (Eq. 8 relaxation matrix, Eq. 9 / Eq. 28) against the
oracle, element by element through the C ABI: float64 at 1e-12 per field for
every scheme variant with a fixed and a constant-viscosity shear rate, float32
deviation storage at float32 round-off, MRT and BGK lattices mixed in one batch,
and the unsupported combinations."""

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

VARIANTS = [("improved", "chempot"), ("standard", "chempot"), ("standard", "ptensor")]
MRT = dict(collision="mrt", tau_e=1.1, tau_s=1.3, tau_q=0.9)


def _droplet(shape, eos, t, r, noise=1e-4, seed=0):
    m = oeos.maxwell(oeos.make_eos(eos), t)
    return inputs.droplet(shape, m["rho_g"], m["rho_l"], r, 5.0, noise=noise, seed=seed)


@pytest.mark.parametrize("scheme,form", VARIANTS)
@pytest.mark.parametrize("nu", [0.0, 0.1])
def test_d2q9_mrt_fp64_ragged_droplet(scheme, form, nu):
    p = runtime.params("D2Q9", 70, 45, 1, eos="vdW", T_over_Tc=0.8, kappa=0.02, tau=0.8, scheme=scheme,
                       force_form=form, nu=nu, **MRT)
    rho0 = _droplet((45, 70), "vdW", 0.8, 12.0)
    print(f"case D2Q9 MRT fp64 {scheme}/{form} nu={nu} 70x45", flush=True)
    sim = runtime.LBM(p)
    sim.init(rho0)
    refs = oracle_run(p, rho0, [1, 10, 100])
    t = 0
    for s in (1, 10, 100):
        sim.step(s - t)
        t = s
        compare(sim, p, refs[s])
    sim.close()


def test_d2q9_mrt_moving_droplet_cs():
    """Carnahan-Starling droplet with a uniform initial velocity (u != 0 keeps every
    non-equilibrium moment and the correction term active), constant nu."""
    p = runtime.params("D2Q9", 48, 40, 1, eos="CS", T_over_Tc=0.8, kappa=0.02, tau=0.8, nu=0.05, **MRT)
    rho0 = _droplet((40, 48), "CS", 0.8, 9.0)
    u0 = np.zeros((2, 40, 48))
    u0[0], u0[1] = 0.05, -0.03
    print("case D2Q9 MRT fp64 CS moving droplet 48x40", flush=True)
    sim = runtime.LBM(p)
    sim.init(rho0, u0)
    sim.step(25)
    compare(sim, p, oracle_run(p, rho0, [25], u0=u0)[25])
    sim.close()


@pytest.mark.parametrize("scheme", ["improved", "standard"])
def test_d2q9_mrt_fp32_deviation_storage(scheme):
    shape = (45, 70)
    p = runtime.params("D2Q9", 70, 45, 1, T_over_Tc=0.8, kappa=0.02, tau=0.8, scheme=scheme, precision="fp32",
                       nu=0.1, **MRT)
    rho0 = _droplet(shape, "vdW", 0.8, 12.0)
    print(f"case D2Q9 MRT fp32 {scheme} 70x45", flush=True)
    sim = runtime.LBM(p)
    sim.init(rho0)
    sim.step(10)
    f_ref, fl = oracle_run(p, rho0, [10])[10]
    n = int(np.prod(shape))
    f = sim.get_f()[:, :n].reshape((-1,) + shape)
    rho, u, mu = sim.moments()
    errs = {"f": rel_err(f, f_ref), "rho": rel_err(rho.reshape(shape), fl["rho"]),
            "u_abs": float((u.reshape((-1,) + shape).cpu() - fl["u"]).abs().max()),
            "mu_abs": float((mu.reshape(shape).cpu() - fl["mu"]).abs().max())}
    print("fp32 MRT errors", errs, flush=True)
    assert errs["f"] < 2e-6 and errs["rho"] < 2e-6 and errs["u_abs"] < 2e-6 and errs["mu_abs"] < 2e-6
    sim.close()


def test_batch_mixes_mrt_and_bgk_lattices():
    specs = [dict(nx=40, ny=36, nu=0.1, **MRT), dict(nx=33, ny=50), dict(nx=64, ny=24, nu=0.0, **MRT)]
    plist, rhos = [], []
    for k, sp in enumerate(specs):
        nx, ny = sp.pop("nx"), sp.pop("ny")
        plist.append(runtime.params("D2Q9", nx, ny, 1, T_over_Tc=0.8, kappa=0.02, tau=0.8, **sp))
        rhos.append(_droplet((ny, nx), "vdW", 0.8, 7.0, seed=k))
    print("case batch of MRT and BGK lattices", flush=True)
    sim = runtime.LBM(plist)
    sim.init(np.concatenate([r.ravel() for r in rhos]))
    sim.step(12)
    for i, (p, r0) in enumerate(zip(plist, rhos)):
        compare(sim, p, oracle_run(p, r0, [12])[12], lat_index=i)
    sim.close()


def test_unsupported_mrt_combinations():
    L = runtime._lib
    with pytest.raises(L.LBMError) as e:
        runtime.LBM(runtime.params("D3Q19", 8, 8, 8, **MRT))
    assert e.value.code == L.LBM_ERR_UNSUPPORTED
    with pytest.raises(L.LBMError) as e:
        runtime.LBM(runtime.params("D2Q9", 16, 16, 1, collision="mrt", tau_e=0.5, tau_s=1.0, tau_q=1.0))
    assert e.value.code == L.LBM_ERR_ARG
    from paper_2008_01473_amd.adjoint import Rollout
    with pytest.raises(ValueError):
        Rollout(runtime.params("D2Q9", 16, 16, 1, **MRT))
