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


def _bench():
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location(
        "bench", os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    return bench


def test_c0_keeps_more_of_the_coexistence_sweep_healthy():
    """The 96-lattice sweep (T/Tc down to 0.5, kappa down to 0.005, float32) for 2e4
    steps: with the paper's c0 = 1, 60 lattices stay healthy (measured); with c0 = 0.4,
    77.  The healthy flat-interface lattices sit on the Maxwell construction to within
    5 % in the gas and 0.5 % in the liquid (measured 4.4 % and 0.48 % at most, the
    thinnest interfaces; the median is 0.1 %)."""
    bench = _bench()
    specs = inputs.batch_specs(96, 0)
    healthy = {}
    for c0 in (1.0, 0.4):
        spec = bench.batch_spec(runtime, inputs, c0=c0)
        print(f"case sweep c0={c0}", flush=True)
        sim = runtime.LBM(spec["params"])
        sim.init(spec["rho0"])
        sim.step(20000)
        rho, _, _ = sim.moments()
        diag = sim.diagnostics()
        healthy[c0] = sum(d["status"] == 0 for d in diag)
        if c0 != 1.0:
            offs = sim.offsets()
            dg, dl = [], []
            for i, (p, s) in enumerate(zip(spec["params"], specs)):
                if diag[i]["status"] or s["shape"] != "slab":
                    continue
                r = rho[offs[i]:offs[i] + p.nx * p.ny].view(p.ny, p.nx)
                m = oeos.maxwell(oeos.make_eos("vdW"), p.T_over_Tc)
                dg.append(abs(float(r[:, 0].mean()) / m["rho_g"] - 1))
                dl.append(abs(float(r[:, p.nx // 2].mean()) / m["rho_l"] - 1))
            print(f"  healthy slabs {len(dg)}: gas max {max(dg):.2e} median {np.median(dg):.2e}; "
                  f"liquid max {max(dl):.2e} median {np.median(dl):.2e}", flush=True)
            assert len(dg) >= 40
            assert max(dg) < 5e-2 and max(dl) < 5e-3
            assert np.median(dg) < 5e-3 and np.median(dl) < 1e-3
        sim.close()
    print(f"  healthy: {healthy}", flush=True)
    assert healthy[1.0] <= 64 and healthy[0.4] >= 74


@pytest.mark.parametrize("T", [0.6, 0.5])
def test_c0_does_not_stabilise_the_cs_droplet_below_0_7(T):
    """The 512^2 Carnahan-Starling droplet (kappa = 0.01, tau = 0.8) at T/Tc = 0.6 and
    0.5 blows up within 1e4 steps for every c0 tried (0.1 to 1; with c0 < |mu_sat| the
    gas p_m is negative), float64 as float32: flagged, as with the paper's c0 = 1."""
    m = oeos.maxwell(oeos.make_eos("CS"), T)
    rho0 = inputs.droplet((512, 512), m["rho_g"], m["rho_l"], 80.0, 5.0, noise=0.0)
    for c0 in (0.1, 0.3, 0.5):
        p = runtime.params("D2Q9", 512, 512, 1, eos="CS", T_over_Tc=T, kappa=0.01, tau=0.8, c0=c0)
        sim = runtime.LBM(p)
        sim.init(rho0)
        sim.step(10000)
        d = sim.diagnostics()[0]
        print(f"  T/Tc {T} c0 {c0}: status {d['status']}", flush=True)
        assert d["status"] != 0
        sim.close()
