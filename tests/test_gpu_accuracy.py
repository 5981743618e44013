"""Accuracy at the configurations' full lengths, on the GPU through the C ABI:

* the 256 x 4 flat interface after 20 000 steps: GPU = oracle on the
  translation-invariant quantities to round-off, whole fields to 1e-8 (the
  interface position random-walks at round-off level); the improved scheme sits on
  the discrete uniform-mu equilibrium (Newton), which on this thin interface lies
  0.85 % from Maxwell; the standard scheme's chemical potential is not uniform;
* float32 deviation storage against float64 at the configurations' lengths, with
  the gates of the benchmark's accuracy object (coexistence densities within 1e-4;
  spurious-current maxima within 5 % whenever float64's is above 1e-10, else float32
  at most 1e-5): the 512^2 Carnahan-Starling droplet after 50 000 steps in the
  improved scheme (densities pass; the spurious-current gate fails and is marked as
  an expected failure with the measured numbers) and in the standard scheme at
  T/Tc = 0.9 (all gates pass), the 256^3 D3Q19 droplet (T/Tc = 0.85) after 10 000
  steps (all gates pass); T/Tc = 0.6 and 0.5 blow up and are flagged.
"""

import numpy as np
import pytest
import torch

from oracle import discrete_equilibrium as de
from oracle import eos as oeos
from oracle.lattice import D2Q9
from paper_2008_01473_amd import inputs
from parity_util import compare, oracle_run

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2008_01473_amd import runtime  # noqa: E402  (raises if liblbm.so is missing)


@pytest.mark.parametrize("scheme", ["improved", "standard"])
def test_flat_interface_config_at_20000_steps(scheme):
    E = oeos.make_eos("vdW", 9.0 / 49.0)
    m = oeos.maxwell(E, 0.9)
    p = runtime.params("D2Q9", 256, 4, 1, eos="vdW", a=9.0 / 49.0, T_over_Tc=0.9, kappa=0.01, tau=1.0,
                       scheme=scheme)
    rho0 = inputs.slab((4, 256), m["rho_g"], m["rho_l"], 4.0, noise=1e-4, seed=0)
    print(f"case 256x4 slab {scheme}, 20000 steps", flush=True)
    sim = runtime.LBM(p)
    sim.init(rho0)
    sim.step(20000)
    f_ref, fl = oracle_run(p, rho0, [20000])[20000]
    # The flat interface can translate at no cost (the discrete equilibrium is unique
    # only up to translation), so round-off differences random-walk its position:
    # whole fields agree to ~3e-10 after 2e4 steps (1e-12 holds through step 1000,
    # test_gpu_parity); translation-invariant quantities agree to round-off.
    compare(sim, p, (f_ref, fl), f_tol=1e-8, fields_tol=1e-8)
    rho, u, mu = sim.moments()
    ref_rho = fl["rho"].numpy()
    assert float(rho.min()) == pytest.approx(float(ref_rho.min()), rel=1e-11)
    assert float(rho.max()) == pytest.approx(float(ref_rho.max()), rel=1e-11)
    assert float(mu.mean()) == pytest.approx(float(fl["mu"].mean()), rel=1e-11, abs=1e-13)
    rho = rho.view(4, 256).cpu().numpy()
    rg, rl = rho.min(), rho.max()
    dev = max(abs(rg / m["rho_g"] - 1), abs(rl / m["rho_l"] - 1))
    print(f"  rho_g {rg:.7f} (Maxwell {m['rho_g']:.7f}), rho_l {rl:.7f} (Maxwell {m['rho_l']:.7f}), "
          f"max rel dev {dev:.2e}, mu spread {float(mu.max() - mu.min()):.2e}", flush=True)
    if scheme == "improved":
        rn, _, res = de.solve(rho, E, 0.9 * E.Tc, 0.01, D2Q9)
        assert res < 1e-12
        # still relaxing after 2e4 steps: mu spread 2e-8, and the largest distance to the
        # Newton profile (3e-7) sits in the interface, where d rho/dx ~ 1 per node
        assert np.abs(rho - rn).max() < 1e-6
        assert float(mu.max() - mu.min()) < 1e-7
        # a = 9/49, kappa = 0.01 make the interface thin (sqrt(kappa/a) ~ 0.23 nodes against
        # ~0.9 at the paper's a = 9/392, kappa = 0.02, whose Table II agreement the oracle's
        # pins cover): the discrete equilibrium itself sits 0.85 % from Maxwell here
        assert dev < 1.5e-2
    else:
        assert float(mu.max() - mu.min()) > 1e-4
    sim.close()


def _bench():
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location(
        "bench", os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    return bench


_CASES = {}


def _case(name):
    """float64 and float32 runs of one accuracy workload, with the benchmark's gates
    (computed once per test session)."""
    if name not in _CASES:
        bench = _bench()
        c = (slice(246, 266), slice(246, 266))
        g = (slice(0, 20), slice(0, 20))
        if name == "c2_improved":
            fn = lambda p: bench.primary_spec(runtime, inputs, precision=p)            # noqa: E731
            _CASES[name] = bench.run_accuracy_case(torch, runtime, fn, 50000, (512, 512), c, g)
        elif name == "c2_standard":
            fn = lambda p: bench.primary_spec(runtime, inputs, precision=p, scheme="standard", T=0.9)  # noqa: E731
            _CASES[name] = bench.run_accuracy_case(torch, runtime, fn, 50000, (512, 512), c, g)
        else:
            fn = lambda p: bench.d3q19_spec(runtime, inputs, precision=p)              # noqa: E731
            _CASES[name] = bench.run_accuracy_case(torch, runtime, fn, 10000, (256, 256, 256),
                                                   (slice(120, 136),) * 3, (slice(0, 16),) * 3)
        a = _CASES[name]
        print(f"  {name}: fp64 {a['fp64']}\n  fp32 {a['fp32']}\n  gates {a['gates']}", flush=True)
    return _CASES[name]


def _c2(precision, T=0.8, steps=50000):
    m = oeos.maxwell(oeos.make_eos("CS"), T)
    p = runtime.params("D2Q9", 512, 512, 1, eos="CS", T_over_Tc=T, kappa=0.01, tau=0.8, precision=precision)
    rho0 = inputs.droplet((512, 512), m["rho_g"], m["rho_l"], 80.0, 5.0, noise=0.0)
    sim = runtime.LBM(p)
    sim.init(rho0)
    sim.step(steps)
    d = sim.diagnostics()[0]
    sim.close()
    return {"status": d["status"], "max_u": d["max_u"]}, m


def test_c2_improved_fp32_coexistence_densities_and_mass():
    """512^2 CS droplet, improved scheme, 5e4 steps: float32 densities within 1e-4 of
    float64 (measured ~2e-7); float64 conserves mass to round-off, float32 keeps the
    float32 representation of the initial state (-4e-8, constant after step 0)."""
    a = _case("c2_improved")
    assert a["fp64"]["status"] == 0 and a["fp32"]["status"] == 0
    assert a["gates"]["rho_l"] and a["gates"]["rho_g"]
    assert abs(a["fp64"]["mass_drift"]) < 1e-10
    assert abs(a["fp32"]["mass_drift"]) < 1e-7
    # the droplet's densities stay near the Maxwell values (Laplace pressure and kappa = 0.01 shift them)
    m = oeos.maxwell(oeos.make_eos("CS"), 0.8)
    assert a["fp64"]["rho_l"] == pytest.approx(m["rho_l"], rel=2e-2)
    assert a["fp64"]["rho_g"] == pytest.approx(m["rho_g"], rel=5e-2)


@pytest.mark.xfail(strict=True, reason=(
    "measured: after 5e4 steps float64's spurious maximum is 2.1e-8 and still decaying, float32's 7-8e-7 (~35x); "
    "float32 storage alone leaves 2.5e-7 (measured with float64 arithmetic on the same float32 state), so the 5 % "
    "gate cannot be met by float32 storage on this workload"))
def test_c2_improved_fp32_spurious_current_gate():
    a = _case("c2_improved")
    assert a["gates"]["max_u"], a["gates"]


def test_c2_improved_fp32_spurious_current_floor():
    """What float32 does reach on that workload: below 1.5e-6 (measured 7-8e-7 with
    the float32 arithmetic in deviation form; 2.9e-6 with plain float32 arithmetic)."""
    a = _case("c2_improved")
    assert a["fp32"]["max_u"] < 1.5e-6


def test_c2_standard_fp32_gates():
    """The standard scheme's spurious currents are O(1e-4): every gate passes (T/Tc = 0.9,
    where this droplet is stable in the standard scheme)."""
    a = _case("c2_standard")
    assert a["fp64"]["status"] == 0 and a["fp32"]["status"] == 0
    assert a["gates"]["all"], a["gates"]
    assert a["fp64"]["max_u"] > 1e-5


def test_c3_d3q19_fp32_gates():
    """The 256^3 D3Q19 droplet at T/Tc = 0.85 (the benchmark's 3D workload; 0.7 blows
    up within ~50 steps and 0.8 after ~4000 at this size, float32 and float64 alike),
    10 000 steps: float32 against float64 passes every gate; mass drift of float32 is
    the representation of its initial state; densities within 2 % (liquid) and 5 %
    (gas) of Maxwell."""
    a = _case("c3_d3q19")
    assert a["fp64"]["status"] == 0 and a["fp32"]["status"] == 0
    assert a["gates"]["all"], a["gates"]
    assert abs(a["fp32"]["mass_drift"]) < 1e-7 and abs(a["fp64"]["mass_drift"]) < 1e-10
    assert a["fp64"]["max_u"] < 1e-3
    m = oeos.maxwell(oeos.make_eos("vdW"), 0.85)
    assert a["fp32"]["rho_l"] == pytest.approx(m["rho_l"], rel=2e-2)
    assert a["fp32"]["rho_g"] == pytest.approx(m["rho_g"], rel=5e-2)


@pytest.mark.parametrize("T", [0.6, 0.5])
def test_c2_droplet_blows_up_and_is_flagged_at_low_temperature(T):
    """The stability warning: at T/Tc = 0.6 and 0.5 the improved scheme's gas rest
    population is negative; the run blows up and the lattice is flagged and frozen."""
    out, _ = _c2("fp64", T=T, steps=5000)
    print(f"  T/Tc {T}: status {out['status']}", flush=True)
    assert out["status"] != 0
