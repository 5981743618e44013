"""Accuracy at the configurations' full lengths, on the GPU through the C ABI:

* the 256 x 4 flat interface after 20 000 steps: GPU = oracle on the
  translation-invariant quantities to round-off, whole fields to 1e-8 (the
  interface position random-walks at round-off level); the improved scheme sits on
  the discrete uniform-mu equilibrium (Newton), which on this thin interface lies
  0.85 % from Maxwell; the standard scheme's chemical potential is not uniform;
* the 512^2 Carnahan-Starling droplet after 50 000 steps: float32 deviation storage
  against float64 -- coexistence densities within 1e-4, spurious currents within 5 %
  or, below float32's resolution (1e-5), at that floor; mass drift;
  T/Tc = 0.6 and 0.5 blow up and are flagged;
* the 256^3 D3Q19 droplet (T/Tc = 0.85) after 10 000 float32 steps stays healthy.
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


def _c2(precision, T=0.8, steps=50000):
    m = oeos.maxwell(oeos.make_eos("CS"), T)
    p = runtime.params("D2Q9", 512, 512, 1, eos="CS", T_over_Tc=T, kappa=0.01, tau=0.8, precision=precision)
    rho0 = inputs.droplet((512, 512), m["rho_g"], m["rho_l"], 80.0, 5.0, noise=0.0)
    sim = runtime.LBM(p)
    sim.init(rho0)
    sim.step(steps)
    rho, u, _ = sim.moments()
    d = sim.diagnostics()[0]
    out = {"status": d["status"], "max_u": d["max_u"], "mass": d["mass"], "mass0": float(rho0.sum())}
    if d["status"] == 0:
        r = rho.view(512, 512).cpu().numpy()
        out["rho_l"] = float(r[246:266, 246:266].mean())     # droplet centre
        out["rho_g"] = float(r[:20, :20].mean())             # far corner
    sim.close()
    return out, m


def test_c2_droplet_fp32_matches_fp64_after_50000_steps():
    a, m = _c2("fp64")
    b, _ = _c2("fp32")
    print(f"  fp64: rho_l {a['rho_l']:.8f} rho_g {a['rho_g']:.8f} max_u {a['max_u']:.3e} "
          f"mass drift {a['mass'] / a['mass0'] - 1:.2e}", flush=True)
    print(f"  fp32: rho_l {b['rho_l']:.8f} rho_g {b['rho_g']:.8f} max_u {b['max_u']:.3e} "
          f"mass drift {b['mass'] / b['mass0'] - 1:.2e}", flush=True)
    print(f"  Maxwell: rho_l {m['rho_l']:.8f} rho_g {m['rho_g']:.8f}", flush=True)
    assert a["status"] == 0 and b["status"] == 0
    assert b["rho_l"] == pytest.approx(a["rho_l"], rel=1e-4)
    assert b["rho_g"] == pytest.approx(a["rho_g"], rel=1e-4)
    # float32 storage resolves velocities down to ~5e-6 here: the 5 % rule applies to
    # float64 maxima above that floor, below it float32 must stay at the floor
    if a["max_u"] > 1e-5:
        assert b["max_u"] == pytest.approx(a["max_u"], rel=0.05)
    else:
        assert b["max_u"] <= 1e-5
    assert abs(a["mass"] / a["mass0"] - 1) < 1e-10     # round-off accumulated over 5e4 steps
    assert abs(b["mass"] / b["mass0"] - 1) < 1e-7      # float32: one rounding of f0 per node and step
    # the droplet's densities stay near the Maxwell values (Laplace pressure and kappa = 0.01 shift them)
    assert a["rho_l"] == pytest.approx(m["rho_l"], rel=2e-2)
    assert a["rho_g"] == pytest.approx(m["rho_g"], rel=5e-2)


@pytest.mark.parametrize("T", [0.6, 0.5])
def test_c2_droplet_blows_up_and_is_flagged_at_low_temperature(T):
    """The stability warning: at T/Tc = 0.6 and 0.5 the improved scheme's gas rest
    population is negative; the run blows up and the lattice is flagged and frozen."""
    out, _ = _c2("fp64", T=T, steps=5000)
    print(f"  T/Tc {T}: status {out['status']}", flush=True)
    assert out["status"] != 0


def test_c3_d3q19_fp32_10000_steps_stays_healthy():
    """At T/Tc = 0.85 (the benchmark's 3D workload); 0.7 blows up within ~50 steps
    and 0.8 after ~4000 at this size, float32 and float64 alike."""
    m = oeos.maxwell(oeos.make_eos("vdW"), 0.85)
    p = runtime.params("D3Q19", 256, 256, 256, eos="vdW", T_over_Tc=0.85, kappa=0.02, tau=1.0, precision="fp32")
    rho0 = inputs.droplet((256, 256, 256), m["rho_g"], m["rho_l"], 40.0, 5.0, noise=0.0)
    print("case 256^3 D3Q19 fp32, 10000 steps", flush=True)
    sim = runtime.LBM(p)
    sim.init(rho0)
    sim.step(10000)
    rho, _, _ = sim.moments()
    d = sim.diagnostics()[0]
    drift = d["mass"] / float(rho0.sum()) - 1
    r = rho.view(256, 256, 256)
    rl, rg = float(r[120:136, 120:136, 120:136].mean()), float(r[:16, :16, :16].mean())
    print(f"  status {d['status']} max_u {d['max_u']:.3e} mass drift {drift:.2e} rho_l {rl:.6f} rho_g {rg:.6f}",
          flush=True)
    assert d["status"] == 0
    assert abs(drift) < 1e-7
    assert d["max_u"] < 1e-3
    assert rl == pytest.approx(m["rho_l"], rel=2e-2) and rg == pytest.approx(m["rho_g"], rel=5e-2)
    sim.close()
