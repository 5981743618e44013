"""Per-lattice diagnostics of the GPU path (lbm_diagnostics: mass, momentum
sum (j + F/2) = sum rho u, max |u|, mu_min, mu_max; Eq. 12 and Eq. 2) against the
oracle's diagnostics of the same time level, for single lattices and batches, with
a translating droplet so that the momentum is not trivially zero.

Bar (float64): mass, mu_min, mu_max to 1e-12 relative; each momentum component to
1e-12 of sum |rho u| (a component may cancel to near zero); max |u| to 1e-12 with
the velocity floor of the field parity tests (1e-2, u's rounding is absolute).
Float32 storage: to the float32 parity bars of the populations (2e-5 relative)."""

import math

import numpy as np
import pytest
import torch

from oracle import model
from paper_2008_01473_amd import inputs
from parity_util import oracle_params, shape_of

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2008_01473_amd import _lib, runtime  # noqa: E402
from oracle import eos as oeos  # noqa: E402


def _inputs(p, radius, seed):
    shape = shape_of(p)
    E = oeos.make_eos("vdW" if p.eos == 0 else "CS", p.a, p.b, p.R)
    m = oeos.maxwell(E, p.T_over_Tc)
    rho0 = inputs.droplet(shape, m["rho_g"], m["rho_l"], radius, 5.0, noise=1e-4, seed=seed)
    u0 = np.zeros((len(shape),) + shape)
    u0[0] = 0.04
    u0[1] = -0.015
    if len(shape) == 3:
        u0[2] = 0.01
    return rho0, u0


def _oracle_diag(p, rho0, u0, steps):
    prm = oracle_params(p)
    f = model.init(torch.as_tensor(rho0), prm, torch.as_tensor(u0))
    out, t = {}, 0
    for s in sorted(steps):
        f = model.run(f, prm, s - t)
        t = s
        fl = model.fields(f, prm)
        d = model.diagnostics(f, prm)
        d["mom_scale"] = float((fl["rho"] * fl["u"].abs()).sum())
        out[s] = d
    return out


def _check(got, ref, tol, label):
    print(f"{label}: mass {got['mass']:.15e} vs {ref['mass']:.15e}; mom {got['mom']} vs {ref['mom']}; "
          f"max_u {got['max_u']:.6e} vs {ref['max_u']:.6e}; mu [{got['mu_min']:.9e}, {got['mu_max']:.9e}] vs "
          f"[{ref['mu_min']:.9e}, {ref['mu_max']:.9e}]", flush=True)
    assert got["status"] == 0
    assert abs(got["mass"] - ref["mass"]) <= tol * abs(ref["mass"])
    for k, r in enumerate(ref["mom"]):
        assert abs(got["mom"][k] - r) <= tol * ref["mom_scale"]
    assert abs(got["max_u"] - ref["max_u"]) <= tol * max(ref["max_u"], 1e-2)
    for key in ("mu_min", "mu_max"):
        assert abs(got[key] - ref[key]) <= tol * max(abs(ref[key]), 1e-3)


_REFS = {}


def _run_and_check(plist, radii, n, tol, prec_label, tile=None):
    sim = runtime.LBM(plist)
    if tile is not None:
        try:
            sim.set_tile_shape(tile)
        except _lib.LBMError as e:
            sim.close()
            if e.code == _lib.LBM_ERR_UNSUPPORTED:
                pytest.skip(f"tile shape {tile} refused for this lattice: {e}")
            raise
    rho_all, u_all, refs = [], [], []
    for i, p in enumerate(plist):
        rho0, u0 = _inputs(p, radii[i], seed=i)
        rho_all.append(rho0.reshape(-1))
        u_all.append(u0.reshape(len(u0), -1))
        key = (prec_label, i, n)
        if key not in _REFS:
            _REFS[key] = _oracle_diag(p, rho0, u0, [n - 1, n])
        refs.append(_REFS[key])
    D = sim.D
    u_cat = np.concatenate([np.concatenate([u[k] for u in u_all]) for k in range(D)])
    sim.init(np.concatenate(rho_all), u_cat)
    sim.step(n)
    torch.cuda.synchronize()
    got = sim.diagnostics()             # the input time level of the last step: n - 1
    for i, p in enumerate(plist):
        assert got[i]["step"] == n - 1
        _check(got[i], refs[i][n - 1], tol, f"{prec_label} lattice {i} t={n - 1}")
    sim.moments()                        # refreshes the diagnostics at the current level n
    got = sim.diagnostics()
    for i, p in enumerate(plist):
        assert got[i]["step"] == n
        _check(got[i], refs[i][n], tol, f"{prec_label} lattice {i} t={n}")
    sim.close()


@pytest.mark.parametrize("scheme,form", [("improved", "chempot"), ("standard", "chempot"), ("standard", "ptensor")])
def test_d2q9_single_lattice_diagnostics(scheme, form):
    p = runtime.params("D2Q9", 70, 37, 1, eos="CS", T_over_Tc=0.85, kappa=0.02, tau=0.8, scheme=scheme,
                       force_form=form)
    _run_and_check([p], [9.0], 6, 1e-12, f"D2Q9 {scheme}/{form}")


_D2Q9_SHAPES = 12


def test_d2q9_tile_shape_count():
    p = runtime.params("D2Q9", 16, 16, 1)
    sim = runtime.LBM([p])
    assert sim.num_tile_shapes() == _D2Q9_SHAPES
    sim.close()


@pytest.mark.parametrize("tile", range(_D2Q9_SHAPES))
@pytest.mark.parametrize("scheme,form", [("improved", "chempot"), ("standard", "chempot"), ("standard", "ptensor")])
def test_d2q9_diagnostics_every_tile_shape(scheme, form, tile):
    """Every tile shape reduces the diagnostics of its own tiling: one node per
    thread, two nodes per thread, and two threads per node (where the helper
    threads take the float64 diagnostics from LDS)."""
    p = runtime.params("D2Q9", 70, 37, 1, eos="CS", T_over_Tc=0.85, kappa=0.02, tau=0.8, scheme=scheme,
                       force_form=form)
    _run_and_check([p], [9.0], 6, 1e-12, f"D2Q9 {scheme}/{form}", tile=tile)


@pytest.mark.parametrize("tile", range(_D2Q9_SHAPES))
def test_d2q9_batch_with_mrt_and_plates_diagnostics_every_tile_shape(tile):
    """A launch whose lattices use the MRT collision and plates carries both
    features' code: the diagnostics of each lattice through every tile shape."""
    plist = [runtime.params("D2Q9", 48, 40, 1, eos="vdW", T_over_Tc=0.8, kappa=0.02, tau=1.0),
             runtime.params("D2Q9", 64, 64, 1, eos="vdW", T_over_Tc=0.75, kappa=0.018, tau=1.0, collision="mrt",
                            tau_e=0.9, tau_s=1.1, tau_q=1.2),
             runtime.params("D2Q9", 45, 37, 1, eos="vdW", T_over_Tc=0.8, kappa=0.02, tau=0.8,
                            walls=(-0.03, 0.03))]
    _run_and_check(plist, [8.0, 12.0, 7.0], 5, 1e-12, "D2Q9 batch mrt+plates", tile=tile)


@pytest.mark.parametrize("scheme", ["improved", "standard"])
def test_d3q19_single_lattice_diagnostics(scheme):
    p = runtime.params("D3Q19", 20, 18, 22, eos="vdW", T_over_Tc=0.85, kappa=0.02, tau=1.0, scheme=scheme)
    _run_and_check([p], [5.0], 5, 1e-12, f"D3Q19 {scheme}")


def test_d2q9_batch_diagnostics():
    plist = [runtime.params("D2Q9", 48, 40, 1, eos="vdW", T_over_Tc=0.8, kappa=0.02, tau=1.0),
             runtime.params("D2Q9", 33, 70, 1, eos="vdW", T_over_Tc=0.9, kappa=0.012, tau=0.9),
             runtime.params("D2Q9", 64, 64, 1, eos="vdW", T_over_Tc=0.75, kappa=0.018, tau=1.0, collision="mrt",
                            tau_e=0.9, tau_s=1.1, tau_q=1.2)]
    _run_and_check(plist, [8.0, 7.0, 12.0], 5, 1e-12, "D2Q9 batch")


def test_d3q19_batch_diagnostics():
    plist = [runtime.params("D3Q19", 16, 18, 20, eos="vdW", T_over_Tc=0.85, kappa=0.02, tau=1.0),
             runtime.params("D3Q19", 21, 12, 17, eos="vdW", T_over_Tc=0.9, kappa=0.015, tau=0.9)]
    _run_and_check(plist, [4.5, 4.0], 4, 1e-12, "D3Q19 batch")


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_fp32_storage_diagnostics(lattice):
    """Float32 deviation storage: the diagnostics track the float64 oracle to the
    float32 bar of the population parity tests (the sums themselves are float64)."""
    if lattice == "D2Q9":
        p = runtime.params("D2Q9", 70, 37, 1, eos="vdW", T_over_Tc=0.85, kappa=0.02, tau=1.0, precision="fp32")
        r = 9.0
    else:
        p = runtime.params("D3Q19", 20, 18, 22, eos="vdW", T_over_Tc=0.85, kappa=0.02, tau=1.0, precision="fp32")
        r = 5.0
    _run_and_check([p], [r], 4, 2e-5, f"{lattice} fp32")
    assert math.isfinite(r)


def _next_supported_shape(sim):
    cur = _lib.lib().lbm_get_tile_shape(sim.h)
    for k in range(1, sim.num_tile_shapes()):
        try:
            sim.set_tile_shape((cur + k) % sim.num_tile_shapes())
            return
        except _lib.LBMError as e:
            assert e.code == _lib.LBM_ERR_UNSUPPORTED


@pytest.mark.parametrize("lattice,graphs", [("D2Q9", True), ("D2Q9", False), ("D3Q19", True)])
def test_diagnostics_after_steps_read_the_last_input(lattice, graphs):
    """After lbm_step(n) the diagnostics are reduced from the last step's input,
    which the second buffer holds: bit for bit those lbm_moments gives on a copy
    stepped n - 1 times, for odd and even n, and after a change of tile shape
    between the steps and the call."""
    if lattice == "D2Q9":
        p = runtime.params("D2Q9", 70, 37, 1, eos="CS", T_over_Tc=0.85, kappa=0.02, tau=0.8)
        r = 9.0
    else:
        p = runtime.params("D3Q19", 20, 18, 22, eos="vdW", T_over_Tc=0.85, kappa=0.02, tau=1.0)
        r = 5.0
    rho0, u0 = _inputs(p, r, seed=5)
    for n in (5, 6):
        for retile in (False, True):
            print(f"case {lattice} graphs={graphs} n={n} retile={retile}", flush=True)
            a, b = runtime.LBM([p]), runtime.LBM([p])
            for sim in (a, b):
                sim.use_graphs(graphs)
                sim.init(rho0.reshape(-1), u0.reshape(len(u0), -1).reshape(-1))
            a.step(n)
            if retile:
                _next_supported_shape(a)
            b.set_tile_shape(_lib.lib().lbm_get_tile_shape(a.h))
            b.step(n - 1)
            b.moments()
            da, db = a.diagnostics(), b.diagnostics()
            assert da[0]["step"] == db[0]["step"] == n - 1
            assert repr(da) == repr(db)
            a.close()
            b.close()


def test_diagnostics_owed_by_steps_use_the_physics_of_those_steps():
    """A change of kappa and T/Tc between lbm_step and lbm_diagnostics does not
    reach the diagnostics of the last step's input: they are those of a copy
    stepped with the old physics and read out before any change."""
    p = runtime.params("D2Q9", 70, 37, 1, eos="CS", T_over_Tc=0.85, kappa=0.02, tau=0.8)
    rho0, u0 = _inputs(p, 9.0, seed=7)
    a, b = runtime.LBM([p]), runtime.LBM([p])
    for sim in (a, b):
        sim.init(rho0.reshape(-1), u0.reshape(-1))
    b.set_tile_shape(_lib.lib().lbm_get_tile_shape(a.h))
    a.step(6)
    _lib.check(_lib.lib().lbm_set_physics(a.h, 0, 0.03, 0.9), "lbm_set_physics")
    da = a.diagnostics()
    b.step(5)
    b.moments()
    db = b.diagnostics()
    assert da[0]["step"] == db[0]["step"] == 5
    assert repr(da) == repr(db)
    a.close()
    b.close()
