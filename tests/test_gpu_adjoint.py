"""Hand-written adjoint on the GPU vs autograd of the float64 CPU oracle, vs central
finite differences of the GPU forward, and the dot-product identity."""

import ctypes
import math

import numpy as np
import pytest
import torch

from oracle import eos as oeos
from oracle import model
from paper_2008_01473_amd import inputs
from parity_util import EOS_NAMES, rel_err, shape_of

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2008_01473_amd import _lib, runtime  # noqa: E402
from paper_2008_01473_amd.adjoint import Rollout, rollout  # noqa: E402


def _oracle_params(p, kappa, T):
    E = oeos.make_eos(EOS_NAMES[p.eos], p.a, p.b, p.R)
    return model.Params(lattice="D2Q9", eos=E, T_over_Tc=T, kappa=kappa, tau=p.tau,
                        scheme="improved" if p.scheme == 1 else "standard", c0=p.c0 if p.c0 > 0 else 1.0)


def _case(scheme, n=(20, 24), T=0.8, kappa=0.02, tau=0.8, seed=0, c0=1.0):
    ny, nx = n
    p = runtime.params("D2Q9", nx, ny, 1, eos="vdW", T_over_Tc=T, kappa=kappa, tau=tau, scheme=scheme, c0=c0)
    m = oeos.maxwell(oeos.VanDerWaals(), T)
    rho0 = inputs.droplet((ny, nx), m["rho_g"], m["rho_l"], 5.0, 5.0, noise=1e-3, seed=seed)
    return p, rho0


@pytest.mark.parametrize("scheme,c0,n", [("improved", 1.0, (20, 24)), ("standard", 1.0, (20, 24)),
                                         ("improved", 0.7, (20, 24)),
                                         # several 32 x 8 tiles, ragged in both directions
                                         ("improved", 1.0, (19, 70)), ("standard", 1.0, (19, 70))])
def test_adjoint_step_matches_oracle_autograd(scheme, c0, n):
    p, rho0 = _case(scheme, n=n, c0=c0)
    shape = shape_of(p)
    kap = torch.tensor(0.02, dtype=torch.float64, requires_grad=True)
    tt = torch.tensor(0.8, dtype=torch.float64, requires_grad=True)
    prm = _oracle_params(p, kap, tt)
    with torch.no_grad():
        f = model.run(model.init(torch.as_tensor(rho0), _oracle_params(p, 0.02, 0.8)), _oracle_params(p, 0.02, 0.8), 3)
    lam = torch.randn((9,) + shape, dtype=torch.float64, generator=torch.Generator().manual_seed(1))
    fv = f.clone().requires_grad_(True)
    out = model.step(fv, prm)
    gf, gk, gt = torch.autograd.grad(out, [fv, kap, tt], grad_outputs=lam)

    roll = Rollout(p)
    sim = roll.sim
    sim.set_f(f.reshape(9, -1))
    state, _ = sim.get_state()
    lam_d = lam.reshape(-1).cuda().contiguous()
    lam_out = torch.empty_like(lam_d)
    grad = torch.zeros(2, dtype=torch.float64, device="cuda")
    L = _lib.lib()
    _lib.check(L.lbm_adjoint_step(sim.h, state.data_ptr(), lam_d.data_ptr(), lam_out.data_ptr(),
                                  roll.ws.data_ptr(), grad.data_ptr()))
    torch.cuda.synchronize()
    e = rel_err(lam_out.view(9, *shape), gf)
    print(f"adjoint step {scheme} {n}: rel err lambda {e:.2e}, kappa {float(grad[0]):.6e} vs {float(gk):.6e}, "
          f"T {float(grad[1]):.6e} vs {float(gt):.6e}", flush=True)
    assert e < 1e-12
    assert float(grad[0]) == pytest.approx(float(gk), rel=1e-10, abs=1e-14)
    assert float(grad[1]) == pytest.approx(float(gt), rel=1e-10, abs=1e-14)
    roll.close()


@pytest.mark.parametrize("scheme", ["improved", "standard"])
def test_rollout_gradients_match_oracle_autograd(scheme):
    """dL/drho0, dL/dkappa, dL/d(T/Tc) through 30 steps with checkpoints every 6
    steps; L = sum (rho_N - rho*)^2 + sum |u_N|^2."""
    p, rho0 = _case(scheme, n=(24, 28))
    shape = shape_of(p)
    n_steps = 30
    g = np.random.default_rng(3)
    target = torch.as_tensor(rho0 + 0.05 * g.uniform(-1, 1, size=shape))
    # oracle (float64 CPU autograd)
    r0 = torch.as_tensor(rho0).clone().requires_grad_(True)
    kap = torch.tensor(0.02, dtype=torch.float64, requires_grad=True)
    tt = torch.tensor(0.8, dtype=torch.float64, requires_grad=True)
    prm = _oracle_params(p, kap, tt)
    f = model.run(model.init(r0, prm), prm, n_steps)
    fl = model.fields(f, prm)
    loss = ((fl["rho"] - target) ** 2).sum() + (fl["u"] ** 2).sum()
    g_r0, g_k, g_t = torch.autograd.grad(loss, [r0, kap, tt])
    # GPU
    roll = Rollout(p)
    r0d = torch.as_tensor(rho0).reshape(-1).cuda().requires_grad_(True)
    kd = torch.tensor(0.02, dtype=torch.float64, device="cuda", requires_grad=True)
    td = torch.tensor(0.8, dtype=torch.float64, device="cuda", requires_grad=True)
    rho, u = roll.forward(r0d.detach(), 0.02, 0.8, n_steps, checkpoint_every=6)
    rho_n, u_n = rollout(r0d, kd, td, roll, n_steps)
    lossd = ((rho_n - target.reshape(-1).cuda()) ** 2).sum() + (u_n ** 2).sum()
    lossd.backward()
    assert float(lossd) == pytest.approx(float(loss), rel=1e-12)
    e = rel_err(r0d.grad.view(shape), g_r0)
    print(f"rollout {scheme}: dL/drho0 rel err {e:.2e}; kappa {float(kd.grad):.8e} vs {float(g_k):.8e}; "
          f"T {float(td.grad):.8e} vs {float(g_t):.8e}", flush=True)
    assert e < 1e-10
    assert float(kd.grad) == pytest.approx(float(g_k), rel=1e-9)
    assert float(td.grad) == pytest.approx(float(g_t), rel=1e-9)
    roll.close()


def test_rollout_gradients_match_central_differences():
    """Improved scheme, 40 steps: the adjoint gradients against central finite
    differences (h = 1e-6) of the GPU float64 forward, for kappa, T/Tc, eight
    seeded components of rho0 (two of them in the interface) and one random
    direction in rho0."""
    p, rho0 = _case("improved", n=(32, 32))
    n_steps = 40
    target = torch.as_tensor(rho0).reshape(-1).cuda() * 1.01
    roll = Rollout(p)

    def loss_at(r0, k, t):
        rho, u = roll.forward(r0, k, t, n_steps)
        return float(((rho - target) ** 2).sum() + (u ** 2).sum())

    r0d = torch.as_tensor(rho0).reshape(-1).cuda().requires_grad_(True)
    kd = torch.tensor(0.02, dtype=torch.float64, device="cuda", requires_grad=True)
    td = torch.tensor(0.8, dtype=torch.float64, device="cuda", requires_grad=True)
    rho_n, u_n = rollout(r0d, kd, td, roll, n_steps)
    (((rho_n - target) ** 2).sum() + (u_n ** 2).sum()).backward()
    h = 1e-6
    base = torch.as_tensor(rho0).reshape(-1).cuda()
    fd_k = (loss_at(base, 0.02 + h, 0.8) - loss_at(base, 0.02 - h, 0.8)) / (2 * h)
    fd_t = (loss_at(base, 0.02, 0.8 + h) - loss_at(base, 0.02, 0.8 - h)) / (2 * h)
    v = torch.as_tensor(np.random.default_rng(5).standard_normal(base.numel())).cuda()
    fd_v = (loss_at(base + h * v, 0.02, 0.8) - loss_at(base - h * v, 0.02, 0.8)) / (2 * h)
    ad_v = float((r0d.grad * v).sum())
    print(f"FD: kappa {fd_k:.8e} vs {float(kd.grad):.8e}; T {fd_t:.8e} vs {float(td.grad):.8e}; "
          f"dir {fd_v:.8e} vs {ad_v:.8e}", flush=True)
    assert float(kd.grad) == pytest.approx(fd_k, rel=1e-5)
    assert float(td.grad) == pytest.approx(fd_t, rel=1e-5)
    assert ad_v == pytest.approx(fd_v, rel=1e-5)
    # eight seeded components of rho0: six drawn uniformly, two on the interface
    # ring (where the gradient is largest and least linear)
    n = base.numel()
    comps = [int(i) for i in np.random.default_rng(7).choice(n, 6, replace=False)]
    yy, xx = np.divmod(np.arange(n), 32)
    ring = np.flatnonzero(np.abs(np.hypot(xx - 16.0, yy - 16.0) - 5.0) < 0.5)
    comps += [int(i) for i in np.random.default_rng(8).choice(ring, 2, replace=False)]
    g_r0 = r0d.grad.detach().cpu()
    for i in comps:
        e = torch.zeros(n, dtype=torch.float64, device="cuda")
        e[i] = 1.0
        fd_i = (loss_at(base + h * e, 0.02, 0.8) - loss_at(base - h * e, 0.02, 0.8)) / (2 * h)
        print(f"FD: rho0[{i}] {fd_i:.8e} vs {float(g_r0[i]):.8e}", flush=True)
        # absolute floor: components far from the droplet carry tiny gradients whose
        # central difference is limited by the loss's rounding (~1e-16 L / h)
        assert float(g_r0[i]) == pytest.approx(fd_i, rel=1e-5, abs=1e-7)
    roll.close()


def test_second_backward_after_a_physics_change():
    """One Rollout runs forward and backward at kappa = 0.02, then forward and
    backward at kappa = 0.025, T/Tc = 0.82 on the same buffers (segment graphs
    on): the second gradients equal, bit for bit, those of a fresh Rollout at the
    new parameters."""
    p, rho0 = _case("improved", n=(24, 28))
    n_steps = 24
    target = torch.as_tensor(rho0).reshape(-1).cuda() * 1.01

    def grads(roll, k, t):
        r0 = torch.as_tensor(rho0).reshape(-1).cuda().requires_grad_(True)
        kd = torch.tensor(k, dtype=torch.float64, device="cuda", requires_grad=True)
        td = torch.tensor(t, dtype=torch.float64, device="cuda", requires_grad=True)
        rho_n, u_n = rollout(r0, kd, td, roll, n_steps)
        (((rho_n - target) ** 2).sum() + (u_n ** 2).sum()).backward()
        torch.cuda.synchronize()
        return r0.grad.clone(), kd.grad.clone(), td.grad.clone()

    roll = Rollout(p)
    roll.sim.use_graphs(True)
    g_first = grads(roll, 0.02, 0.8)
    g_second = grads(roll, 0.025, 0.82)
    roll.close()
    fresh = Rollout(p)
    fresh.sim.use_graphs(True)
    g_fresh = grads(fresh, 0.025, 0.82)
    fresh.close()
    print(f"second backward: dkappa {float(g_second[1]):.10e} fresh {float(g_fresh[1]):.10e} "
          f"first {float(g_first[1]):.10e}", flush=True)
    assert not torch.equal(g_first[1], g_second[1])
    for a, b in zip(g_second, g_fresh):
        assert torch.equal(a, b)


def test_adjoint_dot_product_identity():
    """<lam, J v> = <J^T lam, v> for one improved step, J v by central differences
    of the GPU float64 step."""
    p, rho0 = _case("improved")
    roll = Rollout(p)
    sim = roll.sim
    sim.init(rho0)
    sim.step(2)
    f0 = sim.get_f().clone()
    g = torch.Generator().manual_seed(9)
    v = torch.randn(f0.shape, dtype=torch.float64, generator=g).cuda() * 1e-2
    lam = torch.randn(f0.shape, dtype=torch.float64, generator=g).cuda()
    eps = 1e-6

    def step_from(f):
        sim.set_f(f)
        sim.step(1)
        return sim.get_f().clone()

    jv = (step_from(f0 + eps * v) - step_from(f0 - eps * v)) / (2 * eps)
    sim.set_f(f0)
    state, _ = sim.get_state()
    out = torch.empty(lam.numel(), dtype=torch.float64, device="cuda")
    grad = torch.zeros(2, dtype=torch.float64, device="cuda")
    L = _lib.lib()
    _lib.check(L.lbm_adjoint_step(sim.h, state.data_ptr(), lam.reshape(-1).contiguous().data_ptr(),
                                  out.data_ptr(), roll.ws.data_ptr(), grad.data_ptr()))
    lhs = float((lam * jv).sum())
    rhs = float((out.view_as(v) * v).sum())
    assert lhs == pytest.approx(rhs, rel=1e-7)
    roll.close()


def test_adjoint_rejects_unsupported_handles():
    p = runtime.params("D3Q19", 8, 8, 8)
    sim = runtime.LBM(p)
    assert _lib.lib().lbm_adjoint_workspace_bytes(sim.h) == 0
    with pytest.raises(ValueError):
        Rollout(p)
    sim.close()


def _c5_inputs():
    """256 x 256 droplet r = 40, vdW T/Tc = 0.75, kappa = 0.02, tau = 1.0; target
    density = the same droplet plus 0.01 (rho_l - rho_g) U(-1, 1) noise (seed 11)."""
    m = oeos.maxwell(oeos.VanDerWaals(), 0.75)
    rho0 = inputs.droplet((256, 256), m["rho_g"], m["rho_l"], 40.0, 5.0, noise=1e-4, seed=0)
    rng = np.random.default_rng(11)
    target = inputs.droplet((256, 256), m["rho_g"], m["rho_l"], 40.0, 5.0) + \
        0.01 * (m["rho_l"] - m["rho_g"]) * rng.uniform(-1, 1, size=(256, 256))
    return rho0, target


def test_full_size_adjoint_config_against_finite_differences():
    """The 256^2, 4000-step adjoint configuration: FP32-forward adjoint gradients
    (sqrt(N) = 64-step checkpoints) against central differences h = 1e-6 of the
    float64 forward; the float64-forward adjoint is held to a tight bar."""
    rho0, target = _c5_inputs()
    n_steps = 4000
    tgt = torch.as_tensor(target).reshape(-1).cuda()
    base = torch.as_tensor(rho0).reshape(-1).cuda()
    v = torch.as_tensor(np.random.default_rng(5).standard_normal(base.numel())).cuda()
    grads = {}
    for prec in ("fp64", "fp32"):
        p = runtime.params("D2Q9", 256, 256, 1, eos="vdW", T_over_Tc=0.75, kappa=0.02, tau=1.0, scheme="improved",
                           precision=prec)
        roll = Rollout(p)
        r0 = base.clone().requires_grad_(True)
        kd = torch.tensor(0.02, dtype=torch.float64, device="cuda", requires_grad=True)
        td = torch.tensor(0.75, dtype=torch.float64, device="cuda", requires_grad=True)
        rho_n, u_n = rollout(r0, kd, td, roll, n_steps)
        (((rho_n - tgt) ** 2).sum() + (u_n ** 2).sum()).backward()
        grads[prec] = (float(kd.grad), float(td.grad), float((r0.grad * v).sum()))
        if prec == "fp64":
            def loss_at(r, k, t):
                rho, u = roll.forward(r, k, t, n_steps)
                return float(((rho - tgt) ** 2).sum() + (u ** 2).sum())
            h = 1e-6
            fd = ((loss_at(base, 0.02 + h, 0.75) - loss_at(base, 0.02 - h, 0.75)) / (2 * h),
                  (loss_at(base, 0.02, 0.75 + h) - loss_at(base, 0.02, 0.75 - h)) / (2 * h),
                  (loss_at(base + h * v, 0.02, 0.75) - loss_at(base - h * v, 0.02, 0.75)) / (2 * h))
        roll.close()
    errs64 = [abs(a - b) / abs(b) for a, b in zip(grads["fp64"], fd)]
    errs32 = [abs(a - b) / abs(b) for a, b in zip(grads["fp32"], fd)]
    print(f"C5 FD {fd}\n fp64 adjoint {grads['fp64']} rel {errs64}\n fp32 adjoint {grads['fp32']} rel {errs32}",
          flush=True)
    assert max(errs64) < 1e-5
    assert max(errs32) < 1e-2


@pytest.mark.parametrize("m,graphs", [(1, True), (5, True), (5, False)])
def test_adjoint_segment_equals_step_by_step(m, graphs):
    """lbm_adjoint_segment (restore, recompute m states, m adjoint steps) gives
    the same lambda and parameter gradients as doing it call by call, bit for bit,
    launched eagerly or replayed from its captured graph (second call), and
    leaves the handle at time level t0 + m with that state."""
    p, rho0 = _case("improved")
    roll = Rollout(p)
    sim = roll.sim
    sim.use_graphs(graphs)
    L = _lib.lib()
    sim.init(rho0)
    sim.step(3)
    ck, t0 = sim.get_state()
    lam0 = torch.randn(9 * sim.N, dtype=torch.float64, generator=torch.Generator().manual_seed(5)).cuda()
    # call by call
    sim.set_state(ck, t0)
    seg = []
    for _ in range(m):
        seg.append(sim.get_state()[0])
        sim.step(1)
    lam, lam2 = lam0.clone(), torch.empty_like(lam0)
    g1 = torch.zeros(2, dtype=torch.float64, device="cuda")
    for s in reversed(seg):
        _lib.check(L.lbm_adjoint_step(sim.h, s.data_ptr(), lam.data_ptr(), lam2.data_ptr(), roll.ws.data_ptr(),
                                      g1.data_ptr()))
        lam, lam2 = lam2, lam
    end_state = sim.get_state()[0].clone()
    # one call, twice on the same buffers (the second replays the captured graph)
    states = torch.empty(m * sim.state_bytes, dtype=torch.uint8, device="cuda")
    lam_b, lam_b2 = torch.empty_like(lam0), torch.empty_like(lam0)
    g2 = torch.zeros(2, dtype=torch.float64, device="cuda")
    for rep in range(2):
        print(f"case adjoint segment m={m} graphs={graphs} call {rep}", flush=True)
        lam_b.copy_(lam0)
        g2.zero_()
        _lib.check(L.lbm_adjoint_segment(sim.h, ck.data_ptr(), t0, m, states.data_ptr(), lam_b.data_ptr(),
                                         lam_b2.data_ptr(), roll.ws.data_ptr(), g2.data_ptr()))
        torch.cuda.synchronize()
        assert torch.equal(lam_b, lam)
        assert torch.equal(g1, g2)
        assert sim.time == t0 + m
        assert torch.equal(sim.get_state()[0], end_state)
    roll.close()


@pytest.mark.parametrize("graphs", [True, False])
def test_adjoint_sweep_equals_segment_by_segment(graphs):
    """lbm_adjoint_sweep (every segment in one call, the recomputation of segment i
    on a second stream overlapping the adjoint steps of segment i+1, two arenas)
    gives the lambda and parameter gradients of lbm_adjoint_segment called segment
    by segment in reverse, bit for bit: three segments of 4, 4 and 3 steps, eager
    and from captured graphs, twice on the same buffers (the second call replays),
    and leaves the handle's state and time level unchanged."""
    p, rho0 = _case("improved")
    roll = Rollout(p)
    sim = roll.sim
    sim.use_graphs(graphs)
    L = _lib.lib()
    sim.init(rho0)
    ms = [4, 4, 3]
    t0s, cks = [], []
    for m in ms:
        ck, t = sim.get_state()
        t0s.append(t)
        cks.append(ck.clone())
        sim.step(m)
    end_state, t_end = sim.get_state()
    end_state = end_state.clone()
    lam0 = torch.randn(9 * sim.N, dtype=torch.float64, generator=torch.Generator().manual_seed(7)).cuda()
    # segment by segment
    states = torch.empty(max(ms) * sim.state_bytes, dtype=torch.uint8, device="cuda")
    lam, lam2 = lam0.clone(), torch.empty_like(lam0)
    g1 = torch.zeros(2, dtype=torch.float64, device="cuda")
    for ck, t0, m in reversed(list(zip(cks, t0s, ms))):
        _lib.check(L.lbm_adjoint_segment(sim.h, ck.data_ptr(), t0, m, states.data_ptr(), lam.data_ptr(),
                                         lam2.data_ptr(), roll.ws.data_ptr(), g1.data_ptr()))
    torch.cuda.synchronize()
    sim.set_state(end_state, t_end)
    # one sweep call, twice on the same buffers
    arenas = torch.empty(2 * max(ms) * sim.state_bytes, dtype=torch.uint8, device="cuda")
    lam_b, lam_b2 = torch.empty_like(lam0), torch.empty_like(lam0)
    g2 = torch.zeros(2, dtype=torch.float64, device="cuda")
    n = len(ms)
    ptrs = (ctypes.c_void_p * n)(*[c.data_ptr() for c in cks])
    for rep in range(2):
        print(f"case adjoint sweep graphs={graphs} call {rep}", flush=True)
        lam_b.copy_(lam0)
        g2.zero_()
        _lib.check(L.lbm_adjoint_sweep(sim.h, ptrs, (ctypes.c_longlong * n)(*t0s), (ctypes.c_int * n)(*ms), n,
                                       arenas.data_ptr(), lam_b.data_ptr(), lam_b2.data_ptr(), roll.ws.data_ptr(),
                                       g2.data_ptr()))
        torch.cuda.synchronize()
        assert torch.equal(lam_b, lam)
        assert torch.equal(g1, g2)
        assert sim.time == t_end
        assert torch.equal(sim.get_state()[0], end_state)
    roll.close()
