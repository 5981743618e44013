"""Throughput benchmark of the fused free-energy LB step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-secondary] [--no-cpu-baseline] [--no-accuracy]

Primary workload (the metric's configuration): D2Q9 512 x 512 periodic lattice,
Carnahan-Starling droplet of radius 80 at T/Tc = 0.8, kappa = 0.01, tau = 0.8,
improved scheme, float64.  One step = one fused kernel launch over the lattice
(pull streaming, rho, mu, forces, correction, collision).  `value` is million
lattice updates per second over exactly K timed steps (inputs resident in HBM).

`roofline`: algorithmic HBM bytes of the step kernel (read and write each
population once: 2 * Q * word bytes per node) divided by the kernel's average
duration from HIP events recorded on the launch stream, against 8 TB/s.
`traffic` is the HBM bytes per launch that rocprofv3 counted (FETCH_SIZE +
WRITE_SIZE, scaled by a copy-kernel calibration) for this workload and tile
shape, read from the `traffic-record:` lines of profiles/*.md; null when no
record matches the current kernel sources (SHA-256 over the csrc directory).
`cpu_baseline`: the CPU oracle on a bounded number of steps of the same lattice.
`secondary`: the same measurement for FP32 deviation storage, the MRT collision
at constant viscosity, moving plates, the p_m offset at T/Tc = 0.7, the standard
scheme, the 256^3 D3Q19 droplet, 4096^2 lattices and a batched coexistence
sweep, plus the adjoint's cost.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline: FP64 plain vs FP32/batched/adjoint, same accuracy"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2008_01473_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


def kernel_sources_sha256():
    """Hash of every source the step kernels and their tiling are built from; a
    counter record taken on other sources no longer describes these kernels."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def traffic_records():
    """`traffic-record:` lines of the committed rocprofv3 summaries: HBM bytes per
    launch from FETCH_SIZE and WRITE_SIZE, already scaled by the copy-kernel
    calibration factors."""
    recs = []
    if not os.path.isdir(PROFILES):
        return recs
    for name in sorted(os.listdir(PROFILES)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(PROFILES, name)) as fh:
            for line in fh:
                if line.startswith("traffic-record:"):
                    recs.append(json.loads(line.split(":", 1)[1]))
    return recs


def traffic_for(name, tile, sha, recs):
    for r in recs:
        if r["workload"] == name and list(r["tile"]) == list(tile) and r["sources_sha256"] == sha:
            return r["fetch_bytes"] + r["write_bytes"]
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default="", help="comma list of secondary names to run")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-graphs", action="store_true", help="one kernel launch per step (for counter runs)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile shape (no autotuning)")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the 5e4-step float32/float64 accuracy runs")
    ap.add_argument("--tile", type=int, default=-1, help="force this tile-shape index (no autotuning)")
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="only run the plain copy kernel on this many MiB, 5 times (traffic-counter calibration)")
    return ap.parse_args()


def timed_steps(torch, sim, steps, warmup):
    """Warm up, capture graphs outside the timed region, then time exactly `steps`
    steps with HIP events on the launch stream.  Returns ms per step."""
    sim.step(warmup)
    sim.prepare(steps)
    torch.cuda.synchronize()
    s = sim.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    sim.step(steps)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def measure(torch, runtime, inputs, spec, steps, warmup, graphs=True, tune=0, tile=-1):
    """Build one workload, time it, return a result record.  A workload with a
    `settle` count first runs that many steps and reads the diagnostics, so that
    lattices that blow up early have left the plan before tuning and timing."""
    p_list, rho0 = spec["params"], spec["rho0"]
    sim = runtime.LBM(p_list)
    sim.use_graphs(graphs)
    sim.init(rho0)
    live0 = len(p_list)
    if spec.get("settle", 0):
        sim.step(spec["settle"])
        live0 = sum(d["status"] == 0 for d in sim.diagnostics())
    if tile >= 0:
        sim.set_tile_shape(tile)
    elif tune:
        sim.autotune(tune)          # times every tile shape (and store mode) on this state, keeps the fastest
    shape = sim.tile_shape()
    stores = sim.store_mode()
    ms = timed_steps(torch, sim, steps, warmup)
    Q = sim.Q
    word = 8 if p_list[0].precision == 0 else 4
    diag = sim.diagnostics()
    # lattices that blew up are frozen by the kernel: count only the live ones
    live = [d["status"] == 0 for d in diag]
    blown = len(live) - sum(live)
    nodes = sum(p.nx * p.ny * p.nz for p, ok in zip(p_list, live) if ok)
    bytes_per_launch = 2 * Q * word * nodes
    achieved = bytes_per_launch / (ms * 1e-3) / 1e9
    extra = spec["post"](sim, diag) if spec.get("post") else {}
    sim.close()
    return {**extra, 
        "name": spec["name"],
        "workload": spec["workload"],
        "mlups": nodes / (ms * 1e-3) / 1e6,
        "ms_per_step": ms,
        "nodes": nodes,
        "bytes_per_lup": 2 * Q * word,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS},
        "tile": list(shape),
        "stores": stores,
        "blown_up_lattices": blown,
        "live_lattices_at_start": live0,
        "max_u": max(d["max_u"] for d in diag),
    }


def primary_spec(runtime, inputs, precision="fp64", scheme="improved", T=0.8):
    m = runtime.maxwell("CS", T)
    p = runtime.params("D2Q9", 512, 512, 1, eos="CS", T_over_Tc=T, kappa=0.01, tau=0.8, scheme=scheme,
                       precision=precision)
    rho0 = inputs.droplet((512, 512), m["rho_g"], m["rho_l"], 80.0, 5.0, noise=0.0)
    return {"name": f"d2q9_512_cs_{scheme}_{precision}", "params": [p], "rho0": rho0,
            "workload": f"D2Q9 512x512 periodic, Carnahan-Starling droplet r=80 W=5, T/Tc={T}, kappa=0.01, "
                        f"tau=0.8, {scheme} scheme, {precision}"}


def mrt_spec(runtime, inputs, nu=0.15):
    """The primary's droplet with the MRT collision of Eq. 8 at constant kinematic
    viscosity nu (Fig. 1 uses 0.15 and 0.03); tau_e = tau_s = tau_q = 1."""
    m = runtime.maxwell("CS", 0.8)
    p = runtime.params("D2Q9", 512, 512, 1, eos="CS", T_over_Tc=0.8, kappa=0.01, tau=0.8, collision="mrt",
                       tau_e=1.0, tau_s=1.0, tau_q=1.0, nu=nu)
    rho0 = inputs.droplet((512, 512), m["rho_g"], m["rho_l"], 80.0, 5.0, noise=0.0)
    return {"name": "d2q9_512_cs_improved_mrt_fp64", "params": [p], "rho0": rho0,
            "workload": f"D2Q9 512x512 periodic, Carnahan-Starling droplet r=80 W=5, T/Tc=0.8, kappa=0.01, improved "
                        f"scheme, MRT (Eq. 8) tau_e = tau_s = tau_q = 1, constant nu = {nu}, fp64"}


def plates_spec(runtime, inputs):
    """The primary's droplet in a channel: plates at y = -1/2 and 511.5 moving at
    +0.05 and -0.05 along x (halfway bounce-back), improved scheme, fp64."""
    m = runtime.maxwell("CS", 0.8)
    p = runtime.params("D2Q9", 512, 512, 1, eos="CS", T_over_Tc=0.8, kappa=0.01, tau=0.8, walls=(-0.05, 0.05))
    rho0 = inputs.droplet((512, 512), m["rho_g"], m["rho_l"], 80.0, 5.0, noise=0.0)
    return {"name": "d2q9_512_cs_improved_plates_fp64", "params": [p], "rho0": rho0,
            "workload": "D2Q9 512x512, periodic in x, plates moving at -0.05 / +0.05 bounding y, Carnahan-Starling "
                        "droplet r=80 W=5, T/Tc=0.8, kappa=0.01, tau=0.8, improved scheme, fp64"}


def c0_spec(runtime, inputs):
    """vdW droplet at T/Tc = 0.7 with the p_m offset c0 = 0.6 (an extension that keeps
    the gas rest population positive; the paper's c0 = 1 blows up here), fp64."""
    m = runtime.maxwell("vdW", 0.7)
    p = runtime.params("D2Q9", 512, 512, 1, eos="vdW", T_over_Tc=0.7, kappa=0.02, tau=1.0, c0=0.6)
    rho0 = inputs.droplet((512, 512), m["rho_g"], m["rho_l"], 80.0, 5.0, noise=0.0)
    return {"name": "d2q9_512_vdw_improved_c0_fp64", "params": [p], "rho0": rho0,
            "workload": "D2Q9 512x512 periodic, van der Waals droplet r=80 W=5, T/Tc=0.7, kappa=0.02, tau=1, "
                        "improved scheme with p_m = (0.6 + mu)/3, fp64"}


def d2q9_large_spec(runtime, inputs, precision="fp64", n=4096):
    """The primary's physics on a lattice large enough to leave the launch-latency
    regime: n x n CS droplet of radius 80 n / 512."""
    m = runtime.maxwell("CS", 0.8)
    p = runtime.params("D2Q9", n, n, 1, eos="CS", T_over_Tc=0.8, kappa=0.01, tau=0.8, scheme="improved",
                       precision=precision)
    rho0 = inputs.droplet((n, n), m["rho_g"], m["rho_l"], 80.0 * n / 512, 5.0, noise=0.0)
    return {"name": f"d2q9_{n}_cs_improved_{precision}", "params": [p], "rho0": rho0,
            "workload": f"D2Q9 {n}x{n} periodic, CS droplet r={80 * n // 512}, T/Tc=0.8, kappa=0.01, tau=0.8, "
                        f"improved, {precision}"}


def d3q19_spec(runtime, inputs, T=0.85, precision="fp32"):
    # At T/Tc = 0.7 this droplet blows up within ~50 steps (the oracle too): the
    # rest population rho - 2 p_m of the gas is negative; at 0.8 it blows up after
    # ~4000 steps (float32 and float64 alike).  The kernel does the same work at any
    # temperature, so throughput is timed at T/Tc = 0.85, stable over 10^4 steps.
    m = runtime.maxwell("vdW", T)
    p = runtime.params("D3Q19", 256, 256, 256, eos="vdW", T_over_Tc=T, kappa=0.02, tau=1.0,
                       scheme="improved", precision=precision)
    rho0 = inputs.droplet((256, 256, 256), m["rho_g"], m["rho_l"], 40.0, 5.0, noise=0.0)
    storage = "fp32 deviation storage" if precision == "fp32" else "fp64"
    return {"name": f"d3q19_256_vdw_improved_{precision}", "params": [p], "rho0": rho0,
            "workload": f"D3Q19 256^3 periodic, vdW droplet r=40 W=5, T/Tc={T}, kappa=0.02, tau=1.0, improved, "
                        f"{storage}"}


def d3q19_shard_spec(runtime, inputs, T=0.85):
    """One GPU's share of the 256^3 droplet split into 8 slabs along z: 256 x 256 x 32,
    the slab through the droplet's centre, periodic in z (standing in for the
    neighbours' faces; the face exchange itself is not part of a one-GPU step)."""
    m = runtime.maxwell("vdW", T)
    p = runtime.params("D3Q19", 256, 256, 32, eos="vdW", T_over_Tc=T, kappa=0.02, tau=1.0,
                       scheme="improved", precision="fp32")
    rho0 = inputs.droplet((256, 256, 256), m["rho_g"], m["rho_l"], 40.0, 5.0, noise=0.0)[112:144].copy()
    return {"name": "d3q19_256x256x32_shard_fp32", "params": [p], "rho0": rho0,
            "workload": f"D3Q19 256x256x32 (one of 8 z-slabs of the 256^3 vdW droplet, periodic in z), T/Tc={T}, "
                        "kappa=0.02, tau=1.0, improved, fp32 deviation storage"}


def batch_spec(runtime, inputs, count=96, seed=0, c0=1.0):
    specs = inputs.batch_specs(count, seed)
    ps, rhos = [], []
    for s in specs:
        n = s["n"]
        m = runtime.maxwell("vdW", s["T_over_Tc"])
        ps.append(runtime.params("D2Q9", n, n, 1, eos="vdW", T_over_Tc=s["T_over_Tc"], kappa=s["kappa"],
                                 tau=1.0, scheme="improved", precision="fp32", c0=c0))
        if s["shape"] == "droplet":
            rhos.append(inputs.droplet((n, n), m["rho_g"], m["rho_l"], 0.2 * n, 5.0, noise=1e-4, seed=s["seed"]))
        else:
            rhos.append(inputs.slab((n, n), m["rho_g"], m["rho_l"], 4.0, noise=1e-4, seed=s["seed"]))
    # the lattices below T/Tc ~ 0.6 blow up within the first ~2000 steps (the
    # improved scheme's stability limit); timing starts once they have been frozen
    out = {"name": "batch96_d2q9_fp32", "params": ps, "rho0": np.concatenate([r.ravel() for r in rhos]),
           "settle": 3000,
           "workload": f"{count} D2Q9 lattices n in {{64,128,256,512}} (seed {seed}), slabs/droplets, "
                       "T/Tc in [0.5,0.95], kappa in [0.005,0.02], tau=1.0, improved, fp32, one launch per step; "
                       "timed after 3000 settling steps, blown-up lattices frozen and not counted"}
    if c0 != 1.0:
        # the p_m offset (not the paper's method): more of the sweep stays healthy;
        # the record adds the healthy count and the healthy slabs' bulk densities
        # against the Maxwell construction
        out["name"] = f"batch96_d2q9_fp32_c0_{c0:g}"
        out["settle"] = 20000
        out["workload"] = out["workload"].replace("improved,", f"improved with p_m = ({c0:g} + mu)/3,").replace(
            "3000 settling", "20000 settling")

        def post(sim, diag):
            rho = sim.moments()[0]
            offs = sim.offsets()
            dev_g, dev_l = [], []
            for i, (p, sp) in enumerate(zip(ps, specs)):
                if diag[i]["status"] or sp["shape"] != "slab":
                    continue
                r = rho[offs[i]:offs[i] + p.nx * p.ny].view(p.ny, p.nx)
                mm = runtime.maxwell("vdW", p.T_over_Tc)
                dev_g.append(abs(float(r[:, 0].mean()) / mm["rho_g"] - 1))
                dev_l.append(abs(float(r[:, p.nx // 2].mean()) / mm["rho_l"] - 1))
            return {"c0": c0, "healthy_lattices": sum(d["status"] == 0 for d in diag),
                    "healthy_slabs": len(dev_g), "slab_rho_g_vs_maxwell_max": max(dev_g, default=None),
                    "slab_rho_l_vs_maxwell_max": max(dev_l, default=None),
                    "slab_rho_g_vs_maxwell_median": float(np.median(dev_g)) if dev_g else None,
                    "slab_rho_l_vs_maxwell_median": float(np.median(dev_l)) if dev_l else None}
        out["post"] = post
    return out


def adjoint_measure(torch, runtime, inputs, n_steps=4000):
    """256 x 256 vdW droplet (r = 40, T/Tc = 0.75, kappa = 0.02, tau = 1.0), FP32
    forward with sqrt(N) checkpoints, loss sum (rho_N - rho*)^2 + sum |u_N|^2:
    times the forward and the backward (recompute + adjoint) passes."""
    from paper_2008_01473_amd.adjoint import Rollout, rollout

    m = runtime.maxwell("vdW", 0.75)
    rho0 = inputs.droplet((256, 256), m["rho_g"], m["rho_l"], 40.0, 5.0, noise=1e-4, seed=0)
    rng = np.random.default_rng(11)
    target = inputs.droplet((256, 256), m["rho_g"], m["rho_l"], 40.0, 5.0) + \
        0.01 * (m["rho_l"] - m["rho_g"]) * rng.uniform(-1, 1, size=(256, 256))
    p = runtime.params("D2Q9", 256, 256, 1, eos="vdW", T_over_Tc=0.75, kappa=0.02, tau=1.0, scheme="improved",
                       precision="fp32")
    roll = Rollout(p)
    tgt = torch.as_tensor(target).reshape(-1).cuda()
    r0 = torch.as_tensor(rho0).reshape(-1).cuda().requires_grad_(True)
    kd = torch.tensor(0.02, dtype=torch.float64, device="cuda", requires_grad=True)
    td = torch.tensor(0.75, dtype=torch.float64, device="cuda", requires_grad=True)
    # warm-up: a whole forward and backward, so that graph capture and the first
    # allocation of the checkpoint and segment buffers stay out of the timing
    rho_w, u_w = rollout(r0, kd, td, roll, n_steps)
    (((rho_w - tgt) ** 2).sum() + (u_w ** 2).sum()).backward()
    r0.grad, kd.grad, td.grad = None, None, None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rho_n, u_n = rollout(r0, kd, td, roll, n_steps)
    loss = ((rho_n - tgt) ** 2).sum() + (u_n ** 2).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    roll.close()
    fwd, bwd = t1 - t0, t2 - t1
    return {"name": "adjoint_d2q9_256_fp32", "steps": n_steps,
            "workload": "D2Q9 256x256 vdW droplet r=40, T/Tc=0.75, kappa=0.02, tau=1.0, improved, fp32 forward, "
                        f"{n_steps} steps, sqrt(N) checkpoints, float64 adjoint",
            "forward_s": fwd, "backward_s": bwd, "fwd_plus_bwd_over_fwd": (fwd + bwd) / fwd,
            "mlups": 65536 * n_steps / (fwd + bwd) / 1e6,
            "grad_kappa": float(kd.grad), "grad_T_over_Tc": float(td.grad)}


GATE_RHO = 1e-4           # coexistence densities: float32 within 1e-4 relative of float64
GATE_U = 0.05             # spurious-current maxima within 5 % of float64 ...
GATE_U_FLOOR = 1e-10      # ... whenever the float64 maximum is above this round-off level
GATE_U_ROUNDOFF = 1e-5    # below it, float32 must stay at or below float32's round-off level


def accuracy_gates(a, b):
    """Gates of float32 run `b` against float64 run `a` (dicts with rho_l, rho_g, max_u):
    densities within 1e-4 relative; max |u| within 5 % when float64's is above 1e-10,
    else float32's at most 1e-5 (the reading for round-off spurious currents)."""
    rel = {k: b[k] / a[k] - 1 for k in ("rho_l", "rho_g", "max_u")}
    if a["max_u"] > GATE_U_FLOOR:
        u_ok, u_rule = abs(rel["max_u"]) <= GATE_U, "within 5 % of float64"
    else:
        u_ok, u_rule = b["max_u"] <= GATE_U_ROUNDOFF, "float64 at round-off: float32 <= 1e-5"
    return {"rel": rel, "rho_l": abs(rel["rho_l"]) <= GATE_RHO, "rho_g": abs(rel["rho_g"]) <= GATE_RHO,
            "max_u": u_ok, "max_u_rule": u_rule,
            "all": abs(rel["rho_l"]) <= GATE_RHO and abs(rel["rho_g"]) <= GATE_RHO and u_ok}


def run_accuracy_case(torch, runtime, spec_fn, steps, shape, liquid, gas):
    """One workload in float64 and in float32 deviation storage for `steps` steps:
    the mean density over the `liquid` and `gas` boxes (slices of the field), max |u|,
    mass drift and status of each, and the gates."""
    out = {"steps": steps}
    for prec in ("fp64", "fp32"):
        spec = spec_fn(prec)
        sim = runtime.LBM(spec["params"])
        sim.init(spec["rho0"])
        sim.step(steps)
        rho, _, _ = sim.moments()
        d = sim.diagnostics()[0]
        r = rho.view(*shape)
        out[prec] = {"rho_l": float(r[liquid].mean()), "rho_g": float(r[gas].mean()), "max_u": d["max_u"],
                     "mass_drift": d["mass"] / float(spec["rho0"].sum()) - 1, "status": d["status"]}
        out["workload"] = spec["workload"].rsplit(",", 1)[0]
        sim.close()
        del rho, r
        torch.cuda.empty_cache()
    out["gates"] = accuracy_gates(out["fp64"], out["fp32"])
    return out


def accuracy(torch, runtime, inputs, steps=50000, d3_steps=10000):
    """float32 deviation storage against float64 at the configurations' lengths: the
    primary's 512^2 droplet (improved scheme, 5e4 steps), the same droplet in the
    standard scheme at T/Tc = 0.9 (where it is stable), and the 256^3 D3Q19 droplet
    (1e4 steps); coexistence densities (droplet centre, far corner), spurious-current
    maxima, mass drift, and the pass/fail gates of each."""
    c = (slice(246, 266), slice(246, 266))
    g = (slice(0, 20), slice(0, 20))
    out = {
        "c2_improved": run_accuracy_case(torch, runtime, lambda p: primary_spec(runtime, inputs, precision=p),
                                         steps, (512, 512), c, g),
        "c2_standard_T0.9": run_accuracy_case(
            torch, runtime, lambda p: primary_spec(runtime, inputs, precision=p, scheme="standard", T=0.9),
            steps, (512, 512), c, g),
        "c3_d3q19": run_accuracy_case(torch, runtime, lambda p: d3q19_spec(runtime, inputs, precision=p), d3_steps,
                                      (256, 256, 256), (slice(120, 136),) * 3, (slice(0, 16),) * 3),
    }
    m = runtime.maxwell("CS", 0.8)
    out["c2_improved"]["maxwell"] = {"rho_l": m["rho_l"], "rho_g": m["rho_g"]}
    m = runtime.maxwell("vdW", 0.85)
    out["c3_d3q19"]["maxwell"] = {"rho_l": m["rho_l"], "rho_g": m["rho_g"]}
    return out


def copy_ceiling(torch, runtime, mib=2048, reps=10):
    """Device-to-device bandwidth of the library's plain copy kernel (read + write
    bytes over the event-timed duration): the achievable side of the HBM roofline."""
    nbytes = mib * 2**20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    runtime.copy_kernel(dst, src, nbytes, s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        runtime.copy_kernel(dst, src, nbytes, s)
    e1.record(s)
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return {"GB/s": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS, "bytes_per_launch": 2 * nbytes,
            "kernel": "lbm_copy_kernel (one 16-byte vector per thread, one pass, non-temporal stores)"}


def cpu_baseline(torch, inputs, seconds):
    """The oracle (float64, CPU) on the primary lattice, as many whole steps as fit
    in about `seconds` (at least 2)."""
    from oracle import eos as oeos
    from oracle import model

    # the CPUs this process may run on (capped by OMP_NUM_THREADS when it is set)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = max(1, min(threads, int(os.environ["OMP_NUM_THREADS"])))
    torch.set_num_threads(threads)
    model_name = "unknown CPU"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model_name = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    E = oeos.CarnahanStarling()
    m = oeos.maxwell(E, 0.8)
    rho0 = inputs.droplet((512, 512), m["rho_g"], m["rho_l"], 80.0, 5.0, noise=0.0)
    prm = model.Params(lattice="D2Q9", eos=E, T_over_Tc=0.8, kappa=0.01, tau=0.8, scheme="improved")

    def timed(secs):
        f = model.init(torch.as_tensor(rho0), prm)
        f = model.step(f, prm)      # first-call overheads outside the timing
        n, t0 = 0, time.perf_counter()
        while True:
            f = model.step(f, prm)
            n += 1
            el = time.perf_counter() - t0
            if (el >= secs and n >= 2) or n >= 2000:
                return n, el

    n, el = timed(seconds)
    out = {"value": 512 * 512 * n / el / 1e6, "unit": "MLUPS", "cores": threads,
           "kind": "oracle", "sample": f"{n} steps of the 512x512 D2Q9 CS droplet (improved, float64), "
                                       f"{el:.1f} s on {threads} threads of {model_name}"}
    # the same oracle on one thread
    torch.set_num_threads(1)
    n1, el1 = timed(seconds / 3)
    torch.set_num_threads(threads)
    out["single_thread"] = {"value": 512 * 512 * n1 / el1 / 1e6, "unit": "MLUPS", "cores": 1,
                            "sample": f"{n1} steps, {el1:.1f} s on 1 thread"}
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (lattices of a batch are "
              "independent and would be split between GPUs by the caller); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2008_01473_amd import inputs, runtime

    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        nbytes = int(args.copy_calibration * 2**20)
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            runtime.copy_kernel(dst, src, nbytes)
        torch.cuda.synchronize()
        assert torch.equal(dst, src)
        print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 5}))
        return
    graphs = not args.no_graphs
    tune = 0 if args.no_tune else 20
    sha, recs = kernel_sources_sha256(), traffic_records()
    prim = measure(torch, runtime, inputs, primary_spec(runtime, inputs), args.steps, args.warmup, graphs, tune,
                   args.tile)
    prim["roofline"]["traffic"] = traffic_for(prim["name"], prim["tile"], sha, recs)
    print(f"[bench] primary {prim['workload']}: {prim['mlups']:.1f} MLUPS, {prim['ms_per_step'] * 1e3:.2f} us/step"
          f" (tile {prim['tile']}, {prim['stores']} stores)", file=sys.stderr, flush=True)
    secondary = []
    if not args.no_secondary:
        only = set(filter(None, args.only.split(",")))
        jobs = [
            ("fp32", lambda: primary_spec(runtime, inputs, precision="fp32"), args.steps),
            ("mrt", lambda: mrt_spec(runtime, inputs), args.steps),
            ("plates", lambda: plates_spec(runtime, inputs), args.steps),
            ("c0", lambda: c0_spec(runtime, inputs), args.steps),
            # the standard scheme blows up for this droplet at T/Tc = 0.8 (oracle too); 0.9 is stable
            ("standard", lambda: primary_spec(runtime, inputs, scheme="standard", T=0.9), args.steps),
            ("d3q19", lambda: d3q19_spec(runtime, inputs), max(20, args.steps // 40)),
            ("d3q19_shard", lambda: d3q19_shard_spec(runtime, inputs), max(20, args.steps // 10)),
            ("d2q9_4096_fp64", lambda: d2q9_large_spec(runtime, inputs, "fp64"), max(20, args.steps // 40)),
            ("d2q9_4096_fp32", lambda: d2q9_large_spec(runtime, inputs, "fp32"), max(20, args.steps // 40)),
            ("batch", lambda: batch_spec(runtime, inputs), max(20, args.steps // 20)),
            ("batch_c0", lambda: batch_spec(runtime, inputs, c0=0.4), max(20, args.steps // 20)),
        ]
        if not only or "adjoint" in only:
            r = adjoint_measure(torch, runtime, inputs)
            r["vs_primary_mlups"] = r["mlups"] / prim["mlups"]
            secondary.append(r)
            print(f"[bench] adjoint: fwd {r['forward_s'] * 1e3:.1f} ms, bwd {r['backward_s'] * 1e3:.1f} ms, "
                  f"(fwd+bwd)/fwd = {r['fwd_plus_bwd_over_fwd']:.1f}", file=sys.stderr, flush=True)
        for name, mk, k in jobs:
            if only and name not in only:
                continue
            try:
                r = measure(torch, runtime, inputs, mk(), k, min(args.warmup, k), graphs, tune, args.tile)
            except runtime._lib.LBMError as e:        # a forced tile shape this workload does not support
                print(f"[bench] {name}: skipped ({e})", file=sys.stderr, flush=True)
                continue
            r["steps"] = k
            r["vs_primary_mlups"] = r["mlups"] / prim["mlups"]
            r["roofline"]["traffic"] = traffic_for(r["name"], r["tile"], sha, recs)
            secondary.append(r)
            print(f"[bench] {name}: {r['mlups']:.1f} MLUPS ({r['roofline']['frac'] * 100:.1f}% of 8 TB/s;"
                  f" tile {r['tile']}, {r['stores']} stores)", file=sys.stderr, flush=True)
    acc = None
    if not args.no_secondary and not args.no_accuracy and not args.no_graphs:
        acc = accuracy(torch, runtime, inputs)
        for k, a in acc.items():
            g = a["gates"]
            print(f"[bench] accuracy {k} after {a['steps']} steps: fp32 vs fp64 rho_l {g['rel']['rho_l']:.1e}, "
                  f"rho_g {g['rel']['rho_g']:.1e}; max_u fp64 {a['fp64']['max_u']:.2e}, fp32 {a['fp32']['max_u']:.2e}; "
                  f"gates rho {g['rho_l'] and g['rho_g']}, max_u {g['max_u']} ({g['max_u_rule']})",
                  file=sys.stderr, flush=True)
    ceiling = copy_ceiling(torch, runtime)
    print(f"[bench] copy ceiling: {ceiling['GB/s']:.0f} GB/s ({ceiling['frac_of_peak'] * 100:.1f}% of 8 TB/s)",
          file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(torch, inputs, args.cpu_seconds)
    line = {
        "metric": METRIC,
        "value": prim["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": prim["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": prim["workload"], "lattice": "D2Q9", "nodes": prim["nodes"],
                   "bytes_per_lup": prim["bytes_per_lup"], "tile": prim["tile"], "stores": prim["stores"]},
        "roofline": prim["roofline"],
        "copy_ceiling": ceiling,
        "accuracy": acc,
        "cpu_baseline": cpu,
        "secondary": secondary,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
