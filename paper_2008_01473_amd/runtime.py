"""Python face of the C ABI: parameter records, one handle per lattice or batch,
device buffers from PyTorch, calls into liblbm.so.  Every step of the method
runs in the HIP kernels; this module only marshals arguments."""

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, lbm_diag, lbm_params

_LATTICE = {"D2Q9": _lib.LBM_D2Q9, "D3Q19": _lib.LBM_D3Q19}
_EOS = {"vdW": _lib.LBM_EOS_VDW, "CS": _lib.LBM_EOS_CS}
_SCHEME = {"standard": _lib.LBM_STANDARD, "improved": _lib.LBM_IMPROVED}
_FORCE = {"chempot": _lib.LBM_FORCE_CHEMPOT, "ptensor": _lib.LBM_FORCE_PTENSOR}
_PREC = {"fp64": _lib.LBM_FP64, "fp32": _lib.LBM_FP32_DEV}
_COLLISION = {"bgk": _lib.LBM_BGK, "mrt": _lib.LBM_MRT}

# default EOS constants: the paper's vdW values (Sec. IV A) and the CS reading
# with the same critical density 3.5 and critical temperature 1/14
EOS_DEFAULTS = {"vdW": (9.0 / 392.0, 2.0 / 21.0), "CS": (0.0282217394824, 0.149078724791)}


def params(lattice="D2Q9", nx=64, ny=64, nz=1, eos="vdW", a=None, b=None, R=1.0, T_over_Tc=0.8,
           kappa=0.02, tau=1.0, scheme="improved", force_form="chempot", precision="fp64",
           rho_ref=0.0, pm_ref=0.0, collision="bgk", tau_e=1.0, tau_s=1.0, tau_q=1.0, nu=0.0, walls=None,
           c0=1.0):
    """An lbm_params record (see include/lbm.h).  collision="mrt" selects the
    relaxation matrix of Eq. 8 with rates 1/tau_e, 1/tau_s, 1/tau_q and a shear
    rate from tau (nu <= 0) or from a constant kinematic viscosity nu.
    walls=(U_bottom, U_top) bounds a D2Q9 lattice in y by plates moving along x.
    c0 (improved scheme): p_m = (c0 + mu)/3; the paper's method is c0 = 1."""
    da, db = EOS_DEFAULTS[eos]
    p = lbm_params()
    p.lattice, p.nx, p.ny, p.nz = _LATTICE[lattice], nx, ny, nz
    p.eos, p.a, p.b, p.R = _EOS[eos], da if a is None else a, db if b is None else b, R
    p.T_over_Tc, p.kappa, p.tau = T_over_Tc, kappa, tau
    p.scheme, p.force_form, p.precision = _SCHEME[scheme], _FORCE[force_form], _PREC[precision]
    p.rho_ref, p.pm_ref = rho_ref, pm_ref
    p.collision = _COLLISION[collision]
    p.tau_e, p.tau_s, p.tau_q, p.nu = tau_e, tau_s, tau_q, nu
    if walls is not None:
        p.walls, p.wall_u_bottom, p.wall_u_top = 1, float(walls[0]), float(walls[1])
    p.c0 = c0
    return p


def maxwell(eos="vdW", T_over_Tc=0.8, a=None, b=None, R=1.0):
    """Host float64 Maxwell construction of the library (dict rho_g, rho_l, mu, p)."""
    da, db = EOS_DEFAULTS[eos]
    out = [ctypes.c_double() for _ in range(4)]
    check(_lib.lib().lbm_maxwell(_EOS[eos], da if a is None else a, db if b is None else b, R, T_over_Tc,
                                 *[ctypes.byref(x) for x in out]), "lbm_maxwell")
    return {"rho_g": out[0].value, "rho_l": out[1].value, "mu": out[2].value, "p": out[3].value}


def critical_temperature(eos="vdW", a=None, b=None, R=1.0):
    da, db = EOS_DEFAULTS[eos]
    return _lib.lib().lbm_critical_temperature(_EOS[eos], da if a is None else a, db if b is None else b, R)


class LBM:
    """One lattice or a batch of lattices advanced together on one GPU stream."""

    def __init__(self, prm, device="cuda", stream=None):
        L = _lib.lib()
        plist = prm if isinstance(prm, (list, tuple)) else [prm]
        arr = (lbm_params * len(plist))(*plist)
        self.params = list(plist)
        self.device = torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        check(L.lbm_create_batch(arr, len(plist), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)),
              "lbm_create_batch")
        self.h = h
        self.D = 2 if plist[0].lattice == _lib.LBM_D2Q9 else 3
        self.Q = 9 if self.D == 2 else 19
        self.N = L.lbm_num_nodes(h)
        self.count = L.lbm_count(h)
        sb, wb = L.lbm_state_bytes(h), L.lbm_workspace_bytes(h)
        self.state_bytes = sb
        self.f_a = torch.empty(sb, dtype=torch.uint8, device=self.device)
        self.f_b = torch.empty(sb, dtype=torch.uint8, device=self.device)
        self.ws = torch.empty(wb, dtype=torch.uint8, device=self.device)
        check(L.lbm_bind(h, self.f_a.data_ptr(), self.f_b.data_ptr(), self.ws.data_ptr()), "lbm_bind")

    # -- helpers -------------------------------------------------------------
    def _dev64(self, x, n):
        t = torch.as_tensor(np.ascontiguousarray(x) if isinstance(x, np.ndarray) else x)
        t = t.to(device=self.device, dtype=torch.float64).contiguous().reshape(-1)
        if t.numel() != n:
            raise ValueError(f"expected {n} values, got {t.numel()}")
        return t

    def offsets(self):
        L = _lib.lib()
        return [L.lbm_node_offset(self.h, i) for i in range(self.count)]

    def shape_of(self, i=0):
        p = self.params[i]
        return (p.ny, p.nx) if self.D == 2 else (p.nz, p.ny, p.nx)

    # -- method --------------------------------------------------------------
    def init(self, rho0, u0=None):
        """rho0: concatenated float64 densities of all lattices (array or tensor)."""
        self._rho0 = self._dev64(rho0, self.N)
        self._u0 = None if u0 is None else self._dev64(u0, self.D * self.N)
        check(_lib.lib().lbm_init(self.h, self._rho0.data_ptr(),
                                  None if self._u0 is None else self._u0.data_ptr()), "lbm_init")

    def step(self, n=1):
        check(_lib.lib().lbm_step(self.h, int(n)), "lbm_step")

    def prepare(self, n):
        """Capture the graphs lbm_step(n) will replay (no work is enqueued)."""
        check(_lib.lib().lbm_prepare_steps(self.h, int(n)), "lbm_prepare_steps")

    def moments(self):
        rho = torch.empty(self.N, dtype=torch.float64, device=self.device)
        u = torch.empty(self.D * self.N, dtype=torch.float64, device=self.device)
        mu = torch.empty(self.N, dtype=torch.float64, device=self.device)
        check(_lib.lib().lbm_moments(self.h, rho.data_ptr(), u.data_ptr(), mu.data_ptr()), "lbm_moments")
        return rho, u.view(self.D, self.N), mu

    def diagnostics(self, raise_on_blowup=False):
        out = (lbm_diag * self.count)()
        rc = _lib.lib().lbm_diagnostics(self.h, out)
        if rc != _lib.LBM_ERR_BLOWUP or raise_on_blowup:
            check(rc, "lbm_diagnostics")
        return [{"mass": d.mass, "mom": list(d.mom)[: self.D], "max_u": d.max_u, "mu_min": d.mu_min,
                 "mu_max": d.mu_max, "step": d.step, "status": d.status} for d in out]

    def get_f(self):
        f = torch.empty(self.Q * self.N, dtype=torch.float64, device=self.device)
        check(_lib.lib().lbm_get_f(self.h, f.data_ptr()), "lbm_get_f")
        return f.view(self.Q, self.N)

    def set_f(self, f):
        self._fset = self._dev64(f, self.Q * self.N)
        check(_lib.lib().lbm_set_f(self.h, self._fset.data_ptr()), "lbm_set_f")

    def get_state(self):
        dst = torch.empty(self.state_bytes, dtype=torch.uint8, device=self.device)
        t = ctypes.c_longlong()
        check(_lib.lib().lbm_get_state(self.h, dst.data_ptr(), ctypes.byref(t)), "lbm_get_state")
        return dst, t.value

    def set_state(self, state, t):
        self._sset = state
        check(_lib.lib().lbm_set_state(self.h, state.data_ptr(), int(t)), "lbm_set_state")

    @property
    def time(self):
        return _lib.lib().lbm_time(self.h)

    def num_tile_shapes(self):
        return _lib.lib().lbm_num_tile_shapes(self.h)

    def set_tile_shape(self, s):
        check(_lib.lib().lbm_set_tile_shape(self.h, int(s)), "lbm_set_tile_shape")

    def tile_shape(self, s=None):
        L = _lib.lib()
        s = L.lbm_get_tile_shape(self.h) if s is None else s
        bx, by, bz = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(L.lbm_describe_tile_shape(self.h, s, ctypes.byref(bx), ctypes.byref(by), ctypes.byref(bz)))
        return bx.value, by.value, bz.value

    def set_zchunk(self, bz):
        """D3Q19: fix the z-chunk each work group sweeps (>= 16), or 0 for automatic."""
        check(_lib.lib().lbm_set_zchunk(self.h, int(bz)), "lbm_set_zchunk")

    def use_graphs(self, on=True):
        check(_lib.lib().lbm_set_use_graphs(self.h, 1 if on else 0))

    _STORES = {"streaming": _lib.LBM_STORES_STREAMING, "device": _lib.LBM_STORES_DEVICE}

    def set_store_mode(self, mode):
        """"streaming" (non-temporal stores) or "device" (device-scope stores)."""
        check(_lib.lib().lbm_set_store_mode(self.h, self._STORES[mode]), "lbm_set_store_mode")

    def store_mode(self):
        m = _lib.lib().lbm_get_store_mode(self.h)
        return {v: k for k, v in self._STORES.items()}[m]

    def autotune(self, steps=20):
        scratch = torch.empty(self.state_bytes, dtype=torch.uint8, device=self.device)
        return check(_lib.lib().lbm_autotune(self.h, int(steps), scratch.data_ptr()), "lbm_autotune")

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            torch.cuda.synchronize(self.device)
            _lib.lib().lbm_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def copy_kernel(dst, src, nbytes, stream=None):
    stream = stream or torch.cuda.current_stream()
    check(_lib.lib().lbm_copy_kernel(dst.data_ptr(), src.data_ptr(), int(nbytes), ctypes.c_void_p(stream.cuda_stream)))
