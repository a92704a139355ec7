"""Python binding of the gfx950 library libns.so (C ABI in include/ns.h).

Argument marshalling only: PyTorch provides device memory (the state arrays
and the workspace) and the HIP stream; every arithmetic step of the time
step runs in the library's kernels.  There is no CPU fallback: if the
library or a GPU is missing, construction raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libns.so")

NS_OK, NS_EINVAL, NS_ENOCONV, NS_ENAN, NS_EHIP, NS_ESTATE, NS_EUNSTABLE = 0, -1, -2, -3, -4, -5, -6
STATUS = {0: "NS_OK", -1: "NS_EINVAL", -2: "NS_ENOCONV", -3: "NS_ENAN", -4: "NS_EHIP", -5: "NS_ESTATE",
          -6: "NS_EUNSTABLE"}
PREC_FP64, PREC_MIXED = 0, 1
X0_ZERO, X0_PREV, X0_LEARNED, X0_AUTO = 0, 1, 2, 3
BUF = {"us": 0, "vs": 1, "ws": 2, "bx": 3, "by": 4, "bz": 5, "rhs": 6, "rho": 7, "mu": 8, "chi": 9,
       "rho_flow": 10, "bxf": 11, "byf": 12, "bzf": 13}


class NSBody(C.Structure):
    _fields_ = [("kind", C.c_int), ("c", C.c_double * 3), ("half", C.c_double * 3),
                ("heave_amp", C.c_double), ("heave_omega", C.c_double), ("heave_phase", C.c_double),
                ("free_heave", C.c_int), ("mass", C.c_double), ("pto_damping", C.c_double),
                ("zeta0", C.c_double), ("zdot0", C.c_double)]


class NSWave(C.Structure):
    _fields_ = [("a", C.c_double), ("kappa", C.c_double), ("omega", C.c_double), ("phase", C.c_double)]


class NSParams(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("h", C.c_double),
                ("rho_w", C.c_double), ("mu_w", C.c_double), ("rho_a", C.c_double), ("mu_a", C.c_double),
                ("rho_s", C.c_double), ("mu_s", C.c_double), ("g", C.c_double),
                ("n_cells", C.c_double), ("inv_kappa_p", C.c_double), ("proj_penalty_weight", C.c_double),
                ("n_bodies", C.c_int), ("body", NSBody * 4),
                ("reinit_iters", C.c_int), ("reinit_dtau_over_h", C.c_double),
                ("nu_pre", C.c_int), ("nu_post", C.c_int), ("coarse_sweeps", C.c_int),
                ("max_iters", C.c_int), ("rtol", C.c_double), ("prec", C.c_int), ("x0", C.c_int),
                ("p_scale", C.c_double),
                ("depth", C.c_double), ("gen_len", C.c_double), ("damp_len", C.c_double),
                ("vort_width", C.c_double), ("n_waves", C.c_int), ("waves", NSWave * 64),
                ("consistent", C.c_int), ("cn_sweeps", C.c_int), ("cn_tol", C.c_double)]


class NSFields(C.Structure):
    _fields_ = [("sigma", C.c_void_p), ("u", C.c_void_p), ("v", C.c_void_p), ("w", C.c_void_p),
                ("p", C.c_void_p)]


class NSStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("rel_resid0", C.c_double),
                ("rel_resid", C.c_double), ("true_rel_resid", C.c_double), ("ms", C.c_double),
                ("x0_fallback", C.c_int), ("cn_sweeps", C.c_int), ("t_ms", C.c_double * 8),
                ("x0_used", C.c_int), ("x0_gain", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["t_ms"] = list(self.t_ms)
        return d


class NSError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} -> {STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib() -> C.CDLL:
    """Load libns.so (built by paper_2206_07732_amd.build); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2206_07732_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, d, i = C.c_void_p, C.c_double, C.c_int
        P = C.POINTER(NSParams)
        S = C.POINTER(NSStats)
        sig = {
            "ns_workspace_bytes": ([P], C.c_size_t),
            "ns_init": ([P, NSFields, vp, C.c_size_t, vp, C.POINTER(vp)], i),
            "levelset_advect_reinit": ([vp, d], i),
            "momentum_step": ([vp, d, d], i),
            "projection_solve": ([vp, d, S], i),
            "ns_step": ([vp, d, d, S], i),
            "ns_pcg_solve": ([vp, S], i),
            "ns_apply_A": ([vp, vp, vp], i),
            "ns_vcycle": ([vp, vp, vp], i),
            "ns_buffer": ([vp, i, C.POINTER(vp), C.POINTER(C.c_size_t)], i),
            "ns_diagnostics": ([vp, C.POINTER(C.c_double)], i),
            "ns_num_levels": ([i, i, i], i),
            "ns_set_launch_mode": ([vp, i], i),
            "ns_body_state": ([vp, i, C.POINTER(C.c_double)], i),
            "ns_timing_enable": ([vp, i, i], i),
            "ns_timing_read": ([vp, C.POINTER(C.c_double), C.POINTER(C.c_int)], i),
            "ns_time_kernel": ([vp, i, i, C.POINTER(C.c_double)], i),
            "ns_net_param_count": ([], C.c_size_t),
            "ns_net_workspace_bytes": ([i, i, i, i], C.c_size_t),
            "ns_net_create": ([i, i, i, i, vp, C.c_size_t, vp, C.POINTER(vp)], i),
            "ns_net_destroy": ([vp], None),
            "ns_net_last_error": ([vp], C.c_char_p),
            "ns_net_set_params": ([vp, C.POINTER(C.c_float), C.c_size_t], i),
            "ns_net_get_params": ([vp, C.POINTER(C.c_float), C.c_size_t], i),
            "ns_net_get_grads": ([vp, C.POINTER(C.c_float), C.c_size_t], i),
            "ns_net_set_input": ([vp, vp], i),
            "ns_net_forward": ([vp, vp], i),
            "ns_net_train_step": ([vp, vp, vp, vp, vp, vp, C.c_float, i, C.POINTER(C.c_double)], i),
            "ns_attach_net": ([vp, vp], i),
            "ns_features": ([vp, d, vp, vp], i),
            "ns_target": ([vp, vp, vp], i),
            "ns_cfl_dt": ([vp, d, d, C.POINTER(C.c_double)], i),
            "ns_cfl_dt_noalloc": ([i, i, i, d, vp, vp, vp, d, d, vp, vp], i),
            "ns_phase_timing": ([vp, i], i),
            "ns_set_fine_sweep": ([vp, i], i),
            "ns_get_fine_sweep": ([vp, C.POINTER(i)], i),
            "ns_set_face_tables": ([vp, i], i),
            "ns_get_face_tables": ([vp, C.POINTER(i)], i),
            "ns_last_error": ([vp], C.c_char_p),
            "ns_destroy": ([vp], None),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


EXPORTED = ["ns_workspace_bytes", "ns_init", "levelset_advect_reinit", "momentum_step",
            "projection_solve", "ns_step", "ns_pcg_solve", "ns_apply_A", "ns_vcycle", "ns_buffer",
            "ns_diagnostics", "ns_num_levels", "ns_last_error", "ns_destroy", "ns_set_launch_mode",
            "ns_body_state", "ns_timing_enable", "ns_timing_read", "ns_time_kernel", "ns_net_param_count", "ns_net_workspace_bytes",
            "ns_net_create", "ns_net_destroy", "ns_net_last_error", "ns_net_set_params",
            "ns_net_get_params", "ns_net_get_grads", "ns_net_set_input", "ns_net_forward",
            "ns_net_train_step", "ns_attach_net", "ns_features", "ns_target", "ns_cfl_dt", "ns_phase_timing", "ns_cfl_dt_noalloc",
            "ns_set_fine_sweep", "ns_get_fine_sweep", "ns_set_face_tables", "ns_get_face_tables"]
TIME_SMOOTH0, TIME_SPMV = 0, 1
LAUNCH_STREAM, LAUNCH_GRAPH = 0, 1

SOLVER_DEFAULTS = dict(reinit_iters=5, reinit_dtau_over_h=0.25, nu_pre=2, nu_post=2, coarse_sweeps=10,
                       max_iters=200, rtol=1e-10, prec=PREC_FP64, x0=X0_PREV, p_scale=0.0, cn_tol=1e-10)


def params(wl, **opts) -> NSParams:
    """ns_params for a workload (paper_2206_07732_amd.inputs.Workload)."""
    P = NSParams()
    P.nx, P.ny, P.nz, P.h = wl.nx, wl.ny, wl.nz, wl.h
    P.rho_w, P.mu_w, P.rho_a, P.mu_a, P.rho_s, P.mu_s, P.g = (
        wl.rho_w, wl.mu_w, wl.rho_a, wl.mu_a, wl.rho_s, wl.mu_s, wl.g)
    P.n_cells, P.inv_kappa_p, P.proj_penalty_weight = wl.n_cells, wl.inv_kappa_p, wl.proj_penalty_weight
    P.n_bodies = len(wl.bodies)
    for m, b in enumerate(wl.bodies):
        P.body[m].kind = b.kind
        for q in range(3):
            P.body[m].c[q] = b.c[q]
            P.body[m].half[q] = b.half[q]
        P.body[m].heave_amp, P.body[m].heave_omega, P.body[m].heave_phase = (
            b.heave_amp, b.heave_omega, b.heave_phase)
        P.body[m].free_heave, P.body[m].mass, P.body[m].pto_damping = int(b.free_heave), b.mass, b.pto_damping
        P.body[m].zeta0, P.body[m].zdot0 = b.zeta0, b.zdot0
    P.depth = wl.depth
    P.consistent = int(wl.consistent)
    P.cn_sweeps = int(wl.cn_sweeps)
    if wl.nwt:                                      # numerical wave tank
        from . import inputs as I
        P.gen_len, P.damp_len, P.vort_width = wl.nwt.get("gen", 0.0), wl.nwt.get("damp", 0.0), wl.nwt.get("vort", 0.0)
        a, k, om, ph = I.wave_components(wl)
        P.n_waves = len(a)
        for q in range(len(a)):
            P.waves[q].a, P.waves[q].kappa, P.waves[q].omega, P.waves[q].phase = a[q], k[q], om[q], ph[q]
    o = dict(SOLVER_DEFAULTS)
    o["p_scale"] = wl.rho_w * wl.g * wl.depth      # P0 = rho_w g d
    o.update(opts)
    for k, v in o.items():
        setattr(P, k, v)
    return P


def num_levels(nx, ny, nz) -> int:
    return lib().ns_num_levels(nx, ny, nz)


def _dev_f64(t: torch.Tensor, name: str):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    return t.data_ptr()


class Solver:
    """One time-stepping context bound to caller-owned device fields.

    fields: dict with 'sigma', 'u', 'v', 'w', 'p' float64 CUDA tensors of
    shapes (nz,ny,nx), (nz,ny,nx+1), (nz,ny+1,nx), (nz+1,ny,nx), (nz,ny,nx).
    """

    def __init__(self, P: NSParams, fields: dict, stream: Optional[torch.cuda.Stream] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the solver runs only on the gfx950 library")
        L = lib()
        self.P = P
        self.fields = fields
        self.device = fields["p"].device
        nx, ny, nz = P.nx, P.ny, P.nz
        shapes = {"sigma": (nz, ny, nx), "u": (nz, ny, nx + 1), "v": (nz, ny + 1, nx),
                  "w": (nz + 1, ny, nx), "p": (nz, ny, nx)}
        for k, s in shapes.items():
            if tuple(fields[k].shape) != s:
                raise ValueError(f"{k} has shape {tuple(fields[k].shape)}, expected {s}")
            if fields[k].device != self.device:
                raise ValueError(f"{k} is on {fields[k].device}, the others on {self.device}")
        F = NSFields(*[_dev_f64(fields[k], k) for k in ("sigma", "u", "v", "w", "p")])
        nbytes = L.ns_workspace_bytes(C.byref(P))
        if nbytes == 0:
            raise ValueError("invalid ns_params")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        st = L.ns_init(C.byref(P), F, C.c_void_p(base + self._ws_off), nbytes,
                       C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if st != NS_OK:
            raise NSError("ns_init", st, "invalid parameters, fields or workspace")
        self.ctx = ctx

    # -- helpers
    def _chk(self, fn, st, allow=(NS_OK,)):
        if st not in allow:
            msg = lib().ns_last_error(self.ctx)
            raise NSError(fn, st, msg.decode() if msg else "")
        return st

    def close(self):
        if getattr(self, "ctx", None):
            lib().ns_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the ABI calls
    def levelset_advect_reinit(self, dt: float):
        self._chk("levelset_advect_reinit", lib().levelset_advect_reinit(self.ctx, dt))

    def momentum_step(self, dt: float, t_np1: float):
        self._chk("momentum_step", lib().momentum_step(self.ctx, dt, t_np1))

    def projection_solve(self, dt: float, allow_noconv: bool = False) -> dict:
        S = NSStats()
        st = lib().projection_solve(self.ctx, dt, C.byref(S))
        self._chk("projection_solve", st, (NS_OK, NS_ENOCONV) if allow_noconv else (NS_OK,))
        d = S.as_dict()
        d["status"] = st
        return d

    def step(self, dt: float, t_n: float, allow_noconv: bool = False) -> dict:
        S = NSStats()
        st = lib().ns_step(self.ctx, dt, t_n, C.byref(S))
        self._chk("ns_step", st, (NS_OK, NS_ENOCONV) if allow_noconv else (NS_OK,))
        d = S.as_dict()
        d["status"] = st
        return d

    def pcg_solve(self, allow_noconv: bool = False) -> dict:
        S = NSStats()
        st = lib().ns_pcg_solve(self.ctx, C.byref(S))
        self._chk("ns_pcg_solve", st, (NS_OK, NS_ENOCONV) if allow_noconv else (NS_OK,))
        d = S.as_dict()
        d["status"] = st
        return d

    def apply_A(self, x: torch.Tensor, y: torch.Tensor):
        self._chk("ns_apply_A", lib().ns_apply_A(self.ctx, _dev_f64(x, "x"), _dev_f64(y, "y")))

    def vcycle(self, r: torch.Tensor, z: torch.Tensor):
        self._chk("ns_vcycle", lib().ns_vcycle(self.ctx, _dev_f64(r, "r"), _dev_f64(z, "z")))

    def buffer(self, name: str) -> torch.Tensor:
        """A view of an internal workspace array (float64, or float32 for the
        *f beta copies), shaped like its field."""
        ptr, cnt = C.c_void_p(), C.c_size_t()
        self._chk("ns_buffer", lib().ns_buffer(self.ctx, BUF[name], C.byref(ptr), C.byref(cnt)))
        off = ptr.value - self.workspace.data_ptr()
        f32 = name in ("bxf", "byf", "bzf")
        w = 4 if f32 else 8
        flat = self.workspace[off: off + w * cnt.value].view(torch.float32 if f32 else torch.float64)
        nx, ny, nz = self.P.nx, self.P.ny, self.P.nz
        key = name[:-1] if f32 else name
        shape = {"us": (nz, ny, nx + 1), "bx": (nz, ny, nx + 1), "vs": (nz, ny + 1, nx),
                 "by": (nz, ny + 1, nx), "ws": (nz + 1, ny, nx), "bz": (nz + 1, ny, nx)}.get(
            key, (nz, ny, nx))
        return flat.view(shape)

    def set_launch_mode(self, mode: int):
        """LAUNCH_GRAPH (default): each V-cycle of the CG loop, with the dot
        product after it, is one replay of a recorded HIP graph;
        LAUNCH_STREAM: the same kernels launched one by one."""
        self._chk("ns_set_launch_mode", lib().ns_set_launch_mode(self.ctx, mode))

    def set_fine_sweep(self, fused: bool):
        """The finest level's red-black sweeps as one launch each (True) or
        as two colour passes (False, the library's default)."""
        self._chk("ns_set_fine_sweep", lib().ns_set_fine_sweep(self.ctx, 1 if fused else 0))

    def fine_sweep(self) -> bool:
        """Whether the finest level's red-black sweeps run as one launch each."""
        v = C.c_int()
        self._chk("ns_get_fine_sweep", lib().ns_get_fine_sweep(self.ctx, C.byref(v)))
        return bool(v.value)

    def set_face_tables(self, on: bool):
        """Whether the finest level's kernels read face lines of one value
        through their line tables (the default from 2^21 cells) or load every
        face."""
        self._chk("ns_set_face_tables", lib().ns_set_face_tables(self.ctx, 1 if on else 0))

    def face_tables(self) -> bool:
        """Whether the line tables are used."""
        v = C.c_int()
        self._chk("ns_get_face_tables", lib().ns_get_face_tables(self.ctx, C.byref(v)))
        return bool(v.value)

    def timing_enable(self, kernel: int, max_launches: int):
        self._chk("ns_timing_enable", lib().ns_timing_enable(self.ctx, kernel, max_launches))

    def timing_read(self):
        """(total ms, launches) of the timed kernel since the last read."""
        ms, n = C.c_double(), C.c_int()
        self._chk("ns_timing_read", lib().ns_timing_read(self.ctx, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def time_kernel(self, kernel: int, reps: int) -> float:
        """Average ms of `reps` back-to-back dispatches of a kernel (events around the batch)."""
        ms = C.c_double()
        self._chk("ns_time_kernel", lib().ns_time_kernel(self.ctx, kernel, reps, C.byref(ms)))
        return ms.value

    def attach_net(self, net):
        self._chk("ns_attach_net", lib().ns_attach_net(self.ctx, net.net if net is not None else None))
        self._net = net

    def features(self, dt: float, p_prev: torch.Tensor, feat4: torch.Tensor):
        if not (feat4.is_cuda and feat4.dtype == torch.float32 and feat4.is_contiguous()):
            raise TypeError("feat4 must be a contiguous float32 CUDA tensor")
        self._chk("ns_features", lib().ns_features(self.ctx, dt, _dev_f64(p_prev, "p_prev"), feat4.data_ptr()))

    def target(self, p_prev: torch.Tensor, t: torch.Tensor):
        self._chk("ns_target", lib().ns_target(self.ctx, _dev_f64(p_prev, "p_prev"), t.data_ptr()))

    def body_state(self, m: int) -> dict:
        """Heave offset and velocity of body m, the last hydrodynamic force
        (Fx, Fy, Fz) and power take-off force (free bodies)."""
        out = (C.c_double * 6)()
        self._chk("ns_body_state", lib().ns_body_state(self.ctx, m, out))
        return {"zeta": out[0], "zdot": out[1], "F": (out[2], out[3], out[4]), "f_pto": out[5]}

    def cfl_dt(self, cfl: float, dt_max: float = 0.05) -> float:
        """Time step of the CFL rule on the current fields (ns_cfl_dt)."""
        dt = C.c_double()
        self._chk("ns_cfl_dt", lib().ns_cfl_dt(self.ctx, cfl, dt_max, C.byref(dt)))
        return dt.value

    def phase_timing(self, on: bool):
        """Per-phase device times in the stats' t_ms while on."""
        self._chk("ns_phase_timing", lib().ns_phase_timing(self.ctx, 1 if on else 0))

    def diagnostics(self):
        out = (C.c_double * 4)()
        self._chk("ns_diagnostics", lib().ns_diagnostics(self.ctx, out))
        return list(out)


def cfl_dt_noalloc(nx: int, ny: int, nz: int, h: float, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor,
                   cfl: float, dt_max: float, dt_out: torch.Tensor, stream: Optional[torch.cuda.Stream] = None):
    """ns_cfl_dt_noalloc: the CFL rule's time step into dt_out (one float64
    CUDA element), stream-ordered, without a context or any allocation."""
    if not (dt_out.is_cuda and dt_out.dtype == torch.float64 and dt_out.numel() >= 1):
        raise TypeError("dt_out must be a float64 CUDA tensor")
    st = stream if stream is not None else torch.cuda.current_stream(dt_out.device)
    s = lib().ns_cfl_dt_noalloc(nx, ny, nz, h, _dev_f64(u, "u"), _dev_f64(v, "v"), _dev_f64(w, "w"), cfl, dt_max,
                                dt_out.data_ptr(), C.c_void_p(st.cuda_stream))
    if s != NS_OK:
        raise NSError("ns_cfl_dt_noalloc", s, "invalid sizes, pointers or values, or a HIP failure")


def device_fields(host_fields: dict, device="cuda") -> dict:
    """Copy numpy initial fields to float64 device tensors."""
    return {k: torch.from_numpy(host_fields[k]).to(device=device, dtype=torch.float64).contiguous()
            for k in ("sigma", "u", "v", "w", "p")}


def net_param_count() -> int:
    return lib().ns_net_param_count()


class Net:
    """The learned-guess network on an nx*ny*nz grid (device workspace owned
    by this object's torch tensor)."""

    def __init__(self, nx: int, ny: int, nz: int, training: bool = False, device="cuda",
                 stream: Optional[torch.cuda.Stream] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the network runs only on the gfx950 library")
        L = lib()
        nbytes = L.ns_net_workspace_bytes(nx, ny, nz, 1 if training else 0)
        if nbytes == 0:
            raise ValueError("network grid sizes must be multiples of 4")
        self.shape = (nz, ny, nx)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
        net = C.c_void_p()
        st = L.ns_net_create(nx, ny, nz, 1 if training else 0, C.c_void_p(base + off), nbytes,
                             C.c_void_p(self.stream.cuda_stream), C.byref(net))
        if st != NS_OK:
            raise NSError("ns_net_create", st, "invalid sizes or workspace")
        self.net = net
        self.n = L.ns_net_param_count()

    def _chk(self, fn, st):
        if st != NS_OK:
            msg = lib().ns_net_last_error(self.net)
            raise NSError(fn, st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "net", None):
            lib().ns_net_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        import numpy as np
        a = np.ascontiguousarray(flat, dtype=np.float32)
        assert a.size == self.n
        self._chk("ns_net_set_params",
                  lib().ns_net_set_params(self.net, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))

    def get_params(self):
        import numpy as np
        a = np.empty(self.n, dtype=np.float32)
        self._chk("ns_net_get_params",
                  lib().ns_net_get_params(self.net, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))
        return a

    def get_grads(self):
        import numpy as np
        a = np.empty(self.n, dtype=np.float32)
        self._chk("ns_net_get_grads",
                  lib().ns_net_get_grads(self.net, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))
        return a

    def forward(self, feat4: torch.Tensor) -> torch.Tensor:
        """delta (float32, (nz, ny, nx)) for features (float32, (4, nz, ny, nx))."""
        assert feat4.is_cuda and feat4.dtype == torch.float32 and feat4.is_contiguous()
        out = torch.empty(self.shape, dtype=torch.float32, device=feat4.device)
        self._chk("ns_net_set_input", lib().ns_net_set_input(self.net, feat4.data_ptr()))
        self._chk("ns_net_forward", lib().ns_net_forward(self.net, out.data_ptr()))
        return out

    def train_step(self, feat4: torch.Tensor, target: torch.Tensor, beta, lr: float, update: bool = True) -> float:
        """beta: (bx, by, bz) float32 face tensors of the sample's operator."""
        bx, by, bz = beta
        for t in (feat4, target, bx, by, bz):
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
        loss = C.c_double()
        self._chk("ns_net_train_step", lib().ns_net_train_step(
            self.net, feat4.data_ptr(), target.data_ptr(), bx.data_ptr(), by.data_ptr(), bz.data_ptr(),
            lr, 1 if update else 0, C.byref(loss)))
        return loss.value
