"""Thin ctypes binding of ``libadg.so`` (C ABI in ``include/adg.h``).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory and streams.  If the library is
missing, loading fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libadg.so")

ADG_OK, ADG_EINVAL, ADG_ENOMEM, ADG_EHIP, ADG_ESTATE, ADG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
ADG_BC_PERIODIC, ADG_BC_WALL = 0, 1
ADG_VAR_THETA, ADG_VAR_RHO = 0, 1
ADG_BATCH_PER_ORDER, ADG_BATCH_PERSISTENT = 0, 1

EXPORTED = [
    "adg_init_mesh", "adg_destroy", "adg_mesh_info", "adg_workspace_bytes", "adg_set_state",
    "adg_init_state", "adg_compute_dt", "adg_predictor", "adg_corrector", "adg_step",
    "adg_tv_indicator", "adg_check_health", "adg_last_error", "adg_basis", "adg_set_launch", "adg_step_static",
    "adg_autotune", "adg_batch_create", "adg_batch_destroy", "adg_batch_info", "adg_batch_scenario",
    "adg_batch_set_state", "adg_batch_init_state", "adg_batch_compute_dt", "adg_batch_step",
    "adg_batch_step_graph", "adg_batch_autotune", "adg_batch_set_launch", "adg_batch_set_mode", "adg_get_leaves",
    "adg_regrid_plan", "adg_regrid_apply", "adg_adjoint_workspace_bytes", "adg_step_adjoint",
    "adg_ic_theta", "adg_ic_theta_adjoint", "adg_loss_theta", "adg_loss_theta_adjoint",
    "adg_keep_bytes", "adg_step_keep", "adg_step_adjoint_kept",
    "adg3_init_mesh", "adg3_destroy", "adg3_mesh_info", "adg3_workspace_bytes", "adg3_set_state",
    "adg3_init_state", "adg3_compute_dt", "adg3_predictor", "adg3_corrector", "adg3_step",
    "adg3_check_health",
    "adg_fv_init", "adg_fv_destroy", "adg_fv_info", "adg_fv_workspace_bytes", "adg_fv_set_state",
    "adg_fv_init_state", "adg_fv_compute_dt", "adg_fv_predictor", "adg_fv_corrector", "adg_fv_step",
    "adg_fv_check_health",
    "adg_peaks_sink_bytes", "adg_measure_peaks", "adg_measure_fp64_sharing", "adg_step_to",
]


class AdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"adg error {code}: {msg}")
        self.code = code


class adg_params(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int), ("picard_iters", ctypes.c_int),
        ("gamma", ctypes.c_double), ("Pr", ctypes.c_double), ("R", ctypes.c_double),
        ("cp", ctypes.c_double), ("mu", ctypes.c_double), ("g", ctypes.c_double),
        ("p0", ctypes.c_double), ("theta_bg", ctypes.c_double),
        ("gravity", ctypes.c_int), ("mms", ctypes.c_int),
        ("mms_amp", ctypes.c_double), ("mms_u", ctypes.c_double), ("mms_w", ctypes.c_double),
        ("mms_kx", ctypes.c_double), ("mms_kz", ctypes.c_double), ("mms_p", ctypes.c_double),
        ("cfl", ctypes.c_double), ("fixed_dt", ctypes.c_int),
    ]


class adg_mesh_desc(ctypes.Structure):
    _fields_ = [
        ("x0", ctypes.c_double), ("z0", ctypes.c_double), ("Lx", ctypes.c_double),
        ("Lz", ctypes.c_double), ("nx", ctypes.c_int), ("nz", ctypes.c_int),
        ("max_level", ctypes.c_int), ("bc", ctypes.c_int * 4), ("n_leaves", ctypes.c_int),
        ("leaf_level", ctypes.POINTER(ctypes.c_int32)), ("leaf_i", ctypes.POINTER(ctypes.c_int32)),
        ("leaf_j", ctypes.POINTER(ctypes.c_int32)),
    ]


class adg3_mesh_desc(ctypes.Structure):
    _fields_ = [
        ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("z0", ctypes.c_double), ("h", ctypes.c_double),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("bc", ctypes.c_int * 6),
    ]


class adg_fv_desc(ctypes.Structure):
    _fields_ = [
        ("x0", ctypes.c_double), ("z0", ctypes.c_double), ("h", ctypes.c_double),
        ("nx", ctypes.c_int), ("nz", ctypes.c_int), ("bc", ctypes.c_int * 4),
    ]


_lib = None


# kinds of adg_init_state: the bubble states, the manufactured advected
# density wave, the paper's manufactured solution
INIT_KINDS = {"bubbles": 0, "mms": 1, "paper_mms": 2}

def lib():
    """Load libadg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1905_05524_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        L.adg_init_mesh.argtypes = [ctypes.POINTER(adg_params), ctypes.POINTER(adg_mesh_desc),
                                    ctypes.POINTER(vp)]
        L.adg_destroy.argtypes = [vp]
        L.adg_mesh_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.adg_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.adg_set_state.argtypes = [vp, vp, vp, vp]
        L.adg_init_state.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_double, vp]
        for name in ("adg_compute_dt", "adg_predictor", "adg_corrector", "adg_step", "adg_check_health"):
            getattr(L, name).argtypes = [vp, vp]
        L.adg_tv_indicator.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp]
        L.adg_step_static.argtypes = [vp, vp, vp, vp]
        L.adg_last_error.restype = ctypes.c_char_p
        L.adg_basis.argtypes = [vp, dp, dp, dp, dp]
        ip = ctypes.POINTER(ctypes.c_int)
        L.adg_set_launch.argtypes = [vp, ctypes.c_int, ctypes.c_int]
        L.adg_autotune.argtypes = [vp, ctypes.c_int, vp, ip, ip]
        L.adg_batch_create.argtypes = [ctypes.POINTER(adg_params), ctypes.POINTER(adg_mesh_desc), ctypes.c_int,
                                       ctypes.POINTER(vp)]
        L.adg_batch_destroy.argtypes = [vp]
        L.adg_batch_info.argtypes = [vp, ip, ip, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
        L.adg_batch_scenario.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t), ip, ip]
        L.adg_batch_set_state.argtypes = [vp, vp, vp, vp]
        L.adg_batch_init_state.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ctypes.c_double, vp]
        for name in ("adg_batch_compute_dt", "adg_batch_step", "adg_batch_step_graph"):
            getattr(L, name).argtypes = [vp, vp]
        L.adg_batch_autotune.argtypes = [vp, ctypes.c_int, vp, ip, ip]
        L.adg_batch_set_launch.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.adg_batch_set_mode.argtypes = [vp, ctypes.c_int]
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.adg_get_leaves.argtypes = [vp, i32p, i32p, i32p]
        L.adg_regrid_plan.argtypes = [vp, vp, ip, ctypes.POINTER(ctypes.c_size_t)]
        L.adg_regrid_apply.argtypes = [vp, vp, vp, vp, vp]
        L.adg_adjoint_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.adg_step_adjoint.argtypes = [vp, vp, vp, vp, vp, vp]
        L.adg_ic_theta.argtypes = [vp, vp, vp]
        L.adg_ic_theta_adjoint.argtypes = [vp, vp, vp, vp, vp]
        L.adg_loss_theta.argtypes = [vp, vp, vp, vp]
        L.adg_loss_theta_adjoint.argtypes = [vp, vp, vp, vp, vp]
        L.adg_keep_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
        L.adg_step_keep.argtypes = [vp, vp, vp, vp]
        L.adg_step_to.argtypes = [vp, vp, vp, vp, vp]
        L.adg_step_adjoint_kept.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.adg3_init_mesh.argtypes = [ctypes.POINTER(adg_params), ctypes.POINTER(adg3_mesh_desc), ctypes.POINTER(vp)]
        L.adg3_destroy.argtypes = [vp]
        L.adg3_mesh_info.argtypes = [vp, ip, ip]
        L.adg3_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.adg3_set_state.argtypes = [vp, vp, vp, vp]
        L.adg3_init_state.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_double, vp]
        for name in ("adg3_compute_dt", "adg3_predictor", "adg3_corrector", "adg3_step", "adg3_check_health"):
            getattr(L, name).argtypes = [vp, vp]
        L.adg_fv_init.argtypes = [ctypes.POINTER(adg_params), ctypes.POINTER(adg_fv_desc), ctypes.POINTER(vp)]
        L.adg_fv_destroy.argtypes = [vp]
        L.adg_fv_info.argtypes = [vp, ip]
        L.adg_fv_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.adg_fv_set_state.argtypes = [vp, vp, vp, vp]
        L.adg_fv_init_state.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_double, vp]
        for name in ("adg_fv_compute_dt", "adg_fv_predictor", "adg_fv_corrector", "adg_fv_step",
                     "adg_fv_check_health"):
            getattr(L, name).argtypes = [vp, vp]
        L.adg_peaks_sink_bytes.argtypes = [ctypes.POINTER(ctypes.c_size_t)]
        L.adg_measure_peaks.argtypes = [vp, vp, vp, ctypes.c_size_t, dp, vp]
        L.adg_measure_fp64_sharing.argtypes = [vp, dp, vp]
        _lib = L
    return _lib


def _check(rc):
    if rc != ADG_OK:
        raise AdgError(rc, lib().adg_last_error().decode())


def make_params(phys: dict, fixed_dt: bool = False) -> adg_params:
    p = adg_params()
    p.order = int(phys["N"])
    p.picard_iters = int(phys.get("picard_iters", 0))
    for k in ("gamma", "Pr", "R", "cp", "mu", "g", "p0", "theta_bg", "mms_amp", "mms_u", "mms_w",
              "mms_kx", "mms_kz", "mms_p", "cfl"):
        setattr(p, k, float(phys.get(k, 0.0)))
    p.gravity = int(phys.get("gravity", 0))
    p.mms = int(phys.get("mms", 0))
    p.fixed_dt = 1 if fixed_dt else 0
    return p


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_mesh_desc(mesh: dict, keep: list) -> adg_mesh_desc:
    """Fill an adg_mesh_desc; leaf arrays are appended to `keep` (they must
    outlive the call that reads them)."""
    d = adg_mesh_desc()
    d.x0, d.z0 = float(mesh.get("x0", 0.0)), float(mesh.get("z0", 0.0))
    d.Lx, d.Lz = float(mesh["Lx"]), float(mesh["Lz"])
    d.nx, d.nz = int(mesh["nx"]), int(mesh["nz"])
    d.max_level = int(mesh.get("max_level", 0))
    for k, b in enumerate(mesh.get("bc", [ADG_BC_WALL] * 4)):
        d.bc[k] = int(b)
    leaves = mesh.get("leaves")
    if leaves is not None:
        lv = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 3))
        cols = [np.ascontiguousarray(lv[:, k]) for k in range(3)]
        keep.extend(cols)
        d.n_leaves = lv.shape[0]
        d.leaf_level, d.leaf_i, d.leaf_j = (c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) for c in cols)
    return d


class Mesh:
    """Handle of one mesh + parameters; owns nothing on the device beyond the
    library's constant tables.  State buffers are torch tensors owned here."""

    def __init__(self, phys: dict, mesh: dict, fixed_dt: bool = False, device="cuda"):
        import torch
        self.phys, self.mesh_desc = dict(phys), dict(mesh)
        self._p = make_params(phys, fixed_dt)
        self._keep = []
        d = make_mesh_desc(mesh, self._keep)
        self._d = d
        h = ctypes.c_void_p()
        _check(lib().adg_init_mesh(ctypes.byref(self._p), ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        nc, nn = ctypes.c_int(), ctypes.c_int()
        _check(lib().adg_mesh_info(h, ctypes.byref(nc), ctypes.byref(nn)))
        self.C, self.n = nc.value, nn.value
        wb = ctypes.c_size_t()
        _check(lib().adg_workspace_bytes(h, ctypes.byref(wb)))
        self.ws_bytes = wb.value
        self.device = torch.device(device)
        self.Q = torch.zeros((self.C, 4, self.n, self.n), dtype=torch.float64, device=self.device)
        # 256-byte aligned workspace (torch allocations are at least 512-aligned)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)
        self.clock = torch.zeros(4, dtype=torch.float64, device=self.device)
        self.bind()

    def bind(self):
        _check(lib().adg_set_state(self.h, ctypes.c_void_p(self.Q.data_ptr()),
                                   ctypes.c_void_p(self.ws.data_ptr()),
                                   ctypes.c_void_p(self.clock.data_ptr())))

    def bind_state(self, Q):
        """Bind another state tensor (same shape) with the same workspace and
        clock: a host-side pointer change, no device work.  bind() rebinds
        self.Q."""
        _check(lib().adg_set_state(self.h, ctypes.c_void_p(Q.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                                   ctypes.c_void_p(self.clock.data_ptr())))

    def bind_clock(self, clock):
        """Bind another device clock (double[4] tensor) with the same state
        and workspace: a host-side pointer change, no device work."""
        _check(lib().adg_set_state(self.h, ctypes.c_void_p(self.Q.data_ptr()),
                                   ctypes.c_void_p(self.ws.data_ptr()), ctypes.c_void_p(clock.data_ptr())))

    @property
    def fixed_dt(self):
        return bool(self._p.fixed_dt)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().adg_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # -- calls with the C names --------------------------------------------
    def init_state(self, kind="bubbles", bubbles=(), t0=0.0, stream=None):
        bb = np.ascontiguousarray(np.asarray(bubbles, dtype=np.float64).reshape(-1, 6))
        k = INIT_KINDS[kind]
        _check(lib().adg_init_state(self.h, k, bb.shape[0],
                                    bb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(t0),
                                    _stream_ptr(stream)))

    def set_state(self, Q, t=None, dt=None):
        """Copy a state (numpy or tensor [C,4,n,n]) into the bound buffer."""
        import torch
        self.Q.copy_(torch.as_tensor(np.asarray(Q) if not torch.is_tensor(Q) else Q, dtype=torch.float64))
        if t is not None:
            self.clock[0] = float(t)
        if dt is not None:
            self.clock[1] = float(dt)

    def compute_dt(self, stream=None):
        _check(lib().adg_compute_dt(self.h, _stream_ptr(stream)))

    def predictor(self, stream=None):
        _check(lib().adg_predictor(self.h, _stream_ptr(stream)))

    def corrector(self, stream=None):
        _check(lib().adg_corrector(self.h, _stream_ptr(stream)))

    def step(self, stream=None):
        _check(lib().adg_step(self.h, _stream_ptr(stream)))

    def step_to(self, Q_out, store=None, fd=None, stream=None):
        """adg_step_to: one step from the bound state into Q_out (keeping the
        iterates in store/fd when given); the bound state is left as it was."""
        vp = ctypes.c_void_p
        _check(lib().adg_step_to(self.h, vp(Q_out.data_ptr()), vp(store.data_ptr()) if store is not None else None,
                                 vp(fd.data_ptr()) if fd is not None else None, _stream_ptr(stream)))

    def step_static(self, Q, clock, stream=None):
        """adg_step_static: one step of the caller's Q and clock (device
        tensors) with the library's static workspace; allocates nothing."""
        _check(lib().adg_step_static(self.h, ctypes.c_void_p(Q.data_ptr()), ctypes.c_void_p(clock.data_ptr()),
                                     _stream_ptr(stream)))

    def tv_indicator(self, var, T_refine, T_coarsen, tv, flags, stats, stream=None):
        _check(lib().adg_tv_indicator(self.h, int(var), float(T_refine), float(T_coarsen),
                                      ctypes.c_void_p(tv.data_ptr()), ctypes.c_void_p(flags.data_ptr()),
                                      ctypes.c_void_p(stats.data_ptr()), _stream_ptr(stream)))

    def check_health(self, stream=None):
        _check(lib().adg_check_health(self.h, _stream_ptr(stream)))

    def leaves(self):
        lv = np.zeros((self.C, 3), dtype=np.int32)
        cols = [np.zeros(self.C, dtype=np.int32) for _ in range(3)]
        p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        _check(lib().adg_get_leaves(self.h, p(cols[0]), p(cols[1]), p(cols[2])))
        for k in range(3):
            lv[:, k] = cols[k]
        return lv

    def regrid(self, flags, stream=None):
        """Regrid with per-cell flags (host array or tensor of -1/0/+1); the
        state moves to newly allocated buffers.  Returns the new cell count."""
        import torch
        f = np.ascontiguousarray(np.asarray(flags.cpu() if torch.is_tensor(flags) else flags, dtype=np.int8))
        if f.shape != (self.C,):
            raise ValueError("flags must have one entry per cell")
        nc, wb = ctypes.c_int(), ctypes.c_size_t()
        _check(lib().adg_regrid_plan(self.h, ctypes.c_void_p(f.ctypes.data), ctypes.byref(nc), ctypes.byref(wb)))
        Qn = torch.empty((nc.value, 4, self.n, self.n), dtype=torch.float64, device=self.device)
        wsn = torch.empty(max(wb.value, 256), dtype=torch.uint8, device=self.device)
        _check(lib().adg_regrid_apply(self.h, ctypes.c_void_p(Qn.data_ptr()), ctypes.c_void_p(wsn.data_ptr()),
                                      ctypes.c_void_p(self.clock.data_ptr()), _stream_ptr(stream)))
        self.Q, self.ws, self.C, self.ws_bytes = Qn, wsn, nc.value, wb.value
        return self.C

    # -- adjoint ---------------------------------------------------------------
    def adjoint_workspace(self):
        import torch
        if getattr(self, "_adj_ws", None) is None:
            b = ctypes.c_size_t()
            _check(lib().adg_adjoint_workspace_bytes(self.h, ctypes.byref(b)))
            self._adj_ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device=self.device)
        return self._adj_ws

    def step_adjoint(self, Q_n, lam_np1, lam_n, stream=None):
        ws = self.adjoint_workspace()
        _check(lib().adg_step_adjoint(self.h, ctypes.c_void_p(Q_n.data_ptr()), ctypes.c_void_p(lam_np1.data_ptr()),
                                      ctypes.c_void_p(lam_n.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                      _stream_ptr(stream)))

    def keep_bytes(self):
        """(store bytes, face-data bytes) of one kept step."""
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().adg_keep_bytes(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def step_keep(self, store, fd, stream=None):
        _check(lib().adg_step_keep(self.h, ctypes.c_void_p(store.data_ptr()), ctypes.c_void_p(fd.data_ptr()),
                                   _stream_ptr(stream)))

    def step_adjoint_kept(self, Q_n, store, fd, lam_np1, lam_n, stream=None):
        ws = self.adjoint_workspace()
        _check(lib().adg_step_adjoint_kept(self.h, ctypes.c_void_p(Q_n.data_ptr()), ctypes.c_void_p(store.data_ptr()),
                                           ctypes.c_void_p(fd.data_ptr()), ctypes.c_void_p(lam_np1.data_ptr()),
                                           ctypes.c_void_p(lam_n.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                           _stream_ptr(stream)))

    def ic_theta(self, theta_prime, stream=None):
        _check(lib().adg_ic_theta(self.h, ctypes.c_void_p(theta_prime.data_ptr()), _stream_ptr(stream)))

    def ic_theta_adjoint(self, theta_prime, lam, grad, stream=None):
        _check(lib().adg_ic_theta_adjoint(self.h, ctypes.c_void_p(theta_prime.data_ptr()),
                                          ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                                          _stream_ptr(stream)))

    def loss_theta(self, out, stream=None):
        ws = self.adjoint_workspace()
        _check(lib().adg_loss_theta(self.h, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                    _stream_ptr(stream)))

    def loss_theta_adjoint(self, loss, grad_loss, lam, stream=None):
        _check(lib().adg_loss_theta_adjoint(self.h, ctypes.c_void_p(loss.data_ptr()),
                                            ctypes.c_void_p(grad_loss.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
                                            _stream_ptr(stream)))

    def set_launch(self, cells_per_wave: int, waves_per_block: int):
        _check(lib().adg_set_launch(self.h, int(cells_per_wave), int(waves_per_block)))

    def autotune(self, reps: int = 5, stream=None):
        c, w = ctypes.c_int(), ctypes.c_int()
        _check(lib().adg_autotune(self.h, int(reps), _stream_ptr(stream), ctypes.byref(c), ctypes.byref(w)))
        return c.value, w.value

    def basis(self):
        n = self.n
        xi, w, D, P = np.zeros(n), np.zeros(n), np.zeros((n, n)), np.zeros((n, n))
        dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        _check(lib().adg_basis(self.h, dp(xi), dp(w), dp(D), dp(P)))
        return dict(xi=xi, w=w, D=D, P=P)

    # -- views of the workspace (predictor outputs) --------------------------
    def qstar(self):
        nn = self.n * self.n
        return self.ws[:self.C * 4 * nn * 8].view(torch_float64()).view(self.C, 4, self.n, self.n)

    def face_data(self):
        import torch
        n = self.n
        off = _align256(self.C * 4 * n * n * 8)
        return self.ws[off:off + self.C * 32 * n * 8].view(torch.float64).view(self.C, 4, 2, 4, n)

    @property
    def t(self):
        return float(self.clock[0].item())

    @property
    def dt(self):
        return float(self.clock[1].item())


def make_mesh3_desc(mesh: dict) -> adg3_mesh_desc:
    d = adg3_mesh_desc()
    d.x0, d.y0, d.z0 = (float(mesh.get(k, 0.0)) for k in ("x0", "y0", "z0"))
    d.h = float(mesh["h"])
    d.nx, d.ny, d.nz = int(mesh["nx"]), int(mesh["ny"]), int(mesh["nz"])
    for k, b in enumerate(mesh.get("bc", [ADG_BC_WALL] * 6)):
        d.bc[k] = int(b)
    return d


class Mesh3:
    """Handle of a three-dimensional uniform grid + parameters (C ABI in
    ``include/adg3.h``); state buffers are torch tensors owned here."""

    def __init__(self, phys: dict, mesh: dict, fixed_dt: bool = False, device="cuda"):
        import torch
        self.phys, self.mesh_desc = dict(phys), dict(mesh)
        self._p = make_params(phys, fixed_dt)
        self._d = make_mesh3_desc(mesh)
        h = ctypes.c_void_p()
        _check(lib().adg3_init_mesh(ctypes.byref(self._p), ctypes.byref(self._d), ctypes.byref(h)))
        self.h = h
        nc, nn = ctypes.c_int(), ctypes.c_int()
        _check(lib().adg3_mesh_info(h, ctypes.byref(nc), ctypes.byref(nn)))
        self.C, self.n = nc.value, nn.value
        wb = ctypes.c_size_t()
        _check(lib().adg3_workspace_bytes(h, ctypes.byref(wb)))
        self.ws_bytes = wb.value
        self.device = torch.device(device)
        n = self.n
        self.Q = torch.zeros((self.C, 5, n, n, n), dtype=torch.float64, device=self.device)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)
        self.clock = torch.zeros(4, dtype=torch.float64, device=self.device)
        _check(lib().adg3_set_state(self.h, ctypes.c_void_p(self.Q.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                                    ctypes.c_void_p(self.clock.data_ptr())))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().adg3_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def init_state(self, kind="bubbles", bubbles=(), t0=0.0, stream=None):
        bb = np.ascontiguousarray(np.asarray(bubbles, dtype=np.float64).reshape(-1, 7))
        _check(lib().adg3_init_state(self.h, 1 if kind == "abc" else 0, bb.shape[0],
                                     bb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(t0),
                                     _stream_ptr(stream)))

    def set_state(self, Q, t=None, dt=None):
        """Copy a state (numpy or tensor [C,5,n,n,n]) into the bound buffer."""
        import torch
        self.Q.copy_(torch.as_tensor(np.asarray(Q) if not torch.is_tensor(Q) else Q, dtype=torch.float64))
        if t is not None:
            self.clock[0] = float(t)
        if dt is not None:
            self.clock[1] = float(dt)

    def compute_dt(self, stream=None):
        _check(lib().adg3_compute_dt(self.h, _stream_ptr(stream)))

    def predictor(self, stream=None):
        _check(lib().adg3_predictor(self.h, _stream_ptr(stream)))

    def corrector(self, stream=None):
        _check(lib().adg3_corrector(self.h, _stream_ptr(stream)))

    def step(self, stream=None):
        _check(lib().adg3_step(self.h, _stream_ptr(stream)))

    def check_health(self, stream=None):
        _check(lib().adg3_check_health(self.h, _stream_ptr(stream)))

    # -- views of the workspace (predictor outputs) --------------------------
    def qstar(self):
        import torch
        n = self.n
        return self.ws[:self.C * 5 * n ** 3 * 8].view(torch.float64).view(self.C, 5, n, n, n)

    def face_data(self):
        import torch
        n = self.n
        off = _align256(self.C * 5 * n ** 3 * 8)
        return self.ws[off:off + self.C * 60 * n * n * 8].view(torch.float64).view(self.C, 6, 2, 5, n, n)

    def cell_dt(self):
        import torch
        n = self.n
        off = _align256(self.C * 5 * n ** 3 * 8)
        off = _align256(off + self.C * 60 * n * n * 8)
        return self.ws[off:off + self.C * 8].view(torch.float64)

    @property
    def t(self):
        return float(self.clock[0].item())

    @property
    def dt(self):
        return float(self.clock[1].item())


def make_fv_desc(mesh: dict) -> adg_fv_desc:
    """Finite-volume grid from the 2D mesh dict (nx, nz, x0, z0, Lx, Lz, bc)."""
    d = adg_fv_desc()
    d.x0, d.z0 = float(mesh.get("x0", 0.0)), float(mesh.get("z0", 0.0))
    d.h = float(mesh["Lx"]) / int(mesh["nx"]) if int(mesh["nx"]) > 0 else 0.0
    d.nx, d.nz = int(mesh["nx"]), int(mesh["nz"])
    for k, b in enumerate(mesh.get("bc", [ADG_BC_WALL] * 4)):
        d.bc[k] = int(b)
    return d


class FV:
    """Handle of the MUSCL-Hancock finite-volume scheme (C ABI in
    ``include/adg_fv.h``); Q [C][4] and the workspace are torch tensors."""

    def __init__(self, phys: dict, mesh: dict, fixed_dt: bool = False, device="cuda"):
        import torch
        self.phys, self.mesh_desc = dict(phys), dict(mesh)
        self._p = make_params(dict(phys, N=0), fixed_dt)
        self._d = make_fv_desc(mesh)
        h = ctypes.c_void_p()
        _check(lib().adg_fv_init(ctypes.byref(self._p), ctypes.byref(self._d), ctypes.byref(h)))
        self.h = h
        nc = ctypes.c_int()
        _check(lib().adg_fv_info(h, ctypes.byref(nc)))
        self.C = nc.value
        wb = ctypes.c_size_t()
        _check(lib().adg_fv_workspace_bytes(h, ctypes.byref(wb)))
        self.ws_bytes = wb.value
        self.device = torch.device(device)
        self.Q = torch.zeros((self.C, 4), dtype=torch.float64, device=self.device)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)
        self.clock = torch.zeros(4, dtype=torch.float64, device=self.device)
        _check(lib().adg_fv_set_state(self.h, ctypes.c_void_p(self.Q.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                                      ctypes.c_void_p(self.clock.data_ptr())))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().adg_fv_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def init_state(self, kind="bubbles", bubbles=(), t0=0.0, stream=None):
        bb = np.ascontiguousarray(np.asarray(bubbles, dtype=np.float64).reshape(-1, 6))
        _check(lib().adg_fv_init_state(self.h, 1 if kind == "wave" else 0, bb.shape[0],
                                       bb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(t0),
                                       _stream_ptr(stream)))

    def set_state(self, Q, t=None, dt=None):
        import torch
        self.Q.copy_(torch.as_tensor(np.asarray(Q) if not torch.is_tensor(Q) else Q, dtype=torch.float64))
        if t is not None:
            self.clock[0] = float(t)
        if dt is not None:
            self.clock[1] = float(dt)

    def compute_dt(self, stream=None):
        _check(lib().adg_fv_compute_dt(self.h, _stream_ptr(stream)))

    def predictor(self, stream=None):
        _check(lib().adg_fv_predictor(self.h, _stream_ptr(stream)))

    def corrector(self, stream=None):
        _check(lib().adg_fv_corrector(self.h, _stream_ptr(stream)))

    def step(self, stream=None):
        _check(lib().adg_fv_step(self.h, _stream_ptr(stream)))

    def check_health(self, stream=None):
        _check(lib().adg_fv_check_health(self.h, _stream_ptr(stream)))

    def face_values(self):
        """Evolved face values as [C][4 faces][4 vars] (a copy)."""
        import torch
        E = self.ws[:16 * self.C * 8].view(torch.float64).view(4, 4, self.C)
        return E.permute(2, 0, 1).contiguous()

    @property
    def t(self):
        return float(self.clock[0].item())

    @property
    def dt(self):
        return float(self.clock[1].item())


class Batch:
    """Many independent scenarios stepped together (scenarios grouped by
    order; one device state array, one clock per scenario)."""

    def __init__(self, workloads: list, fixed_dt: bool = False, device="cuda"):
        import torch
        S = len(workloads)
        self.workloads = workloads
        P = (adg_params * S)()
        D = (adg_mesh_desc * S)()
        self._keep = []
        for s, w in enumerate(workloads):
            P[s] = make_params(w["phys"], fixed_dt)
            D[s] = make_mesh_desc(w["mesh"], self._keep)
        h = ctypes.c_void_p()
        _check(lib().adg_batch_create(P, D, S, ctypes.byref(h)))
        self.h = h
        self.S = S
        ng, tc = ctypes.c_int(), ctypes.c_int()
        qd, wb = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().adg_batch_info(h, ctypes.byref(ng), ctypes.byref(tc), ctypes.byref(qd), ctypes.byref(wb)))
        self.n_groups, self.C_total, self.q_doubles, self.ws_bytes = ng.value, tc.value, qd.value, wb.value
        self.device = torch.device(device)
        self.Q = torch.zeros(max(self.q_doubles, 1), dtype=torch.float64, device=self.device)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)
        self.clock = torch.zeros((S, 4), dtype=torch.float64, device=self.device)
        self.scen = []
        for s in range(S):
            off, nc, nn = ctypes.c_size_t(), ctypes.c_int(), ctypes.c_int()
            _check(lib().adg_batch_scenario(h, s, ctypes.byref(off), ctypes.byref(nc), ctypes.byref(nn)))
            self.scen.append((off.value, nc.value, nn.value))
        _check(lib().adg_batch_set_state(h, ctypes.c_void_p(self.Q.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                                         ctypes.c_void_p(self.clock.data_ptr())))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().adg_batch_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def state(self, s):
        """View of scenario s's state [C][4][n][n]."""
        off, C, n = self.scen[s]
        return self.Q[off:off + C * 4 * n * n].view(C, 4, n, n)

    def init_state(self, s, kind="bubbles", bubbles=(), t0=0.0, stream=None):
        bb = np.ascontiguousarray(np.asarray(bubbles, dtype=np.float64).reshape(-1, 6))
        _check(lib().adg_batch_init_state(self.h, int(s), INIT_KINDS[kind], bb.shape[0],
                                          bb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(t0),
                                          _stream_ptr(stream)))

    def compute_dt(self, stream=None):
        _check(lib().adg_batch_compute_dt(self.h, _stream_ptr(stream)))

    def step(self, stream=None):
        _check(lib().adg_batch_step(self.h, _stream_ptr(stream)))

    def step_graph(self, stream):
        _check(lib().adg_batch_step_graph(self.h, _stream_ptr(stream)))

    def autotune(self, reps: int = 5, stream=None):
        G = self.n_groups
        c, w = (ctypes.c_int * G)(), (ctypes.c_int * G)()
        _check(lib().adg_batch_autotune(self.h, int(reps), _stream_ptr(stream), c, w))
        return list(c), list(w)

    def set_launch(self, group: int, cells_per_wave: int, waves_per_block: int):
        _check(lib().adg_batch_set_launch(self.h, int(group), int(cells_per_wave), int(waves_per_block)))

    def set_mode(self, mode: int):
        """ADG_BATCH_PER_ORDER (0) or ADG_BATCH_PERSISTENT (1) predictor."""
        _check(lib().adg_batch_set_mode(self.h, int(mode)))


def measure_peaks(copy_mib: int = 1024, stream=None) -> dict:
    """Measured FP64 vector and matrix-core rates and copy bandwidth of the
    current device (``include/adg_peaks.h``), beside the published figures."""
    import torch
    nb = ctypes.c_size_t()
    _check(lib().adg_peaks_sink_bytes(ctypes.byref(nb)))
    sink = torch.empty(nb.value // 8, dtype=torch.float64, device="cuda")
    n = (copy_mib << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    out = (ctypes.c_double * 3)()
    _check(lib().adg_measure_peaks(ctypes.c_void_p(sink.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                   ctypes.c_void_p(dst.data_ptr()), n * 8, out, _stream_ptr(stream)))
    if not torch.equal(src[:1024], dst[:1024]) or not torch.equal(src[-1024:], dst[-1024:]):
        raise AdgError(ADG_ESTATE, "peak copy produced wrong data")
    sh = (ctypes.c_double * 5)()
    _check(lib().adg_measure_fp64_sharing(ctypes.c_void_p(sink.data_ptr()), sh, _stream_ptr(stream)))
    pr = torch.cuda.get_device_properties(torch.cuda.current_device())
    return {"fp64_sharing": {"mfma_4x4x4_tflops": sh[0], "fma_tflops": sh[1], "half_and_half_tflops": sh[2],
                             "half_and_half_mfma_part": sh[3], "half_and_half_fma_part": sh[4]},
            "fp64_vector_tflops": out[0], "fp64_vector_tflops_spec": 78.6,
            "fp64_mfma_tflops": out[1], "fp64_mfma_tflops_spec": 78.6,
            "copy_GBps": out[2], "hbm_GBps_spec": 8000.0, "copy_bytes": n * 8,
            "device": {"name": pr.name, "arch": getattr(pr, "gcnArchName", ""),
                       "compute_units": pr.multi_processor_count, "memory_bytes": pr.total_memory,
                       "lds_per_block_bytes": pr.shared_memory_per_block, "wavefront": pr.warp_size,
                       "l2_bytes": getattr(pr, "L2_cache_size", None)}}


def _align256(x):
    return (x + 255) & ~255


def torch_float64():
    import torch
    return torch.float64
