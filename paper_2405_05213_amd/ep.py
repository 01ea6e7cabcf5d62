"""Thin ctypes binding of libep.so (include/ep.h).

Argument marshalling only: every numerical step runs in the HIP library.  PyTorch is
used for device memory (the workspace and device vectors) and the stream.
Importing works without a GPU; calls that need the library raise if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libep.so")

EP_OK, EP_ERR_ARG, EP_ERR_ORDER, EP_ERR_HIP, EP_ERR_KRYLOV = 0, -1, -2, -3, -4
EP_ERR_INVERTED, EP_ERR_NONFINITE, EP_ERR_WORKSPACE, EP_ERR_DEVICE = -5, -6, -7, -8
MODELS = {"linear": 0, "nh": 1, "yeoh": 2, "svk": 3}
S0_AUTO, S0_SCALED = -1.0, -2.0          # ep_set_krylov's s0 modes (include/ep.h)
PRECISIONS = {"f64": 0, "mixed_f32": 1, "mixed_bf16": 2}

_i64, _i32, _dbl, _vp = C.c_int64, C.c_int32, C.c_double, C.c_void_p
_P = C.POINTER


class EPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ep error {code}: {msg}")
        self.code = code


_lib = None

_SIGS = {
    "ep_create": [_P(_vp), C.c_int],
    "ep_destroy": [_vp],
    "ep_last_error": [_vp],
    "ep_version": [],
    "ep_set_stream": [_vp, _vp],
    "ep_set_mesh_hex8": [_vp, _i64, _vp, _i64, _vp],
    "ep_set_mesh_hex27": [_vp, _i64, _vp, _i64, _vp],
    "ep_set_material": [_vp, C.c_int, _vp, C.c_int, _dbl],
    "ep_set_dirichlet": [_vp, _i64, _vp],
    "ep_set_traction": [_vp, _i64, _vp, _vp, _i64, _vp, _vp],
    "ep_set_krylov": [_vp, _dbl, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _dbl],
    "ep_set_precision": [_vp, C.c_int],
    "ep_set_scheme": [_vp, C.c_int],
    "ep_set_orthogonalization": [_vp, C.c_int],
    "ep_get_launch": [_vp, _P(C.c_int), _P(C.c_int), _P(C.c_int), _P(C.c_int)],
    "ep_get_orthogonalization": [_vp, _P(C.c_int)],
    "ep_set_launch": [_vp, C.c_int],
    "ep_autotune": [_vp, _dbl, C.c_int, C.c_int, _P(C.c_int), _P(_dbl)],
    "ep_workspace_size": [_vp, _P(C.c_size_t)],
    "ep_bind_workspace": [_vp, _vp, C.c_size_t],
    "ep_set_state": [_vp, _dbl, _vp, _vp],
    "ep_step": [_vp, _dbl, _i64],
    "ep_sync": [_vp],
    "ep_get_state": [_vp, _P(_dbl), _vp, _vp],
    "ep_get_energy": [_vp, _P(_dbl), _P(_dbl), _P(_dbl)],
    "ep_checkpoint_size": [_vp, _P(C.c_size_t)],
    "ep_save_checkpoint": [_vp, _vp, C.c_size_t],
    "ep_load_checkpoint": [_vp, _vp, C.c_size_t],
    "ep_get_stats": [_vp, _P(_i64), _P(C.c_int), _P(_dbl), _P(C.c_int), _P(_dbl)],
    "ep_get_step_log": [_vp, C.c_int, _vp, _vp, _vp, _vp],
    "ep_apply_H": [_vp, _vp, _vp, _vp],
    "ep_form_tangents": [_vp, _vp],
    "ep_apply_A": [_vp, _vp, _dbl, _dbl, _vp, _vp],
    "ep_vector_length": [_vp, _P(_i64), _P(_i64)],
    "ep_expm": [_vp, C.c_int, _vp, _vp],
    "ep_expm_noalloc": [C.c_int, _vp, _vp, _vp],
    "ep_arnoldi": [_vp, _vp, _dbl, _dbl, _vp, C.c_int, _vp, _vp, _P(C.c_int)],
    "ep_expv": [_vp, _vp, _dbl, _dbl, _vp, _vp, _P(C.c_int), _P(C.c_int), _P(_dbl)],
    "ep_batch_add_instance": [_vp, _i64, _vp, _i64, _vp, C.c_int, _vp, C.c_int, _dbl, _i64, _vp, _i64, _vp,
                              _vp, _i64, _vp, _vp, _P(_i32)],
    "ep_batch_set_state": [_vp, _i32, _dbl, _vp, _vp],
    "ep_batch_step": [_vp, _dbl, _i64],
    "ep_batch_get_state": [_vp, _i32, _P(_dbl), _vp, _vp],
    "ep_batch_get_stats": [_vp, _i32, _P(_i64), _P(C.c_int), _P(C.c_int), _P(_dbl), _P(_i64), _P(C.c_int),
                           _P(C.c_int)],
    "ep_batch_get_energy": [_vp, _i32, _P(_dbl), _P(_dbl), _P(_dbl)],
    "ep_batch_plan": [_vp, C.c_int, _dbl],
    "ep_batch_autotune": [_vp, _dbl, C.c_int, _P(C.c_int), _P(_dbl)],
    "ep_batch_get_plan": [_vp, _i32, _P(C.c_int), _P(C.c_int)],
    "ep_batch_get_time": [_vp, _i32, _P(_dbl), _P(_i64)],
    "ep_batch_checkpoint_size": [_vp, _i32, _P(C.c_size_t)],
    "ep_batch_save_checkpoint": [_vp, _i32, _vp, C.c_size_t],
    "ep_batch_load_checkpoint": [_vp, _i32, _vp, C.c_size_t],
}
EXPORTED = sorted(_SIGS)


def lib():
    """Load libep.so; raises (loudly) if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2405_05213_amd.build")
        # torch's HIP runtime must be initialised first: loading the library's device code
        # before it leaves torch without visible GPUs
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_char_p if name in ("ep_last_error", "ep_version") else C.c_int
        _lib = L
    return _lib


def _ptr(a):
    """Host numpy array or torch tensor -> void pointer (None stays None)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32a(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


class Context:
    """One ep_ctx.  device=-1 gives a host-only context (validation only)."""

    def __init__(self, device: int = 0, stream=None):
        self._L = lib()
        h = C.c_void_p()
        rc = self._L.ep_create(C.byref(h), device)
        if rc != EP_OK:
            raise EPError(rc, f"ep_create(device={device}) failed")
        self.h = h
        self.device = device
        self.workspace = None
        if stream is not None:
            self._call("ep_set_stream", C.c_void_p(stream))

    def close(self):
        """Release the context (its HIP graphs and host state) now."""
        h = getattr(self, "h", None)
        if h is not None and getattr(self, "_L", None) is not None:
            self._L.ep_destroy(h)
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        # during interpreter shutdown the HIP runtime (and a profiler attached to it) may
        # already be finalised: destroying graphs then is unsafe, and the process is ending
        if sys.is_finalizing():
            return
        self.close()

    def _call(self, name, *args):
        rc = getattr(self._L, name)(self.h, *args)
        if rc != EP_OK:
            msg = self._L.ep_last_error(self.h)
            raise EPError(rc, msg.decode() if msg else name)
        return rc

    # ---------------------------------------------------------------- setup
    def set_mesh(self, xyz, conn):
        """hex8 (conn n_e x 8) or quadratic 27-node hexahedra (conn n_e x 27)."""
        self._xyz, self._conn = _f64(xyz), _i32a(conn)
        name = "ep_set_mesh_hex27" if self._conn.shape[1] == 27 else "ep_set_mesh_hex8"
        self._call(name, self._xyz.shape[0], _ptr(self._xyz), self._conn.shape[0], _ptr(self._conn))
        self.n_nodes = self._xyz.shape[0]

    def set_material(self, model: str, params, rho: float):
        p = _f64(params)
        self._call("ep_set_material", MODELS[model], _ptr(p), p.size, float(rho))

    def set_dirichlet(self, dofs):
        d = _i32a(dofs)
        self._call("ep_set_dirichlet", d.size, _ptr(d))

    def set_traction(self, faces, t0, knots_t, knots_s):
        f = _i32a(faces)
        f = f.reshape(-1, f.shape[-1] if f.ndim == 2 else 4)
        t = _f64(t0)
        kt, ks = _f64(knots_t), _f64(knots_s)
        self._call("ep_set_traction", f.shape[0], _ptr(f), _ptr(t), kt.size, _ptr(kt), _ptr(ks))

    def set_krylov(self, tol=1e-10, m_max=64, check_every=4, m_fixed=0, k_fixed=0, max_substeps=64, s0=-1.0):
        self._call("ep_set_krylov", float(tol), int(m_max), int(check_every), int(m_fixed), int(k_fixed),
                   int(max_substeps), float(s0))

    def set_precision(self, prec: str):
        self._call("ep_set_precision", PRECISIONS[prec])

    def set_scheme(self, order: int):
        """Time integrator: 2 (the paper's second-order step) or 4 (two-term Magnus)."""
        self._call("ep_set_scheme", int(order))

    def set_orthogonalization(self, mode: int):
        """-1 automatic, 0 sequential MGS, 1 MGS in compact-WY form (see include/ep.h)."""
        self._call("ep_set_orthogonalization", int(mode))

    def orthogonalization(self) -> int:
        m = C.c_int()
        self._call("ep_get_orthogonalization", C.byref(m))
        return m.value

    def launch(self):
        """(workgroups, entries per workgroup, mesh class: 0 general, 1 congruent, 2 lattice)."""
        g, ch, sg, cg = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        self._call("ep_get_launch", C.byref(g), C.byref(ch), C.byref(sg), C.byref(cg))
        return g.value, ch.value, cg.value

    def slices_in_device_memory(self) -> bool:
        sg = C.c_int()
        self._call("ep_get_launch", None, None, C.byref(sg), None)
        return bool(sg.value)

    def set_launch(self, workgroups: int):
        self._call("ep_set_launch", int(workgroups))

    def autotune(self, dt, m_trial=16, trials=3):
        g, ms = C.c_int(), C.c_double()
        self._call("ep_autotune", float(dt), int(m_trial), int(trials), C.byref(g), C.byref(ms))
        return g.value, ms.value

    def workspace_size(self) -> int:
        n = C.c_size_t()
        self._call("ep_workspace_size", C.byref(n))
        return n.value

    def bind(self):
        import torch
        n = self.workspace_size()
        self.workspace = torch.empty(n + 256, dtype=torch.uint8, device=f"cuda:{self.device}")
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._call("ep_bind_workspace", C.c_void_p(base + off), n)

    # ---------------------------------------------------------------- state
    def set_state(self, t, u, v):
        u, v = _f64(u), _f64(v)
        self._call("ep_set_state", float(t), _ptr(u), _ptr(v))

    def step(self, dt, n_steps=1):
        self._call("ep_step", float(dt), int(n_steps))

    def sync(self):
        self._call("ep_sync")

    def get_state(self):
        t = C.c_double()
        u = np.empty(3 * self.n_nodes)
        v = np.empty(3 * self.n_nodes)
        self._call("ep_get_state", C.byref(t), _ptr(u), _ptr(v))
        return t.value, u, v

    def save_checkpoint(self) -> bytes:
        """Opaque image of the whole stepping state (ep_save_checkpoint)."""
        n = C.c_size_t()
        self._call("ep_checkpoint_size", C.byref(n))
        buf = C.create_string_buffer(n.value)
        self._call("ep_save_checkpoint", buf, n.value)
        return buf.raw

    def load_checkpoint(self, image: bytes):
        """Resume from an image of save_checkpoint (ep_load_checkpoint)."""
        buf = C.create_string_buffer(bytes(image), len(image))
        self._call("ep_load_checkpoint", buf, len(image))

    def energy(self):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        self._call("ep_get_energy", C.byref(a), C.byref(b), C.byref(c))
        return a.value, b.value, c.value

    def stats(self):
        mv, m, k = C.c_int64(), C.c_int(), C.c_int()
        eps, dr = C.c_double(), C.c_double()
        self._call("ep_get_stats", C.byref(mv), C.byref(m), C.byref(eps), C.byref(k), C.byref(dr))
        return {"matvecs": mv.value, "m": m.value, "eps": eps.value, "k": k.value, "drift": dr.value}

    def step_log(self, n):
        mc, mp, kc = (np.zeros(n, np.int32) for _ in range(3))
        ec = np.zeros(n)
        self._call("ep_get_step_log", int(n), _ptr(mc), _ptr(mp), _ptr(kc), _ptr(ec))
        return {"m_corr": mc, "m_pred": mp, "k_corr": kc, "eps_corr": ec}

    # ---------------------------------------------------------------- stages (device tensors)
    def vector_length(self):
        a, b = C.c_int64(), C.c_int64()
        self._call("ep_vector_length", C.byref(a), C.byref(b))
        return a.value, b.value

    def apply_H(self, u_lin, x, y, sync=True):
        self._call("ep_apply_H", _ptr(u_lin), _ptr(x), _ptr(y))
        if sync:
            self.sync()

    def form_tangents(self, u_lin, sync=True):
        self._call("ep_form_tangents", _ptr(u_lin))
        if sync:
            self.sync()

    def apply_A(self, u_lin, tau, pscale, x, y):
        self._call("ep_apply_A", _ptr(u_lin), float(tau), float(pscale), _ptr(x), _ptr(y))

    def expm(self, H):
        H = _f64(H)
        m = H.shape[0]
        E = np.empty((m, m))
        self._call("ep_expm", int(m), _ptr(H), _ptr(E))
        return E

    def arnoldi(self, u_lin, tau, pscale, w, m, V=None):
        H = np.zeros((m + 1, m))
        steps = C.c_int()
        self._call("ep_arnoldi", _ptr(u_lin), float(tau), float(pscale), _ptr(w), int(m), _ptr(V), _ptr(H),
                   C.byref(steps))
        return H, steps.value

    def expv(self, u_lin, tau, pscale, w, y):
        m, k, e = C.c_int(), C.c_int(), C.c_double()
        self._call("ep_expv", _ptr(u_lin), float(tau), float(pscale), _ptr(w), _ptr(y), C.byref(m), C.byref(k),
                   C.byref(e))
        return m.value, k.value, e.value


def expm_noalloc(m, H_dev, E_dev, stream=None):
    """ep_expm_noalloc: E = exp(H) on device tensors (m x m FP64, row-major) of the current
    device, enqueued on `stream` (a raw HIP stream handle; None = null stream)."""
    rc = lib().ep_expm_noalloc(int(m), _ptr(H_dev), _ptr(E_dev), C.c_void_p(stream) if stream else None)
    if rc != EP_OK:
        raise EPError(rc, "ep_expm_noalloc failed")


class Batch(Context):
    """A batch context: many independent instances advanced together (one launch per step)."""

    def __init__(self, device: int = 0, stream=None):
        super().__init__(device, stream)
        self.n_nodes_of = []

    def add(self, prob) -> int:
        xyz, conn = _f64(prob.xyz), _i32a(prob.conn)
        p = _f64(prob.params)
        cl = _i32a(prob.clamped)
        f = _i32a(prob.faces).reshape(-1, 4)
        t0 = _f64(prob.t0)
        kt, ks = _f64(prob.knots_t), _f64(prob.knots_s)
        iid = C.c_int32()
        self._call("ep_batch_add_instance", xyz.shape[0], _ptr(xyz), conn.shape[0], _ptr(conn), MODELS[prob.model],
                   _ptr(p), p.size, float(prob.rho), cl.size, _ptr(cl), f.shape[0], _ptr(f), _ptr(t0), kt.size,
                   _ptr(kt), _ptr(ks), C.byref(iid))
        self.n_nodes_of.append(xyz.shape[0])
        return iid.value

    def set_state(self, iid, t, u, v):
        u, v = _f64(u), _f64(v)
        self._call("ep_batch_set_state", int(iid), float(t), _ptr(u), _ptr(v))

    def step(self, dt, n_steps=1):
        self._call("ep_batch_step", float(dt), int(n_steps))

    def get_state(self, iid):
        t = C.c_double()
        n = 3 * self.n_nodes_of[iid]
        u, v = np.empty(n), np.empty(n)
        self._call("ep_batch_get_state", int(iid), C.byref(t), _ptr(u), _ptr(v))
        return t.value, u, v

    def plan(self, max_workgroups=0, serial=0.35):
        """Re-plan the launch: teams for costly instances, lists of cheap ones (ep_batch_plan)."""
        self._call("ep_batch_plan", int(max_workgroups), float(serial))

    def autotune(self, dt, steps=5):
        """Time candidate launch plans and keep the fastest (ep_batch_autotune); the states are
        restored afterwards.  Returns (workgroups per launch, ms per step)."""
        w, ms = C.c_int(), C.c_double()
        self._call("ep_batch_autotune", float(dt), int(steps), C.byref(w), C.byref(ms))
        return w.value, ms.value

    def plan_of(self, iid):
        """(team size of instance iid, workgroups per launch) of the current plan."""
        g, w = C.c_int(), C.c_int()
        self._call("ep_batch_get_plan", int(iid), C.byref(g), C.byref(w))
        return g.value, w.value

    def time_of(self, iid):
        """(device microseconds per step, steps timed) of instance iid (ep_batch_get_time)."""
        us, n = C.c_double(), C.c_int64()
        self._call("ep_batch_get_time", int(iid), C.byref(us), C.byref(n))
        return us.value, n.value

    def save_checkpoint(self, iid) -> bytes:
        """Opaque image of one instance's stepping state (ep_batch_save_checkpoint)."""
        n = C.c_size_t()
        self._call("ep_batch_checkpoint_size", int(iid), C.byref(n))
        buf = C.create_string_buffer(n.value)
        self._call("ep_batch_save_checkpoint", int(iid), buf, n.value)
        return buf.raw

    def load_checkpoint(self, iid, image: bytes):
        """Resume one instance from an image of save_checkpoint (ep_batch_load_checkpoint)."""
        buf = C.create_string_buffer(bytes(image), len(image))
        self._call("ep_batch_load_checkpoint", int(iid), buf, len(image))

    def stats(self, iid):
        mv, m, k, e = C.c_int64(), C.c_int(), C.c_int(), C.c_double()
        mvp, mp, kp = C.c_int64(), C.c_int(), C.c_int()
        self._call("ep_batch_get_stats", int(iid), C.byref(mv), C.byref(m), C.byref(k), C.byref(e), C.byref(mvp),
                   C.byref(mp), C.byref(kp))
        return {"matvecs": mv.value, "m": m.value, "k": k.value, "eps": e.value, "matvecs_pred": mvp.value,
                "m_pred": mp.value, "k_pred": kp.value}

    def energy(self, iid):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        self._call("ep_batch_get_energy", int(iid), C.byref(a), C.byref(b), C.byref(c))
        return a.value, b.value, c.value


def batch_from_problems(probs, device=0, tol=None, m_max=32, check_every=4, m_fixed=0, k_fixed=0,
                        max_substeps=64, s0=-1.0, precision="f64", stream=None):
    """Batch context with one instance per workloads.Problem, bound and at the initial states."""
    b = Batch(device, stream=stream)
    for p in probs:
        b.add(p)
    b.set_krylov(probs[0].tol if tol is None else tol, m_max, check_every, m_fixed, k_fixed, max_substeps, s0)
    b.set_precision(precision)
    b.bind()
    for i, p in enumerate(probs):
        b.set_state(i, 0.0, p.u0, p.v0)
    return b


def solver_from_problem(prob, device=0, tol=None, m_max=64, check_every=4, m_fixed=0, k_fixed=0,
                        max_substeps=64, s0=-1.0, precision="f64", workgroups=0, stream=None, ortho=-1, scheme=2):
    """Context set up from a workloads.Problem, bound and at the problem's initial state."""
    ctx = Context(device, stream=stream)
    ctx.set_mesh(prob.xyz, prob.conn)
    ctx.set_material(prob.model, prob.params, prob.rho)
    if len(prob.clamped):
        ctx.set_dirichlet(prob.clamped)
    if len(prob.faces):
        ctx.set_traction(prob.faces, prob.t0, prob.knots_t, prob.knots_s)
    ctx.set_krylov(prob.tol if tol is None else tol, m_max, check_every, m_fixed, k_fixed, max_substeps, s0)
    ctx.set_precision(precision)
    ctx.set_scheme(scheme)
    ctx.set_launch(workgroups)
    ctx.set_orthogonalization(ortho)
    ctx.bind()
    ctx.set_state(0.0, prob.u0, prob.v0)
    return ctx
