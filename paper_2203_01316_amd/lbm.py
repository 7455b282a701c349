"""Thin ctypes binding of liblbm.so (C ABI in include/lbm.h).

Argument marshalling only: every step of the lattice Boltzmann path runs in the
HIP kernels of the library.  PyTorch provides device memory (the workspace and
field tensors) and the stream.  There is no fallback: if the library is not
built, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# torch first: it loads the HIP runtime that the library then shares (loading
# the library first brings in a second runtime copy, whose device calls fail)
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc, gfx950)")

_lib = C.CDLL(LIB_PATH)

# enums (include/lbm.h)
OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EUNSUPPORTED, EDIVERGED = 0, -1, -2, -3, -4, -5, -6
D2Q9, D3Q27 = 9, 27
FP64, FP32, FP32_DEV, FP16_DEV, FP32_SR, FP16_SR = 0, 1, 2, 3, 4, 5
STREAM_AB, STREAM_AA = 0, 1
CM_SRT, CM_1ST, CM_TRT, CM_NS, CM_CUSTOM = 0, 1, 2, 3, 4
FLUID, SOLID, EQ, OUTLET = 0, 1, 2, 3
BB, IBB = 0, 1
ABB, IABB = 0, 1
_STATUS = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ESTATE: "ESTATE",
           EUNSUPPORTED: "EUNSUPPORTED", EDIVERGED: "EDIVERGED"}
_RELAX = {"srt": CM_SRT, "1st": CM_1ST, "trt": CM_TRT, "ns": CM_NS, "custom": CM_CUSTOM}
_STORAGE = {"fp64": FP64, "fp32": FP32, "fp32_dev": FP32_DEV, "fp16_dev": FP16_DEV, "fp32_sr": FP32_SR,
            "fp16_sr": FP16_SR}


class Params(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("with_ns", C.c_int32), ("storage", C.c_int32), ("stream", C.c_int32),
                ("relax_f", C.c_int32), ("relax_h", C.c_int32), ("u_mode", C.c_int32),
                ("with_source", C.c_int32), ("max_links", C.c_int32), ("max_special", C.c_int32),
                ("cumulant", C.c_int32), ("nu", C.c_double), ("k", C.c_double),
                ("rho_ref", C.c_double), ("H_ref", C.c_double), ("u0", C.c_double * 3),
                ("s_custom_f", C.c_double * 27), ("s_custom_h", C.c_double * 27), ("s_bulk_f", C.c_double)]


class Group(C.Structure):
    _fields_ = [("f_scheme", C.c_int32), ("h_scheme", C.c_int32), ("rho_w", C.c_double),
                ("u_w", C.c_double * 3), ("H_w", C.c_double)]


class Link(C.Structure):
    _fields_ = [("node", C.c_int32), ("dir", C.c_int32), ("group", C.c_int32),
                ("xf_solid", C.c_int32), ("q", C.c_double)]


LINK_DTYPE = np.dtype([("node", np.int32), ("dir", np.int32), ("group", np.int32),
                       ("xf_solid", np.int32), ("q", np.float64)])

_P = C.POINTER
_vp = C.c_void_p
_sig = {
    "lbm_version": (C.c_char_p, []),
    "lbm_workspace_bytes": (C.c_size_t, [_P(Params)]),
    "lbm_relaxation_rates": (C.c_int, [_P(Params), _vp, _vp, _vp]),
    "lbm_count_geometry": (C.c_int, [_P(Params), _vp, _P(C.c_int64), _P(C.c_int64)]),
    "lbm_build_links": (C.c_int, [_P(Params), _vp, _vp, C.c_int32, _vp, C.c_int64, _P(C.c_int64)]),
    "lbm_last_error": (C.c_char_p, [_vp]),
    "lbm_create": (C.c_int, [_P(Params), _vp, _vp, _P(_vp)]),
    "lbm_destroy": (None, [_vp]),
    "lbm_set_geometry": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int32]),
    "lbm_get_links": (C.c_int, [_vp, _vp, C.c_int64, _P(C.c_int64)]),
    "lbm_set_velocity": (C.c_int, [_vp, _vp]),
    "lbm_set_source": (C.c_int, [_vp, _vp]),
    "lbm_init_equilibrium": (C.c_int, [_vp, _vp, _vp, _vp]),
    "lbm_step": (C.c_int, [_vp, C.c_int32]),
    "lbm_macroscopic": (C.c_int, [_vp, _vp, _vp, _vp]),
    "lbm_get_populations": (C.c_int, [_vp, C.c_int32, C.c_int32, _vp]),
    "lbm_set_populations": (C.c_int, [_vp, C.c_int32, _vp, C.c_int64]),
    "lbm_reduce": (C.c_int, [_vp, C.c_int32, _vp, C.c_int32, _vp, C.c_int32]),
    "lbm_nusselt": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double, _vp, C.c_int32]),
    "lbm_reduce_noalloc": (C.c_int, [_vp, C.c_int32, _vp, C.c_int32, _vp, C.c_int32]),
    "lbm_device_copy": (C.c_int, [_vp, _vp, C.c_size_t, C.c_int32, _vp]),
    "lbm_state_bytes": (C.c_size_t, [_vp]),
    "lbm_save_state": (C.c_int, [_vp, _vp]),
    "lbm_load_state": (C.c_int, [_vp, _vp]),
    "lbm_time": (C.c_int64, [_vp]),
    "lbm_sync": (C.c_int, [_vp]),
    "lbm_objective": (C.c_int, [_vp, _vp, _vp, _vp, _P(C.c_double)]),
    "lbm_objective_residual": (C.c_int, [_vp, _vp, _vp, _P(C.c_double)]),
    "lbm_adjoint_seed": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int32]),
    "lbm_adjoint_step": (C.c_int, [_vp, _vp, _vp, _vp]),
    "lbm_profile_begin": (C.c_int, [_vp, C.c_int32]),
    "lbm_profile_end": (C.c_int, [_vp, _P(C.c_double), _P(C.c_double), _P(C.c_int64)]),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_sig)


class LBMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(status, ctx=None):
    if status != OK:
        msg = _lib.lbm_last_error(ctx)
        raise LBMError(status, msg.decode() if msg else "")


def version() -> str:
    return _lib.lbm_version().decode()


def make_params(lattice=D2Q9, nx=64, ny=64, nz=1, *, with_ns=False, storage="fp64", stream=STREAM_AB,
                relax_f="ns", relax_h="trt", nu=0.0, k=0.01, u0=(0.0, 0.0, 0.0), u_mode=0,
                with_source=False, max_links=0, max_special=0, rho_ref=0.0, H_ref=0.0,
                s_custom_f=None, s_custom_h=None, cumulant_f=False, cumulant_h=False, s_bulk_f=0.0) -> Params:
    """Library parameters.  cumulant_f / cumulant_h select the cumulant
    collision for that lattice (relax_h="1st" is the paper's Cumulants-1st);
    s_bulk_f the trace rate of f's second-order block (0: the library's
    default, see lbm_params)."""
    p = Params()
    p.lattice, p.nx, p.ny, p.nz = int(lattice), int(nx), int(ny), int(nz)
    p.with_ns = int(bool(with_ns))
    p.storage = _STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.stream = int(stream)
    p.relax_f = _RELAX[relax_f] if isinstance(relax_f, str) else int(relax_f)
    p.relax_h = _RELAX[relax_h] if isinstance(relax_h, str) else int(relax_h)
    p.u_mode = int(u_mode)
    p.with_source = int(bool(with_source))
    p.cumulant = (1 if cumulant_h else 0) | (2 if cumulant_f else 0)
    p.max_links, p.max_special = int(max_links), int(max_special)
    p.nu, p.k = float(nu), float(k)
    p.rho_ref, p.H_ref = float(rho_ref), float(H_ref)
    p.s_bulk_f = float(s_bulk_f)
    for d in range(3):
        p.u0[d] = float(u0[d]) if d < len(u0) else 0.0
    for k_ in range(27):
        p.s_custom_f[k_] = float(s_custom_f[k_]) if s_custom_f is not None and k_ < len(s_custom_f) else 1.0
        p.s_custom_h[k_] = float(s_custom_h[k_]) if s_custom_h is not None and k_ < len(s_custom_h) else 1.0
    return p


def workspace_bytes(p: Params) -> int:
    n = _lib.lbm_workspace_bytes(C.byref(p))
    if n == 0:
        _check(EINVAL)
    return int(n)


def relaxation_rates(p: Params):
    """Per-moment rates (s_f[27], s_h[27]) in the header's moment order."""
    sf = np.zeros(27)
    sh = np.zeros(27)
    _check(_lib.lbm_relaxation_rates(C.byref(p), sf.ctypes.data, sh.ctypes.data, None))
    return sf, sh


def bulk_rate(p: Params) -> float:
    """Trace rate of f's second-order block (0: no separate rate)."""
    sb = C.c_double()
    _check(_lib.lbm_relaxation_rates(C.byref(p), None, None, C.byref(sb)))
    return float(sb.value)


def device_copy(dst, src, blocks=0, hip_stream=None):
    """lbm_device_copy of the torch tensor src into dst (same byte size)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("dst and src sizes differ")
    _check(_lib.lbm_device_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes, int(blocks),
                                hip_stream))


def _host_flags(flags):
    if flags is None:
        return None
    return np.ascontiguousarray(np.asarray(flags).reshape(-1), dtype=np.uint16)


def _host_q(q, Q):
    if q is None:
        return None
    return np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(Q, -1))


def count_geometry(p: Params, flags):
    fl = _host_flags(flags)
    nl = C.c_int64()
    ns = C.c_int64()
    _check(_lib.lbm_count_geometry(C.byref(p), None if fl is None else fl.ctypes.data, C.byref(nl), C.byref(ns)))
    return int(nl.value), int(ns.value)


def build_links(p: Params, flags, q=None, n_groups=256):
    """Cut-link table built on the host by the library (no GPU needed)."""
    fl = _host_flags(flags)
    qq = _host_q(q, p.lattice)
    cnt = C.c_int64()
    _check(_lib.lbm_build_links(C.byref(p), fl.ctypes.data, None if qq is None else qq.ctypes.data,
                                int(n_groups), None, 0, C.byref(cnt)))
    out = np.zeros(cnt.value, dtype=LINK_DTYPE)
    if cnt.value:
        _check(_lib.lbm_build_links(C.byref(p), fl.ctypes.data, None if qq is None else qq.ctypes.data,
                                    int(n_groups), out.ctypes.data, cnt.value, C.byref(cnt)))
    return out


def _groups_struct(groups):
    arr = (Group * max(1, len(groups)))()
    for i, g in enumerate(groups):
        arr[i].f_scheme = int(g.get("f_scheme", BB))
        arr[i].h_scheme = int(g.get("h_scheme", ABB))
        arr[i].rho_w = float(g.get("rho_w", 1.0))
        uw = g.get("u_w", (0.0, 0.0, 0.0))
        for d in range(3):
            arr[i].u_w[d] = float(uw[d]) if d < len(uw) else 0.0
        arr[i].H_w = float(g.get("H_w", 0.0))
    return arr


class LBM:
    """One context of liblbm.so on one device and stream.

    The workspace and every field the library borrows are torch tensors held by
    this object for its lifetime.
    """

    def __init__(self, lattice=D2Q9, nx=64, ny=64, nz=1, *, device="cuda:0", hip_stream=None, flags=None,
                 q=None, groups=(), **kw):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        p = make_params(lattice, nx, ny, nz, **kw)
        fl = _host_flags(flags)
        if fl is not None:
            nl, ns = count_geometry(p, fl)
            p.max_links = max(p.max_links, nl)
            p.max_special = max(p.max_special, ns)
        self.params = p
        self.Q = int(lattice)
        self.n = int(nx) * int(ny) * int(nz)
        self.shape = (int(nz), int(ny), int(nx))
        self.rdtype = torch.float64 if p.storage in (FP64, FP32_SR) else torch.float32
        nbytes = workspace_bytes(p)
        with torch.cuda.device(self.device):
            self.stream = hip_stream if hip_stream is not None else torch.cuda.current_stream(self.device)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            ctx = C.c_void_p()
            _check(_lib.lbm_create(C.byref(p), C.c_void_p(self.workspace.data_ptr()),
                                   C.c_void_p(self.stream.cuda_stream), C.byref(ctx)))
        self.ctx = ctx
        self._keep = {}
        if fl is not None or groups:
            self.set_geometry(fl, q, groups)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx and _lib is not None:
            _lib.lbm_destroy(ctx)
            self.ctx = None

    def _ck(self, status):
        _check(status, self.ctx)

    def _dev(self, t, dtype):
        torch = self.torch
        t = torch.as_tensor(t)
        return t.to(device=self.device, dtype=dtype).contiguous()

    # -- set-up ----------------------------------------------------------------
    def set_geometry(self, flags, q=None, groups=()):
        fl = _host_flags(flags)
        qq = _host_q(q, self.Q)
        g = _groups_struct(groups)
        self._ck(_lib.lbm_set_geometry(self.ctx, None if fl is None else fl.ctypes.data,
                                       None if qq is None else qq.ctypes.data, C.cast(g, C.c_void_p),
                                       len(groups)))

    def links(self):
        cnt = C.c_int64()
        self._ck(_lib.lbm_get_links(self.ctx, None, 0, C.byref(cnt)))
        out = np.zeros(cnt.value, dtype=LINK_DTYPE)
        if cnt.value:
            self._ck(_lib.lbm_get_links(self.ctx, out.ctypes.data, cnt.value, C.byref(cnt)))
        return out

    def set_velocity(self, u):
        t = self._dev(u, self.rdtype).reshape(3, self.n)
        self._keep["u"] = t
        self._ck(_lib.lbm_set_velocity(self.ctx, C.c_void_p(t.data_ptr())))

    def set_source(self, Qsrc):
        t = self._dev(Qsrc, self.rdtype).reshape(self.n)
        self._keep["src"] = t
        self._ck(_lib.lbm_set_source(self.ctx, C.c_void_p(t.data_ptr())))

    def init(self, H, u=None, rho=None):
        torch = self.torch
        Ht = self._dev(H, torch.float64).reshape(self.n)
        ut = None if u is None else self._dev(u, torch.float64).reshape(3, self.n)
        rt = None if rho is None else self._dev(rho, torch.float64).reshape(self.n)
        self._ck(_lib.lbm_init_equilibrium(self.ctx, None if rt is None else rt.data_ptr(),
                                           None if ut is None else ut.data_ptr(), Ht.data_ptr()))
        self._keep["init"] = (Ht, ut, rt)  # alive until the kernel has run
        self.sync()
        self._keep.pop("init")

    # -- evolution ---------------------------------------------------------------
    def step(self, n=1):
        self._ck(_lib.lbm_step(self.ctx, int(n)))

    @property
    def t(self):
        return int(_lib.lbm_time(self.ctx))

    def sync(self):
        self._ck(_lib.lbm_sync(self.ctx))

    # -- outputs --------------------------------------------------------------------
    def macroscopic(self):
        torch = self.torch
        rho = torch.empty(self.n, dtype=torch.float64, device=self.device)
        u = torch.empty(3, self.n, dtype=torch.float64, device=self.device)
        H = torch.empty(self.n, dtype=torch.float64, device=self.device)
        self._ck(_lib.lbm_macroscopic(self.ctx, rho.data_ptr(), u.data_ptr(), H.data_ptr()))
        self.sync()
        return rho, u, H

    def populations(self, lattice="h", which="pre"):
        torch = self.torch
        out = torch.empty(self.Q, self.n, dtype=torch.float64, device=self.device)
        lat = 0 if lattice == "f" else 1
        w = 0 if which == "pre" else 1
        self._ck(_lib.lbm_get_populations(self.ctx, lat, w, out.data_ptr()))
        self.sync()
        return out

    def set_populations(self, lattice, g, t=0):
        torch = self.torch
        gt = self._dev(g, torch.float64).reshape(self.Q, self.n)
        self._ck(_lib.lbm_set_populations(self.ctx, 0 if lattice == "f" else 1, gt.data_ptr(), int(t)))
        self.sync()

    def reduce(self, group=0, columns=()):
        cols = np.ascontiguousarray(np.asarray(columns, dtype=np.int32).reshape(-1))
        out = np.zeros(3 + len(cols))
        self._ck(_lib.lbm_reduce(self.ctx, int(group), cols.ctypes.data if len(cols) else None, len(cols),
                                 out.ctypes.data, len(out)))
        return out

    def reduce_noalloc(self, group=0, columns=()):
        """lbm_reduce_noalloc: reduce() with its scratch in the library's static
        device array (no allocation by the library)."""
        cols = np.ascontiguousarray(np.asarray(columns, dtype=np.int32).reshape(-1))
        out = np.zeros(3 + len(cols))
        self._ck(_lib.lbm_reduce_noalloc(self.ctx, int(group), cols.ctypes.data if len(cols) else None, len(cols),
                                         out.ctypes.data, len(out)))
        return out

    def nusselt(self, group, x_in, x_out, T_wall, T_in):
        """lbm_nusselt: (Nu, Nu from the heater flux alone, q_surface, q_in,
        q_out) of the canonical state at the current time."""
        out = np.zeros(5)
        self._ck(_lib.lbm_nusselt(self.ctx, int(group), int(x_in), int(x_out), float(T_wall), float(T_in),
                                  out.ctypes.data, 5))
        return tuple(float(v) for v in out)

    def profile_begin(self, max_steps):
        """Time the bulk and boundary kernels of the next max_steps steps."""
        self._ck(_lib.lbm_profile_begin(self.ctx, int(max_steps)))

    def profile_end(self):
        """(bulk_ms, boundary_ms, steps) summed over the timed steps."""
        b = C.c_double()
        s = C.c_double()
        k = C.c_int64()
        self._ck(_lib.lbm_profile_end(self.ctx, C.byref(b), C.byref(s), C.byref(k)))
        return b.value, s.value, int(k.value)

    # -- discrete adjoint (advection-only, periodic) ------------------------------
    def objective(self, H_target):
        """(J, lam, dJdQ): J = 1/2 sum (H - H*)^2 of the canonical state, the adjoint
        seed lam [Q, n] (arithmetic dtype) and the direct part of dJ/dQ (FP64)."""
        torch = self.torch
        Ht = self._dev(H_target, torch.float64).reshape(self.n)
        lam = torch.empty(self.Q, self.n, dtype=self.rdtype, device=self.device)
        dq = torch.empty(self.n, dtype=torch.float64, device=self.device)
        J = C.c_double()
        self._ck(_lib.lbm_objective(self.ctx, Ht.data_ptr(), lam.data_ptr(), dq.data_ptr(), C.byref(J)))
        return J.value, lam, dq

    def objective_residual(self, H_target, resid=None):
        """(J, resid): resid = H - H* of the canonical state (FP64 [n], zero at
        solid nodes) and J = 1/2 sum resid^2."""
        torch = self.torch
        Ht = self._dev(H_target, torch.float64).reshape(self.n)
        if resid is None:
            resid = torch.empty(self.n, dtype=torch.float64, device=self.device)
        J = C.c_double()
        self._ck(_lib.lbm_objective_residual(self.ctx, Ht.data_ptr(), resid.data_ptr(), C.byref(J)))
        return J.value, resid

    def adjoint_seed(self, resid, lam, dJdQ, accumulate=True):
        """lam (+)= resid in every direction, dJdQ (+)= resid / 2."""
        self._ck(_lib.lbm_adjoint_seed(self.ctx, resid.data_ptr(), lam.data_ptr(), dJdQ.data_ptr(),
                                       1 if accumulate else 0))

    def adjoint_step(self, lam_next, lam_prev, dJdQ=None):
        """One reverse step into lam_prev; dJdQ (if given) accumulates."""
        self._ck(_lib.lbm_adjoint_step(self.ctx, lam_next.data_ptr(), lam_prev.data_ptr(),
                                       None if dJdQ is None else dJdQ.data_ptr()))

    def state_bytes(self):
        return int(_lib.lbm_state_bytes(self.ctx))

    def save_state(self):
        torch = self.torch
        buf = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        self._ck(_lib.lbm_save_state(self.ctx, buf.data_ptr()))
        return buf

    def load_state(self, buf):
        self._ck(_lib.lbm_load_state(self.ctx, buf.data_ptr()))
        self.sync()
