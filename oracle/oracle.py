"""Python binding of the FP64 CPU oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it to check and time the GPU library.  Nothing in the
product path imports this module, and it imports nothing from the product.

Time convention (shared with the GPU library's documented semantics, not its
code): ``post`` holds the post-collision state of step t-1; the canonical
state at time t is its streamed form ``pre = stream(post)``.  One step is
``pre = stream(post); post = collide(pre)``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")

FLUID, SOLID, EQ, OUTLET = 0, 1, 2, 3
BB, IBB = 0, 1
ABB, IABB = 0, 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
             "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Group(C.Structure):
    _fields_ = [("f_scheme", C.c_int32), ("h_scheme", C.c_int32), ("rho_w", C.c_double),
                ("u_w", C.c_double * 3), ("H_w", C.c_double)]


class Cfg(C.Structure):
    _fields_ = [("Q", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("with_ns", C.c_int32), ("u_field", C.c_int32),
                ("s_f", C.c_double * 27), ("s_h", C.c_double * 27), ("u0", C.c_double * 3),
                ("uvel", C.c_void_p), ("src", C.c_void_p), ("flags", C.c_void_p),
                ("qlink", C.c_void_p), ("n_groups", C.c_int32), ("collide_off", C.c_int32),
                ("groups", C.c_void_p), ("cu_f", C.c_int32), ("cu_h", C.c_int32), ("s_bulk_f", C.c_double)]


class Link(C.Structure):
    _fields_ = [("node", C.c_int32), ("dir", C.c_int32), ("group", C.c_int32),
                ("xf_solid", C.c_int32), ("q", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        dp = C.POINTER(C.c_double)
        _lib.ora_section_flux.restype = C.c_double
        _lib.ora_links.restype = C.c_long
        for name in ("ora_collide", "ora_stream", "ora_init_post", "ora_macroscopic"):
            getattr(_lib, name).restype = C.c_int
        del dp
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------------------
# Small matrix / table accessors (used by the pins)
# ---------------------------------------------------------------------------
def lattice(Q: int):
    e = np.zeros((Q, 3), np.int32)
    opp = np.zeros(Q, np.int32)
    mo = np.zeros((Q, 3), np.int32)
    assert lib().ora_lattice(Q, _p(e), _p(opp), _p(mo)) == 0
    return e, opp, mo


def matrix(name: str, Q: int, u=None):
    out = np.zeros((Q, Q))
    fn = getattr(lib(), "ora_matrix_" + name)
    if u is None:
        assert fn(Q, _p(out)) == 0
    else:
        uu = np.ascontiguousarray(u, dtype=np.float64)
        assert fn(Q, _p(uu), _p(out)) == 0
    return out


def equilibrium(Q: int, psi: float, u):
    out = np.zeros(Q)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    assert lib().ora_equilibrium(Q, C.c_double(psi), _p(uu), _p(out)) == 0
    return out


def cm_equilibrium(Q: int, psi: float):
    out = np.zeros(Q)
    assert lib().ora_cm_equilibrium(Q, C.c_double(psi), _p(out)) == 0
    return out


def collision_matrix(Q: int, u, s):
    """Per-node affine collision g* = A g + b Q (advection-diffusion)."""
    uu = np.ascontiguousarray(u, dtype=np.float64)
    ss = np.ascontiguousarray(s, dtype=np.float64)
    A = np.zeros((Q, Q))
    b = np.zeros(Q)
    assert lib().ora_collision_matrix(Q, _p(uu), _p(ss), _p(A), _p(b)) == 0
    return A, b


def collide_node(Q: int, g, u, s, src: float = 0.0, s_bulk: float = 0.0):
    """One central-moment collision; s_bulk > 0 relaxes the trace of the
    second-order block at that rate and its deviator at s[200]."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    ss = np.ascontiguousarray(s, dtype=np.float64)
    out = np.zeros(Q)
    assert lib().ora_collide_node(Q, _p(g), _p(uu), _p(ss), C.c_double(src), C.c_double(s_bulk), _p(out)) == 0
    return out


def cumulants(Q: int, g):
    """Cumulants of a population set (moment order of the oracle's tables):
    c[0] = sum g, the others those of the normalised distribution."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    out = np.zeros(Q)
    assert lib().ora_cumulants(Q, _p(g), _p(out)) == 0
    return out


def from_cumulants(Q: int, c):
    c = np.ascontiguousarray(c, dtype=np.float64)
    out = np.zeros(Q)
    assert lib().ora_from_cumulants(Q, _p(c), _p(out)) == 0
    return out


def collide_node_cu(Q: int, g, u, s, src: float = 0.0, s_bulk: float = 0.0):
    g = np.ascontiguousarray(g, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    ss = np.ascontiguousarray(s, dtype=np.float64)
    out = np.zeros(Q)
    assert lib().ora_collide_node_cu(Q, _p(g), _p(uu), _p(ss), C.c_double(src), C.c_double(s_bulk), _p(out)) == 0
    return out


# ---------------------------------------------------------------------------
# Relaxation presets (Sec. 2.1.1) -- moment order of the oracle's tables
# ---------------------------------------------------------------------------
def s_main(k: float) -> float:
    """Main rate s = 1 / (k / (cs^2 dt) + 1/2), cs^2 = 1/3, dt = 1."""
    return 1.0 / (3.0 * k + 0.5)


def preset(Q: int, kind: str, rate: float) -> np.ndarray:
    """Per-moment rates. kind: 'srt', '1st', 'trt' (h lattice) or 'ns' (f)."""
    _, _, mo = lattice(Q)
    order = mo.sum(axis=1)
    s = np.ones(27)
    for k in range(Q):
        o = order[k]
        if kind == "srt":
            s[k] = rate
        elif kind == "1st":
            s[k] = rate if o == 1 else 1.0
        elif kind == "trt":
            s[k] = rate if o % 2 == 1 else 1.0
        elif kind == "ns":
            s[k] = rate if o == 2 else 1.0
        else:
            raise ValueError(kind)
    return s


# ---------------------------------------------------------------------------
# Whole-lattice simulation
# ---------------------------------------------------------------------------
class Sim:
    def __init__(self, Q, nx, ny, nz=1, *, with_ns=False, s_f=None, s_h=None, u0=(0.0, 0.0, 0.0),
                 uvel=None, src=None, flags=None, qlink=None, groups=(), collide_off=False, cu_f=False,
                 cu_h=False, s_bulk_f=0.0):
        self.Q, self.nx, self.ny, self.nz = Q, nx, ny, nz
        self.N = nx * ny * nz
        self.with_ns = bool(with_ns)
        self.cfg = Cfg()
        c = self.cfg
        c.Q, c.nx, c.ny, c.nz = Q, nx, ny, nz
        c.with_ns = int(with_ns)
        c.collide_off = int(collide_off)
        c.cu_f = int(cu_f)
        c.cu_h = int(cu_h)
        c.s_bulk_f = float(s_bulk_f)
        sf = np.ones(27) if s_f is None else np.asarray(s_f, float)
        sh = np.ones(27) if s_h is None else np.asarray(s_h, float)
        for k in range(27):
            c.s_f[k] = float(sf[k]) if k < len(sf) else 1.0
            c.s_h[k] = float(sh[k]) if k < len(sh) else 1.0
        for d in range(3):
            c.u0[d] = float(u0[d]) if d < len(u0) else 0.0
        self._keep = []
        if uvel is not None:
            self.uvel = np.ascontiguousarray(np.broadcast_to(np.asarray(uvel, float).reshape(3, -1), (3, self.N)))
            c.u_field = 1
            c.uvel = _p(self.uvel)
        else:
            self.uvel = None
        self.set_source(src)
        if flags is not None:
            self.flags = np.ascontiguousarray(flags, dtype=np.uint16).reshape(-1)
            assert self.flags.size == self.N
            c.flags = _p(self.flags)
        else:
            self.flags = None
        if qlink is not None:
            self.qlink = np.ascontiguousarray(qlink, dtype=np.float64).reshape(Q, self.N)
            c.qlink = _p(self.qlink)
        else:
            self.qlink = None
        self.groups = (Group * max(1, len(groups)))()
        for i, g in enumerate(groups):
            self.groups[i].f_scheme = g.get("f_scheme", BB)
            self.groups[i].h_scheme = g.get("h_scheme", ABB)
            self.groups[i].rho_w = g.get("rho_w", 1.0)
            uw = g.get("u_w", (0.0, 0.0, 0.0))
            for d in range(3):
                self.groups[i].u_w[d] = uw[d] if d < len(uw) else 0.0
            self.groups[i].H_w = g.get("H_w", 0.0)
        c.n_groups = len(groups)
        c.groups = C.cast(self.groups, C.c_void_p)
        shape = (Q, self.N)
        self.post_f = np.zeros(shape)
        self.post_h = np.zeros(shape)
        self.t = 0

    def set_source(self, src):
        if src is not None:
            self.src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1)
            self.cfg.src = _p(self.src)
        else:
            self.src = None
            self.cfg.src = None

    # -- state -----------------------------------------------------------------
    def init(self, H, u=None, rho=None):
        """Equilibrium initial state at t = 0 from the fields H [n], u [3,n], rho [n]."""
        N = self.N
        H = np.ascontiguousarray(np.broadcast_to(np.asarray(H, float).reshape(-1), (N,)))
        if u is None:
            if self.uvel is not None:
                u = self.uvel
            else:
                u = np.repeat(np.asarray(self.cfg.u0[:], float).reshape(3, 1), N, axis=1)
        u = np.ascontiguousarray(np.broadcast_to(np.asarray(u, float).reshape(3, -1), (3, N)))
        rho = np.ones(N) if rho is None else np.ascontiguousarray(
            np.broadcast_to(np.asarray(rho, float).reshape(-1), (N,)))
        assert lib().ora_init_post(C.byref(self.cfg), _p(rho), _p(u), _p(H),
                                   _p(self.post_f), _p(self.post_h)) == 0
        self.t = 0

    def set_post(self, f=None, h=None, t=0):
        if f is not None:
            self.post_f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.Q, self.N).copy()
        if h is not None:
            self.post_h = np.ascontiguousarray(h, dtype=np.float64).reshape(self.Q, self.N).copy()
        self.t = t

    def pre(self, with_flux=False):
        """Canonical pre-collision state at the current time (and link fluxes)."""
        f = self.post_f.copy()
        h = self.post_h.copy()
        flux = None
        if with_flux:
            nl = self.nlinks()
            flux = np.zeros(max(nl, 1))
        assert lib().ora_stream(C.byref(self.cfg), _p(self.post_f), _p(self.post_h),
                                _p(f), _p(h), _p(flux)) == 0
        if with_flux:
            return f, h, flux[: self.nlinks()]
        return f, h

    def collide(self, f, h):
        fs = np.zeros_like(h)
        hs = np.zeros_like(h)
        assert lib().ora_collide(C.byref(self.cfg), _p(f), _p(h), _p(fs), _p(hs)) == 0
        return fs, hs

    def step(self, n=1):
        for _ in range(n):
            f, h = self.pre()
            self.post_f, self.post_h = self.collide(f, h)
            self.t += 1

    # -- observables ---------------------------------------------------------------
    def macroscopic(self):
        f, h = self.pre()
        N = self.N
        rho = np.zeros(N)
        u = np.zeros((3, N))
        H = np.zeros(N)
        assert lib().ora_macroscopic(C.byref(self.cfg), _p(f), _p(h), _p(rho), _p(u), _p(H)) == 0
        return rho, u, H

    def nlinks(self):
        return int(lib().ora_links(C.byref(self.cfg), None, C.c_long(0)))

    def links(self):
        n = self.nlinks()
        arr = (Link * max(n, 1))()
        lib().ora_links(C.byref(self.cfg), arr, C.c_long(n))
        out = np.zeros(n, dtype=[("node", np.int32), ("dir", np.int32), ("group", np.int32),
                                 ("xf_solid", np.int32), ("q", np.float64)])
        for i in range(n):
            out[i] = (arr[i].node, arr[i].dir, arr[i].group, arr[i].xf_solid, arr[i].q)
        return out

    def adjoint_step(self, lam_next, dJdQ=None):
        """lam_next = dJ/dpre(t+1) -> dJ/dpre(t); dJdQ (if given) accumulates."""
        lam_next = np.ascontiguousarray(lam_next, dtype=np.float64).reshape(self.Q, self.N)
        out = np.zeros_like(lam_next)
        assert lib().ora_adjoint_step(C.byref(self.cfg), _p(lam_next), _p(out), _p(dJdQ)) == 0
        return out

    def adjoint_step_dense(self, lam_next, dJdQ=None):
        """The adjoint step as the plain transpose of the one-step map from the
        canonical state at t to that at t + 1 (collision, then streaming with
        the wall rules, EQ nodes and the source).  For a prescribed velocity
        that map is affine in the state and in the source, so each column is
        the forward step of a unit vector minus the step of zero.  Small
        lattices only; the advection-diffusion lattice only."""
        assert not self.with_ns
        Q, N = self.Q, self.N
        lam = np.array(lam_next, dtype=np.float64).reshape(Q, N)
        solid = self._solid()
        lam[:, solid] = 0.0  # solid nodes carry no state
        src0 = None if self.src is None else self.src.copy()
        saved = (self.post_f, self.post_h, self.t)
        zero = np.zeros((Q, N))

        def F(h, src):
            self.set_source(src)
            _, hs = self.collide(zero, h)
            self.post_h = hs
            return self.pre()[1]

        try:
            base = F(zero, src0)
            out = np.zeros(Q * N)
            e = np.zeros(Q * N)
            for k in range(Q * N):
                e[k] = 1.0
                out[k] = float(((F(e.reshape(Q, N), src0) - base) * lam).sum())
                e[k] = 0.0
            if dJdQ is not None:
                b0 = F(zero, np.zeros(N))
                unit = np.zeros(N)
                for m in range(N):
                    unit[m] = 1.0
                    dJdQ[m] += float(((F(zero, unit) - b0) * lam).sum())
                    unit[m] = 0.0
        finally:
            self.set_source(src0)
            self.post_f, self.post_h, self.t = saved
        out = out.reshape(Q, N)
        out[:, solid] = 0.0
        return out

    def _solid(self):
        if self.flags is None:
            return np.zeros(self.N, dtype=bool)
        return (self.flags & 15) == 1

    def objective(self, H_target):
        """J = 1/2 sum over the non-solid nodes of (H - H*)^2 of the canonical
        state, dJ/dpre (all directions equal H - H*) and the direct part of
        dJ/dQ (Q enters H as Q/2)."""
        _, _, H = self.macroscopic()
        r = H - np.asarray(H_target, dtype=np.float64).reshape(-1)
        r[self._solid()] = 0.0
        lam = np.repeat(r[None, :], self.Q, axis=0)
        return 0.5 * float((r * r).sum()), lam, 0.5 * r

    def gradient_source(self, H_target, steps, dense=False):
        """J and dJ/dQ after `steps` steps from the current post state (which
        must be the initial one): forward, objective, then reverse steps
        (dense: with adjoint_step_dense, which also covers geometry)."""
        self.step(steps)
        J, lam, dJdQ = self.objective(H_target)
        dJdQ = np.ascontiguousarray(dJdQ)
        for _ in range(steps):
            lam = self.adjoint_step_dense(lam, dJdQ) if dense else self.adjoint_step(lam, dJdQ)
        return J, dJdQ

    def gradient_source_tracking(self, H_target, steps, every, dense=False):
        """J = sum over t = every, 2 every, ... <= steps of 1/2 sum (H_t - H*)^2
        and dJ/dQ, from the current post state (the initial one): the forward
        keeps the seed of every observation time, the reverse sweep adds the
        seed of time t to lambda once a reverse step has carried lambda back
        to t."""
        seeds, J = {}, 0.0
        for t in range(1, steps + 1):
            self.step(1)
            if t % every == 0:
                Jt, lam_t, dq_t = self.objective(H_target)
                J += Jt
                seeds[t] = (lam_t, dq_t)
        lam = np.zeros((self.Q, self.N))
        dJdQ = np.zeros(self.N)
        if steps in seeds:
            lam += seeds[steps][0]
            dJdQ += seeds[steps][1]
        for t in range(steps - 1, -1, -1):
            lam = self.adjoint_step_dense(lam, dJdQ) if dense else self.adjoint_step(lam, dJdQ)
            if t in seeds:
                lam = lam + seeds[t][0]
                dJdQ += seeds[t][1]
        return J, dJdQ

    def nusselt(self, group, x_in, x_out, k, T_wall, T_in):
        """(Nu, Nu from the heater flux alone, q_surface, q_in, q_out) of the
        canonical state at the current time (Sec. 4.4)."""
        out = np.zeros(5)
        assert lib().ora_nusselt(C.byref(self.cfg), _p(self.post_f), _p(self.post_h), int(group), int(x_in),
                                 int(x_out), C.c_double(k), C.c_double(T_wall), C.c_double(T_in), _p(out)) == 0
        return tuple(float(v) for v in out)

    def section_flux(self, X, h=None):
        if h is None:
            _, h = self.pre()
        return float(lib().ora_section_flux(C.byref(self.cfg), _p(np.ascontiguousarray(h)), int(X)))
