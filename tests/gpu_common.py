"""Shared set-up of the GPU parity tests: the same seeded inputs handed to the
HIP library (through its C ABI binding) and to the FP64 oracle."""
import numpy as np

from paper_2203_01316_amd import workloads as W


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def f32(a):
    """Values as the FP32 arithmetic sees them (inputs rounded once)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def fluid_only(arr, flags):
    """Populations with solid nodes zeroed (solid nodes carry no state)."""
    a = np.array(arr, dtype=np.float64, copy=True)
    if flags is not None:
        a[..., (np.asarray(flags).reshape(-1) & 15) == W.SOLID] = 0.0
    return a


def pair(L, O, *, Q, dims, storage="fp64", with_ns=False, relax_h="trt", nu=0.0, k=0.01, u0=(0, 0, 0),
         uvel=None, src=None, flags=None, q=None, groups=(), H0=None, u_init=None, rho0=None, oracle_init=True,
         cu_f=False, cu_h=False, stream=0, rho_ref=0.0, H_ref=0.0, relax_f="ns"):
    """GPU context and oracle simulation over identical inputs, both at t = 0."""
    nx, ny, nz = dims
    n = nx * ny * nz
    lowp = storage != "fp64"
    cast = f32 if lowp else (lambda a: np.asarray(a, dtype=np.float64))
    uv = None if uvel is None else cast(np.asarray(uvel).reshape(3, n))
    sr = None if src is None else cast(np.asarray(src).reshape(n))
    kw = dict(with_ns=with_ns, storage=storage, relax_h=relax_h, relax_f=relax_f, nu=nu, k=k, u0=u0,
              u_mode=1 if uv is not None and not with_ns else 0, with_source=src is not None,
              cumulant_f=cu_f, cumulant_h=cu_h, stream=stream, rho_ref=rho_ref, H_ref=H_ref)
    g = L.LBM(Q, nx, ny, nz, flags=flags, q=q, groups=groups, **kw)
    if uv is not None:
        g.set_velocity(uv)
    if sr is not None:
        g.set_source(sr)
    sf, sh = L.relaxation_rates(g.params)
    o = O.Sim(Q, nx, ny, nz, with_ns=with_ns, s_f=sf, s_h=sh, u0=u0, uvel=uv, src=sr, flags=flags, qlink=q,
              groups=list(groups), cu_f=cu_f, cu_h=cu_h, s_bulk_f=L.bulk_rate(g.params))
    H0 = np.ones(n) if H0 is None else np.asarray(H0, float).reshape(n)
    g.init(H0, u=u_init, rho=rho0)
    if oracle_init:
        o.init(H0, u=u_init, rho=rho0)
    return g, o


def gpu_pre(g, lattice="h"):
    return g.populations(lattice, "pre").cpu().numpy()


def gpu_post(g, lattice="h"):
    return g.populations(lattice, "post").cpu().numpy()
