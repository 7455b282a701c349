"""Seeded synthetic inputs: geometry (node flags, per-link wall distances) and
initial fields for the lattice Boltzmann workloads.

This module builds inputs only.  It holds none of the method's arithmetic (no
collision, streaming or boundary formula) and is shared by the GPU tests, the
oracle tests and the benchmark.

Node-flag encoding (the library's geometry input): bits 0-3 node type,
bits 4-11 boundary group.

  FLUID  = 0  ordinary node
  SOLID  = 1  wall interior; links from a non-solid node into it are cut links
              handled by the group's wall scheme
  EQ     = 2  equilibrium node: its populations are replaced by the
              equilibrium at the group's wall values after streaming
  OUTLET = 3  zero-gradient outlet node (unknown e_x < 0 populations copied
              from the upstream x - 1 neighbour)

Per-link wall distances ``q`` are stored as a ``[Q, n]`` array: ``q[i, x_b]``
is the fraction of the link vector e_i from the boundary node x_b to the wall.
The D2Q9 direction order is (0,0),(1,0),(0,1),(1,1),(-1,0),(0,-1),(1,-1),
(-1,1),(-1,-1); D3Q27 follows the paper's Sec. 2.1 order.
"""
from __future__ import annotations

import math

import numpy as np

FLUID, SOLID, EQ, OUTLET = 0, 1, 2, 3

# Velocity sets used to locate cut links (inputs only).
D2Q9_E = np.array([(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0), (-1, 0, 0), (0, -1, 0),
                   (1, -1, 0), (-1, 1, 0), (-1, -1, 0)], dtype=np.int64)
D3Q27_E = np.array([
    (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1),
    (-1, 0, 0), (0, -1, 0), (0, 0, -1), (1, -1, 0), (1, 0, -1), (-1, 1, 0), (-1, 0, 1),
    (0, 1, -1), (0, -1, 1), (1, 1, 1), (-1, -1, 0), (-1, 0, -1), (0, -1, -1), (-1, 1, 1),
    (1, -1, 1), (1, 1, -1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1), (-1, -1, -1)],
    dtype=np.int64)


def flag(kind: int, group: int = 0) -> int:
    return int(kind) | (int(group) << 4)


def circle_q(nx: int, ny: int, flags: np.ndarray, circles, Q: int = 9) -> np.ndarray:
    """Wall distance of every cut link whose solid end lies in one of ``circles``.

    ``circles`` is a list of (cx, cy, r, inside) tuples: the wall of a disc
    (inside=True, solid for |x-c| <= r) or of the outside of a circle
    (inside=False, solid for |x-c| >= r).  For a cut link from fluid x_b along
    e_i, q is the smallest t in (0, 1] with |x_b + t e_i - c| = r, solved with
    the textbook quadratic formula in FP64.  Links not on a circle keep q=0.5.
    """
    E = D2Q9_E if Q == 9 else D3Q27_E
    n = nx * ny
    q = np.full((Q, n), 0.5)
    f2 = flags.reshape(ny, nx) & 15
    ys, xs = np.nonzero(f2 != SOLID)
    for a in range(1, Q):
        ex, ey = int(E[a, 0]), int(E[a, 1])
        tx = (xs + ex) % nx
        ty = (ys + ey) % ny
        cut = f2[ty, tx] == SOLID
        for x, y, sx, sy in zip(xs[cut], ys[cut], tx[cut], ty[cut]):
            best = None
            for (cx, cy, r, inside) in circles:
                d_end = math.hypot(sx - cx, sy - cy)
                if (inside and d_end > r) or ((not inside) and d_end < r):
                    continue
                dx, dy = x - cx, y - cy
                A = ex * ex + ey * ey
                B = 2.0 * (dx * ex + dy * ey)
                Cc = dx * dx + dy * dy - r * r
                disc = B * B - 4.0 * A * Cc
                if disc < 0:
                    continue
                sq = math.sqrt(disc)
                for t in ((-B - sq) / (2 * A), (-B + sq) / (2 * A)):
                    if 0.0 < t <= 1.0 and (best is None or t < best):
                        best = t
            if best is not None:
                q[a, x + nx * y] = best
    return q


def sphere_box(nx: int, ny: int, nz: int, center, r: float, inlet: bool = False):
    """D3Q27 box, periodic, with a solid sphere (group 0, IBB/IABB, H = 2) and
    optionally an EQ inlet plane x = 0 (group 1) and an outlet plane x = nx-1.
    Returns (flags [n], q [27, n], groups); q is the smallest t in (0, 1] with
    |x_b + t e_i - c| = r for links into the sphere (textbook quadratic, FP64)."""
    n = nx * ny * nz
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx]
    cx, cy, cz = center
    flags = np.zeros((nz, ny, nx), np.uint16)
    if inlet:
        flags[:, :, 0] = flag(EQ, 1)
        flags[:, :, nx - 1] = flag(OUTLET, 0)
    ball = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 <= r * r
    flags[ball] = flag(SOLID, 0)
    flags = flags.reshape(-1)
    q = np.full((27, n), 0.5)
    solid = (flags & 15) == SOLID
    X, Y, Z = x.reshape(-1), y.reshape(-1), z.reshape(-1)
    for a in range(1, 27):
        ex, ey, ez = (int(v) for v in D3Q27_E[a])
        tgt = ((X + ex) % nx) + nx * (((Y + ey) % ny) + ny * ((Z + ez) % nz))
        cut = (~solid) & solid[tgt]
        for m in np.nonzero(cut)[0]:
            dx, dy, dz = X[m] - cx, Y[m] - cy, Z[m] - cz
            A = ex * ex + ey * ey + ez * ez
            B = 2.0 * (dx * ex + dy * ey + dz * ez)
            Cc = dx * dx + dy * dy + dz * dz - r * r
            disc = B * B - 4.0 * A * Cc
            if disc < 0:
                continue
            sq = math.sqrt(disc)
            ts = [t for t in ((-B - sq) / (2 * A), (-B + sq) / (2 * A)) if 0.0 < t <= 1.0]
            if ts:
                q[a, m] = min(ts)
    groups = [dict(f_scheme=1, h_scheme=1, H_w=2.0), dict(f_scheme=0, h_scheme=0, rho_w=1.0,
                                                           u_w=(0.02, 0.0, 0.0), H_w=1.0)]
    return flags, q, groups


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
def gaussian_hill(L: int = 64, sigma: float = 8.0, amp: float = 0.5, center=None, u=(0.05, 0.02),
                  k: float = 0.01, t: float = 0.0, images: int = 1) -> np.ndarray:
    """Advected-diffusing Gaussian hill H(x, t) = 1 + amp * sigma0^2/(sigma0^2 + 2kt) *
    exp(-|x - x0 - u t|^2 / (2 (sigma0^2 + 2 k t))), summed over periodic images
    (closed form of Sec. 4.1 for N = 2 dimensions).  Nodes at integer x, y."""
    if center is None:
        center = (L / 2, L / 2)
    x = np.arange(L, dtype=np.float64)
    X, Y = np.meshgrid(x, x, indexing="xy")
    s2 = sigma * sigma + 2.0 * k * t
    acc = np.zeros_like(X)
    for mx in range(-images, images + 1):
        for my in range(-images, images + 1):
            dx = X - center[0] - u[0] * t - mx * L
            dy = Y - center[1] - u[1] * t - my * L
            acc += np.exp(-(dx * dx + dy * dy) / (2.0 * s2))
    return (1.0 + amp * sigma * sigma / s2 * acc).reshape(-1)


def channel(nx: int = 1024, ny: int = 256, cx: float = 256, cy: float = 128, r: float = 20,
            u_max: float = 0.05, H_wall: float = 0.0, H_in: float = 1.0, H_cyl: float = 2.0):
    """Channel with walls at y = 0 and y = ny-1 (group 0, ABB, H_wall), inlet column
    x = 0 (EQ, group 1, H_in), outlet column x = nx-1, and a disc (group 2, IABB,
    H_cyl) solid iff (x-cx)^2 + (y-cy)^2 <= r^2.  Returns (flags, q, groups, u)
    with a Poiseuille velocity field u[3, n]."""
    n = nx * ny
    flags = np.zeros((ny, nx), np.uint16)
    y, x = np.mgrid[0:ny, 0:nx]
    flags[:, 0] = flag(EQ, 1)
    flags[:, nx - 1] = flag(OUTLET, 0)
    flags[0, :] = flag(SOLID, 0)
    flags[ny - 1, :] = flag(SOLID, 0)
    disc = (x - cx) ** 2 + (y - cy) ** 2 <= r * r
    flags[disc] = flag(SOLID, 2)
    flags = flags.reshape(-1)
    q = circle_q(nx, ny, flags, [(cx, cy, r, True)])
    h = float(ny - 2)
    yy = y.astype(np.float64)
    ux = 4.0 * u_max * (yy - 0.5) * (h + 0.5 - yy) / (h * h)
    ux[0, :] = 0.0
    ux[ny - 1, :] = 0.0
    u = np.zeros((3, n))
    u[0] = ux.reshape(-1)
    groups = [
        dict(f_scheme=0, h_scheme=0, H_w=H_wall),
        dict(f_scheme=0, h_scheme=0, H_w=H_in),
        dict(f_scheme=1, h_scheme=1, H_w=H_cyl),
    ]
    return flags, q, groups, u


def walled_box(nx: int = 24, ny: int = 14, cx: float = 8.3, cy: float = 6.6, r: float = 2.7,
               u_max: float = 0.04):
    """The channel above made periodic in x (no inlet or outlet column): walls at
    y = 0 and y = ny-1 (group 0, ABB, H = 0.5), a disc (group 2, IABB, H = 2),
    a 2 x 2 patch of EQ nodes (group 1, H = 1.5) at x = 0.7 nx and two EQ nodes
    on the lower wall (they have cut links).  Returns (flags, q, groups, u)."""
    flags, q, groups, u = channel(nx, ny, cx, cy, r, u_max, H_wall=0.5, H_in=1.5, H_cyl=2.0)
    f2 = flags.reshape(ny, nx).copy()
    f2[1:ny - 1, 0] = flag(FLUID, 0)
    f2[1:ny - 1, nx - 1] = flag(FLUID, 0)
    ex, ey = int(0.7 * nx), ny // 2
    f2[ey:ey + 2, ex:ex + 2] = flag(EQ, 1)
    f2[1, 3:5] = flag(EQ, 1)
    return f2.reshape(-1), q, groups, u


def gap_box(nx: int = 20, ny: int = 16, H_w: float = 1.7, seed: int = 5, Q: int = 9):
    """Periodic box with two one-node gaps, so that cut links have a solid x_f:
    a horizontal slit (solid rows y = ny/4 and ny/4 + 2 for nx/8 <= x < 3nx/4,
    fluid row between them) and a vertical one (solid columns x = 0.8nx and
    0.8nx + 2 for ny/2 <= y < 7ny/8).  All solid nodes are group 0 (IBB/IABB,
    H = H_w).  Returns (flags, q_lo, q_hi, groups): q_lo holds seeded uniform
    wall distances in [0.1, 0.45] on every cut link, q_hi in [0.55, 1]
    (numpy PCG64(seed)); other entries are 1/2.  For D3Q27 (Q = 27) the same
    cross-section is extruded along z (ny/4 layers, periodic)."""
    nz = 1 if Q == 9 else max(ny // 4, 2)
    f = np.zeros((nz, ny, nx), np.uint16)
    y0, x0, x1 = ny // 4, nx // 8, (3 * nx) // 4
    f[:, y0, x0:x1] = flag(SOLID, 0)
    f[:, y0 + 2, x0:x1] = flag(SOLID, 0)
    xc, ya, yb = int(0.8 * nx), ny // 2, (7 * ny) // 8
    f[:, ya:yb, xc] = flag(SOLID, 0)
    f[:, ya:yb, xc + 2] = flag(SOLID, 0)
    flags = f.reshape(-1)
    n = flags.size
    E = D2Q9_E if Q == 9 else D3Q27_E
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = rng.uniform(0.1, 0.45, size=(Q, n))
    hi = rng.uniform(0.55, 1.0, size=(Q, n))
    q_lo = np.full((Q, n), 0.5)
    q_hi = np.full((Q, n), 0.5)
    solid = (f & 15) == SOLID
    for a in range(1, Q):
        ex, ey, ez = (int(v) for v in E[a])
        cut = (~solid) & np.roll(solid, shift=(-ez, -ey, -ex), axis=(0, 1, 2))
        cut = cut.reshape(-1)
        q_lo[a, cut] = lo[a, cut]
        q_hi[a, cut] = hi[a, cut]
    groups = [dict(f_scheme=1, h_scheme=1, rho_w=1.0, H_w=H_w)]
    return flags, q_lo, q_hi, groups


def heated_cylinder(nx: int = 2048, ny: int = 2048, r: float = 64, cx=None, cy=None,
                    u_in: float = 0.04, amp: float = 1e-3, seed: int = 0, T_in: float = 10.0,
                    T_cyl: float = 11.0):
    """Coupled flow + heat: periodic in y, EQ inlet column x = 0 (group 0: rho = 1,
    u = (u_in + amp*xi(y), 0) with xi ~ U(-1, 1) from numpy PCG64(seed), H = T_in),
    zero-gradient outlet column x = nx-1, heated disc (group 1: IBB for f, IABB for
    h, H = T_cyl).  Returns (flags, q, groups, u_inlet[3, n], init fields)."""
    if cx is None:
        cx = nx // 4
    if cy is None:
        cy = ny // 2
    n = nx * ny
    flags = np.zeros((ny, nx), np.uint16)
    flags[:, 0] = flag(EQ, 0)
    flags[:, nx - 1] = flag(OUTLET, 0)
    y, x = np.mgrid[0:ny, 0:nx]
    disc = (x - cx) ** 2 + (y - cy) ** 2 <= r * r
    flags[disc] = flag(SOLID, 1)
    flags = flags.reshape(-1)
    q = circle_q(nx, ny, flags, [(cx, cy, r, True)])
    xi = np.random.Generator(np.random.PCG64(seed)).uniform(-1.0, 1.0, size=ny)
    u = np.zeros((3, ny, nx))
    u[0] = (u_in + amp * xi)[:, None]
    u[:, disc] = 0.0
    u = u.reshape(3, n)
    groups = [dict(f_scheme=0, h_scheme=0, rho_w=1.0, H_w=T_in),
              dict(f_scheme=1, h_scheme=1, rho_w=1.0, H_w=T_cyl)]
    rho0 = np.ones(n)
    H0 = np.full(n, T_in)
    return flags, q, groups, u, rho0, H0


def boundary_mix(nx: int = 33, ny: int = 40, u_in: float = 0.03, seed: int = 4):
    """Short coupled channel whose inlet and outlet nodes come in every local
    configuration: walls at y = 0 and y = ny-1 (group 0: BB/ABB, H = 0); EQ
    inlet column x = 0 (group 1: H = 1) touching the walls, with one node of
    group 252 (H = 1.5) at y = 12 and one OUTLET node at y = 7 whose upstream
    node wraps to x = nx-1 (left FLUID there); outlet column x = nx-1 (with
    nx = 33 the node at y = 32 has n = 1088, a multiple of 64); a solid block
    (group 2) at x = nx-3, y = 20..21 that gives the upstream nodes of four
    outlets cut links; a disc of radius 4 at (14, 20) (group 2: IBB/IABB,
    H = 2).  Velocity: u_x = u_in (1 + 0.1 xi(y)), xi ~ U(-1, 1) from numpy
    PCG64(seed), zero in solids.  Returns (flags, q, groups, u[3, n], rho0, H0).
    """
    n = nx * ny
    f = np.zeros((ny, nx), np.uint16)
    f[:, 0] = flag(EQ, 1)
    f[:, nx - 1] = flag(OUTLET, 0)
    f[12, 0] = flag(EQ, 252)
    f[7, 0] = flag(OUTLET, 0)
    f[7, nx - 1] = flag(FLUID, 0)
    f[20:22, nx - 3] = flag(SOLID, 2)
    yy, xx = np.mgrid[0:ny, 0:nx]
    disc = (xx - 14) ** 2 + (yy - 20) ** 2 <= 16
    f[disc] = flag(SOLID, 2)
    f[0, :] = flag(SOLID, 0)
    f[ny - 1, :] = flag(SOLID, 0)
    flags = f.reshape(-1)
    q = circle_q(nx, ny, flags, [(14.0, 20.0, 4.0, True)])
    xi = np.random.Generator(np.random.PCG64(seed)).uniform(-1.0, 1.0, size=ny)
    u = np.zeros((3, ny, nx))
    u[0] = (u_in * (1.0 + 0.1 * xi))[:, None]
    u[:, (f & 15) == SOLID] = 0.0
    groups = [dict(f_scheme=0, h_scheme=0, rho_w=1.0, H_w=0.0),
              dict(f_scheme=0, h_scheme=0, rho_w=1.0, H_w=1.0),
              dict(f_scheme=1, h_scheme=1, rho_w=1.0, H_w=2.0)]
    groups += [dict(f_scheme=0, h_scheme=0, rho_w=1.0, H_w=0.0)] * (252 - len(groups))
    groups.append(dict(f_scheme=0, h_scheme=0, rho_w=1.0, H_w=1.5))
    return flags, q, groups, u.reshape(3, n), np.ones(n), np.zeros(n)


def confined_cylinder(S: int = 1, Pr: float = 10.0, second_order: bool = True, xc_frac: float = 0.2):
    """Steady forced convection from a confined cylinder (Sec. 4.4, case table):
    lattice (1000 S) x (150 S), D = 30 S, U = 0.01 / S, nu = 0.03, k = nu / Pr,
    Re = U D / nu = 10.  Inlet: EQ column x = 0 (group 0: rho = 1, u = (U, 0),
    H = T_in = 10), standing in for the paper's Zou-He inlet.  Outlet:
    zero-gradient column x = nx - 1.  Top and bottom: periodic in y; the steady
    flow is symmetric about the channel axis, where the periodic images then
    meet with zero normal velocity and zero normal gradients, as on the
    paper's symmetry planes.  Cylinder (group 1, H = T_cyl = 11): centre
    (xc_frac nx, ny / 2 - 1/2), solid iff |x - c| <= D / 2, IBB/IABB when
    second_order else BB/ABB; q from circle_q.  Returns (flags, q, groups,
    u[3, n], rho0, H0, info) with info holding nu, k, D, U, T_in, T_cyl and
    the section columns 50 lu after the inlet and 100 lu before the outlet."""
    nx, ny = 1000 * S, 150 * S
    D, U, nu = 30.0 * S, 0.01 / S, 0.03
    k = nu / Pr
    r = D / 2.0
    cx, cy = xc_frac * nx, ny / 2.0 - 0.5
    n = nx * ny
    f = np.zeros((ny, nx), np.uint16)
    f[:, 0] = flag(EQ, 0)
    f[:, nx - 1] = flag(OUTLET, 0)
    yy, xx = np.mgrid[0:ny, 0:nx]
    disc = (xx - cx) ** 2 + (yy - cy) ** 2 <= r * r
    f[disc] = flag(SOLID, 1)
    flags = f.reshape(-1)
    q = circle_q(nx, ny, flags, [(cx, cy, r, True)])
    u = np.zeros((3, ny, nx))
    u[0] = U
    u[:, disc] = 0.0
    T_in, T_cyl = 10.0, 11.0
    scheme = 1 if second_order else 0
    groups = [dict(f_scheme=0, h_scheme=0, rho_w=1.0, H_w=T_in),
              dict(f_scheme=scheme, h_scheme=scheme, rho_w=1.0, H_w=T_cyl)]
    info = dict(nx=nx, ny=ny, nu=nu, k=k, D=D, U=U, T_in=T_in, T_cyl=T_cyl, sections=(50, nx - 101))
    return flags, q, groups, u.reshape(3, n), np.ones(n), np.full(n, T_in), info


def taylor_green_3d(L: int = 256, u0: float = 0.04):
    """Taylor-Green vortex on an L^3 periodic box: u = u0 (sin kx cos ky cos kz,
    -cos kx sin ky cos kz, 0), rho = 1 + 3 p with p = u0^2/16 (cos 2kx + cos 2ky)
    (cos 2kz + 2), H = 1 + 0.1 sin kx sin ky sin kz, k = 2 pi / L.
    Returns (rho[n], u[3, n], H[n]) with x fastest."""
    kk = 2.0 * math.pi / L
    c = np.arange(L, dtype=np.float64) * kk
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    ux = u0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    uy = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    p = u0 * u0 / 16.0 * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
    rho = 1.0 + 3.0 * p
    H = 1.0 + 0.1 * np.sin(X) * np.sin(Y) * np.sin(Z)
    u = np.stack([ux, uy, np.zeros_like(ux)]).reshape(3, -1)
    return rho.reshape(-1), u, H.reshape(-1)


def concentric_cylinders(R: int, T_in: float = 2.0, T_out: float = 1.0, eq_layer: bool = False,
                         offset=(0.31, 0.17)):
    """Heater disc of radius R/2 inside a cooler circle of radius R (Sec. 4.3), on an
    (2R+6)^2 periodic box with an off-grid centre.  Groups: 0 inner (H = T_in),
    1 outer (H = T_out).  With eq_layer, every solid node linked to a fluid node
    becomes an EQ node of its wall.  Returns (L, flags, q, groups_h_values, T_exact, fluid)."""
    L = 2 * R + 6
    cx, cy = L / 2 + offset[0], L / 2 + offset[1]
    ri, ro = R / 2.0, float(R)
    y, x = np.mgrid[0:L, 0:L]
    r = np.hypot(x - cx, y - cy)
    inner = r <= ri
    outer = r >= ro
    fluid = ~inner & ~outer
    flags = np.zeros((L, L), np.uint16)
    flags[inner] = flag(SOLID, 0)
    flags[outer] = flag(SOLID, 1)
    if eq_layer:
        near = np.zeros_like(fluid)
        for a in range(1, 9):
            near |= np.roll(np.roll(fluid, -int(D2Q9_E[a, 1]), axis=0), -int(D2Q9_E[a, 0]), axis=1)
        layer = near & ~fluid
        flags[layer & inner] = flag(EQ, 0)
        flags[layer & outer] = flag(EQ, 1)
    flags = flags.reshape(-1)
    q = circle_q(L, L, flags, [(cx, cy, ri, True), (cx, cy, ro, False)])
    T = np.where(fluid, (T_out - T_in) * np.log(np.maximum(r, 1e-12) / ri) / math.log(ro / ri) + T_in,
                 np.where(inner, T_in, T_out))
    return L, flags, q, (T_in, T_out), T.reshape(-1), fluid.reshape(-1)
