"""In-place (AA) streaming against two-array (AB) streaming: the same
arithmetic on every node, so the canonical states, the stored post-collision
states, the macroscopic fields and the reductions agree bit for bit after odd
and even step counts, with walls, interpolated walls, EQ nodes and outlets.
With stochastic rounding (FP32-SR) the draws follow the updating node and
the value's direction, so both layouts make the same draws and agree bit for
bit too."""
import numpy as np
import pytest

from paper_2203_01316_amd import workloads as W

from gpu_common import f32, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    from paper_2203_01316_amd import lbm
    return lbm


def _both(L, make):
    return make(L.STREAM_AB), make(L.STREAM_AA)


def _same(L, ab, aa, lattices, exact=True, cols=(), group=0):
    for lat in lattices:
        for which in ("pre", "post"):
            x = ab.populations(lat, which).cpu().numpy()
            y = aa.populations(lat, which).cpu().numpy()
            if exact:
                assert np.array_equal(x, y), (lat, which, np.abs(x - y).max())
            else:
                assert rel_l2(y, x) < 1e-6, (lat, which, rel_l2(y, x))
    ra = ab.reduce(group=group, columns=cols)
    rb = aa.reduce(group=group, columns=cols)
    if exact:
        assert np.array_equal(ra, rb), (ra, rb)
    _, ua, Ha = ab.macroscopic()
    _, ub, Hb = aa.macroscopic()
    if exact:
        assert np.array_equal(Ha.cpu().numpy(), Hb.cpu().numpy())


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp32_sr"])
def test_aa_periodic_hill(L, storage):
    H0 = W.gaussian_hill(64, 8.0, 0.5, None, (0.05, 0.02), 0.01, 0.0)

    def make(stream):
        g = L.LBM(9, 64, 64, storage=storage, k=0.01, u0=(0.05, 0.02, 0), stream=stream)
        g.init(H0)
        return g

    ab, aa = _both(L, make)
    for k in (1, 6, 13):
        ab.step(k)
        aa.step(k)
        _same(L, ab, aa, ("h",))


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp32_sr"])
def test_aa_channel(L, storage):
    flags, q, groups, u = W.channel(160, 48, 40, 24, 7.5, 0.05)
    uu = f32(u) if storage == "fp32" else u

    def make(stream):
        g = L.LBM(9, 160, 48, storage=storage, k=0.005, u_mode=1, flags=flags, q=q, groups=groups, stream=stream)
        g.set_velocity(uu)
        g.init(np.zeros(160 * 48))
        return g

    ab, aa = _both(L, make)
    for k in (1, 2, 37):
        ab.step(k)
        aa.step(k)
        _same(L, ab, aa, ("h",), cols=(10, 80, 159), group=2)


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp32_sr"])
def test_aa_coupled_cylinder(L, storage):
    flags, q, groups, u, rho0, H0 = W.heated_cylinder(192, 96, 9.5, u_in=0.04, amp=1e-3, seed=0)
    uu = f32(u) if storage == "fp32" else u

    def make(stream):
        g = L.LBM(9, 192, 96, storage=storage, with_ns=True, nu=0.04, k=0.06, flags=flags, q=q, groups=groups,
                  stream=stream)
        g.set_velocity(uu)
        g.init(H0, u=uu, rho=rho0)
        return g

    ab, aa = _both(L, make)
    for k in (1, 4, 51):
        ab.step(k)
        aa.step(k)
        _same(L, ab, aa, ("f", "h"), cols=(5, 150), group=1)


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp32_sr"])
def test_aa_boundary_mix(L, storage):
    """Listed outlets (the thread also updates the upstream node) next to
    bulk-handled ones (the upstream populations come from the previous lane)."""
    flags, q, groups, u, rho0, H0 = W.boundary_mix()
    uu = f32(u) if storage == "fp32" else u

    def make(stream):
        g = L.LBM(9, 33, 40, storage=storage, with_ns=True, nu=0.04, k=0.05, flags=flags, q=q, groups=groups,
                  stream=stream)
        g.set_velocity(uu)
        g.init(H0, u=uu, rho=rho0)
        return g

    ab, aa = _both(L, make)
    for k in (1, 2, 37):
        ab.step(k)
        aa.step(k)
        _same(L, ab, aa, ("f", "h"), cols=(2, 31, 32), group=2)


@pytest.mark.parametrize("storage", ["fp32", "fp64", "fp32_sr"])
def test_aa_d3q27_sphere(L, storage):
    nx, ny, nz = 20, 14, 12
    flags, q, groups = W.sphere_box(nx, ny, nz, (9.3, 6.6, 5.8), 3.4, inlet=True)
    n = nx * ny * nz
    rng = np.random.default_rng(60)
    u = np.zeros((3, n))
    u[0] = 0.02
    u = f32(u) if storage == "fp32" else u
    H0 = 1 + 0.1 * rng.uniform(size=n)

    def make(stream):
        g = L.LBM(27, nx, ny, nz, storage=storage, with_ns=True, nu=0.03, k=0.02, flags=flags, q=q, groups=groups,
                  stream=stream)
        g.init(H0, u=u, rho=np.ones(n))
        return g

    ab, aa = _both(L, make)
    for k in (1, 2, 9):
        ab.step(k)
        aa.step(k)
        _same(L, ab, aa, ("f", "h"), cols=(3, 15), group=0)


@pytest.mark.parametrize("cu", [False, True])
@pytest.mark.parametrize("storage", ["fp32", "fp64", "fp32_sr"])
def test_aa_d3q27_several_tiles(L, storage, cu):
    """Several population tiles with a ragged last one (19,200 nodes), sphere,
    inlet and outlet, central-moment or cumulant kernels (the in-place steps
    run under their residency cap)."""
    nx, ny, nz = 40, 30, 16
    flags, q, groups = W.sphere_box(nx, ny, nz, (17.3, 14.6, 7.8), 5.2, inlet=True)
    n = nx * ny * nz
    u = np.zeros((3, n))
    u[0] = 0.02
    u = f32(u) if storage == "fp32" else u
    H0 = 1 + 0.1 * np.random.default_rng(63).uniform(size=n)

    def make(stream):
        g = L.LBM(27, nx, ny, nz, storage=storage, with_ns=True, nu=0.03, k=0.02, flags=flags, q=q, groups=groups,
                  stream=stream, cumulant_f=cu, cumulant_h=cu, relax_h="1st" if cu else "trt")
        g.init(H0, u=u, rho=np.ones(n))
        return g

    ab, aa = _both(L, make)
    for k in (1, 4):
        ab.step(k)
        aa.step(k)
        _same(L, ab, aa, ("f", "h"), cols=(3, 31), group=0)


def test_aa_full_size_cylinder(L):
    """2048^2 coupled FP32 heated cylinder (the benchmark configuration): the
    in-place layout equals the two-array one bit for bit after 1 and 3 steps."""
    nx = ny = 2048
    nu = 0.0512
    flags, q, groups, u, rho0, H0 = W.heated_cylinder(nx, ny, 64, u_in=0.04, amp=1e-3, seed=0)
    uu = f32(u)

    def make(stream):
        g = L.LBM(9, nx, ny, storage="fp32", with_ns=True, nu=nu, k=nu / 0.71, flags=flags, q=q, groups=groups,
                  stream=stream, rho_ref=1.0, H_ref=10.0)
        g.set_velocity(uu)
        g.init(H0, u=uu, rho=rho0)
        return g

    ab, aa = _both(L, make)
    for k in (1, 2):
        ab.step(k)
        aa.step(k)
        _same(L, ab, aa, ("f", "h"), cols=(50, nx - 101), group=1)


def test_aa_restart_and_set_at_odd_phase(L):
    flags, q, groups, u, rho0, H0 = W.heated_cylinder(96, 48, 6.5, cx=24, cy=24, u_in=0.04, amp=1e-3, seed=0)
    uu = f32(u)

    def make(stream):
        g = L.LBM(9, 96, 48, storage="fp32", with_ns=True, nu=0.04, k=0.05, flags=flags, q=q, groups=groups,
                  stream=stream)
        g.set_velocity(uu)
        g.init(H0, u=uu, rho=rho0)
        return g

    ab, aa = _both(L, make)
    ab.step(7)
    aa.step(7)
    snap = aa.save_state()
    aa.step(10)
    ref = aa.populations("h", "post").cpu().numpy()
    aa.load_state(snap)
    assert aa.t == 7
    aa.step(10)
    assert np.array_equal(aa.populations("h", "post").cpu().numpy(), ref)
    # replace the state of both contexts at odd AA phase, then continue
    fpost = ab.populations("f", "post")
    hpost = ab.populations("h", "post")
    ab.step(3)
    aa2 = make(L.STREAM_AA)
    aa2.step(1)
    aa2.set_populations("f", fpost, t=17)
    aa2.set_populations("h", hpost, t=17)
    ab2 = make(L.STREAM_AB)
    ab2.set_populations("f", fpost, t=17)
    ab2.set_populations("h", hpost, t=17)
    ab2.step(3)
    aa2.step(3)
    _same(L, ab2, aa2, ("f", "h"))


def test_aa_fp16_dev_close_to_ab(L):
    flags, q, groups, u, rho0, H0 = W.heated_cylinder(192, 96, 9.5, u_in=0.04, amp=1e-3, seed=0)
    uu = f32(u)

    def make(stream):
        g = L.LBM(9, 192, 96, storage="fp16_dev", with_ns=True, nu=0.04, k=0.06, flags=flags, q=q, groups=groups,
                  stream=stream, rho_ref=1.0, H_ref=10.0)
        g.set_velocity(uu)
        g.init(H0, u=uu, rho=rho0)
        return g

    ab, aa = _both(L, make)
    ab.step(41)
    aa.step(41)
    _same(L, ab, aa, ("f", "h"), exact=False)


def _random_state(n, D, seed):
    rng = np.random.default_rng(seed)
    u = np.zeros((3, n))
    u[0] = 0.03 + 0.01 * rng.standard_normal(n)
    u[1] = 0.01 * rng.standard_normal(n)
    if D == 3:
        u[2] = 0.01 * rng.standard_normal(n)
    return u, 1 + 1e-3 * rng.standard_normal(n), 10 + rng.standard_normal(n)


@pytest.mark.parametrize("storage", ["fp32", "fp32_dev", "fp16_dev", "fp16_sr"])
@pytest.mark.parametrize("case", ["d2q9_one_block_rows", "d2q9_two_block_rows", "d2q9_ade_two_block_rows",
                                  "d3q27_one_block_rows", "d3q27_cumulant"])
def test_aa_realigned_pushes(L, case, storage):
    """Lattices without geometry whose x-rows are whole blocks of 256 nodes,
    where the swapped in-place phase hands its x-pushes to the thread that
    stores them through LDS: rows of one block (the periodic wrap stays in the
    block) and of two blocks (one push per direction leaves each block, and
    the last block of a row wraps to the row's start), coupled or
    advection-diffusion only, central moments or cumulants.  AA equals AB bit
    for bit after odd and even step counts."""
    D = 3 if case.startswith("d3q27") else 2
    dims = {"d2q9_one_block_rows": (256, 5, 1), "d2q9_two_block_rows": (512, 6, 1),
            "d2q9_ade_two_block_rows": (512, 4, 1), "d3q27_one_block_rows": (256, 3, 4),
            "d3q27_cumulant": (256, 4, 3)}[case]
    n = dims[0] * dims[1] * dims[2]
    u, rho, H = _random_state(n, D, 71)
    ns = "ade" not in case
    cu = case == "d3q27_cumulant"
    u = f32(u)

    def make(stream):
        kw = dict(storage=storage, stream=stream, rho_ref=1.0, H_ref=10.0, k=0.02)
        if ns:
            kw.update(with_ns=True, nu=0.03, cumulant_f=cu, cumulant_h=cu, relax_h="1st" if cu else "trt")
        else:
            kw.update(u0=(0.05, 0.02, 0.0))
        g = L.LBM(9 if D == 2 else 27, *(dims[:2] if D == 2 else dims), **kw)
        g.init(H, u=u if ns else None, rho=rho if ns else None)
        return g

    ab, aa = _both(L, make)
    for k in (1, 2, 5):
        ab.step(k)
        aa.step(k)
        _same(L, ab, aa, ("f", "h") if ns else ("h",))


@pytest.mark.parametrize("storage", ["fp32", "fp32_dev", "fp16_dev", "fp16_sr"])
@pytest.mark.parametrize("nx", [256, 512])
def test_aa_rows_of_whole_blocks_with_geometry(L, nx, storage):
    """Rows of one and two whole blocks with geometry (heated cylinder with
    walls, an EQ inlet and an outlet column), where the in-place step keeps
    the plain push (the realignment is for lattices without geometry): AA
    equals AB bit for bit (FP16: within rounding of the stored deviations)."""
    ny = 64
    flags, q, groups, u, rho0, H0 = W.heated_cylinder(nx, ny, 9.5, cx=nx // 3, cy=31.3, u_in=0.04, amp=1e-3,
                                                       seed=4)
    uu = f32(u)

    def make(stream):
        g = L.LBM(9, nx, ny, storage=storage, with_ns=True, nu=0.04, k=0.06, flags=flags, q=q, groups=groups,
                  stream=stream, rho_ref=1.0, H_ref=10.0)
        g.set_velocity(uu)
        g.init(H0, u=uu, rho=rho0)
        return g

    ab, aa = _both(L, make)
    for k in (1, 2, 7):
        ab.step(k)
        aa.step(k)
        _same(L, ab, aa, ("f", "h"), exact=storage not in ("fp16_dev", "fp16_sr"), cols=(3, nx - 20), group=1)


def test_aa_rows_of_whole_blocks_d3q27_sphere(L):
    """D3Q27 with a sphere, an EQ inlet plane and an outlet plane on rows of
    256 nodes (bulk and boundary launches): AA equals AB bit for bit."""
    nx, ny, nz = 256, 12, 10
    flags, q, groups = W.sphere_box(nx, ny, nz, (60.3, 5.6, 4.8), 3.4, inlet=True)
    n = nx * ny * nz
    u = np.zeros((3, n))
    u[0] = 0.02
    H0 = 1 + 0.1 * np.random.default_rng(64).uniform(size=n)

    def make(stream):
        g = L.LBM(27, nx, ny, nz, storage="fp32", with_ns=True, nu=0.03, k=0.02, flags=flags, q=q, groups=groups,
                  stream=stream)
        g.init(H0, u=f32(u), rho=np.ones(n))
        return g

    ab, aa = _both(L, make)
    for k in (1, 2, 5):
        ab.step(k)
        aa.step(k)
        _same(L, ab, aa, ("f", "h"), cols=(3, nx - 20), group=0)
