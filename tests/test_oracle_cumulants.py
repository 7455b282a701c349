"""Pins of the oracle's cumulant transform and cumulant collision (Sec. 2.1.1,
Eqs. hydro_cu_collision, H_cu_collision; App. D for the source).

The cumulants are checked against quantities defined without the oracle's
recursion: the paper's equilibrium cumulant vector, statistical independence,
the textbook central-moment formulas of the low-order cumulants, and the
mean / variance of the post-collision populations.
"""
import math

import numpy as np
import pytest

from paper_2203_01316_amd import workloads as W

CS2 = 1.0 / 3.0


def _moments_by_definition(e, g):
    """Mean, and central moments E[prod (x_d - mean_d)^n_d] of g / sum g."""
    p = g / g.sum()
    mean = e.T.astype(float) @ p
    d = e - mean

    def central(n):
        return float((p * np.prod(d ** np.asarray(n), axis=1)).sum())

    return mean, central


@pytest.mark.parametrize("Q", [9, 27])
def test_round_trip(oracle, Q):
    rng = np.random.default_rng(3)
    for _ in range(5):
        g = rng.uniform(0.01, 0.3, Q)
        c = oracle.cumulants(Q, g)
        assert np.abs(oracle.from_cumulants(Q, c) - g).max() < 1e-13


@pytest.mark.parametrize("Q", [9, 27])
def test_equilibrium_cumulants_are_the_paper_vector(oracle, Q):
    """The discrete equilibrium has the cumulants listed in Sec. 2.1.1: psi,
    the velocity at first order, cs^2 on 200/020/002, zero elsewhere."""
    _, _, mo = oracle.lattice(Q)
    for psi, u in ((1.0, (0.0, 0.0, 0.0)), (1.7, (0.08, -0.05, 0.03)), (0.4, (-0.1, 0.02, -0.07))):
        uu = np.array(u)
        if Q == 9:
            uu[2] = 0.0
        c = oracle.cumulants(Q, oracle.equilibrium(Q, psi, uu))
        want = np.zeros(Q)
        for k, n in enumerate(mo):
            order = n.sum()
            if order == 0:
                want[k] = psi
            elif order == 1:
                want[k] = uu[int(np.argmax(n))]
            elif order == 2 and n.max() == 2:
                want[k] = CS2
        assert np.abs(c - want).max() < 1e-13, (psi, u)


@pytest.mark.parametrize("Q", [9, 27])
def test_independent_axes(oracle, Q):
    """A product distribution g = rho prod_d p_d(e_d): every cumulant with two
    or more nonzero indices vanishes, and the pure ones are the mean and
    variance of the one-dimensional factors."""
    e, _, mo = oracle.lattice(Q)
    D = 2 if Q == 9 else 3
    rng = np.random.default_rng(11)
    p = [rng.uniform(0.1, 1.0, 3) for _ in range(D)]
    p = [v / v.sum() for v in p]
    rho = 1.37
    g = np.array([rho * np.prod([p[d][e[a, d] + 1] for d in range(D)]) for a in range(Q)])
    c = oracle.cumulants(Q, g)
    vals = np.array([-1.0, 0.0, 1.0])
    for k, n in enumerate(mo):
        nz = np.nonzero(n)[0]
        if len(nz) == 0:
            assert c[k] == pytest.approx(rho, rel=1e-14)
        elif len(nz) >= 2:
            assert abs(c[k]) < 1e-14, n
        else:
            d = nz[0]
            m1 = (p[d] * vals).sum()
            if n[d] == 1:
                assert c[k] == pytest.approx(m1, abs=1e-15)
            else:
                assert c[k] == pytest.approx((p[d] * vals ** 2).sum() - m1 ** 2, abs=1e-15)


def test_low_order_cumulants_by_definition(oracle):
    """Covariance, third central moments and the fourth-order formulas
    k22 = m22 - m20 m02 - 2 m11^2 and k211 = m211 - m200 m011 - 2 m110 m101
    (central moments of the normalised distribution)."""
    rng = np.random.default_rng(5)
    for Q in (9, 27):
        e, _, mo = oracle.lattice(Q)
        g = rng.uniform(0.02, 0.2, Q)
        c = oracle.cumulants(Q, g)
        mean, m = _moments_by_definition(e, g)
        idx = {tuple(n): k for k, n in enumerate(mo)}
        assert c[idx[(1, 0, 0)]] == pytest.approx(mean[0], abs=1e-15)
        assert c[idx[(1, 1, 0)]] == pytest.approx(m((1, 1, 0)), abs=1e-15)
        assert c[idx[(2, 1, 0)]] == pytest.approx(m((2, 1, 0)), abs=1e-15)
        k22 = m((2, 2, 0)) - m((2, 0, 0)) * m((0, 2, 0)) - 2 * m((1, 1, 0)) ** 2
        assert c[idx[(2, 2, 0)]] == pytest.approx(k22, abs=1e-15)
        if Q == 27:
            k211 = m((2, 1, 1)) - m((2, 0, 0)) * m((0, 1, 1)) - 2 * m((1, 1, 0)) * m((1, 0, 1))
            assert c[idx[(2, 1, 1)]] == pytest.approx(k211, abs=1e-15)
            assert c[idx[(1, 1, 1)]] == pytest.approx(m((1, 1, 1)), abs=1e-15)


@pytest.mark.parametrize("Q", [9, 27])
def test_full_relaxation_gives_equilibrium(oracle, Q):
    rng = np.random.default_rng(7)
    g = rng.uniform(0.02, 0.2, Q)
    u = np.array([0.04, -0.06, 0.05 if Q == 27 else 0.0])
    out = oracle.collide_node_cu(Q, g, u, np.ones(27))
    assert np.abs(out - oracle.equilibrium(Q, g.sum(), u)).max() < 1e-15


@pytest.mark.parametrize("Q", [9, 27])
def test_cumulants_first_relaxes_the_mean(oracle, Q):
    """Cumulants-1st (Sec. 2.1.1): only the first cumulants move, at s^H,
    towards u; every other cumulant is set to equilibrium, so after the
    collision the mean is c1 + s (u - c1), the variance along each axis is
    cs^2 and sum g grows by the source Q."""
    e, _, _ = oracle.lattice(Q)
    D = 2 if Q == 9 else 3
    rng = np.random.default_rng(9)
    g = rng.uniform(0.02, 0.2, Q)
    u = np.array([0.03, 0.07, -0.02 if Q == 27 else 0.0])
    s = oracle.preset(Q, "1st", 1.7)
    src = 0.013
    out = oracle.collide_node_cu(Q, g, u, s, src)
    mean0, _ = _moments_by_definition(e, g)
    mean1, m1 = _moments_by_definition(e, out)
    assert out.sum() == pytest.approx(g.sum() + src, rel=1e-14)
    for d in range(D):
        assert mean1[d] == pytest.approx(mean0[d] + 1.7 * (u[d] - mean0[d]), abs=1e-14)
        var = m1(tuple(2 if i == d else 0 for i in range(3)))
        assert var == pytest.approx(CS2, abs=1e-14)


@pytest.mark.parametrize("Q", [9, 27])
def test_cumulant_ns_conserves_mass_and_momentum(oracle, Q):
    e, _, _ = oracle.lattice(Q)
    rng = np.random.default_rng(13)
    f = rng.uniform(0.02, 0.2, Q)
    u = (e.T.astype(float) @ f) / f.sum()
    out = oracle.collide_node_cu(Q, f, u, oracle.preset(Q, "ns", 1.6))
    assert out.sum() == pytest.approx(f.sum(), rel=1e-14)
    assert np.abs(e.T @ out - e.T @ f).max() < 1e-14


def _hill_error_cu(oracle, L, n, k, u, sigma):
    sim = oracle.Sim(9, L, L, s_h=oracle.preset(9, "1st", oracle.s_main(k)), u0=(u[0], u[1], 0.0), cu_h=True)
    sim.init(W.gaussian_hill(L, sigma, 0.5, None, u, k, 0.0))
    sim.step(n)
    _, _, H = sim.macroscopic()
    a = W.gaussian_hill(L, sigma, 0.5, None, u, k, float(n))
    return math.sqrt(((a - H) ** 2).sum() / (a ** 2).sum())


def test_cumulants_first_gaussian_hill(oracle):
    """Sec. 4.1 with the Cumulants-1st kernel: the advected hill follows the
    closed form, and the error falls by four under diffusive scaling."""
    assert _hill_error_cu(oracle, 64, 1000, 0.01, (0.05, 0.02), 8.0) < 6e-4
    e1 = _hill_error_cu(oracle, 32, 100, 0.02, (0.04, 0.02), 4.0)
    e2 = _hill_error_cu(oracle, 64, 400, 0.02, (0.02, 0.01), 8.0)
    assert 3.5 < e1 / e2 < 4.5, (e1, e2)


def test_cumulant_shear_wave_gives_viscosity(oracle):
    """f with the cumulant collision, second-order cumulants at s_nu: a shear
    wave decays as exp(-nu k^2 t)."""
    for Q, dims in ((9, (2, 32, 1)), (27, (2, 32, 2))):
        nx, ny, nz = dims
        nu = 0.05
        N = nx * ny * nz
        y = (np.arange(N) // nx) % ny
        A = 1e-3
        kk = 2 * math.pi / ny
        u = np.zeros((3, N))
        u[0] = A * np.sin(kk * y)
        sim = oracle.Sim(Q, nx, ny, nz, with_ns=True, s_f=oracle.preset(Q, "ns", oracle.s_main(nu)),
                         s_h=oracle.preset(Q, "1st", 1.0), cu_f=True, cu_h=True)
        sim.init(np.ones(N), u=u, rho=np.ones(N))
        T = 300
        sim.step(T)
        _, uu, _ = sim.macroscopic()
        amp = 2.0 / N * (uu[0] * np.sin(kk * y)).sum()
        rate = -math.log(amp / A) / (kk * kk * (T + 0.5))
        assert rate == pytest.approx(nu, rel=0.01), (Q, rate)
