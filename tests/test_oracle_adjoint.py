"""Pins of the oracle's discrete adjoint (advection-diffusion with a source).

The adjoint is not in the paper; it is defined as the exact transpose of the
forward step.  The forward step is affine in (state, Q), so the checks are
exact identities up to rounding: the transpose identity against the oracle's
own forward step, and central finite differences of the objective (quadratic
in Q, so the central difference has no truncation error)."""
import numpy as np
import pytest

from paper_2203_01316_amd import workloads as W


def _sim(oracle, L=10, Q=9, u=(0.03, -0.02, 0.0), src=None, kind="trt", k=0.02):
    n = L * L if Q == 9 else L ** 3
    dims = (L, L, 1) if Q == 9 else (L, L, L)
    return oracle.Sim(Q, *dims, s_h=oracle.preset(Q, kind, oracle.s_main(k)), u0=u,
                      src=np.zeros(n) if src is None else src), n


def _forward_pre(sim, pre, src):
    """F(pre; Q) = stream(collide(pre)) with source Q."""
    sim.set_source(src)
    fz = np.zeros_like(pre)
    _, post = sim.collide(fz, pre)
    sim.set_post(h=post)
    return sim.pre()[1]


@pytest.mark.parametrize("Q,kind", [(9, "trt"), (9, "srt"), (27, "trt")])
def test_adjoint_is_transpose_of_forward(oracle, Q, kind):
    L = 8 if Q == 9 else 4
    sim, n = _sim(oracle, L, Q, kind=kind)
    rng = np.random.default_rng(40)
    p = rng.uniform(0.0, 0.3, (Q, n))
    d = rng.standard_normal((Q, n))
    src = 0.01 * rng.standard_normal(n)
    dq = rng.standard_normal(n)
    lam = rng.standard_normal((Q, n))
    sim.set_source(src)
    dJdQ = np.zeros(n)
    adj = sim.adjoint_step(lam, dJdQ)
    F0 = _forward_pre(sim, p, src)
    F1 = _forward_pre(sim, p + d, src)
    F2 = _forward_pre(sim, p, src + dq)
    lhs = float((lam * (F1 - F0)).sum())
    assert lhs == pytest.approx(float((adj * d).sum()), rel=1e-11)
    lhs = float((lam * (F2 - F0)).sum())
    assert lhs == pytest.approx(float((dJdQ * dq).sum()), rel=1e-10)


def test_adjoint_gradient_matches_central_differences(oracle):
    L, T = 8, 25
    rng = np.random.default_rng(41)
    src = 0.01 * rng.standard_normal(L * L)
    target = 1.0 + 0.01 * rng.standard_normal(L * L)
    H0 = W.gaussian_hill(L, 2.0, 0.2, None, (0.0, 0.0), 0.0, 0.0)

    def run(q):
        sim, _ = _sim(oracle, L, src=q)
        sim.init(H0)
        return sim

    sim = run(src)
    J, g = sim.gradient_source(target, T)
    eps = 1e-3
    for node in rng.integers(0, L * L, 6):
        qp = src.copy()
        qp[node] += eps
        qm = src.copy()
        qm[node] -= eps
        sp = run(qp)
        sp.step(T)
        sm = run(qm)
        sm.step(T)
        Jp, _, _ = sp.objective(target)
        Jm, _, _ = sm.objective(target)
        fd = (Jp - Jm) / (2 * eps)
        assert fd == pytest.approx(g[node], rel=1e-7, abs=1e-12)
    assert J > 0


@pytest.mark.parametrize("every", [1, 4])
def test_tracking_gradient_matches_central_differences(oracle, every):
    """An objective summed over observation times (every `every` steps, the
    last one at T or before it): the reverse sweep with the seed of each time
    added once lambda is carried back to it equals central differences of J
    (quadratic in Q, so exact up to rounding).  Seeds at the wrong time, or a
    missing one, fail by O(1)."""
    L, T = 8, 23
    rng = np.random.default_rng(42 + every)
    src = 0.01 * rng.standard_normal(L * L)
    target = 1.0 + 0.01 * rng.standard_normal(L * L)
    H0 = W.gaussian_hill(L, 2.0, 0.2, None, (0.0, 0.0), 0.0, 0.0)

    def run(q):
        sim, _ = _sim(oracle, L, src=q)
        sim.init(H0)
        return sim

    def J_of(q):
        sim = run(q)
        J = 0.0
        for t in range(1, T + 1):
            sim.step(1)
            if t % every == 0:
                J += sim.objective(target)[0]
        return J

    J, g = run(src).gradient_source_tracking(target, T, every)
    assert J == pytest.approx(J_of(src), rel=1e-14)
    eps = 1e-3
    for node in rng.integers(0, L * L, 6):
        qp = src.copy()
        qp[node] += eps
        qm = src.copy()
        qm[node] -= eps
        fd = (J_of(qp) - J_of(qm)) / (2 * eps)
        assert fd == pytest.approx(g[node], rel=1e-7, abs=1e-12)
    # the final-state objective is the special case every = T
    J1, g1 = run(src).gradient_source_tracking(target, T, T)
    J2, g2 = run(src).gradient_source(target, T)
    assert J1 == J2 and np.array_equal(g1, g2)


@pytest.mark.parametrize("Q,L", [(9, 8), (27, 4)])
def test_dense_adjoint_equals_periodic_adjoint(oracle, Q, L):
    """Two independent constructions of the periodic adjoint agree: the
    per-node transposed matrices and the transpose probed from the forward
    step column by column."""
    sim, n = _sim(oracle, L, Q)
    rng = np.random.default_rng(42)
    sim.set_source(0.01 * rng.standard_normal(n))
    lam = rng.standard_normal((Q, n))
    d1 = np.zeros(n)
    d2 = np.zeros(n)
    a1 = sim.adjoint_step(lam, d1)
    a2 = sim.adjoint_step_dense(lam, d2)
    assert np.abs(a1 - a2).max() < 1e-12 * np.abs(a1).max()
    assert np.abs(d1 - d2).max() < 1e-12 * np.abs(d1).max()


@pytest.mark.parametrize("case", ["walled", "channel"])
def test_dense_adjoint_with_walls_vs_central_differences(oracle, case):
    """Walls (ABB, IABB on a disc), EQ nodes with and without cut links, an EQ
    inlet and an outlet column (channel), with a prescribed Poiseuille
    velocity: the gradient of J from the probed adjoint equals central
    differences of the forward oracle (J is quadratic in Q)."""
    nx, ny, T = 16, 12, 10
    if case == "walled":
        flags, q, groups, u = W.walled_box(nx, ny, 6.3, 5.6, 2.2)
    else:
        flags, q, groups, u = W.channel(nx, ny, 6.3, 5.6, 2.2, H_wall=0.5)
    n = nx * ny
    rng = np.random.default_rng(43)
    src = 0.01 * rng.standard_normal(n)
    target = 1.0 + 0.01 * rng.standard_normal(n)
    H0 = 1.0 + 0.1 * rng.uniform(size=n)
    sh = oracle.preset(9, "trt", oracle.s_main(0.02))

    def run(qv):
        sim = oracle.Sim(9, nx, ny, s_h=sh, uvel=u, src=qv, flags=flags, qlink=q, groups=groups)
        sim.init(H0)
        return sim

    J, g = run(src).gradient_source(target, T, dense=True)
    t = flags & 15
    fluid = np.nonzero(t == W.FLUID)[0]
    eqs = np.nonzero(t == W.EQ)[0]
    nodes = list(rng.choice(fluid, 5, replace=False)) + [int(eqs[0]), int(eqs[-1])]
    outs = np.nonzero(t == W.OUTLET)[0]
    if outs.size:
        nodes += [int(outs[1]), int(outs[-2]), int(outs[1]) - 1]
    eps = 1e-3
    for node in nodes:
        qp = src.copy()
        qp[node] += eps
        qm = src.copy()
        qm[node] -= eps
        sp = run(qp)
        sp.step(T)
        sm = run(qm)
        sm.step(T)
        Jp, _, _ = sp.objective(target)
        Jm, _, _ = sm.objective(target)
        fd = (Jp - Jm) / (2 * eps)
        assert fd == pytest.approx(g[node], rel=1e-7, abs=1e-12), node
    assert J > 0


def test_dense_adjoint_ignores_solid_nodes(oracle):
    """Solid nodes carry no state: lambda there is ignored on input and zero on
    output."""
    nx, ny = 12, 10
    flags, q, groups, u = W.walled_box(nx, ny, 4.3, 4.6, 1.8)
    n = nx * ny
    sim = oracle.Sim(9, nx, ny, s_h=oracle.preset(9, "trt", oracle.s_main(0.02)), uvel=u, src=np.zeros(n),
                     flags=flags, qlink=q, groups=groups)
    rng = np.random.default_rng(44)
    lam = rng.standard_normal((9, n))
    solid = (flags & 15) == W.SOLID
    lam2 = lam.copy()
    lam2[:, solid] = rng.standard_normal((9, int(solid.sum())))
    a1 = sim.adjoint_step_dense(lam)
    a2 = sim.adjoint_step_dense(lam2)
    assert np.array_equal(a1, a2)
    assert not a1[:, solid].any()
