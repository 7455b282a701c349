"""GPU discrete adjoint against the oracle's adjoint (periodic, and with walls
and EQ nodes) and against central finite differences of the GPU's own FP64
forward (the objective is quadratic in the source, so the central difference
has no truncation error)."""
import numpy as np
import pytest

from gpu_common import f32, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    from paper_2203_01316_amd import lbm
    return lbm


def _ctx(L, Q, dims, storage, u0=(0.03, 0.0, 0.0), uvel=None, k=0.01):
    kw = dict(storage=storage, k=k, u0=u0, with_source=True, u_mode=1 if uvel is not None else 0)
    g = L.LBM(Q, *dims, **kw)
    if uvel is not None:
        g.set_velocity(uvel)
    return g


@pytest.mark.parametrize("Q,dims,storage,tol", [(9, (37, 21, 1), "fp64", 1e-12), (9, (37, 21, 1), "fp32", 1e-5),
                                                (27, (9, 7, 6), "fp64", 1e-12), (27, (9, 7, 6), "fp32", 1e-5)])
def test_adjoint_step_matches_oracle(L, oracle, Q, dims, storage, tol):
    import torch
    n = int(np.prod(dims))
    rng = np.random.default_rng(50)
    u = np.zeros((3, n))
    u[: (2 if Q == 9 else 3)] = rng.uniform(-0.04, 0.04, (2 if Q == 9 else 3, n))
    if storage == "fp32":
        u = f32(u)
    g = _ctx(L, Q, dims, storage, uvel=u)
    g.set_source(np.zeros(n))
    sf, sh = L.relaxation_rates(g.params)
    o = oracle.Sim(Q, *dims, s_h=sh, uvel=u, src=np.zeros(n))
    lam = rng.standard_normal((Q, n))
    if storage == "fp32":
        lam = f32(lam)
    dt = g.rdtype
    lt = torch.as_tensor(lam, dtype=dt, device=g.device)
    out = torch.empty_like(lt)
    dq = torch.zeros(n, dtype=torch.float64, device=g.device)
    g.adjoint_step(lt, out, dq)
    g.sync()
    dq_o = np.zeros(n)
    ref = o.adjoint_step(lam, dq_o)
    assert rel_l2(out.cpu().numpy(), ref) < tol
    assert rel_l2(dq.cpu().numpy(), dq_o) < tol


def test_gradient_matches_oracle_adjoint(L, oracle):
    """J and dJ/dQ after 150 steps on 48^2 (FP64) equal the oracle's discrete adjoint."""
    import torch
    from paper_2203_01316_amd.adjoint import source_objective
    n1, T = 48, 150
    n = n1 * n1
    rng = np.random.default_rng(51)
    src = 0.01 * rng.standard_normal(n)
    target = 1.0 + 0.01 * rng.standard_normal(n)
    H0 = np.ones(n)
    g = _ctx(L, 9, (n1, n1, 1), "fp64", k=0.02)
    q = torch.tensor(src, dtype=torch.float64, device=g.device, requires_grad=True)
    J = source_objective(q, g, H0, target, T, recompute=True)
    J.backward()
    _, sh = L.relaxation_rates(g.params)
    o = oracle.Sim(9, n1, n1, s_h=sh, u0=(0.03, 0.0, 0.0), src=src)
    o.init(H0)
    Jo, go = o.gradient_source(target, T)
    assert float(J.detach()) == pytest.approx(Jo, rel=1e-12)
    assert rel_l2(q.grad.cpu().numpy(), go) < 1e-11


def test_c5_gradient_vs_central_differences(L):
    """512^2, 2000 steps, u = (0.03, 0), source ~ N(0, 0.01^2): the FP32 adjoint
    gradient (checkpoints every 45 steps, with and without replay) matches FP64
    central differences (eps = 1e-3) on 16 random nodes: at every node within
    1e-4 of the largest |dJ/dQ| of the sample, and within 1e-4 relative at
    every node whose |dJ/dQ| is at least a tenth of that largest value (the
    relative error of a near-zero gradient measures only its cancellation)."""
    import torch
    from paper_2203_01316_amd.adjoint import source_objective
    n1, T, k = 512, 2000, 0.01
    n = n1 * n1
    src = 0.01 * np.random.Generator(np.random.PCG64(1)).standard_normal(n)
    target = 1.0 + 0.01 * np.random.Generator(np.random.PCG64(2)).standard_normal(n)
    nodes = np.random.Generator(np.random.PCG64(3)).choice(n, 16, replace=False)
    H0 = np.ones(n)
    g32 = _ctx(L, 9, (n1, n1, 1), "fp32", k=k)
    grads = []
    for rec in (True, False):
        q = torch.tensor(f32(src), dtype=torch.float32, device=g32.device, requires_grad=True)
        J = source_objective(q, g32, H0, target, T, interval=45, recompute=rec)
        J.backward()
        grads.append(q.grad.double().cpu().numpy())
    np.testing.assert_array_equal(grads[0], grads[1])
    g64 = _ctx(L, 9, (n1, n1, 1), "fp64", k=k)
    eps = 1e-3

    def J64(qv):
        g64.set_source(qv)
        g64.init(H0)
        g64.step(T)
        Jv, _, _ = g64.objective(target)
        return Jv

    fd = []
    for m in nodes:
        qp = src.copy()
        qp[m] += eps
        qm = src.copy()
        qm[m] -= eps
        fd.append((J64(qp) - J64(qm)) / (2 * eps))
    fd = np.array(fd)
    adj = grads[0][nodes]
    scale = np.abs(fd).max()
    per_node = np.abs(adj - fd) / np.abs(fd)
    big = np.abs(fd) >= 0.1 * scale
    print("C5 gradient vs FD: rel L2 %.2e, max |adj - fd| / max |fd| %.2e, max relative on %d nodes %.2e, "
          "max relative on all %.2e" % (rel_l2(adj, fd), np.abs(adj - fd).max() / scale, big.sum(),
                                        per_node[big].max(), per_node.max()))
    assert np.abs(adj - fd).max() < 1e-4 * scale, (adj, fd)
    assert per_node[big].max() < 1e-4, (adj, fd)
    assert big.sum() >= 8


def test_tracking_gradient_fp32_vs_central_differences(L):
    """512^2, 400 steps, the objective summed every 20 steps against one
    target: the FP32 checkpointed sweep (snapshots every 20 steps, replayed
    for the residuals) against FP64 central differences of the same objective
    on 16 random nodes, with the bounds of the final-state test above."""
    import torch
    from paper_2203_01316_amd.adjoint import tracking_objective
    n1, T, every, k = 512, 400, 20, 0.01
    n = n1 * n1
    src = 0.01 * np.random.Generator(np.random.PCG64(11)).standard_normal(n)
    target = 1.0 + 0.01 * np.random.Generator(np.random.PCG64(12)).standard_normal(n)
    nodes = np.random.Generator(np.random.PCG64(13)).choice(n, 16, replace=False)
    H0 = np.ones(n)
    g32 = _ctx(L, 9, (n1, n1, 1), "fp32", k=k)
    q = torch.tensor(f32(src), dtype=torch.float32, device=g32.device, requires_grad=True)
    J = tracking_objective(q, g32, H0, target, T, every, interval=20)
    J.backward()
    adj = q.grad.double().cpu().numpy()[nodes]
    g64 = _ctx(L, 9, (n1, n1, 1), "fp64", k=k)
    eps = 1e-3

    def J64(qv):
        g64.set_source(qv)
        g64.init(H0)
        Jv = 0.0
        for _ in range(T // every):
            g64.step(every)
            Jv += g64.objective_residual(target)[0]
        return Jv

    fd = []
    for m in nodes:
        qp = src.copy()
        qp[m] += eps
        qm = src.copy()
        qm[m] -= eps
        fd.append((J64(qp) - J64(qm)) / (2 * eps))
    fd = np.array(fd)
    scale = np.abs(fd).max()
    per_node = np.abs(adj - fd) / np.abs(fd)
    big = np.abs(fd) >= 0.1 * scale
    print("tracking gradient vs FD: max |adj - fd| / max |fd| %.2e, max relative on %d nodes %.2e"
          % (np.abs(adj - fd).max() / scale, big.sum(), per_node[big].max()))
    assert float(J.detach()) == pytest.approx(J64(src), rel=1e-4)
    assert np.abs(adj - fd).max() < 1e-4 * scale, (adj, fd)
    assert per_node[big].max() < 1e-4, (adj, fd)
    assert big.sum() >= 8


def _walls(W, case):
    if case == "walled":
        dims = (24, 14, 1)
        flags, q, groups, u = W.walled_box(*dims[:2])
    elif case == "mix":
        dims = (33, 40, 1)
        flags, q, groups, u, _, _ = W.boundary_mix()
    elif case == "gap":
        dims = (20, 16, 1)
        flags, q_lo, q_hi, groups = W.gap_box(*dims[:2], H_w=2.0)
        q = np.where(np.random.default_rng(9).uniform(size=q_lo.shape) < 0.5, q_lo, q_hi)
        u = np.zeros((3, int(np.prod(dims))))
        u[0] = 0.03
        u[1] = -0.01
        u[:, (flags & 15) == W.SOLID] = 0.0
    else:
        dims = (8, 7, 6)
        flags, q, groups = W.sphere_box(*dims, (3.6, 3.3, 2.8), 1.7, inlet=case == "sphere_io")
        u = np.zeros((3, int(np.prod(dims))))
        u[0] = 0.03
        u[1] = -0.01
    return dims, flags, q, groups, u


@pytest.mark.parametrize("case,storage,tol", [("walled", "fp64", 1e-12), ("walled", "fp32", 1e-5),
                                              ("mix", "fp64", 1e-12), ("mix", "fp32", 1e-5),
                                              ("sphere", "fp64", 1e-12), ("sphere_io", "fp64", 1e-12),
                                              ("sphere_io", "fp32", 1e-5), ("gap", "fp64", 1e-12),
                                              ("gap", "fp32", 1e-5)])
def test_adjoint_step_with_walls_matches_oracle(L, oracle, case, storage, tol):
    """Walls (ABB and IABB on a disc, IABB on a sphere), EQ nodes with and
    without cut links, bulk-handled and listed outlets (the mixed inlet and
    outlet geometry, the sphere with an inlet and an outlet plane), one-node
    gaps with wall distances below and above 1/2: one GPU adjoint step against
    the oracle's transpose of its own forward step."""
    import torch
    from paper_2203_01316_amd import workloads as W
    dims, flags, q, groups, u = _walls(W, case)
    Q = 9 if dims[2] == 1 else 27
    n = int(np.prod(dims))
    if storage == "fp32":
        u = f32(u)
    g = L.LBM(Q, *dims, storage=storage, k=0.02, with_source=True, u_mode=1, flags=flags, q=q, groups=groups)
    g.set_velocity(u)
    g.set_source(np.zeros(n))
    _, sh = L.relaxation_rates(g.params)
    o = oracle.Sim(Q, *dims, s_h=sh, uvel=u, src=np.zeros(n), flags=flags, qlink=q, groups=groups)
    rng = np.random.default_rng(52)
    lam = rng.standard_normal((Q, n))
    if storage == "fp32":
        lam = f32(lam)
    lt = torch.as_tensor(lam, dtype=g.rdtype, device=g.device)
    out = torch.empty_like(lt)
    dq = torch.zeros(n, dtype=torch.float64, device=g.device)
    g.adjoint_step(lt, out, dq)
    g.sync()
    dq_o = np.zeros(n)
    ref = o.adjoint_step_dense(lam, dq_o)
    assert rel_l2(out.cpu().numpy(), ref) < tol
    assert rel_l2(dq.cpu().numpy(), dq_o) < tol


def test_gradient_with_walls_matches_oracle(L, oracle):
    """J and dJ/dQ after 12 steps of the walled box (FP64) equal the oracle's."""
    import torch
    from paper_2203_01316_amd import workloads as W
    from paper_2203_01316_amd.adjoint import source_objective
    T = 12
    dims, flags, q, groups, u = _walls(W, "walled")
    n = int(np.prod(dims))
    rng = np.random.default_rng(53)
    src = 0.01 * rng.standard_normal(n)
    target = 1.0 + 0.01 * rng.standard_normal(n)
    H0 = 1.0 + 0.1 * rng.uniform(size=n)
    g = L.LBM(9, *dims, storage="fp64", k=0.02, with_source=True, u_mode=1, flags=flags, q=q, groups=groups)
    g.set_velocity(u)
    qt = torch.tensor(src, dtype=torch.float64, device=g.device, requires_grad=True)
    J = source_objective(qt, g, H0, target, T, recompute=True)
    J.backward()
    _, sh = L.relaxation_rates(g.params)
    o = oracle.Sim(9, *dims, s_h=sh, uvel=u, src=src, flags=flags, qlink=q, groups=groups)
    o.init(H0)
    Jo, go = o.gradient_source(target, T, dense=True)
    assert float(J.detach()) == pytest.approx(Jo, rel=1e-12)
    assert rel_l2(qt.grad.cpu().numpy(), go) < 1e-11


@pytest.mark.parametrize("recompute,interval", [(True, 10), (True, 12), (False, 10)])
def test_tracking_gradient_matches_oracle(L, oracle, recompute, interval):
    """J summed every 7 steps over 150 steps on 48^2 (FP64) and dJ/dQ.  The
    checkpointed sweep (snapshots every `interval` steps; the residual of each
    observation time recomputed by replaying its segment, with observation
    times on and off segment starts) and the sweep over stored residuals
    both equal the oracle's reverse sweep."""
    import torch
    from paper_2203_01316_amd.adjoint import tracking_objective
    n1, T, every = 48, 150, 7
    n = n1 * n1
    rng = np.random.default_rng(57)
    src = 0.01 * rng.standard_normal(n)
    target = 1.0 + 0.01 * rng.standard_normal(n)
    H0 = np.ones(n)
    g = _ctx(L, 9, (n1, n1, 1), "fp64", k=0.02)
    q = torch.tensor(src, dtype=torch.float64, device=g.device, requires_grad=True)
    J = tracking_objective(q, g, H0, target, T, every, interval=interval, recompute=recompute)
    J.backward()
    _, sh = L.relaxation_rates(g.params)
    o = oracle.Sim(9, n1, n1, s_h=sh, u0=(0.03, 0.0, 0.0), src=src)
    o.init(H0)
    Jo, go = o.gradient_source_tracking(target, T, every)
    assert float(J.detach()) == pytest.approx(Jo, rel=1e-12)
    assert rel_l2(q.grad.cpu().numpy(), go) < 1e-11


def test_tracking_gradient_with_walls_matches_oracle(L, oracle):
    """The same objective (every 3 steps over 13, one target per time) on the
    walled box against the oracle's dense reverse sweep."""
    import torch
    from paper_2203_01316_amd import workloads as W
    from paper_2203_01316_amd.adjoint import tracking_objective
    T, every = 13, 3
    dims, flags, q, groups, u = _walls(W, "walled")
    n = int(np.prod(dims))
    rng = np.random.default_rng(58)
    src = 0.01 * rng.standard_normal(n)
    targets = [1.0 + 0.01 * rng.standard_normal(n) for _ in range(T // every)]
    H0 = 1.0 + 0.1 * rng.uniform(size=n)
    g = L.LBM(9, *dims, storage="fp64", k=0.02, with_source=True, u_mode=1, flags=flags, q=q, groups=groups)
    g.set_velocity(u)
    qt = torch.tensor(src, dtype=torch.float64, device=g.device, requires_grad=True)
    J = tracking_objective(qt, g, H0, targets, T, every, interval=4)
    J.backward()
    _, sh = L.relaxation_rates(g.params)
    o = oracle.Sim(9, *dims, s_h=sh, uvel=u, src=src, flags=flags, qlink=q, groups=groups)
    o.init(H0)
    # the oracle's sweep with one target per time, written out here
    seeds, Jo = {}, 0.0
    for t in range(1, T + 1):
        o.step(1)
        if t % every == 0:
            Jt, lam_t, dq_t = o.objective(targets[t // every - 1])
            Jo += Jt
            seeds[t] = (lam_t, dq_t)
    lam = np.zeros((9, n))
    go = np.zeros(n)
    for t in range(T - 1, -1, -1):
        lam = o.adjoint_step_dense(lam, go)
        if t in seeds:
            lam = lam + seeds[t][0]
            go += seeds[t][1]
    assert float(J.detach()) == pytest.approx(Jo, rel=1e-12)
    assert rel_l2(qt.grad.cpu().numpy(), go) < 1e-11


def test_walls_gradient_vs_central_differences(L):
    """Walled box with a disc and EQ nodes, 96 x 48, 300 steps: the FP32
    adjoint gradient (checkpoints every 17 steps) matches FP64 central
    differences (eps = 1e-3) of the GPU forward on 10 nodes (fluid nodes next
    to the walls and the disc, and EQ nodes) within 1e-4 relative L2."""
    import torch
    from paper_2203_01316_amd import workloads as W
    from paper_2203_01316_amd.adjoint import source_objective
    nx, ny, T = 96, 48, 300
    flags, q, groups, u = W.walled_box(nx, ny, 30.3, 22.6, 8.2)
    n = nx * ny
    rng = np.random.default_rng(54)
    src = 0.01 * rng.standard_normal(n)
    target = 1.0 + 0.01 * rng.standard_normal(n)
    H0 = np.ones(n)
    t = flags & 15
    near = np.nonzero((t == W.FLUID) & ((np.arange(n) // nx == 1) | (np.arange(n) // nx == ny - 2)))[0]
    nodes = list(rng.choice(near, 4, replace=False)) + list(rng.choice(np.nonzero(t == W.FLUID)[0], 4,
                                                                         replace=False))
    eqs = np.nonzero(t == W.EQ)[0]
    nodes += [int(eqs[0]), int(eqs[-1])]

    def ctx(storage):
        g = L.LBM(9, nx, ny, storage=storage, k=0.02, with_source=True, u_mode=1, flags=flags, q=q, groups=groups)
        g.set_velocity(f32(u) if storage == "fp32" else u)
        return g

    g32 = ctx("fp32")
    qt = torch.tensor(f32(src), dtype=torch.float32, device=g32.device, requires_grad=True)
    J = source_objective(qt, g32, H0, target, T, interval=17, recompute=True)
    J.backward()
    adj = qt.grad.double().cpu().numpy()[nodes]
    g64 = ctx("fp64")
    eps = 1e-3

    def J64(qv):
        g64.set_source(qv)
        g64.init(H0)
        g64.step(T)
        Jv, _, _ = g64.objective(target)
        return Jv

    fd = []
    for m in nodes:
        qp = src.copy()
        qp[m] += eps
        qm = src.copy()
        qm[m] -= eps
        fd.append((J64(qp) - J64(qm)) / (2 * eps))
    fd = np.array(fd)
    assert rel_l2(adj, fd) < 1e-4, (adj, fd)


def test_adjoint_rejects_flow(L):
    """The hydrodynamic lattice has no adjoint."""
    import torch
    lam = torch.zeros(9, 64, dtype=torch.float32, device="cuda:0")
    g = L.LBM(9, 8, 8, k=0.01, nu=0.02, with_ns=True)
    with pytest.raises(L.LBMError) as e:
        g.adjoint_step(lam, torch.empty_like(lam))
    assert e.value.status == L.EUNSUPPORTED
