"""Host-side checks of the C-ABI library (no GPU): every symbol declared in
include/lbm.h is exported, parameter validation, relaxation presets, and the
cut-link table built by the library's host code against the oracle's own
(bit-exact)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2203_01316_amd import lbm
    return lbm


def _declared():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L._lib, name), name
    assert set(L.EXPORTED) == set(names)


def test_version_and_workspace(L):
    assert "gfx950" in L.version()
    p = L.make_params(L.D2Q9, 64, 32, with_ns=True, storage="fp32", nu=0.01, k=0.02)
    n = L.workspace_bytes(p)
    # two lattices x two copies x 9 x 4 B per node, plus tables and scratch
    assert n >= 2 * 2 * 9 * 4 * 64 * 32
    p.nz = 2
    with pytest.raises(L.LBMError) as e:
        L.workspace_bytes(p)
    assert "nz" in str(e.value)


@pytest.mark.parametrize("kw,msg", [
    (dict(k=-0.1), "conductivity"),
    (dict(with_ns=True, nu=0.0), "viscosity"),
    (dict(storage=7), "storage"),
    (dict(lattice=15), "lattice"),
    (dict(stream=7), "stream mode"),
    (dict(nx=0), "nx, ny, nz"),
    (dict(cumulant_f=True), "cumulant f collision needs with_ns"),
    (dict(ny=-3), "nx, ny, nz"),
    (dict(with_source=True, with_ns=True, nu=0.1), "source"),
])
def test_param_validation(L, kw, msg):
    base = dict(lattice=L.D2Q9, nx=8, ny=8, k=0.01)
    base.update(kw)
    lat = base.pop("lattice")
    p = L.make_params(lat, base.pop("nx"), base.pop("ny"), **base)
    with pytest.raises(L.LBMError) as e:
        L.workspace_bytes(p)
    assert msg in str(e.value)


@pytest.mark.parametrize("Q", [9, 27])
def test_presets_match_oracle(L, oracle, Q):
    nz = 1 if Q == 9 else 4
    for rh, name in ((L.CM_SRT, "srt"), (L.CM_1ST, "1st"), (L.CM_TRT, "trt")):
        p = L.make_params(Q, 4, 4, nz, with_ns=True, nu=0.013, k=0.0021, relax_h=rh, relax_f="ns")
        sf, sh = L.relaxation_rates(p)
        np.testing.assert_array_equal(sh[:Q], oracle.preset(Q, name, oracle.s_main(0.0021))[:Q])
        np.testing.assert_array_equal(sf[:Q], oracle.preset(Q, "ns", oracle.s_main(0.013))[:Q])
        assert L.bulk_rate(p) == 1.0


def test_bulk_rate_choices(L):
    """s_bulk_f: 0 selects 1 for the hydrodynamic preset and no separate trace
    rate for the others; an explicit rate is kept; a custom f needs equal
    diagonal rates; rates outside (0, 2) are refused."""
    assert L.bulk_rate(L.make_params(9, 4, 4, with_ns=True, nu=0.01)) == 1.0
    assert L.bulk_rate(L.make_params(9, 4, 4, with_ns=True, nu=0.01, s_bulk_f=1.3)) == 1.3
    assert L.bulk_rate(L.make_params(9, 4, 4, with_ns=True, nu=0.01, relax_f="srt")) == 0.0
    assert L.bulk_rate(L.make_params(9, 4, 4, k=0.01)) == 0.0
    s = np.full(27, 1.2)
    assert L.bulk_rate(L.make_params(27, 4, 4, 4, with_ns=True, relax_f="custom", s_custom_f=s,
                                     s_bulk_f=0.8)) == 0.8
    s[8] = 1.3  # D3Q27 moment 020
    for bad in (dict(relax_f="custom", s_custom_f=s, s_bulk_f=0.8), dict(nu=0.01, s_bulk_f=2.0),
                dict(nu=0.01, s_bulk_f=-0.5)):
        with pytest.raises(L.LBMError) as e:
            L.relaxation_rates(L.make_params(27, 4, 4, 4, with_ns=True, **bad))
        assert e.value.status == L.EINVAL


def _random_geometry(rng, nx, ny, nz, Q):
    n = nx * ny * nz
    t = rng.choice([0, 0, 0, 0, 1, 1, 2, 3], size=n).astype(np.uint16)
    g = rng.integers(0, 3, size=n).astype(np.uint16)
    flags = t | (g << 4)
    q = rng.uniform(0.01, 1.0, size=(Q, n))
    return flags, q


@pytest.mark.parametrize("Q,dims", [(9, (13, 11, 1)), (27, (6, 5, 4))])
def test_link_table_bit_exact_vs_oracle(L, oracle, Q, dims):
    rng = np.random.default_rng(21)
    flags, q = _random_geometry(rng, *dims, Q)
    # an outlet needs a non-solid upstream node: clear those
    nx = dims[0]
    for n in np.nonzero((flags & 15) == 3)[0]:
        up = n - 1 if n % nx else n + nx - 1
        if flags[up] & 15 == 1:
            flags[n] = 0
    p = L.make_params(Q, *dims, k=0.01)
    mine = L.build_links(p, flags, q, n_groups=3)
    sim = oracle.Sim(Q, *dims, flags=flags, qlink=q, groups=[{}] * 3)
    ref = sim.links()
    assert len(mine) > 50
    assert mine.tobytes() == ref.tobytes()
    nl, ns = L.count_geometry(p, flags)
    assert nl == len(ref)
    assert ns == _expected_records(flags, ref, dims[0])


def _expected_records(flags, links, nx):
    """Boundary-node records: every non-solid node with cut links, EQ nodes
    with cut links, and outlet nodes unless the bulk threads take them (no cut
    links on the node or on its upstream node n - 1, which is FLUID, x != 0 and
    n % 64 != 0).  EQ nodes without cut links and of a group below 252 are
    bulk-handled."""
    t = flags & 15
    has_link = np.zeros(len(flags), bool)
    has_link[links["node"]] = True
    count = 0
    for n in range(len(flags)):
        if t[n] == 1:
            continue
        if t[n] == 3:
            bulk = (not has_link[n] and n % nx != 0 and n % 64 != 0 and t[n - 1] == 0
                    and not has_link[n - 1])
            count += not bulk
        elif has_link[n] or (t[n] == 2 and (flags[n] >> 4) > 251):
            count += 1
    return count


def test_bulk_handled_boundary_nodes(L, oracle):
    """A lattice with every inlet/outlet configuration: records exist exactly
    for the nodes the rule above lists (the outlet at y = 32 starts a 64-node
    group, the outlet at x = 0 has a periodic upstream, four outlets have an
    upstream node with cut links, corner EQ nodes have cut links, one EQ node
    is in group 252)."""
    from paper_2203_01316_amd import workloads as W
    flags, q, groups, _, _, _ = W.boundary_mix()
    nx, ny = 33, 40
    assert (32 + nx * 32) % 64 == 0
    p = L.make_params(L.D2Q9, nx, ny, k=0.01, with_ns=True, nu=0.04)
    links = oracle.Sim(9, nx, ny, flags=flags, qlink=q, groups=groups).links()
    nl, ns = L.count_geometry(p, flags)
    assert nl == len(links)
    t = (flags & 15).reshape(ny, nx)
    g = (flags >> 4).reshape(ny, nx)
    exp = _expected_records(flags, links, nx)
    # the group-252 EQ node has no cut link but keeps a record
    assert t[12, 0] == L.EQ and g[12, 0] == 252
    assert ns == exp
    n_out = int(np.count_nonzero(t == L.OUTLET))
    assert n_out == ny - 3 + 1


def test_aa_layout_geometry(L, oracle):
    """In the in-place (AA) layout an outlet's thread also updates its upstream
    node, which must then be a plain fluid node; the cut links are unchanged."""
    flags, q, groups, u = __import__("paper_2203_01316_amd.workloads", fromlist=["x"]).channel(64, 24, 20, 12, 4.0)
    pab = L.make_params(L.D2Q9, 64, 24, k=0.01)
    paa = L.make_params(L.D2Q9, 64, 24, k=0.01, stream=L.STREAM_AA)
    assert L.build_links(paa, flags, q, 3).tobytes() == L.build_links(pab, flags, q, 3).tobytes()
    nl_ab, ns_ab = L.count_geometry(pab, flags)
    nl_aa, ns_aa = L.count_geometry(paa, flags)
    assert nl_aa == nl_ab and ns_aa <= ns_ab
    bad = flags.copy().reshape(24, 64)
    bad[5, 62] = L.EQ  # upstream of the outlet node (63, 5)
    with pytest.raises(L.LBMError) as e:
        L.build_links(paa, bad.reshape(-1), q, 3)
    assert "AA layout" in str(e.value) and "outlet node" in str(e.value)
    L.build_links(pab, bad.reshape(-1), q, 3)  # fine for two arrays


def test_geometry_errors_name_the_index(L):
    p = L.make_params(L.D2Q9, 8, 8, k=0.01)
    flags = np.zeros(64, np.uint16)
    flags[9] = 1 | (2 << 4)  # solid, group 2
    q = np.full((9, 64), 0.5)
    with pytest.raises(L.LBMError) as e:
        L.build_links(p, flags, q, n_groups=2)
    assert "node 9" in str(e.value) and "group 2" in str(e.value)
    q[1, 8] = 0.0  # link (node 8, dir 1) points into node 9
    with pytest.raises(L.LBMError) as e:
        L.build_links(p, flags, q, n_groups=3)
    assert "node 8" in str(e.value) and "q =" in str(e.value)
    flags[:] = 0
    flags[0] = 3
    flags[7] = 1  # upstream of the outlet at x = 0 wraps to x = 7
    with pytest.raises(L.LBMError) as e:
        L.build_links(p, flags, None, n_groups=1)
    assert "outlet node 0" in str(e.value)
