"""GPU parity of the HIP path against the CPU oracle (through the C ABI).

Tolerances:
  * tree structure, keys, sort order, node moments: bit-exact (the same
    FP64 operations in the same order, no FMA, on both sides);
  * FP64 walk vs the oracle tree walk (same tree, groups and opening rule):
    1e-6 relative per particle (only the summation order differs);
  * theta = 0 vs direct summation: 1e-12 (FP64) -- the tree reduces to the
    direct sum (Section 2.4);
  * mixed walk vs FP64 direct summation at theta = 0.5: median 1e-3;
  * neighbour lists: identical sets.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2110_11658_amd import ic

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0) if torch.cuda.is_available() else None


def _pbh(**kw):
    from paper_2110_11658_amd.api import Pbh
    return Pbh(0, **kw)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _rel(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def _sets_equal(g_off, g_idx, o_off, o_idx):
    assert np.array_equal(g_off, o_off)
    for i in range(g_off.size - 1):
        got = np.sort(g_idx[g_off[i]:g_off[i + 1]])
        if not np.array_equal(got, o_idx[o_off[i]:o_off[i + 1]]):
            raise AssertionError(f"neighbour set of {i} differs")


def _run(p, c, r_in, r_out, theta, eps, nbr=True):
    p.build(_t(c.pos), _t(c.mass))
    acc, pot, off, idx = p.force(r_in, r_out, theta, eps, neighbours=nbr)
    torch.cuda.synchronize()
    out = [acc.cpu().numpy(), pot.cpu().numpy()]
    if nbr:
        out += [off.cpu().numpy(), idx.cpu().numpy()]
    return out


# ---------------------------------------------------------------- tree stages
@pytest.mark.parametrize("n,n_leaf,seed", [(4096, 16, 1), (3001, 8, 2), (700, 1, 3)])
def test_tree_bit_exact(n, n_leaf, seed):
    print(f"tree n={n} n_leaf={n_leaf}", flush=True)
    c = ic.plummer(n, seed=seed, masses="kroupa")
    p = _pbh(leaf_size=n_leaf, n_crit=64)
    p.build(_t(c.pos), _t(c.mass))
    order, keys, ni, nd = p.debug_tree()
    okeys = oracle.keys(c.pos, 21)
    oorder, oi, od = oracle.tree_nodes(c.pos, c.mass, n_leaf=n_leaf, D=21)
    assert np.array_equal(order.astype(np.int64), oorder)
    assert np.array_equal(keys, okeys[oorder])
    assert ni.shape == oi.shape
    assert np.array_equal(ni, oi)
    assert np.array_equal(nd, od)   # identical FP64 operation order
    st = p.stats()
    assert st["n_nodes"] == oi.shape[0] and st["n_leaves"] == int((oi[:, 2] == 0).sum())
    assert st["error_flags"] == 0
    gb, gc, gbox = p.debug_groups()
    ob, oc = oracle.groups(c.pos, c.mass, n_leaf=n_leaf, n_crit=64)
    assert np.array_equal(gb.astype(np.int64), ob) and np.array_equal(gc.astype(np.int64), oc)
    xs = c.pos[oorder]
    for g in range(0, gb.size, 5):
        pts = xs[gb[g]:gb[g] + gc[g]]
        assert np.array_equal(gbox[g, :3], pts.min(0)) and np.array_equal(gbox[g, 3:], pts.max(0))
    assert st["n_groups"] == gb.size


def test_sort_ties_and_duplicates():
    rng = np.random.default_rng(4)
    base = rng.random((300, 3))
    pos = np.concatenate([base, base, base[::-1], np.zeros((40, 3))])
    mass = np.full(pos.shape[0], 1.0 / pos.shape[0])
    p = _pbh(leaf_size=4)
    p.build(_t(pos), _t(mass))
    order, keys, ni, nd = p.debug_tree()
    okeys = oracle.keys(pos, 21)
    assert np.array_equal(order, np.argsort(okeys, kind="stable"))
    oorder, oi, od = oracle.tree_nodes(pos, mass, n_leaf=4, D=21)
    assert np.array_equal(ni, oi) and np.array_equal(nd, od)


# ---------------------------------------------------------------- forces
CASES = [  # n, seed, masses, eps, r_out, theta, n_leaf, n_crit
    (4096, 1, "equal", 1e-4, 0.05, 0.5, 16, 64),
    (5000, 6, "kroupa", 1e-5, 0.15, 0.5, 16, 64),
    (2077, 7, "kroupa", 0.0, 0.2, 0.7, 8, 32),
    (1500, 8, "two", 1e-3, 0.3, 0.3, 4, 17),
]


@pytest.mark.parametrize("n,seed,masses,eps,r_out,theta,n_leaf,n_crit", CASES)
def test_fp64_walk_matches_oracle_tree(n, seed, masses, eps, r_out, theta, n_leaf, n_crit):
    print(f"fp64 walk n={n} theta={theta}", flush=True)
    c = ic.plummer(n, seed=seed, masses=masses)
    r_in = 0.1 * r_out
    p = _pbh(leaf_size=n_leaf, n_crit=n_crit, prec="fp64")
    acc, pot, off, idx = _run(p, c, r_in, r_out, theta, eps)
    oa, op, ost = oracle.tree(c.pos, c.mass, r_in, r_out, theta, eps, n_leaf=n_leaf, n_crit=n_crit)
    assert _rel(acc, oa).max() < 1e-6
    assert (np.abs(pot - op) / np.abs(op)).max() < 1e-6
    st = p.stats()
    assert (st["n_pn"], st["n_pp_far"], st["n_pp_near"]) == (ost["pn"], ost["pp_far"], ost["pp_near"])
    o_off, o_idx = oracle.nbr_cells(c.pos, r_out)
    _sets_equal(off, idx, o_off, o_idx)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_theta0_equals_direct(prec):
    c = ic.plummer(3000, seed=9, masses="kroupa")
    r_out, eps = 0.1, 1e-4
    p = _pbh(prec=prec)
    acc, pot = _run(p, c, 0.1 * r_out, r_out, 0.0, eps, nbr=False)
    oa, op = oracle.direct(c.pos, c.mass, 0.1 * r_out, r_out, eps)
    tol = 1e-12 if prec == "fp64" else 2e-5
    assert _rel(acc, oa).max() < tol
    assert (np.abs(pot - op) / np.abs(op)).max() < tol
    st = p.stats()
    assert st["n_pn"] == 0 and st["n_pp_far"] + st["n_pp_near"] == c.n * c.n


@pytest.mark.parametrize("n,seed,r_out", [(4096, 1, 0.05), (20000, 10, 0.1)])
def test_mixed_walk_accuracy(n, seed, r_out):
    c = ic.plummer(n, seed=seed, masses="kroupa")
    r_in, eps = 0.1 * r_out, 1e-5
    oa, op = oracle.direct(c.pos, c.mass, r_in, r_out, eps)
    errs = []
    for theta in (0.7, 0.5, 0.3):
        p = _pbh(prec="mixed")
        acc, pot, off, idx = _run(p, c, r_in, r_out, theta, eps)
        e = _rel(acc, oa)
        errs.append(np.median(e))
        if theta == 0.5:
            assert np.median(e) < 1e-3
            assert np.median(np.abs(pot - op) / np.abs(op)) < 1e-3
        o_off, o_idx = oracle.nbr_cells(c.pos, r_out)
        _sets_equal(off, idx, o_off, o_idx)
    assert errs[0] > errs[1] > errs[2]


def test_mixed_matches_fp64_walk_closely():
    c = ic.plummer(8192, seed=12, masses="kroupa")
    args = (0.008, 0.08, 0.5, 1e-5)
    a64, p64 = _run(_pbh(prec="fp64"), c, *args, nbr=False)
    a32, p32 = _run(_pbh(prec="mixed"), c, *args, nbr=False)
    # same interactions; only FP32 rounding differs
    assert np.median(_rel(a32, a64)) < 1e-5
    assert np.median(np.abs(p32 - p64) / np.abs(p64)) < 1e-5


# ---------------------------------------------------------------- edge cases
def test_single_particle_and_pairs():
    p = _pbh()
    c = ic.plummer(1, seed=1)
    acc, pot, off, idx = _run(p, c, 0.01, 0.1, 0.5, 0.0)
    assert np.all(acc == 0) and np.all(pot == 0) and list(off) == [0, 0]
    pos = np.array([[0.0, 0.0, 0.0], [0.055, 0.0, 0.0]])
    mass = np.array([0.3, 0.7])
    p.build(_t(pos), _t(mass))
    for prec in ("fp64", "mixed"):
        p.set_params(prec=prec)
        p.build(_t(pos), _t(mass))
        a, ph, off, idx = p.force(0.01, 0.1, 0.5, 0.0)
        oa, op = oracle.direct(pos, mass, 0.01, 0.1, 0.0)
        tol = 1e-13 if prec == "fp64" else 1e-6
        assert np.allclose(a.cpu().numpy(), oa, rtol=tol, atol=0)
        assert np.allclose(ph.cpu().numpy(), op, rtol=tol, atol=0)
        assert list(off.cpu().numpy()) == [0, 1, 2] and sorted(idx.cpu().numpy()) == [0, 1]


@pytest.mark.parametrize("r_in,r_out", [(0.0, 0.0), (0.05, 0.05), (0.0, 0.08)])
def test_degenerate_radii(r_in, r_out):
    c = ic.plummer(2500, seed=13)
    eps = 1e-3
    oa, op = oracle.direct(c.pos, c.mass, r_in, r_out, eps)
    for prec, tol in (("fp64", 1e-12), ("mixed", 2e-5)):
        p = _pbh(prec=prec)
        acc, pot, off, idx = _run(p, c, r_in, r_out, 0.0, eps)
        assert _rel(acc, oa).max() < tol
        assert (np.abs(pot - op) / np.abs(op)).max() < tol
        o_off, o_idx = oracle.nbr_cells(c.pos, r_out)
        _sets_equal(off, idx, o_off, o_idx)


def test_coincident_particles():
    rng = np.random.default_rng(3)
    base = rng.normal(size=(200, 3)) * 0.1
    pos = np.concatenate([base, base[:50]])
    mass = np.full(pos.shape[0], 1.0 / pos.shape[0])
    r_in, r_out = 0.01, 0.05
    oa, op = oracle.direct(pos, mass, r_in, r_out, 0.0)
    p = _pbh(prec="fp64", leaf_size=2)
    acc, pot, off, idx = _run(p, type("C", (), {"pos": pos, "mass": mass})(), r_in, r_out, 0.0, 0.0)
    assert np.allclose(acc, oa, rtol=1e-12, atol=1e-12 * np.abs(oa).max())
    assert np.allclose(pot, op, rtol=1e-12)
    o_off, o_idx = oracle.nbr_cells(pos, r_out)
    _sets_equal(off, idx, o_off, o_idx)


def test_lattice_ties():
    g = np.arange(6, dtype=float) * 0.1
    pos = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1).T.copy()
    mass = np.full(pos.shape[0], 1.0 / pos.shape[0])
    p = _pbh(leaf_size=4, n_crit=16)
    for r_out in (0.1, 0.1000001, 0.15):
        p.build(_t(pos), _t(mass))
        _, _, off, idx = p.force(0.0, r_out, 0.5, 0.0)
        o_off, o_idx = oracle.nbr_brute(pos, r_out)
        _sets_equal(off.cpu().numpy(), idx.cpu().numpy(), o_off, o_idx)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_neighbour_routes(prec):
    # Lists reach the CSR by two routes: rows the walk staged (whole rows, or
    # per-copy sub-rows of split groups) and the fill traversal (groups with a
    # list longer than its row). A clump where every member has ~1500
    # neighbours overflows the rows, a sparse halo gives split groups, and the
    # Plummer body is staged; every route must give the oracle's sets.
    rng = np.random.default_rng(11)
    r_out = 0.05
    body = ic.plummer(6000, seed=12).pos
    clump = rng.uniform(-1.0, 1.0, size=(1500, 3)) * (r_out / 4) + 0.3
    halo = rng.normal(size=(300, 3)) * 5.0
    pos = np.ascontiguousarray(np.concatenate([body, clump, halo]))
    mass = np.full(pos.shape[0], 1.0 / pos.shape[0])
    print(f"routes n={pos.shape[0]} {prec}", flush=True)
    p = _pbh(leaf_size=8, n_crit=64, prec=prec)
    _, _, off, idx = _run(p, type("C", (), {"pos": pos, "mass": mass})(), 0.1 * r_out, r_out, 0.5, 0.0)
    o_off, o_idx = oracle.nbr_brute(pos, r_out)
    assert o_off[-1] > 1500 * 1499
    _sets_equal(off, idx, o_off, o_idx)
    _, nb = p.debug_wave_log()
    filled = int(nb[:, 0].sum())
    n_groups = p.stats()["n_groups"]
    assert 0 < filled < n_groups, (filled, n_groups)


@pytest.mark.parametrize("spread", [1.0, 300.0])
def test_neighbour_boundary_pairs(spread):
    # Pairs separated by r_out (1 + u 1e-6): the mixed walk decides most pairs
    # in FP32 and those within a rounding band of r_out in FP64; the sets must
    # equal the FP64 definition's. spread = 300 puts the pairs in sparse,
    # large groups (box half-side > 64 r_out), which always take the FP64 test.
    rng = np.random.default_rng(21)
    r_out = 0.01
    m = 1500
    centres = rng.uniform(-1.0, 1.0, size=(m, 3)) * spread * r_out * 20
    d = rng.normal(size=(m, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    sep = r_out * (1.0 + rng.uniform(-1.0, 1.0, size=m) * 1e-6)
    pos = np.ascontiguousarray(np.concatenate([centres, centres + d * sep[:, None]]))
    mass = np.full(pos.shape[0], 1.0 / pos.shape[0])
    print(f"boundary pairs spread={spread}", flush=True)
    p = _pbh(prec="mixed", leaf_size=8, n_crit=64)
    _, _, off, idx = _run(p, type("C", (), {"pos": pos, "mass": mass})(), 0.1 * r_out, r_out, 0.5, 0.0)
    o_off, o_idx = oracle.nbr_brute(pos, r_out)
    assert o_off[-1] > 0
    _sets_equal(off, idx, o_off, o_idx)


# ---------------------------------------------------------------- error paths
def test_error_paths():
    from paper_2110_11658_amd._lib import (PBH_E_ARG, PBH_E_NBR_OVERFLOW, PBH_E_NONFINITE,
                                           PBH_E_STATE, PbhError)
    p = _pbh()
    c = ic.plummer(1000, seed=2)
    pos = c.pos.copy()
    with pytest.raises(PbhError) as e:
        p.force(0.01, 0.1, 0.5, 0.0)
    assert e.value.status == PBH_E_STATE
    pos[17, 1] = np.nan
    with pytest.raises(PbhError) as e:
        p.build(_t(pos), _t(c.mass))
    assert e.value.status == PBH_E_NONFINITE
    m = c.mass.copy()
    m[3] = np.inf
    with pytest.raises(PbhError) as e:
        p.build(_t(c.pos), _t(m))
    assert e.value.status == PBH_E_NONFINITE
    p.build(_t(c.pos), _t(c.mass))
    for bad in ((0.2, 0.1, 0.5, 0.0), (-0.1, 0.1, 0.5, 0.0), (0.01, 0.1, -1.0, 0.0),
                (0.01, 0.1, 0.5, -1e-3), (0.01, float("nan"), 0.5, 0.0)):
        with pytest.raises(PbhError) as e:
            p.force(*bad)
        assert e.value.status == PBH_E_ARG
    with pytest.raises(PbhError) as e:
        p.force(0.02, 0.2, 0.5, 0.0, nbr_cap=10)   # binding retries once with more room
        raise PbhError(PBH_E_NBR_OVERFLOW, "")
    # direct ABI: overflow reports the needed size, forces still valid
    import ctypes as C
    from paper_2110_11658_amd.api import _ptr, _stream
    acc = torch.empty((c.n, 3), dtype=torch.float64, device=DEV)
    pot = torch.empty(c.n, dtype=torch.float64, device=DEV)
    off = torch.empty(c.n + 1, dtype=torch.int64, device=DEV)
    idx = torch.empty(10, dtype=torch.int32, device=DEV)
    tot = C.c_int64(0)
    bp, bm = p._built
    st = p.L.pbh_force(p.ctx, _ptr(bp), _ptr(bm), 0.02, 0.2, 0.5, 0.0, _ptr(acc), _ptr(pot), _ptr(off),
                       _ptr(idx), 10, C.byref(tot), _stream())
    assert st == PBH_E_NBR_OVERFLOW and tot.value > 10
    o_off, _ = oracle.nbr_cells(c.pos, 0.2)
    assert tot.value == o_off[-1]
    assert np.array_equal(off.cpu().numpy(), o_off)
    oa, _ = oracle.direct(c.pos, c.mass, 0.02, 0.2, 0.0)
    assert np.median(_rel(acc.cpu().numpy(), oa)) < 1e-3
    # overflow without a host wait: entries beyond the capacity are dropped and flagged
    st = p.L.pbh_force(p.ctx, _ptr(bp), _ptr(bm), 0.02, 0.2, 0.5, 0.0, _ptr(acc), _ptr(pot), _ptr(off),
                       _ptr(idx), 10, None, _stream())
    assert st == 0 and p.stats()["error_flags"] & 1


def test_force_needs_the_built_arrays():
    # The REGF-style contract: pbh_force takes the particles again; they must be
    # the arrays of the last build, unchanged (PBH_E_STATE otherwise)
    import ctypes as C

    from paper_2110_11658_amd._lib import PBH_E_STATE
    from paper_2110_11658_amd.api import _ptr, _stream
    c = ic.plummer(3000, seed=21)
    p = _pbh()
    pos, mass = _t(c.pos), _t(c.mass)
    acc = torch.empty((c.n, 3), dtype=torch.float64, device=DEV)
    pot = torch.empty(c.n, dtype=torch.float64, device=DEV)
    off = torch.empty(c.n + 1, dtype=torch.int64, device=DEV)
    idx = torch.empty(200000, dtype=torch.int32, device=DEV)
    tot = C.c_int64(0)

    def force(pp, mm, total=True):
        return p.L.pbh_force(p.ctx, _ptr(pp), _ptr(mm), 0.01, 0.1, 0.5, 0.0, _ptr(acc), _ptr(pot),
                             _ptr(off), _ptr(idx), idx.shape[0], C.byref(tot) if total else None,
                             _stream())
    assert force(pos, mass) == PBH_E_STATE            # no build yet
    p.build(pos, mass)
    assert force(pos, mass) == 0
    a0 = acc.clone()
    copy = pos.clone()                                 # same values, other array
    assert force(copy, mass) == PBH_E_STATE
    assert force(pos, mass.clone()) == PBH_E_STATE
    assert b"last build" in p.L.pbh_last_error(p.ctx)
    # moved in place since the build: detected by the walk
    pos[123, 0] += 1e-9
    assert force(pos, mass) == PBH_E_STATE
    assert b"changed" in p.L.pbh_last_error(p.ctx)
    assert force(pos, mass, total=False) == 0         # no wait: reported in the flags
    assert p.stats()["error_flags"] & 32
    mass[7] *= 2.0
    pos[123, 0] -= 1e-9                                # (may not restore the bits exactly)
    p.build(pos, mass)
    assert force(pos, mass) == 0 and not (p.stats()["error_flags"] & 32)
    assert not torch.equal(acc, a0)                   # mass 7 doubled since the first call
    # the core quantities take the built arrays too
    from paper_2110_11658_amd._lib import PbhError
    sample = torch.arange(0, c.n, 3, dtype=torch.int32, device=DEV)
    with pytest.raises(PbhError) as e:
        p.core(copy, mass, sample)
    assert e.value.status == PBH_E_STATE
    p.core(pos, mass, sample)


def test_deterministic_repeat():
    c = ic.plummer(30000, seed=14, masses="kroupa")
    p = _pbh()
    r1 = _run(p, c, 0.01, 0.1, 0.5, 1e-5)
    r2 = _run(p, c, 0.01, 0.1, 0.5, 1e-5)
    for a, b in zip(r1, r2):
        assert np.array_equal(a, b)


def test_context_reuse_across_inputs():
    # One context serves inputs of different sizes and different buffers of
    # the same size (its captured build sequence and level-sized launches are
    # keyed on them): every result equals that of a fresh context.
    cs = [ic.plummer(20000, seed=31, masses="kroupa"), ic.plummer(3000, seed=32),
          ic.plummer(20000, seed=33, masses="kroupa"), ic.plummer(20000, seed=31, masses="kroupa")]
    args = (0.005, 0.05, 0.5, 1e-5)
    p = _pbh()
    for k, c in enumerate(cs):
        print(f"reuse input {k} n={c.mass.size}", flush=True)
        got = _run(p, c, *args)
        ref = _run(_pbh(), c, *args)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)


# ---------------------------------------------------------------- batched
def test_batched_equals_per_cluster():
    e = ic.ensemble(n_clusters=5, nmin=300, nmax=5000, nbar=16)
    theta, eps = 0.5, 1e-5
    from paper_2110_11658_amd.api import Pbh
    pb = Pbh(0, key_bits=19, n_crit=64)   # same groups in both builds whatever the total size
    pb.build_batched(e.offsets, _t(e.pos), _t(e.mass))
    acc, pot, off, idx = pb.force_batched(e.r_in, e.r_out, theta, eps)
    torch.cuda.synchronize()
    acc, pot, off, idx = (t.cpu().numpy() for t in (acc, pot, off, idx))
    assert pb.stats()["n_clusters"] == 5
    ps = Pbh(0, key_bits=19, n_crit=64)
    for k in range(5):
        s = slice(e.offsets[k], e.offsets[k + 1])
        ps.build(_t(e.pos[s]), _t(e.mass[s]))
        a, ph, o, ix = ps.force(e.r_in[k], e.r_out[k], theta, eps)
        assert np.array_equal(acc[s], a.cpu().numpy())
        assert np.array_equal(pot[s], ph.cpu().numpy())
        o = o.cpu().numpy()
        ix = ix.cpu().numpy()
        b0 = e.offsets[k]
        assert np.array_equal(off[s.start:s.stop + 1] - off[s.start], o)
        assert np.array_equal(idx[off[s.start]:off[s.stop]], ix + b0)


def test_batched_many_clusters_equals_per_cluster():
    # 300 clusters: the group size limit then comes from one histogram copy per
    # cluster (fewer clusters spread each over several copies); each cluster's
    # groups, forces and lists must still equal those of a build of its own
    # (9 cluster bits leave 18 key bits per axis, used by both builds)
    e = ic.ensemble(n_clusters=300, seed0=7100, nmin=60, nmax=600, nbar=8)
    theta, eps = 0.5, 1e-5
    from paper_2110_11658_amd.api import Pbh
    pb = Pbh(0, key_bits=18, n_crit=64)
    pb.build_batched(e.offsets, _t(e.pos), _t(e.mass))
    acc, pot, off, idx = pb.force_batched(e.r_in, e.r_out, theta, eps)
    torch.cuda.synchronize()
    acc, pot, off, idx = (t.cpu().numpy() for t in (acc, pot, off, idx))
    assert pb.stats()["n_clusters"] == 300
    ps = Pbh(0, key_bits=18, n_crit=64)
    print("batched 300 clusters", flush=True)
    for k in range(300):
        s = slice(e.offsets[k], e.offsets[k + 1])
        ps.build(_t(e.pos[s]), _t(e.mass[s]))
        a, ph, o, ix = ps.force(e.r_in[k], e.r_out[k], theta, eps)
        assert np.array_equal(acc[s], a.cpu().numpy()), k
        assert np.array_equal(pot[s], ph.cpu().numpy()), k
        o = o.cpu().numpy()
        assert np.array_equal(off[s.start:s.stop + 1] - off[s.start], o), k
        assert np.array_equal(idx[off[s.start]:off[s.stop]], ix.cpu().numpy() + e.offsets[k]), k


# ---------------------------------------------------------------- leapfrog
def test_kdk_graph_equals_eager_and_oracle():
    c = ic.plummer(4096, seed=15, masses="kroupa")
    r_out = ic.r_out_for_nbar(c.n, 16.0)
    r_in, theta, eps, dt, steps = 0.1 * r_out, 0.5, 1e-4, 1.0 / 256, 6
    res = {}
    for mode in ("graph", "eager"):
        p = _pbh(prec="fp64", leaf_size=16, n_crit=64)   # the oracle walk's defaults
        pos, vel, mass = _t(c.pos), _t(c.vel), _t(c.mass)
        en = p.kdk(pos, vel, mass, dt, steps, r_in, r_out, theta, eps, graph=(mode == "graph"))
        torch.cuda.synchronize()
        res[mode] = (pos.cpu().numpy(), vel.cpu().numpy(), en.cpu().numpy())
    for a, b in zip(res["graph"], res["eager"]):
        assert np.array_equal(a, b)
    # oracle leapfrog with the CPU tree walk
    x, v = c.pos.copy(), c.vel.copy()
    a, ph, _ = oracle.tree(x, c.mass, r_in, r_out, theta, eps)
    energies = [0.5 * np.dot(c.mass, (v * v).sum(1)) + 0.5 * np.dot(c.mass, ph)]
    for _ in range(steps):
        v += 0.5 * dt * a
        x += dt * v
        a, ph, _ = oracle.tree(x, c.mass, r_in, r_out, theta, eps)
        v += 0.5 * dt * a
        energies.append(0.5 * np.dot(c.mass, (v * v).sum(1)) + 0.5 * np.dot(c.mass, ph))
    gx, gv, ge = res["graph"]
    assert np.max(np.abs(gx - x)) < 1e-9
    assert np.allclose(ge, energies, rtol=1e-9)


# ---------------------------------------------------------------- autotuner
def test_autotune_choices_valid_and_cached(tmp_path, monkeypatch):
    from paper_2110_11658_amd import autotune
    monkeypatch.setenv("PBH_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    c = ic.plummer(20000, seed=21, masses="kroupa")
    p = _pbh()
    cands, tiles = ((8, 32), (16, 64)), (64, 128)
    r = autotune.tune(p, _t(c.pos), _t(c.mass), 0.01, 0.1, 0.5, 1e-5, candidates=cands, tiles=tiles,
                      reps=1)
    assert (r["leaf_size"], r["n_crit"]) in cands and r["walk_tile"] in tiles and not r["cached"]
    # two (n_leaf, n_crit) pairs at the first tile, both timed again, then the
    # other tile at the better pair
    assert len(r["table"]) == 5 and all(t["ms"] > 0 for t in r["table"])
    got = p.params()
    assert (got["leaf_size"], got["n_crit"], got["walk_tile"]) == (r["leaf_size"], r["n_crit"],
                                                                   r["walk_tile"])
    r2 = autotune.tune(p, _t(c.pos), _t(c.mass), 0.01, 0.1, 0.5, 1e-5, candidates=cands, tiles=tiles,
                       reps=1)
    assert r2["cached"] and (r2["leaf_size"], r2["n_crit"], r2["walk_tile"]) == (
        r["leaf_size"], r["n_crit"], r["walk_tile"])
    # every candidate gives the same neighbour sets
    o_off, o_idx = oracle.nbr_cells(c.pos, 0.1)
    for t in r["table"]:
        p.set_params(leaf_size=t["leaf_size"], n_crit=t["n_crit"], walk_tile=t["walk_tile"])
        acc, pot, off, idx = _run(p, c, 0.01, 0.1, 0.5, 1e-5)
        _sets_equal(off, idx, o_off, o_idx)


def test_walk_clock():
    # pbh_walk_clock: PBH_E_STATE before any walk; afterwards the engine clock
    # of the last walk from its workgroups' cycle and tick counts, within the
    # range an MI355X engine clock can take (its peak is 2400 MHz).
    import ctypes as C
    from paper_2110_11658_amd._lib import PBH_E_STATE
    c = ic.plummer(20000, seed=5)
    p = _pbh(leaf_size=8, n_crit=64)
    v = C.c_double(0.0)
    assert p.L.pbh_walk_clock(p.ctx, C.byref(v)) == PBH_E_STATE
    print("walk clock n=20000", flush=True)
    _run(p, c, 0.004, 0.04, 0.5, 1e-4)
    mhz = p.walk_clock_mhz()
    print("walk clock MHz", mhz, flush=True)
    assert 300.0 < mhz < 2600.0, mhz
