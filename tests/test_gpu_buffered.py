"""GPU parity of the buffered neighbour radius (pbh_force_buffered): lists of
every j != i with r_ij < r_out + r_buff (Section 2.3, R_buff; the run-parameter
rule r_buff = 3 tau sigma), through the C ABI, against the CPU oracle.

Tolerances as for the unbuffered path: neighbour sets identical (FP64
predicate without FMA on both sides); FP64 walk against the oracle tree walk
with the same near rule 1e-6 per particle and identical interaction counts;
mixed walk against FP64 direct summation median 1e-3.
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


def _np(t):
    return None if t is None else t.cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def _sets_equal(g_off, g_idx, o_off, o_idx):
    assert np.array_equal(g_off, o_off)
    for i in range(g_off.size - 1):
        got = np.sort(g_idx[g_off[i]:g_off[i + 1]])
        if not np.array_equal(got, o_idx[o_off[i]:o_off[i + 1]]):
            raise AssertionError(f"neighbour set of {i} differs")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n,buff", [(4096, 0.5), (6000, 1.5)])
def test_buffered_walk_and_lists(prec, n, buff):
    print(f"buffered n={n} r_buff={buff} r_out prec={prec}", flush=True)
    c = ic.plummer(n, seed=51, masses="kroupa")
    r_out = ic.r_out_for_nbar(n, 16.0)
    r_in, r_buff, eps, theta = 0.1 * r_out, buff * r_out, 1e-4, 0.5
    p = _pbh(leaf_size=8, n_crit=32, prec=prec)
    p.build(_t(c.pos), _t(c.mass))
    acc, pot, off, idx = [_np(v) for v in p.force(r_in, r_out, theta, eps, r_buff=r_buff)]
    o_off, o_idx = oracle.nbr_cells(c.pos, r_out + r_buff)
    _sets_equal(off, idx, o_off, o_idx)
    assert off[-1] > n   # the buffer is exercised
    oa, op, ost = oracle.tree(c.pos, c.mass, r_in, r_out, theta, eps, n_leaf=8, n_crit=32,
                              r_buff=r_buff)
    st = p.stats()
    assert (st["n_pn"], st["n_pp_far"], st["n_pp_near"]) == (ost["pn"], ost["pp_far"], ost["pp_near"])
    if prec == "fp64":
        assert _rel(acc, oa).max() < 1e-6
        assert (np.abs(pot - op) / np.abs(op)).max() < 1e-6
    else:
        ref, _ = oracle.direct(c.pos, c.mass, r_in, r_out, eps)
        assert np.median(_rel(acc, ref)) < 1e-3


def test_buffered_lists_survive_a_drift():
    # lists built with r_buff hold every pair inside r_out after each particle
    # moves by at most r_buff / 2; the irregular force from the old lists at
    # the new positions then equals the oracle's over all pairs
    n = 5000
    c = ic.plummer(n, seed=52, masses="kroupa")
    r_out = ic.r_out_for_nbar(n, 32.0)
    r_in, r_buff, eps = 0.1 * r_out, 0.4 * r_out, 1e-4
    p = _pbh()
    p.build(_t(c.pos), _t(c.mass))
    _, _, off, idx = p.force(r_in, r_out, 0.5, eps, r_buff=r_buff)
    vmax = np.linalg.norm(c.vel, axis=1).max()
    dt = 0.49 * r_buff / vmax
    moved = c.pos + dt * c.vel
    acc, jerk, pot = [_np(v) for v in p.irregular(_t(moved), _t(c.vel), _t(c.mass), r_in, r_out,
                                                  eps, off, idx)]
    oa, oj, opot, sc = oracle.irregular(moved, c.vel, c.mass, r_in, r_out, eps)
    assert np.all(np.linalg.norm(acc - oa, axis=1) <= 1e-12 * sc[:, 0])
    assert np.all(np.linalg.norm(jerk - oj, axis=1) <= 1e-12 * sc[:, 1])
    assert np.all(np.abs(pot - opot) <= 1e-12 * sc[:, 2])
    # without the buffer some pair inside r_out at the new positions is missed
    _, _, off0, idx0 = p.force(r_in, r_out, 0.5, eps)
    a0, _, _ = p.irregular(_t(moved), _t(c.vel), _t(c.mass), r_in, r_out, eps, off0, idx0)
    assert np.any(np.linalg.norm(_np(a0) - oa, axis=1) > 1e-9 * sc[:, 0])


def test_buffered_batched_per_cluster():
    ens = ic.ensemble(n_clusters=5, seed0=4200, nmin=800, nmax=4000, nbar=16.0)
    eps = 1e-4
    r_buff = 0.7 * ens.r_out
    p = _pbh(leaf_size=8, n_crit=32, prec="fp64")
    p.build_batched(ens.offsets, _t(ens.pos), _t(ens.mass))
    acc, _, off, idx = [_np(v) for v in p.force_batched(ens.r_in, ens.r_out, 0.5, eps,
                                                        r_buff=r_buff)]
    for k in range(ens.n_clusters):
        a, b = ens.offsets[k], ens.offsets[k + 1]
        o_off, o_idx = oracle.nbr_brute(ens.pos[a:b], ens.r_out[k] + r_buff[k])
        g_off = off[a:b + 1] - off[a]
        g_idx = idx[off[a]:off[b]] - a
        _sets_equal(g_off, g_idx, o_off, o_idx)
        oa, _, _ = oracle.tree(ens.pos[a:b], ens.mass[a:b], ens.r_in[k], ens.r_out[k], 0.5, eps,
                               n_leaf=8, n_crit=32, r_buff=r_buff[k])
        assert _rel(acc[a:b], oa).max() < 1e-6


def test_paper_rule_radii():
    # the paper's run parameters at N = 32k: r_cut = 4 tau, r_buff = 3 tau sigma
    n = 32768
    c = ic.plummer(n, seed=53)
    pr = ic.paper_radii(n)
    r_out, r_buff = pr["r_cut"], pr["r_buff"]
    p = _pbh()
    p.build(_t(c.pos), _t(c.mass))
    _, _, off, idx = [_np(v) for v in p.force(0.1 * r_out, r_out, 0.5, 1e-5, r_buff=r_buff)]
    o_off, o_idx = oracle.nbr_cells(c.pos, r_out + r_buff)
    _sets_equal(off, idx, o_off, o_idx)
    # mean count against the Plummer prediction for the list radius
    pred = ic.NBAR_COEF * n * (r_out + r_buff) ** 3 / ic.PLUMMER_A_HENON ** 3
    assert abs(off[-1] / n - pred) < 0.1 * pred


def test_buffered_rejects_bad_buffer():
    from paper_2110_11658_amd._lib import PBH_E_ARG, PbhError
    c = ic.plummer(100, seed=54)
    p = _pbh()
    p.build(_t(c.pos), _t(c.mass))
    for bad in (-0.01, float("nan"), float("inf")):
        with pytest.raises(PbhError) as e:
            p.force(0.01, 0.1, 0.5, 1e-4, r_buff=bad)
        assert e.value.status == PBH_E_ARG
