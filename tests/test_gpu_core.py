"""GPU parity of the core quantities (pbh_core, through the C ABI) against the
CPU oracle's brute-force 6-nearest-neighbour search.

* per-sample densities: bit-exact (identical FP64 distances without FMA,
  identical tie order, identical mass sum and formula);
* density centre, core radius, core density: 1e-12 relative (sums over the
  sample in a different order on each side);
* N_core: equal up to particles within rounding of the core sphere;
* r_half: one of the particle radii adjacent to the oracle's in distance
  order (the running mass sums differ in order);
* R_min, dT_min: 1e-12 relative given equal r_half.
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


def _check(pos, mass, smp, got_rho, got, eta=0.02, full=True):
    rho, ref = oracle.core(pos, mass, smp.astype(np.int64), eta=eta)
    assert np.array_equal(got_rho, rho)
    if not full:
        return
    assert np.allclose(got["center"], ref["center"], rtol=0, atol=1e-12 * max(1.0, np.abs(pos).max()))
    for k in ("rho_core", "r_core"):
        assert got[k] == pytest.approx(ref[k], rel=1e-12)
    d2 = ((pos - ref["center"]) ** 2).sum(1)
    band = int((np.abs(d2 - ref["r_core"] ** 2) <= 1e-10 * ref["r_core"] ** 2).sum())
    assert abs(got["n_core"] - ref["n_core"]) <= band
    r = np.sqrt(np.sort(d2))
    kk = int(np.searchsorted(r, ref["r_half"]))
    lo, hi = r[max(kk - 1, 0)], r[min(kk + 1, r.size - 1)]
    assert lo * (1 - 1e-12) <= got["r_half"] <= hi * (1 + 1e-12)
    if got["r_half"] == pytest.approx(ref["r_half"], rel=1e-12):
        assert got["r_min"] == pytest.approx(ref["r_min"], rel=1e-12)
        assert got["dt_min"] == pytest.approx(ref["dt_min"], rel=1e-12)


@pytest.mark.parametrize("n,masses,leaf,seed", [(20000, "kroupa", 8, 71), (5000, "equal", 16, 72),
                                                (777, "kroupa", 1, 73)])
def test_core_matches_oracle(n, masses, leaf, seed):
    print(f"core n={n} masses={masses} leaf={leaf}", flush=True)
    c = ic.plummer(n, seed=seed, masses=masses)
    smp = ic.core_sample(n, seed)
    p = _pbh(leaf_size=leaf)
    pos, mass = _t(c.pos), _t(c.mass)
    p.build(pos, mass)
    rho, got = p.core(pos, mass, _t(smp))
    _check(c.pos, c.mass, smp, rho.cpu().numpy(), got)


def test_core_ties_and_small_inputs():
    # a lattice: many exact distance ties (lower index first on both sides)
    g = np.arange(12.0)
    pos = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1).T.copy()
    rng = np.random.default_rng(74)
    perm = rng.permutation(pos.shape[0])
    pos = pos[perm].copy()
    mass = rng.uniform(0.5, 1.5, pos.shape[0])
    smp = np.arange(0, pos.shape[0], 5).astype(np.int32)
    p = _pbh(leaf_size=4)
    pos_d, mass_d = _t(pos), _t(mass)
    p.build(pos_d, mass_d)
    rho, got = p.core(pos_d, mass_d, _t(smp))
    _check(pos, mass, smp, rho.cpu().numpy(), got)
    # seven particles: each one's neighbours are all the others
    pos7 = rng.normal(size=(7, 3))
    m7 = np.ones(7)
    q = _pbh()
    pos7_d, m7_d = _t(pos7), _t(m7)
    q.build(pos7_d, m7_d)
    smp7 = np.arange(7, dtype=np.int32)
    rho7, got7 = q.core(pos7_d, m7_d, _t(smp7))
    _check(pos7, m7, smp7, rho7.cpu().numpy(), got7)


def test_core_full_size_sampled():
    # the 2^20 Plummer/Kroupa workload with the paper's sample size
    # (sqrt(5000 N) = 72 407 particles); the oracle's O(S N) search checks 512
    c, w = ic.workload("plummer1m_kroupa")
    print(f"core full size n={c.n}", flush=True)
    smp = ic.core_sample(c.n, 75)
    p = _pbh()
    pos, mass = _t(c.pos), _t(c.mass)
    p.build(pos, mass)
    rho, got = p.core(pos, mass, _t(smp))
    rho = rho.cpu().numpy()
    sel = np.random.default_rng(76).choice(smp.size, 512, replace=False)
    _check(c.pos, c.mass, smp[sel], rho[sel], got, full=False)
    a = ic.PLUMMER_A_HENON
    assert got["r_core"] == pytest.approx(np.sqrt(0.3) * a, rel=0.07)
    assert np.linalg.norm(got["center"]) < 0.06 * a


def test_core_error_paths():
    from paper_2110_11658_amd._lib import PBH_E_ARG, PBH_E_STATE, PbhError
    c = ic.plummer(500, seed=77)
    pos, mass = _t(c.pos), _t(c.mass)
    p = _pbh()
    with pytest.raises(PbhError) as e:   # no build
        p.core(pos, mass, _t(np.arange(10, dtype=np.int32)))
    assert e.value.status == PBH_E_STATE
    p.build(pos, mass)
    with pytest.raises(PbhError) as e:
        p.core(pos, mass, _t(np.array([1, 600], dtype=np.int32)))
    assert e.value.status == PBH_E_ARG and "sample" in str(e.value)
    with pytest.raises(PbhError) as e:
        p.core(pos, mass, _t(np.arange(10, dtype=np.int32)), eta=0.0)
    assert e.value.status == PBH_E_ARG
    q = _pbh()
    q.build(_t(c.pos[:5]), _t(c.mass[:5]))
    with pytest.raises(PbhError) as e:
        q.core(_t(c.pos[:5]), _t(c.mass[:5]), _t(np.arange(3, dtype=np.int32)))
    assert e.value.status == PBH_E_ARG
    b = _pbh()
    b.build_batched([0, 250, 500], pos, mass)
    with pytest.raises(PbhError) as e:
        b.core(pos, mass, _t(np.arange(10, dtype=np.int32)))
    assert e.value.status == PBH_E_STATE
