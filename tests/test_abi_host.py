"""Host-side checks that need no GPU: the C ABI library loads and exports every
entry point that include/pbh.h declares; the IC generators behave."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2110_11658_amd import _lib, ic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pbh.h")).read()
    return sorted(set(re.findall(r"\b(pbh_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2110_11658_amd import build
        build.build()
    lib = ctypes.CDLL(_lib.LIB_PATH)
    declared = _declared()
    assert len(declared) >= 14
    for name in declared:
        assert hasattr(lib, name), name
    assert set(_lib.EXPORTS) == set(declared)


def test_status_strings_without_gpu():
    lib = _lib.load()
    assert lib.pbh_status_string(0) == b"ok"
    assert lib.pbh_status_string(5) == b"neighbour capacity too small"
    # no device in this container: create must fail cleanly, not crash
    ctx = ctypes.c_void_p()
    import torch
    if not torch.cuda.is_available():
        st = lib.pbh_create(0, None, ctypes.byref(ctx))
        assert st != 0 and not ctx.value


def test_plummer_generator_units_and_determinism():
    a = ic.plummer(20000, seed=5)
    b = ic.plummer(20000, seed=5)
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.vel, b.vel)
    assert a.pos.flags.c_contiguous and a.pos.dtype == np.float64
    assert np.allclose((a.mass[:, None] * a.pos).sum(0), 0, atol=1e-14)
    # kinetic energy of Henon units: T = 1/4 (virial, E = -1/4)
    T = 0.5 * np.dot(a.mass, (a.vel**2).sum(1))
    assert T == pytest.approx(0.25, rel=0.03)
    r = np.linalg.norm(a.pos, axis=1)
    # half-mass radius of a Plummer sphere: a / sqrt(2^(2/3) - 1)
    rh = ic.PLUMMER_A_HENON / np.sqrt(2 ** (2 / 3) - 1)
    assert np.median(r) == pytest.approx(rh, rel=0.03)
    assert r.max() < 38.8 * ic.PLUMMER_A_HENON


def test_kroupa_moments():
    rng = np.random.default_rng(0)
    m = ic.kroupa_masses(rng, 400000, normalise=False)
    assert m.min() >= 0.08 and m.max() <= 100
    # closed-form moments of the two-segment power law
    m0, m1, m2 = 0.08, 0.5, 100.0
    k2 = m1 ** (2.3 - 1.3)
    n1 = (m1**-0.3 - m0**-0.3) / -0.3
    n2 = k2 * (m2**-1.3 - m1**-1.3) / -1.3
    mm1 = (m1**0.7 - m0**0.7) / 0.7
    mm2 = k2 * (m2**-0.3 - m1**-0.3) / -0.3
    assert np.mean(m < 0.5) == pytest.approx(n1 / (n1 + n2), abs=3e-3)
    assert m.mean() == pytest.approx((mm1 + mm2) / (n1 + n2), rel=0.02)
    assert ic.kroupa_masses(rng, 1000).sum() == pytest.approx(1.0)


def test_ensemble_layout():
    e = ic.ensemble(n_clusters=4, nmin=100, nmax=400)
    assert e.offsets[0] == 0 and e.offsets[-1] == e.mass.size
    assert np.all(np.diff(e.offsets) >= 100) and np.all(np.diff(e.offsets) <= 400)
    for k in range(4):
        s = slice(e.offsets[k], e.offsets[k + 1])
        assert e.mass[s].sum() == pytest.approx(1.0)
    assert np.allclose(e.r_in, 0.1 * e.r_out)


def test_r_out_rule():
    r = ic.r_out_for_nbar(1 << 20, 64.0)
    assert r == pytest.approx(0.04077, rel=1e-3)
    assert ic.NBAR_COEF * (1 << 20) * r**3 / ic.PLUMMER_A_HENON**3 == pytest.approx(64.0)
