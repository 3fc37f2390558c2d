"""One context across entry points: buffers of one entry point outlive
calls of the others (GPU, through the C ABI).

A leapfrog call that changes n re-allocates only its own buffers; the
irregular-force flag word and the Hermite state stay valid, so repeating
an irregular-force call and a Hermite integration afterwards gives the same
bits as the first time, and the Hermite batch graph is re-captured when n
changes and reused when nothing does.
"""
import numpy as np
import pytest
import torch

from paper_2110_11658_amd import ic

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0) if torch.cuda.is_available() else None


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _irr_and_hermite(p, c, r_in, r_out, eps, T):
    pos, vel, mass = _t(c.pos), _t(c.vel), _t(c.mass)
    p.build(pos, mass)
    fr, _, off, idx = p.force(r_in, r_out, 0.0, eps, r_buff=0.5 * r_out)
    acc, jerk, pot = p.irregular(pos, vel, mass, r_in, r_out, eps, off, idx)
    st = p.hermite(pos, vel, mass, fr, r_in, r_out, eps, off, idx, T)
    torch.cuda.synchronize()
    return [v.cpu().numpy() for v in (acc, jerk, pot, pos, vel)], st


def test_context_reuse_across_entry_points():
    from paper_2110_11658_amd.api import Pbh
    print("context reuse: irregular, hermite, kdk with another n, again", flush=True)
    c = ic.plummer(700, seed=93, masses="kroupa")
    r_out = ic.r_out_for_nbar(c.n, 12.0)
    r_in, eps, T = 0.1 * r_out, 1e-4, 1.0 / 256
    p = Pbh(0, prec="fp64")
    first, st1 = _irr_and_hermite(p, c, r_in, r_out, eps, T)
    c2 = ic.plummer(333, seed=94)
    p.kdk(_t(c2.pos), _t(c2.vel), _t(c2.mass), 1.0 / 512, 2, r_in, r_out, 0.5, eps)
    again, st2 = _irr_and_hermite(p, c, r_in, r_out, eps, T)
    assert st1 == st2
    for a, b in zip(first, again):
        assert np.array_equal(a, b)
    # a smaller Hermite problem on the same context (graph re-captured), then
    # the first one again (graph re-captured back)
    small, _ = _irr_and_hermite(p, ic.plummer(200, seed=95, masses="kroupa"), r_in, r_out, eps, T)
    assert all(np.all(np.isfinite(v)) for v in small)
    third, st3 = _irr_and_hermite(p, c, r_in, r_out, eps, T)
    assert st3 == st1
    for a, b in zip(first, third):
        assert np.array_equal(a, b)
    p.close()
