"""GPU parity of the Hermite integration of F_I (pbh_hermite) and of the P3T
loop (pbh_p3t), through the C ABI, against the CPU oracle (Section 2.2).

Both sides take the same block-step decisions from FP64 values that differ
only in summation order (the GPU sums F_I over neighbour lists, the oracle
over all pairs), so the block schedules are compared exactly (block count,
particle steps, deepest level) and positions and velocities to 1e-10 of
their scale after one regular step (3 steps for the P3T loop: rounding
differences grow with each step but stay far below the integration error).
"""
import math

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


def _setup(n, seed, nbar):
    c = ic.plummer(n, seed=seed, masses="kroupa")
    r_out = ic.r_out_for_nbar(n, nbar)
    return c, 0.1 * r_out, r_out


def test_hermite_matches_oracle():
    # a regular step of 1/16 (dt_max = 1/64): eq. dt puts a fifth of the
    # particles below dt_max and the deepest at level 8
    c, r_in, r_out = _setup(512, 91, 16.0)
    eps, T, eta = 1e-4, 1.0 / 16, 0.02
    r_buff = 3.0 * np.linalg.norm(c.vel, axis=1).max() * T
    p = _pbh(prec="fp64")
    pos, vel, mass = _t(c.pos), _t(c.vel), _t(c.mass)
    p.build(pos, mass)
    fr, _, off, idx = p.force(r_in, r_out, 0.0, eps, r_buff=r_buff)
    st = p.hermite(pos, vel, mass, fr, r_in, r_out, eps, off, idx, T, eta)
    ofr, _ = oracle.direct(c.pos, c.mass, r_in, r_out, eps)
    ox, ov, ost = oracle.hermite(c.pos, c.vel, c.mass, r_in, r_out, eps, T, eta=eta, fr=ofr)
    assert st == ost and st["kmax"] >= 4
    gx, gv = pos.cpu().numpy(), vel.cpu().numpy()
    assert np.abs(gx - ox).max() <= 1e-10 * np.abs(ox).max()
    assert np.abs(gv - ov).max() <= 1e-10 * np.abs(ov).max()


def _first_step_ticks(want, dtmax, kmax=40):
    # dt_max / 2^k not above the wanted step, k <= 40, as ticks of dt_max / 2^40
    out = np.empty(want.size, dtype=np.int64)
    for i, w in enumerate(want):
        d, k = dtmax, 0
        while d > w and k < kmax:
            d *= 0.5
            k += 1
        out[i] = 1 << (kmax - k)
    return out


@pytest.mark.parametrize("n,seed,nbar,eps", [(2048, 95, 16.0, 1e-4), (1024, 96, 6.0, 0.0)])
def test_first_steps_are_eq_dt(n, seed, nbar, eps):
    # Section 2.1 (after eq. dt): every particle starts the regular step on the
    # step eq. dt asks for with the computed second and third derivatives of
    # F_I. The GPU's first step of each particle equals the oracle's, exactly;
    # particles with no pair inside r_out start on dt_max.
    c, r_in, r_out = _setup(n, seed, nbar)
    T, eta = 1.0 / 16, 0.02
    r_buff = 3.0 * np.linalg.norm(c.vel, axis=1).max() * T
    p = _pbh(prec="fp64")
    pos, vel, mass = _t(c.pos), _t(c.vel), _t(c.mass)
    p.build(pos, mass)
    fr, _, off, idx = p.force(r_in, r_out, 0.0, eps, r_buff=r_buff)
    p.hermite(pos, vel, mass, fr, r_in, r_out, eps, off, idx, T, eta)
    ticks = p.debug_herm_first_steps()
    ofr, _ = oracle.direct(c.pos, c.mass, r_in, r_out, eps)
    _, _, ost = oracle.hermite(c.pos, c.vel, c.mass, r_in, r_out, eps, T, eta=eta, fr=ofr, want=True)
    ref = _first_step_ticks(ost["want_start"], T / 4)
    assert np.array_equal(ticks, ref)
    assert (ref < (1 << 40)).sum() > n // 4      # many particles start below dt_max
    o_off, _ = oracle.nbr_brute(c.pos, r_out)
    lonely = np.diff(o_off) == 0
    if lonely.any():
        assert np.all(ticks[lonely] == 1 << 40)


def test_p3t_matches_oracle():
    c, r_in, r_out = _setup(384, 92, 12.0)
    eps, T, eta, steps = 1e-4, 1.0 / 256, 0.02, 3
    r_buff = 3.0 * np.linalg.norm(c.vel, axis=1).max() * T
    p = _pbh(prec="fp64")
    pos, vel, mass = _t(c.pos), _t(c.vel), _t(c.mass)
    e, st = p.p3t(pos, vel, mass, r_in, r_out, r_buff, 0.0, eps, T, eta, steps)
    ox, ov, oe = oracle.p3t(c.pos, c.vel, c.mass, r_in, r_out, eps, T, eta=eta, steps=steps)
    assert st["steps"] > steps * c.n
    gx, gv = pos.cpu().numpy(), vel.cpu().numpy()
    assert np.abs(gx - ox).max() <= 1e-10 * np.abs(ox).max()
    assert np.abs(gv - ov).max() <= 1e-10 * np.abs(ov).max()
    assert np.allclose(e.cpu().numpy(), oe, rtol=1e-11, atol=0)


@pytest.mark.parametrize("n,seed,T", [(2048, 96, 1.0 / 32), (4096, 97, 1.0 / 16)])
def test_hermite_larger_n(n, seed, T):
    # thousands of particles: blocks from every particle active (the front
    # predicts them all at once) down to a few particles of the deepest level
    # (lane groups per list); the schedule and the states equal the oracle's
    print(f"hermite n={n}", flush=True)
    c, r_in, r_out = _setup(n, seed, 16.0)
    eps, eta = 1e-4, 0.02
    r_buff = 3.0 * np.linalg.norm(c.vel, axis=1).max() * T
    p = _pbh(prec="fp64")
    pos, vel, mass = _t(c.pos), _t(c.vel), _t(c.mass)
    p.build(pos, mass)
    fr, _, off, idx = p.force(r_in, r_out, 0.0, eps, r_buff=r_buff)
    st = p.hermite(pos, vel, mass, fr, r_in, r_out, eps, off, idx, T, eta)
    ofr, _ = oracle.direct(c.pos, c.mass, r_in, r_out, eps)
    ox, ov, ost = oracle.hermite(c.pos, c.vel, c.mass, r_in, r_out, eps, T, eta=eta, fr=ofr)
    assert st == ost and st["steps"] > 2 * n and st["kmax"] >= 4
    gx, gv = pos.cpu().numpy(), vel.cpu().numpy()
    assert np.abs(gx - ox).max() <= 1e-10 * np.abs(ox).max()
    assert np.abs(gv - ov).max() <= 1e-10 * np.abs(ov).max()


def test_p3t_larger_n():
    print("p3t n=1536", flush=True)
    c, r_in, r_out = _setup(1536, 98, 12.0)
    eps, T, eta, steps = 1e-4, 1.0 / 256, 0.02, 2
    r_buff = 3.0 * np.linalg.norm(c.vel, axis=1).max() * T
    p = _pbh(prec="fp64")
    pos, vel, mass = _t(c.pos), _t(c.vel), _t(c.mass)
    e, st = p.p3t(pos, vel, mass, r_in, r_out, r_buff, 0.0, eps, T, eta, steps)
    ox, ov, oe = oracle.p3t(c.pos, c.vel, c.mass, r_in, r_out, eps, T, eta=eta, steps=steps)
    gx, gv = pos.cpu().numpy(), vel.cpu().numpy()
    assert np.abs(gx - ox).max() <= 1e-10 * np.abs(ox).max()
    assert np.abs(gv - ov).max() <= 1e-10 * np.abs(ov).max()
    assert np.allclose(e.cpu().numpy(), oe, rtol=1e-11, atol=0)


def test_p3t_paper_parameters_16k():
    # 16384 particles with the paper's run parameters (tau rule: r_cut = 4 tau,
    # r_buff = 3 tau sigma, dt_reg the largest power of 1/2 not above tau,
    # eta = 0.02; Kroupa masses): two regular steps of the whole loop, FP64 and
    # theta = 0 on the GPU against the oracle loop (direct regular force)
    n = 16384
    print(f"p3t paper parameters n={n}", flush=True)
    c = ic.plummer(n, seed=99, masses="kroupa")
    pr = ic.paper_radii(n)
    r_out, r_buff, T = pr["r_cut"], pr["r_buff"], pr["dt_reg"]
    r_in, eps, eta, steps = 0.1 * r_out, 1e-5, 0.02, 2
    p = _pbh(prec="fp64")
    pos, vel, mass = _t(c.pos), _t(c.vel), _t(c.mass)
    e, st = p.p3t(pos, vel, mass, r_in, r_out, r_buff, 0.0, eps, T, eta, steps)
    ox, ov, oe = oracle.p3t(c.pos, c.vel, c.mass, r_in, r_out, eps, T, eta=eta, steps=steps)
    assert st["steps"] >= steps * 4 * n   # every particle takes at least dt_max = dt_reg / 4
    gx, gv = pos.cpu().numpy(), vel.cpu().numpy()
    assert np.abs(gx - ox).max() <= 1e-10 * np.abs(ox).max()
    assert np.abs(gv - ov).max() <= 1e-10 * np.abs(ov).max()
    assert np.allclose(e.cpu().numpy(), oe, rtol=1e-11, atol=0)


def test_hermite_kepler_order_on_gpu():
    # two bodies, all of the force irregular: the orbit closes after one period
    # with an error falling as eta^2 (4th order)
    m1, m2, ecc = 0.6, 0.4, 0.5
    M = m1 + m2
    rp = 1.0 - ecc
    vp = math.sqrt(M * (1.0 + ecc) / rp)
    pos0 = np.array([[-m2 / M * rp, 0.0, 0.0], [m1 / M * rp, 0.0, 0.0]])
    vel0 = np.array([[0.0, -m2 / M * vp, 0.0], [0.0, m1 / M * vp, 0.0]])
    mass = _t(np.array([m1, m2]))
    P = 2.0 * math.pi / math.sqrt(M)
    off = _t(np.array([0, 1, 2], dtype=np.int64))
    idx = _t(np.array([1, 0], dtype=np.int32))
    p = _pbh()
    errs = []
    for eta in (0.02, 0.02 / 16):
        pos, vel = _t(pos0), _t(vel0)
        p.hermite(pos, vel, mass, None, 100.0, 100.0, 0.0, off, idx, P, eta)
        x = pos.cpu().numpy()
        errs.append(np.linalg.norm((x[1] - x[0]) - (pos0[1] - pos0[0])))
    assert errs[1] < 1e-4 and errs[0] / errs[1] > 100.0


def test_p3t_mixed_tree_energy():
    # the production configuration: mixed precision, theta = 0.5, buffered
    # lists; the energy stays within the leapfrog error of the regular step
    c, r_in, r_out = _setup(20000, 93, 16.0)
    T = 1.0 / 512
    r_buff = 3.0 * np.linalg.norm(c.vel, axis=1).max() * T
    p = _pbh()
    pos, vel, mass = _t(c.pos), _t(c.vel), _t(c.mass)
    e, st = p.p3t(pos, vel, mass, r_in, r_out, r_buff, 0.5, 1e-4, T, 0.02, 4)
    e = e.cpu().numpy()
    assert np.all(np.isfinite(e)) and abs(e[-1] - e[0]) < 1e-5 * abs(e[0])
    assert st["blocks"] >= 16


def test_hermite_error_paths():
    from paper_2110_11658_amd._lib import PBH_E_ARG, PbhError
    c, r_in, r_out = _setup(64, 94, 8.0)
    p = _pbh()
    pos, vel, mass = _t(c.pos), _t(c.vel), _t(c.mass)
    off = _t(np.zeros(65, dtype=np.int64))
    idx = _t(np.zeros(1, dtype=np.int32))
    for bad in (0.0, -1.0, float("nan")):
        with pytest.raises(PbhError) as e:
            p.hermite(pos, vel, mass, None, r_in, r_out, 1e-4, off, idx, bad)
        assert e.value.status == PBH_E_ARG
    with pytest.raises(PbhError) as e:
        p.hermite(pos, vel, mass, None, r_in, r_out, 1e-4, off, idx, 0.01, eta=0.0)
    assert e.value.status == PBH_E_ARG
    # a list entry out of range is reported, never read
    off2 = _t(np.arange(65, dtype=np.int64))
    idx2 = _t(np.full(64, 1000, dtype=np.int32))
    with pytest.raises(PbhError) as e:
        p.hermite(pos, vel, mass, None, r_in, r_out, 1e-4, off2, idx2, 0.01)
    assert e.value.status == PBH_E_ARG
