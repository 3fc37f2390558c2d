"""The block schedule of the Hermite integration, on the CPU.

With block steps dt_i = 2^(K - k_i) ticks (level k_i), each chosen as the
largest such step not above a wanted value that divides the block time, and
never more than twice the old step (Section 2.2; eq. dt and its rounding),
the next block time min(tau_i + dt_i) is the first multiple of the smallest
occupied step after the current time, and the active particles are exactly
the levels k >= K - ctz(t_next). The GPU schedule is built on that rule;
these checks compare it with the plain minimum over random step choices
(small K so that runs end quickly), and check the bounds on level changes
that the bucket moves rely on.
"""
import random

K = 8


def _block_step(want_level, tau):
    t = 1 << (K - want_level)
    if tau:
        t = min(t, tau & -tau)   # the largest power of two dividing tau
    return t


def _level(t):
    return K - (t.bit_length() - 1)


def _by_levels(dt, tcur):
    kmax = max(_level(d) for d in dt)
    sh = K - kmax
    tn = ((tcur >> sh) + 1) << sh
    tz = (tn & -tn).bit_length() - 1
    ks = 0 if tz >= K else K - tz
    return tn, ks


def test_level_rule_equals_minimum():
    for trial in range(200):
        rnd = random.Random(trial)
        n = rnd.randint(1, 40)
        tend = 1 << (K + 2)
        tau = [0] * n
        dt = [_block_step(rnd.randint(0, K), 0) for _ in range(n)]
        tcur = 0
        while tcur < tend:
            tn = min(tau[i] + dt[i] for i in range(n))
            act = [i for i in range(n) if tau[i] + dt[i] == tn]
            tn2, ks = _by_levels(dt, tcur)
            assert tn2 == tn
            assert act == [i for i in range(n) if _level(dt[i]) >= ks]
            for i in act:
                old = _level(dt[i])
                want = max(0, min(K, old + rnd.choice([-3, -1, 0, 0, 1, 2, 3])))
                want = max(want, old - 1)   # the new step is at most twice the old one
                tau[i] = tn
                dt[i] = _block_step(want, tn)
                assert _level(dt[i]) >= ks - 1   # moves land in buckets >= k* - 1
                assert tn % dt[i] == 0
            tcur = tn
        assert tcur == tend   # the last block lands exactly on the end of the step


def test_single_level_is_uniform_stepping():
    # every particle on level k: blocks every 2^(K-k) ticks, all active
    for k in range(K + 1):
        dt = [1 << (K - k)] * 5
        t = 0
        for _ in range(4):
            tn, ks = _by_levels(dt, t)
            assert tn == t + (1 << (K - k)) and ks <= k
            t = tn
