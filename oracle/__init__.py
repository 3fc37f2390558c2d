"""CPU FP64 oracle for the P3T distant-force path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product library never calls it, and the two share no
code: this side is plain C (``pbh_oracle.c``, built with ``-ffp-contract=off``)
driven through ctypes.

Functions follow Arnold, Baumgardt & Wang (2021), Section 2.1 (the P3T force
split, eq. fi and the changeover function eq. duncan) and Section 2.4 (the
Barnes-Hut tree with opening angle theta). See ``pbh_oracle.c`` for the exact
definitions, including the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pbh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = C.c_double
_i64 = C.c_int64
_p = C.c_void_p


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.orc_W.restype = _d
        L.orc_W.argtypes = [_d, _d, _d]
        L.orc_phiR.restype = _d
        L.orc_phiR.argtypes = [_d, _d, _d]
        L.orc_phiR_coeffs.argtypes = [_d, _d, _p, _p]
        L.orc_direct.argtypes = [_i64, _p, _p, _d, _d, _d, _i64, _p, _p, _p]
        L.orc_full_direct.argtypes = [_i64, _p, _p, _d, _p, _p]
        L.orc_irregular.argtypes = [_i64, _p, _p, _p, _d, _d, _d, _i64, _p, _p, _p, _p, _p]
        L.orc_core.argtypes = [_i64, _p, _p, _i64, _p, _d, _p, _p]
        L.orc_irr_derivs.argtypes = [_i64, _p, _p, _p, _p, _p, _d, _d, _d, _i64, _p, _p, _p]
        L.orc_hermite.argtypes = [_i64, _p, _p, _p, _p, _d, _d, _d, _d, _d, _p, _p]
        L.orc_p3t.argtypes = [_i64, _p, _p, _p, _d, _d, _d, _d, _d, C.c_int, _p]
        L.orc_knn6.argtypes = [_i64, _p, _i64, _p, _p, _p]
        L.orc_nbr_brute.restype = _i64
        L.orc_nbr_brute.argtypes = [_i64, _p, _d, _p, _p, _i64]
        L.orc_nbr_cells.restype = _i64
        L.orc_nbr_cells.argtypes = [_i64, _p, _d, _p, _p, _i64]
        L.orc_keys.argtypes = [_i64, _p, C.c_int, _p]
        L.orc_tree.argtypes = [_i64, _p, _p, _d, _d, _d, _d, _d, C.c_int, C.c_int, C.c_int, _p, _p, _p]
        L.orc_tree_nodes.restype = _i64
        L.orc_tree_nodes.argtypes = [_i64, _p, _p, C.c_int, C.c_int, _i64, _p, _p, _p]
        L.orc_groups.restype = _i64
        L.orc_groups.argtypes = [_i64, _p, _p, C.c_int, C.c_int, C.c_int, _i64, _p, _p]
        L.orc_group_limit.restype = _d
        L.orc_group_limit.argtypes = [_i64, _p, _p, C.c_int, C.c_int, C.c_int]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def W(s: float, r_in: float, r_out: float) -> float:
    """Changeover weight W = 1 - K of eq. duncan (Section 2.1)."""
    return lib().orc_W(float(s), float(r_in), float(r_out))


def phiR(s: float, r_in: float, r_out: float) -> float:
    """Regular potential: dPhi_R/ds = W(s)/s^2, Phi_R(s) = -1/s for s >= r_out."""
    return lib().orc_phiR(float(s), float(r_in), float(r_out))


def phiR_coeffs(r_in: float, r_out: float):
    d = np.zeros(8)
    g1 = np.zeros(1)
    lib().orc_phiR_coeffs(float(r_in), float(r_out), _ptr(d), _ptr(g1))
    return d, float(g1[0])


def direct(pos, mass, r_in, r_out, eps, targets=None):
    """O(N^2) regular acceleration and potential (eq. fi with F_R = total - F_I).

    Returns (acc [n_t,3], pot [n_t]) for all particles or the given targets.
    """
    pos = _f64(pos)
    n = pos.shape[0]
    mass = _f64(mass, (n,))
    if targets is None:
        nt = n
        tgt = None
    else:
        tgt = np.ascontiguousarray(targets, dtype=np.int64)
        nt = tgt.size
    acc = np.zeros((nt, 3))
    pot = np.zeros(nt)
    lib().orc_direct(n, _ptr(pos), _ptr(mass), float(r_in), float(r_out), float(eps),
                     nt, None if tgt is None else _ptr(tgt), _ptr(acc), _ptr(pot))
    return acc, pot


def full_direct(pos, mass, eps):
    """Plain softened gravity (whole force, no changeover)."""
    pos = _f64(pos)
    n = pos.shape[0]
    mass = _f64(mass, (n,))
    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    lib().orc_full_direct(n, _ptr(pos), _ptr(mass), float(eps), _ptr(acc), _ptr(pot))
    return acc, pot


def irregular(pos, vel, mass, r_in, r_out, eps, targets=None):
    """O(N^2) irregular force F_I (eq. fi), its time derivative (eq. fidot,
    read as the term-by-term derivative of eq. fi) and the irregular
    potential Phi_I = -1/s - Phi_R(s), summed over every j != i.

    Returns (acc [n_t,3], jerk [n_t,3], pot [n_t], scale [n_t,3]); scale holds
    per-target magnitude sums (acceleration, jerk, potential) over the pairs
    inside r_out, for error bounds.
    """
    pos = _f64(pos)
    n = pos.shape[0]
    vel = _f64(vel, (n, 3))
    mass = _f64(mass, (n,))
    if targets is None:
        nt = n
        tgt = None
    else:
        tgt = np.ascontiguousarray(targets, dtype=np.int64)
        nt = tgt.size
    acc = np.zeros((nt, 3))
    jerk = np.zeros((nt, 3))
    pot = np.zeros(nt)
    scale = np.zeros((nt, 3))
    lib().orc_irregular(n, _ptr(pos), _ptr(vel), _ptr(mass), float(r_in), float(r_out), float(eps),
                        nt, None if tgt is None else _ptr(tgt), _ptr(acc), _ptr(jerk), _ptr(pot),
                        _ptr(scale))
    return acc, jerk, pot, scale


CORE_KEYS = ("center", "rho_core", "r_core", "n_core", "r_half", "r_min", "dt_min")


def core(pos, mass, sample, eta=0.02):
    """Core quantities from the 6 nearest neighbours of a particle sample
    (brute force): per-sample densities rho [n_s] and a dict with the density
    centre, core density, core radius, core count, half-mass radius about the
    density centre, and the regularisation parameters R_min, dT_min."""
    pos = _f64(pos)
    n = pos.shape[0]
    mass = _f64(mass, (n,))
    smp = np.ascontiguousarray(sample, dtype=np.int64)
    rho = np.zeros(smp.size)
    out = np.zeros(9)
    lib().orc_core(n, _ptr(pos), _ptr(mass), smp.size, _ptr(smp), float(eta), _ptr(rho), _ptr(out))
    res = {"center": out[:3].copy(), "rho_core": out[3], "r_core": out[4], "n_core": int(out[5]),
           "r_half": out[6], "r_min": out[7], "dt_min": out[8]}
    return rho, res


def knn6(pos, sample):
    """(d2 [n_s,6] ascending, idx [n_s,6]): 6 nearest neighbours by brute force."""
    pos = _f64(pos)
    smp = np.ascontiguousarray(sample, dtype=np.int64)
    d2 = np.zeros((smp.size, 6))
    idx = np.zeros((smp.size, 6), dtype=np.int64)
    lib().orc_knn6(pos.shape[0], _ptr(pos), smp.size, _ptr(smp), _ptr(d2), _ptr(idx))
    return d2, idx


def irr_derivs(pos, vel, acc, jrk, mass, r_in, r_out, eps, targets=None):
    """Second and third time derivatives of F_I (eq. fi) along the motion on
    which every particle has position pos, velocity vel, acceleration acc and
    its derivative jrk (all [n,3]); sums over every j != i with s < r_out.
    Returns (f2 [n_t,3], f3 [n_t,3])."""
    pos = _f64(pos)
    n = pos.shape[0]
    vel = _f64(vel, (n, 3))
    acc = _f64(acc, (n, 3))
    jrk = _f64(jrk, (n, 3))
    mass = _f64(mass, (n,))
    if targets is None:
        nt, tgt = n, None
    else:
        tgt = np.ascontiguousarray(targets, dtype=np.int64)
        nt = tgt.size
    f2 = np.zeros((nt, 3))
    f3 = np.zeros((nt, 3))
    lib().orc_irr_derivs(n, _ptr(pos), _ptr(vel), _ptr(acc), _ptr(jrk), _ptr(mass), float(r_in),
                         float(r_out), float(eps), nt, None if tgt is None else _ptr(tgt), _ptr(f2),
                         _ptr(f3))
    return f2, f3


def hermite(pos, vel, mass, r_in, r_out, eps, T, eta=0.02, fr=None, want=False):
    """Hermite integration of F_I with block time steps over one regular step
    T (Section 2.2). Returns (x, v, stats) with stats = dict(blocks, steps, kmax).
    With want=True stats also holds, per particle, the step eq. dt asked for at
    the start ("want_start"), at the last corrector step ("want_last", before
    the doubling cap and block rounding), that last step's length ("d_last")
    and the length of the step before it ("d_prev", 0 if none this call)."""
    x = _f64(pos).copy()
    n = x.shape[0]
    v = _f64(vel, (n, 3)).copy()
    mass = _f64(mass, (n,))
    f = None if fr is None else _f64(fr, (n, 3))
    st = np.zeros(3, dtype=np.int64)
    w = np.zeros(4 * n) if want else None
    lib().orc_hermite(n, _ptr(x), _ptr(v), _ptr(mass), None if f is None else _ptr(f), float(r_in),
                      float(r_out), float(eps), float(T), float(eta), _ptr(st),
                      None if w is None else _ptr(w))
    out = {"blocks": int(st[0]), "steps": int(st[1]), "kmax": int(st[2])}
    if want:
        out.update(want_start=w[:n].copy(), want_last=w[n:2 * n].copy(), d_last=w[2 * n:3 * n].copy(),
                   d_prev=w[3 * n:].copy())
    return x, v, out


def p3t(pos, vel, mass, r_in, r_out, eps, T, eta=0.02, steps=1):
    """P3T loop (Section 2.2): kick, Hermite F_I over T, kick, with the direct
    regular force. Returns (x, v, energy [steps+1])."""
    x = _f64(pos).copy()
    n = x.shape[0]
    v = _f64(vel, (n, 3)).copy()
    mass = _f64(mass, (n,))
    e = np.zeros(steps + 1)
    lib().orc_p3t(n, _ptr(x), _ptr(v), _ptr(mass), float(r_in), float(r_out), float(eps), float(T),
                  float(eta), int(steps), _ptr(e))
    return x, v, e


def _nbr(fn, pos, r_out):
    pos = _f64(pos)
    n = pos.shape[0]
    off = np.zeros(n + 1, dtype=np.int64)
    total = fn(n, _ptr(pos), float(r_out), _ptr(off), None, 0)
    idx = np.zeros(max(total, 1), dtype=np.int32)
    fn(n, _ptr(pos), float(r_out), _ptr(off), _ptr(idx), total)
    return off, idx[:total]


def nbr_brute(pos, r_out):
    """Neighbour CSR by brute force: j != i with (dx*dx + dy*dy) + dz*dz < r_out*r_out."""
    return _nbr(lib().orc_nbr_brute, pos, r_out)


def nbr_cells(pos, r_out):
    """Neighbour CSR from a cell list with cells of side r_out (lists ascending)."""
    return _nbr(lib().orc_nbr_cells, pos, r_out)


def keys(pos, D: int = 21) -> np.ndarray:
    """Morton keys of one cluster, D bits per dimension."""
    pos = _f64(pos)
    k = np.zeros(pos.shape[0], dtype=np.uint64)
    lib().orc_keys(pos.shape[0], _ptr(pos), int(D), _ptr(k))
    return k


def tree(pos, mass, r_in, r_out, theta, eps, n_leaf=16, n_crit=64, D=21, r_buff=0.0):
    """CPU Barnes-Hut walk with the same tree, group and opening rules as the GPU.

    Nodes closer than the list radius r_out + r_buff to a group are opened to
    particle pairs. Returns (acc, pot, stats) with stats = dict(nodes, leaves,
    groups, pn, pp_far, pp_near).
    """
    pos = _f64(pos)
    n = pos.shape[0]
    mass = _f64(mass, (n,))
    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    st = np.zeros(6, dtype=np.int64)
    lib().orc_tree(n, _ptr(pos), _ptr(mass), float(r_in), float(r_out), float(r_buff), float(theta),
                   float(eps), int(n_leaf), int(n_crit), int(D), _ptr(acc), _ptr(pot), _ptr(st))
    names = ("nodes", "leaves", "groups", "pn", "pp_far", "pp_near")
    return acc, pot, dict(zip(names, (int(v) for v in st)))


def kdk(pos, vel, mass, r_in, r_out, theta, eps, dt, steps, n_leaf=16, n_crit=64):
    """Kick-drift-kick leapfrog under the regular force (Section 2.2, eq. kick
    and the loop after it), the force from the CPU tree walk (``tree``) after a
    full rebuild at every step:
        a = F_R(x); repeat: v += dt/2 a; x += dt v; a = F_R(x); v += dt/2 a.
    Returns (x, v, energy [steps+1]) with E = sum m v^2/2 + sum m Phi_R/2
    before the first step and after each."""
    x = _f64(pos).copy()
    n = x.shape[0]
    v = _f64(vel, (n, 3)).copy()
    mass = _f64(mass, (n,))

    def energy(ph):
        return 0.5 * np.dot(mass, (v * v).sum(1)) + 0.5 * np.dot(mass, ph)

    a, ph, _ = tree(x, mass, r_in, r_out, theta, eps, n_leaf=n_leaf, n_crit=n_crit)
    e = [energy(ph)]
    for _ in range(steps):
        v += (0.5 * dt) * a
        x += dt * v
        a, ph, _ = tree(x, mass, r_in, r_out, theta, eps, n_leaf=n_leaf, n_crit=n_crit)
        v += (0.5 * dt) * a
        e.append(energy(ph))
    return x, v, np.array(e)


def tree_nodes(pos, mass, n_leaf=16, D=21):
    """Octree export: (order, ints [nodes,4] = begin,count,nchild,level,
    doubles [nodes,16] = M, com[3], q[6] (xx,yy,zz,xy,xz,yz), lo[3], hi[3])."""
    pos = _f64(pos)
    n = pos.shape[0]
    mass = _f64(mass, (n,))
    order = np.zeros(n, dtype=np.int64)
    nn = lib().orc_tree_nodes(n, _ptr(pos), _ptr(mass), int(n_leaf), int(D), 0, _ptr(order), None, None)
    ib = np.zeros((nn, 4), dtype=np.int64)
    db = np.zeros((nn, 16))
    lib().orc_tree_nodes(n, _ptr(pos), _ptr(mass), int(n_leaf), int(D), nn, _ptr(order), _ptr(ib), _ptr(db))
    return order, ib, db


def groups(pos, mass, n_leaf=16, n_crit=64, D=21):
    """Walk groups: (begin [G], count [G]) in sorted-particle positions."""
    pos = _f64(pos)
    n = pos.shape[0]
    mass = _f64(mass, (n,))
    ng = lib().orc_groups(n, _ptr(pos), _ptr(mass), int(n_leaf), int(n_crit), int(D), 0, None, None)
    b = np.zeros(ng, dtype=np.int64)
    c = np.zeros(ng, dtype=np.int64)
    lib().orc_groups(n, _ptr(pos), _ptr(mass), int(n_leaf), int(n_crit), int(D), ng, _ptr(b), _ptr(c))
    return b, c


def group_limit(pos, mass, n_leaf=16, n_crit=64, D=21) -> float:
    """Size limit (largest box side) of the walk groups of one cluster."""
    pos = _f64(pos)
    n = pos.shape[0]
    mass = _f64(mass, (n,))
    return float(lib().orc_group_limit(n, _ptr(pos), _ptr(mass), int(n_leaf), int(n_crit), int(D)))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of later calls (timing only; results do not depend on it)."""
    lib().orc_set_num_threads(int(n))
