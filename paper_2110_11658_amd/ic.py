"""Seeded synthetic initial conditions for the distant-force path.

This module only draws inputs. It holds none of the force method's arithmetic,
so both the HIP path and the CPU oracle can be fed from it.

Everything is generated from ``numpy.random.default_rng(seed)`` (PCG64) with a
fixed draw order, so a (generator, seed, N) triple always gives the same arrays.

* Plummer spheres in Henon N-body units (G = M = 1, E = -1/4) with equal
  masses, as the paper's accuracy and performance runs use (Results,
  "Accuracy and Performance"). Radii follow the inverse cumulative mass
  profile of the Plummer sphere with the mass fraction capped at 0.999;
  speeds follow the isotropic Plummer distribution function by rejection
  sampling; the model is then rescaled from a = 1 to the Henon length unit
  a = 3*pi/16 and its centre of mass is moved to rest at the origin.
* Kroupa (2001) two-segment IMF between 0.08 and 100 (slopes -1.3 and -2.3,
  continuous at 0.5), normalised to total mass 1. Positions do not depend on
  mass.
* The two-component spectrum of the paper's core-collapse run (Results,
  "Core Collapse"): every tenth particle is ten times heavier.
* An ensemble of independent clusters with log-uniform sizes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

#: Plummer scale length in Henon units (E = -1/4 for M = G = 1).
PLUMMER_A_HENON = 3.0 * math.pi / 16.0
#: Mean neighbour count within radius r for a Plummer sphere:
#: n = NBAR_COEF * N * r^3 / a^3, with NBAR_COEF = (4 pi / 3) * 540 / 12288
#: (the integral of rho^2 over the Plummer sphere).
NBAR_COEF = (4.0 * math.pi / 3.0) * 540.0 / 12288.0
#: Largest enclosed-mass fraction drawn (truncates the halo at ~38.7 a).
PLUMMER_XMAX = 0.999

KROUPA_M = (0.08, 0.5, 100.0)
KROUPA_SLOPES = (1.3, 2.3)


def r_out_for_nbar(n: int, nbar: float, a: float = PLUMMER_A_HENON) -> float:
    """Radius whose sphere holds ``nbar`` neighbours on average in a Plummer model."""
    return a * (nbar / (NBAR_COEF * n)) ** (1.0 / 3.0)


def paper_radii(n: int) -> dict:
    """Run-parameter rule of the paper (Results, "Parameters").

    tau = (1/128) (N / 2^14)^(-1/3); r_cut = 4 tau; r_buff = 3 tau sigma with
    sigma = 1/sqrt(2); dt_reg = the largest power of 1/2 not above tau;
    dt_max = dt_reg / 4.
    """
    tau = (1.0 / 128.0) * (n / 2.0**14) ** (-1.0 / 3.0)
    sigma = 1.0 / math.sqrt(2.0)
    k = math.ceil(-math.log2(tau))
    dt_reg = 2.0 ** (-k)
    if dt_reg > tau:  # guard against log2 rounding
        dt_reg *= 0.5
    return {"tau": tau, "r_cut": 4.0 * tau, "r_buff": 3.0 * tau * sigma,
            "dt_reg": dt_reg, "dt_max": dt_reg / 4.0, "sigma": sigma}


def _plummer_unit(rng: np.random.Generator, n: int):
    """Plummer sphere with G = M = a = 1 (Aarseth, Henon & Wielen 1974 recipe)."""
    pos = np.empty((n, 3))
    vel = np.empty((n, 3))
    filled = 0
    while filled < n:
        k = n - filled
        x1 = rng.random(k)
        ok = (x1 > 0.0) & (x1 <= PLUMMER_XMAX)
        x1 = x1[ok]
        k = x1.size
        r = 1.0 / np.sqrt(x1 ** (-2.0 / 3.0) - 1.0)
        x2 = rng.random(k)
        x3 = rng.random(k)
        z = (1.0 - 2.0 * x2) * r
        rho = np.sqrt(np.maximum(r * r - z * z, 0.0))
        phi = 2.0 * math.pi * x3
        pos[filled:filled + k, 0] = rho * np.cos(phi)
        pos[filled:filled + k, 1] = rho * np.sin(phi)
        pos[filled:filled + k, 2] = z
        # speed: q = v / v_esc drawn from q^2 (1 - q^2)^(7/2) by rejection
        q = np.empty(k)
        todo = np.arange(k)
        while todo.size:
            x4 = rng.random(todo.size)
            x5 = rng.random(todo.size)
            acc = 0.1 * x5 < x4 * x4 * (1.0 - x4 * x4) ** 3.5
            q[todo[acc]] = x4[acc]
            todo = todo[~acc]
        v = q * math.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
        x6 = rng.random(k)
        x7 = rng.random(k)
        vz = (1.0 - 2.0 * x6) * v
        vrho = np.sqrt(np.maximum(v * v - vz * vz, 0.0))
        vphi = 2.0 * math.pi * x7
        vel[filled:filled + k, 0] = vrho * np.cos(vphi)
        vel[filled:filled + k, 1] = vrho * np.sin(vphi)
        vel[filled:filled + k, 2] = vz
        filled += k
    return pos, vel


def kroupa_masses(rng: np.random.Generator, n: int, normalise: bool = True) -> np.ndarray:
    """Kroupa (2001) IMF on [0.08, 100]: dN/dm ~ m^-1.3 below 0.5, m^-2.3 above."""
    m0, m1, m2 = KROUPA_M
    a1, a2 = KROUPA_SLOPES
    # piecewise power law, continuous at m1: k2 = k1 * m1^(a2 - a1)
    k1 = 1.0
    k2 = k1 * m1 ** (a2 - a1)
    w1 = k1 * (m1 ** (1 - a1) - m0 ** (1 - a1)) / (1 - a1)
    w2 = k2 * (m2 ** (1 - a2) - m1 ** (1 - a2)) / (1 - a2)
    u_seg = rng.random(n)
    u = rng.random(n)
    low = u_seg < w1 / (w1 + w2)
    m = np.empty(n)
    e1 = 1 - a1
    e2 = 1 - a2
    m[low] = (m0 ** e1 + u[low] * (m1 ** e1 - m0 ** e1)) ** (1.0 / e1)
    hi = ~low
    m[hi] = (m1 ** e2 + u[hi] * (m2 ** e2 - m1 ** e2)) ** (1.0 / e2)
    if normalise:
        m = m / m.sum()
    return m


def two_component_masses(n: int) -> np.ndarray:
    """Mass spectrum of the paper's core-collapse run: m = 10/(1.9N) for i = 0 mod 10, else 1/(1.9N)."""
    m = np.full(n, 1.0 / (1.9 * n))
    m[0::10] = 10.0 / (1.9 * n)
    return m


@dataclass
class Cluster:
    pos: np.ndarray   # (n, 3) float64, C-contiguous
    vel: np.ndarray   # (n, 3) float64
    mass: np.ndarray  # (n,) float64

    @property
    def n(self) -> int:
        return self.mass.shape[0]


def plummer(n: int, seed: int, masses: str = "equal") -> Cluster:
    """Plummer sphere in Henon units. ``masses`` is "equal", "kroupa" or "two".

    Draw order: positions and velocities first (in blocks, with rejection),
    then the masses from the same generator.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.default_rng(seed)
    pos, vel = _plummer_unit(rng, n)
    if masses == "equal":
        m = np.full(n, 1.0 / n)
    elif masses == "kroupa":
        m = kroupa_masses(rng, n)
    elif masses == "two":
        m = two_component_masses(n)
        m = m / m.sum()
    else:
        raise ValueError(f"unknown mass spectrum {masses!r}")
    # Henon scaling: lengths x a, velocities / sqrt(a) (G = M = 1 fixed)
    pos *= PLUMMER_A_HENON
    vel /= math.sqrt(PLUMMER_A_HENON)
    # centre of mass at rest at the origin (mass-weighted)
    mt = m.sum()
    pos -= (m[:, None] * pos).sum(0) / mt
    vel -= (m[:, None] * vel).sum(0) / mt
    return Cluster(np.ascontiguousarray(pos), np.ascontiguousarray(vel), m)


@dataclass
class Ensemble:
    pos: np.ndarray      # (sum n_k, 3)
    vel: np.ndarray
    mass: np.ndarray
    offsets: np.ndarray  # (n_clusters + 1,) int64
    r_out: np.ndarray    # (n_clusters,) per-cluster outer changeover radius
    r_in: np.ndarray

    @property
    def n_clusters(self) -> int:
        return self.offsets.size - 1


def ensemble(n_clusters: int = 64, seed0: int = 4000, nmin: float = 1e4, nmax: float = 2e5,
             nbar: float = 64.0, gamma: float = 0.1, masses: str = "kroupa") -> Ensemble:
    """Independent Plummer clusters with N_k = round(exp(U[ln nmin, ln nmax])).

    Cluster k uses generator seed ``seed0 + k``: its first draw sets N_k, the
    rest build the cluster. Each cluster has total mass 1; its r_out holds
    ``nbar`` neighbours on average and r_in = gamma * r_out.
    """
    parts = []
    sizes = []
    for k in range(n_clusters):
        rng = np.random.default_rng(seed0 + k)
        nk = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        sizes.append(nk)
        c = plummer(nk, seed=int(rng.integers(0, 2**62)), masses=masses)
        parts.append(c)
    offsets = np.zeros(n_clusters + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    pos = np.ascontiguousarray(np.concatenate([c.pos for c in parts]))
    vel = np.ascontiguousarray(np.concatenate([c.vel for c in parts]))
    mass = np.concatenate([c.mass for c in parts])
    r_out = np.array([r_out_for_nbar(s, nbar) for s in sizes])
    return Ensemble(pos, vel, mass, offsets, r_out, gamma * r_out)


def core_sample_size(n: int) -> int:
    """Sample size of the paper's core-radius algorithm: min(N, sqrt(5000 N))."""
    return int(min(n, math.floor(math.sqrt(5000.0 * n))))


def core_sample(n: int, seed: int) -> np.ndarray:
    """Distinct particle indices (int32, ascending) drawn uniformly for the
    core-radius algorithm; the draw is an input, made here with PCG64."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, core_sample_size(n), replace=False)).astype(np.int32)


# Workloads named in the measurement plan: (seed, N, mass spectrum, eps, r_out, theta)
WORKLOADS = {
    "plummer4k_equal": dict(seed=1, n=4096, masses="equal", eps=1e-4, r_out=0.05, theta=0.5),
    "plummer128k_kroupa": dict(seed=2, n=131072, masses="kroupa", eps=1e-5,
                               r_out=r_out_for_nbar(131072, 64.0), theta=0.5),
    "plummer1m_kroupa": dict(seed=3, n=1048576, masses="kroupa", eps=1e-6,
                             r_out=r_out_for_nbar(1048576, 64.0), theta=0.5),
    "plummer4m_kroupa": dict(seed=5, n=4194304, masses="kroupa", eps=1e-6,
                             r_out=r_out_for_nbar(4194304, 64.0), theta=0.5),
}


def workload(name: str):
    """(Cluster, params) for a named workload; r_in = 0.1 r_out throughout."""
    w = dict(WORKLOADS[name])
    c = plummer(w["n"], w["seed"], w["masses"])
    w["r_in"] = 0.1 * w["r_out"]
    return c, w
