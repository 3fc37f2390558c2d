"""Autotuner for the tree and walk parameters: leaf size n_leaf, group size
n_crit and the walk's LDS tile (walk_tile).

Each candidate is timed on the caller's actual input. A candidate is one full
pass: build, walk, and (optionally) neighbour lists. Timing uses the library's
HIP events on torch's current stream. The best is the candidate with the
smallest median time over `reps` passes after one warm-up; before the first
candidate a few untimed passes bring the clocks up, and the three fastest
(n_leaf, n_crit) pairs are timed again with twice the passes before one is
chosen. The search runs in two stages: every (n_leaf, n_crit) pair at the
default tile, then every tile at the best pair. Results are cached in a JSON file keyed by device name,
log2 N, theta, precision, neighbours and cluster count. The cache path comes
from PBH_AUTOTUNE_CACHE, else ~/.cache/pbh/autotune.json.

Every candidate yields the same neighbour lists. Forces differ only within
the tree's approximation: the opening rule and quadrupoles are the same for
all candidates, but different groups see different interaction lists. The
tuner therefore optimises speed alone.
"""
from __future__ import annotations

import json
import math
import os
from typing import Iterable, Optional, Sequence, Tuple

import torch

DEFAULT_CANDIDATES: Tuple[Tuple[int, int], ...] = (
    (8, 32), (8, 48), (8, 64), (16, 32), (16, 48), (16, 64), (32, 48), (32, 64))
DEFAULT_TILES: Tuple[int, ...] = (64, 96, 128)


def _cache_path() -> str:
    p = os.environ.get("PBH_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "pbh", "autotune.json")


def _key(n: int, theta: float, prec: str, neighbours: bool, n_clusters: int) -> str:
    dev = "cpu"
    if torch.cuda.is_available():
        props = torch.cuda.get_device_properties(torch.cuda.current_device())
        # the marketing name can read empty (e.g. under a profiler); the ISA name cannot
        dev = f"{props.name}|{props.gcnArchName}"
    return f"{dev}|log2n={round(math.log2(max(n, 1)))}|theta={theta:.3f}|{prec}|nbr={int(neighbours)}|c={n_clusters}"


def load_cache() -> dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict) -> None:
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def tune(pbh, pos: torch.Tensor, mass: torch.Tensor, r_in, r_out, theta: float, eps: float,
         prec: str = "mixed", neighbours: bool = True, offsets: Optional[Sequence[int]] = None,
         candidates: Iterable[Tuple[int, int]] = DEFAULT_CANDIDATES,
         tiles: Iterable[int] = DEFAULT_TILES, reps: int = 3, use_cache: bool = True) -> dict:
    """Pick (n_leaf, n_crit, walk_tile) for this input; leaves `pbh` configured
    with the winner.

    r_in/r_out are floats for one cluster or sequences for a batched build
    (with `offsets`). Returns {"leaf_size", "n_crit", "walk_tile", "ms", "table",
    "cached"}; `table` lists every timed candidate.
    """
    n = int(pos.shape[0])
    n_clusters = 1 if offsets is None else len(offsets) - 1
    tiles = tuple(tiles)
    key = _key(n, theta, prec, neighbours, n_clusters) + f"|tiles={','.join(map(str, tiles))}"
    cache = load_cache() if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]
        pbh.set_params(leaf_size=best["leaf_size"], n_crit=best["n_crit"],
                       walk_tile=best["walk_tile"], prec=prec)
        return dict(best, cached=True)

    pbh.set_timing(True)
    table = []

    def timed(leaf, ncrit, tile, nrep=reps, record=True):
        pbh.set_params(leaf_size=leaf, n_crit=ncrit, walk_tile=tile, prec=prec)
        times = []
        for r in range(nrep + 1):
            if offsets is None:
                pbh.build(pos, mass)
                pbh.force(r_in, r_out, theta, eps, neighbours=neighbours)
            else:
                pbh.build_batched(offsets, pos, mass)
                pbh.force_batched(r_in, r_out, theta, eps, neighbours=neighbours)
            s = pbh.stats()
            if r > 0:
                times.append(s["ms_build"] + s["ms_walk"] + s["ms_nbr"])
        times.sort()
        row = {"leaf_size": leaf, "n_crit": ncrit, "walk_tile": tile, "ms": times[len(times) // 2]}
        if record:
            table.append(row)
        return row

    candidates = list(candidates)
    timed(*candidates[0], tiles[0], nrep=3, record=False)   # clocks up before anything is timed
    stage1 = sorted((timed(leaf, ncrit, tiles[0]) for leaf, ncrit in candidates), key=lambda t: t["ms"])
    recheck = [timed(t["leaf_size"], t["n_crit"], tiles[0], nrep=2 * reps) for t in stage1[:3]]
    first = min(recheck, key=lambda t: t["ms"])
    best = min([first] + [timed(first["leaf_size"], first["n_crit"], t) for t in tiles[1:]],
               key=lambda t: t["ms"])
    pbh.set_params(leaf_size=best["leaf_size"], n_crit=best["n_crit"], walk_tile=best["walk_tile"],
                   prec=prec)
    result = {"leaf_size": best["leaf_size"], "n_crit": best["n_crit"],
              "walk_tile": best["walk_tile"], "ms": best["ms"], "table": table}
    if use_cache:
        cache[key] = result
        save_cache(cache)
    return dict(result, cached=False)
