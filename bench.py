"""Benchmark of the P3T distant-force path on one MI355X.

One step = one pass of the whole path over a resident synthetic cluster:
tree build (bounding box, Morton keys, radix sort, octree, FP64 moments,
groups) + grouped mixed-precision walk (regular force and potential, written
in caller order) + neighbour lists inside r_out (count, scan, fill).

Default workload: Plummer sphere, N = 2^20, Kroupa masses, Henon units,
eps = 1e-6, r_out for 64 mean neighbours (0.04077), r_in = 0.1 r_out,
theta = 0.5, monopole + quadrupole nodes, FP32 interactions with FP64
positions and sums.

Prints one JSON line. value = all interactions (particle-node + particle-
particle) per second of whole step time. The roofline object covers the walk
kernel, timed with HIP events on its own stream inside the timed region. The
cpu_baseline leg times the CPU oracle (tree walk with the same tree, groups
and opening rule, OpenMP over the host cores) on the full workload and
compares the GPU result with FP64 direct sums on a sample of particles.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic FP32 operations per interaction (add, sub, mul = 1, rsqrt = 1,
# log = 1), counted from the formulas the walk evaluates:
#   particle-node, monopole + traceless quadrupole: 55
#   particle-particle outside r_out (W = 1): 20
#   particle-particle in a near leaf (W(s) and the regular potential): 50
FLOPS_PN, FLOPS_FAR, FLOPS_NEAR = 55, 20, 50
PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32 (256 CU x 256 flop/clk x 2.4 GHz)

WORKLOADS = {
    "plummer1m": ("plummer1m_kroupa", 0.5),
    "plummer128k": ("plummer128k_kroupa", 0.5),
    "plummer4m": ("plummer4m_kroupa", 0.5),
}


def walk_traffic(kernel: str):
    """HBM bytes per walk launch from the committed rocprofv3 counter summary,
    or None when the walk source has changed since the counters were taken."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_2110_11658_amd", "csrc", "walk.hip")
    prof = os.path.join(ROOT, "profiles", "k_walk_plummer1m_hbm_traffic.md")
    if not os.path.exists(prof):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    text = open(prof).read()
    m_sha = re.search(r"walk.hip sha256 prefix: ([0-9a-f]{16})", text)
    m_val = re.search(r"traffic_bytes_per_launch " + re.escape(kernel) + r": ([0-9]+)", text)
    if not m_sha or not m_val or m_sha.group(1) != sha:
        return None
    return float(m_val.group(1))


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plummer1m", choices=sorted(WORKLOADS))
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--prec", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--leaf", type=int, default=16)
    ap.add_argument("--ncrit", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-neighbours", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the timed region, copy a buffer of this many MiB once "
                         "(a plain copy kernel of known size, to scale HBM byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the distant-force "
              "path is measured on a single MI355X.", file=sys.stderr)
        sys.exit(2)

    import ctypes as C

    import torch

    from paper_2110_11658_amd import ic
    from paper_2110_11658_amd._lib import check
    from paper_2110_11658_amd.api import Pbh, _ptr, _stream

    wname, theta = WORKLOADS[args.workload]
    if args.theta is not None:
        theta = args.theta
    cl, w = ic.workload(wname)
    n = cl.n
    dev = torch.device("cuda", 0)
    pos = torch.from_numpy(cl.pos).to(dev)
    mass = torch.from_numpy(cl.mass).to(dev)
    acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
    pot = torch.empty(n, dtype=torch.float64, device=dev)
    off = torch.empty(n + 1, dtype=torch.int64, device=dev)

    p = Pbh(0, leaf_size=args.leaf, n_crit=args.ncrit, prec=args.prec)
    L, ctx = p.L, p.ctx
    neighbours = not args.no_neighbours

    # size the neighbour buffer once (outside the timed region)
    p.build(pos, mass)
    total = C.c_int64(0)
    idx = torch.empty(1, dtype=torch.int32, device=dev)
    st = L.pbh_force(ctx, w["r_in"], w["r_out"], theta, w["eps"], _ptr(acc), _ptr(pot), _ptr(off),
                     _ptr(idx), 0, C.byref(total), _stream())
    cap = int(total.value * 1.05) + 1024
    idx = torch.empty(cap, dtype=torch.int32, device=dev)

    def step():
        check(ctx, L.pbh_build(ctx, n, _ptr(pos), _ptr(mass), _stream()))
        check(ctx, L.pbh_force(ctx, w["r_in"], w["r_out"], theta, w["eps"], _ptr(acc), _ptr(pot),
                               _ptr(off) if neighbours else None, _ptr(idx) if neighbours else None,
                               cap if neighbours else 0, None, _stream()))

    if args.calib_copy_mib:
        src = torch.empty(args.calib_copy_mib << 17, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    p.set_timing(True)
    for _ in range(args.warmup):
        step()
        p.stats()
    torch.cuda.synchronize()

    walk_ms, build_ms, nbr_ms = [], [], []
    inter = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        s = p.stats()   # waits for the step; reads the phase events and counters
        walk_ms.append(s["ms_walk"])
        build_ms.append(s["ms_build"])
        nbr_ms.append(s["ms_nbr"])
        inter += s["n_pn"] + s["n_pp_far"] + s["n_pp_near"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if s["error_flags"]:
        raise RuntimeError(f"device error flags {s['error_flags']:#x}")

    ms_step = 1e3 * (t1 - t0) / args.steps
    flops = FLOPS_PN * s["n_pn"] + FLOPS_FAR * s["n_pp_far"] + FLOPS_NEAR * s["n_pp_near"]
    walk_avg = float(np.mean(walk_ms))
    achieved = flops / (walk_avg * 1e-3) / 1e12
    per_step_inter = s["n_pn"] + s["n_pp_far"] + s["n_pp_near"]

    rec = {
        "metric": "particle-node interactions/s and force evals/s at N=1e6 vs FP32 VALU roofline",
        "value": inter / (t1 - t0),
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{wname}: Plummer N={n} Kroupa eps={w['eps']} r_out={w['r_out']:.5f} "
                               f"r_in={w['r_in']:.6f} theta={theta} quadrupole",
                   "n": n, "theta": theta, "precision": args.prec, "leaf_size": args.leaf,
                   "n_crit": args.ncrit, "neighbours": neighbours},
        "force_evals_per_s": n / (ms_step * 1e-3),
        "force_evals_per_s_walk_only": n / (walk_avg * 1e-3),
        "interactions_per_s_walk_only": per_step_inter / (walk_avg * 1e-3),
        "phase_ms": {"build": float(np.mean(build_ms)), "walk": walk_avg,
                     "neighbours": float(np.mean(nbr_ms))},
        "interactions_per_step": {"pn": s["n_pn"], "pp_far": s["n_pp_far"], "pp_near": s["n_pp_near"]},
        "nbr_total": int(off[-1].item()) if neighbours else None,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": (walk_traffic("k_walk<true>") if args.prec == "mixed"
                                 and wname == "plummer1m_kroupa" else None),
                     "kernel": "k_walk<mixed>" if args.prec == "mixed" else "k_walk<fp64>",
                     "flops_per_launch": flops},
    }

    if not args.no_cpu_baseline:
        rec["cpu_baseline"], rec["accuracy"] = cpu_baseline(cl, w, theta, args, acc, pot)
    p.close()
    print(json.dumps(rec))


def cpu_baseline(cl, w, theta, args, acc, pot):
    """CPU oracle on the same workload: tree walk over all particles (timed), plus
    FP64 direct sums on 512 sampled particles for the GPU result's error."""
    import oracle
    acc_h = acc.cpu().numpy()
    pot_h = pot.cpu().numpy()
    t = time.perf_counter()
    _, _, st = oracle.tree(cl.pos, cl.mass, w["r_in"], w["r_out"], theta, w["eps"],
                           n_leaf=args.leaf, n_crit=args.ncrit)
    dt = time.perf_counter() - t
    inter = st["pn"] + st["pp_far"] + st["pp_near"]
    base = {"value": inter / dt, "unit": "interactions/s", "cores": oracle.num_threads(),
            "kind": "oracle", "seconds": dt,
            "sample": f"full workload ({cl.n} particles) through the CPU FP64 tree walk "
                      f"(tree build + walk), {oracle.num_threads()} OpenMP threads"}
    tg = np.random.default_rng(12345).choice(cl.n, 512, replace=False)
    ra, rp = oracle.direct(cl.pos, cl.mass, w["r_in"], w["r_out"], w["eps"], targets=tg)
    ea = np.linalg.norm(acc_h[tg] - ra, axis=1) / np.linalg.norm(ra, axis=1)
    ep = np.abs(pot_h[tg] - rp) / np.abs(rp)
    q = lambda e: {"median": float(np.median(e)), "p90": float(np.percentile(e, 90)),
                   "p99": float(np.percentile(e, 99)), "max": float(e.max())}
    accuracy = {"vs": "FP64 direct summation on 512 sampled particles",
                "force_rel": q(ea), "pot_rel": q(ep)}
    return base, accuracy


if __name__ == "__main__":
    main()
