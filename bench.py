"""Benchmark of the P3T distant-force path on one MI355X.

One step = one pass of the whole path over resident synthetic input:
tree build (bounding box, Morton keys, radix sort, octree, FP64 moments,
groups) + grouped walk (regular force and potential, written in caller order)
+ neighbour lists inside r_out (count, scan, fill).

Workloads (--workload):
  plummer1m    (default) Plummer sphere N = 2^20, Kroupa masses, Henon units,
               eps = 1e-6, r_out for 64 mean neighbours (0.04077), r_in =
               0.1 r_out, theta = 0.5, quadrupole nodes, FP32 interactions
               with FP64 positions and sums; n_leaf, n_crit and the walk tile
               from the autotuner, timed on this input before the timed
               region (--no-autotune: --leaf, --ncrit)
  plummer128k  N = 131072, eps = 1e-5, n_crit = 32 (run with --prec fp64 and mixed)
  plummer4m    N = 2^22, eps = 1e-6
  ensemble64   64 independent clusters, N log-uniform in [1e4, 2e5], each
               with its own r_out for 64 neighbours; one batched build and one
               persistent walk launch per step
  p3t1m        N = 2^20 with the paper's run parameters (tau = (1/128)(N/2^14)^(-1/3),
               r_cut = 4 tau, r_buff = 3 tau sigma, dt_reg = 2^-9, eta = 0.02,
               theta = 0.4):
               the whole P3T loop (regular force and buffered lists, kicks,
               Hermite F_I on block steps); a step = one regular step
  kdk4m        N = 2^22: 32 kick-drift-kick steps of dt = 1/1024 with a full
               rebuild each step, captured once in a hipGraph; reports the
               relative energy drift (a step = one KDK step)

Prints one JSON line. For the force workloads value = all interactions
(particle-node + particle-particle) per second of whole step time. The
roofline object covers the walk kernel, timed with HIP events on its stream
inside the timed region. The cpu_baseline leg times the CPU oracle (tree walk
with the same tree, groups and opening rule, OpenMP over the host cores) on
the same workload and compares the GPU result with FP64 direct sums on a
sample of particles.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic operations per interaction (add, sub, mul = 1, FMA = 2,
# rsqrt = 1, log = 1), counted from the formulas the walk evaluates:
#   particle-node, monopole + traceless quadrupole: 55
#   particle-particle outside r_out (W = 1): 20
#   particle-particle in a near leaf (W(s) and the regular potential): 50
FLOPS_PN, FLOPS_FAR, FLOPS_NEAR = 55, 20, 50
# Irregular force + jerk + potential per neighbour pair (FP64): separation 3,
# s^2 6, rsqrt and powers 4, changeover K and its slope 19, force 8, jerk 33,
# irregular potential (closed-form Phi_R with log) 22.
FLOPS_IRR = 95
HBM_PEAK_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32 (256 CU x 256 flop/clk x 2.4 GHz)
PEAK_FP64_TFLOPS = 78.6

WORKLOADS = {
    "plummer1m": "plummer1m_kroupa",
    "plummer128k": "plummer128k_kroupa",
    "plummer4m": "plummer4m_kroupa",
    "ensemble64": None,
    "kdk4m": "plummer4m_kroupa",
    "p3t1m": "plummer1m_kroupa",
}
METRIC = "particle-node interactions/s and force evals/s at N=1e6 vs FP32 VALU roofline"
# The paper's own headline, quoted for context only (whole NBODY6+P3T code,
# other hardware, not this metric): abstract and Section 3.1.
CONTEXT = ("paper (context, not comparable): the whole NBODY6+P3T code runs more than 2x faster "
           "than NBODY6 at N = 10^6 on one NVIDIA V100 with 2 x 14-core Intel Xeon Gold 6132 "
           "(abstract; Section 3.1)")


def clock_mhz(torch):
    """Peak engine clock the HIP runtime reports for device 0 (MHz), or None.

    hipDeviceGetAttribute(hipDeviceAttributeClockRate = 5, in kHz) from the HIP
    runtime library torch has loaded."""
    import ctypes
    try:
        hip = ctypes.CDLL("libamdhip64.so")
        v = ctypes.c_int(0)
        if hip.hipDeviceGetAttribute(ctypes.byref(v), 5, 0) == 0 and v.value > 0:
            return v.value / 1000.0
    except OSError:
        pass
    return None


def walk_traffic(kernel: str):
    """HBM bytes per walk launch from the committed rocprofv3 counter summary,
    or None when the walk source has changed since the counters were taken."""
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
    ap.add_argument("--theta", type=float, default=None,
                    help="opening angle (default 0.5; 0.4 for p3t1m, the paper's runs)")
    ap.add_argument("--prec", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--leaf", type=int, default=0,
                    help="n_leaf (tree leaf size; default 8, 16 for kdk4m, the oracle run's)")
    ap.add_argument("--ncrit", type=int, default=0,
                    help="n_crit (largest walk group); 0 = the library's choice by size "
                         "(32 below 2^18 particles, else 64)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use --leaf/--ncrit as given instead of the autotuner's choice of n_leaf, "
                         "n_crit and walk tile (timed on this input before the timed region)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-neighbours", action="store_true")
    ap.add_argument("--valu-probe", action="store_true",
                    help="before the timed region, run the library's VALU calibration kernel once "
                         "(4096 waves x 32032 VALU instructions, to scale instruction counters)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the timed region, copy a buffer of this many MiB once "
                         "(a plain copy kernel of known size, to scale HBM byte counters)")
    return ap.parse_args()


def q(e):
    return {"median": float(np.median(e)), "p90": float(np.percentile(e, 90)),
            "p99": float(np.percentile(e, 99)), "max": float(np.max(e))}


def main():
    args = parse()
    if args.theta is None:
        args.theta = 0.4 if args.workload == "p3t1m" else 0.5
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the distant-force "
              "path is measured on a single MI355X.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "kdk4m":
        return bench_kdk(args)
    if args.workload == "p3t1m":
        return bench_p3t(args)
    return bench_force(args)


def _setup(args, torch):
    from paper_2110_11658_amd import ic
    dev = torch.device("cuda", 0)
    if args.workload == "ensemble64":
        e = ic.ensemble(n_clusters=64)
        inp = {"pos": e.pos, "mass": e.mass, "offsets": e.offsets, "r_in": e.r_in, "r_out": e.r_out,
               "eps": 1e-6, "name": "ensemble64_kroupa",
               "desc": f"64 Plummer clusters, N log-uniform [1e4, 2e5] (total {e.offsets[-1]}), "
                       f"Kroupa, eps=1e-6, per-cluster r_out for 64 neighbours, r_in=0.1 r_out"}
    else:
        wname = WORKLOADS[args.workload]
        cl, w = ic.workload(wname)
        inp = {"pos": cl.pos, "mass": cl.mass, "vel": cl.vel, "offsets": None, "r_in": w["r_in"],
               "r_out": w["r_out"], "eps": w["eps"], "name": wname,
               "desc": f"Plummer N={cl.n} Kroupa eps={w['eps']} r_out={w['r_out']:.5f} "
                       f"r_in={w['r_in']:.6f}"}
    inp["n"] = inp["mass"].size
    # SHA-256 of the generated positions and masses (FP64, C order): the inputs
    # of a record can be regenerated from the seed and checked against it
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(inp["pos"], dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(inp["mass"], dtype=np.float64).tobytes())
    inp["sha256"] = h.hexdigest()
    inp["pos_d"] = torch.from_numpy(inp["pos"]).to(dev)
    inp["mass_d"] = torch.from_numpy(inp["mass"]).to(dev)
    return inp, dev


def bench_force(args):
    import ctypes as C

    import torch

    from paper_2110_11658_amd import autotune
    from paper_2110_11658_amd._lib import check
    from paper_2110_11658_amd.api import Pbh, _ptr, _stream

    inp, dev = _setup(args, torch)
    n, theta, eps = inp["n"], args.theta, inp["eps"]
    pos, mass = inp["pos_d"], inp["mass_d"]
    batched = inp["offsets"] is not None
    neighbours = not args.no_neighbours
    p = Pbh(0, prec=args.prec)
    L, ctx = p.L, p.ctx

    tuned = None
    if args.no_autotune:
        ncrit = args.ncrit or (32 if n < (1 << 18) else 64)   # the library's rule for n_crit = 0
        p.set_params(leaf_size=args.leaf or 8, n_crit=ncrit, prec=args.prec)
    else:
        tuned = autotune.tune(p, pos, mass, inp["r_in"], inp["r_out"], theta, eps, prec=args.prec,
                              neighbours=neighbours, offsets=inp["offsets"])
    prm = p.params()

    acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
    pot = torch.empty(n, dtype=torch.float64, device=dev)
    off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    if batched:
        offs = np.ascontiguousarray(inp["offsets"], dtype=np.int64)
        ri = np.ascontiguousarray(inp["r_in"], dtype=np.float64)
        ro = np.ascontiguousarray(inp["r_out"], dtype=np.float64)
        nc = offs.size - 1

        def build():
            check(ctx, L.pbh_build_batched(ctx, nc, offs.ctypes.data_as(C.c_void_p), _ptr(pos),
                                           _ptr(mass), _stream()))

        def force(o, ix, cap, tot):
            return L.pbh_force_batched(ctx, _ptr(pos), _ptr(mass), ri.ctypes.data_as(C.c_void_p),
                                       ro.ctypes.data_as(C.c_void_p), theta, eps, _ptr(acc),
                                       _ptr(pot), o, ix, cap, tot, _stream())
    else:
        def build():
            check(ctx, L.pbh_build(ctx, n, _ptr(pos), _ptr(mass), _stream()))

        def force(o, ix, cap, tot):
            return L.pbh_force(ctx, _ptr(pos), _ptr(mass), inp["r_in"], inp["r_out"], theta, eps,
                               _ptr(acc), _ptr(pot), o, ix, cap, tot, _stream())

    # size the neighbour buffer once (outside the timed region)
    build()
    total = C.c_int64(0)
    idx = torch.empty(1, dtype=torch.int32, device=dev)
    force(_ptr(off), _ptr(idx), 0, C.byref(total))
    cap = int(total.value * 1.05) + 1024
    idx = torch.empty(cap, dtype=torch.int32, device=dev)

    def step():
        build()
        check(ctx, force(_ptr(off) if neighbours else None, _ptr(idx) if neighbours else None,
                         cap if neighbours else 0, None))

    if args.calib_copy_mib:
        src = torch.empty(args.calib_copy_mib << 17, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.valu_probe:
        probe_out = torch.empty(4096, dtype=torch.float32, device=dev)
        check(ctx, L.pbh_debug_valu_probe(ctx, 4096, 1000, _ptr(probe_out), _stream()))
        torch.cuda.synchronize()

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
    walk_mhz = p.walk_clock_mhz()   # engine clock during the last timed walk
    flops = FLOPS_PN * s["n_pn"] + FLOPS_FAR * s["n_pp_far"] + FLOPS_NEAR * s["n_pp_near"]
    walk_avg = float(np.mean(walk_ms))
    achieved = flops / (walk_avg * 1e-3) / 1e12
    per_step_inter = s["n_pn"] + s["n_pp_far"] + s["n_pp_near"]
    peak = PEAK_FP32_TFLOPS if args.prec == "mixed" else PEAK_FP64_TFLOPS
    kernel = f"k_walk<{'true' if args.prec == 'mixed' else 'false'}, {prm['walk_tile'] or 64}>"

    rec = {
        "metric": METRIC,
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
        "config": {"workload": f"{inp['name']}: {inp['desc']} theta={theta} quadrupole",
                   "n": n, "theta": theta, "precision": args.prec, "leaf_size": prm["leaf_size"],
                   "n_crit": prm["n_crit"], "walk_tile": prm["walk_tile"] or 64,
                   "neighbours": neighbours, "autotuned": tuned is not None,
                   "clusters": 64 if batched else 1},
        "inputs_sha256": inp["sha256"],
        "force_evals_per_s": n / (ms_step * 1e-3),
        "force_evals_per_s_build_walk": n / ((float(np.mean(build_ms)) + walk_avg) * 1e-3),
        "force_evals_per_s_walk_only": n / (walk_avg * 1e-3),
        "interactions_per_s_walk_only": per_step_inter / (walk_avg * 1e-3),
        "phase_ms": {"build": float(np.mean(build_ms)), "walk": walk_avg,
                     "neighbours": float(np.mean(nbr_ms))},
        "interactions_per_step": {"pn": s["n_pn"], "pp_far": s["n_pp_far"], "pp_near": s["n_pp_near"]},
        "rates_walk_only": {k: v / (walk_avg * 1e-3) for k, v in
                            (("pn_per_s", s["n_pn"]), ("pp_per_s", s["n_pp_far"] + s["n_pp_near"]),
                             ("interactions_per_s", per_step_inter))},
        "groups": s["n_groups"],
        "nbr_total": int(off[-1].item()) if neighbours else None,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": (walk_traffic(kernel) if inp["name"] == "plummer1m_kroupa" else None),
                     "kernel": kernel, "flops_per_launch": flops,
                     # the same rate against the FP32 vector peak without packed
                     # instructions (4 SIMD16 x 2 flop x 256 CUs x 2.4 GHz)
                     "peak_unpacked": 78.6, "frac_unpacked": achieved / 78.6,
                     "clock_mhz": clock_mhz(torch),
                     # the device cycle counter (clock64) over the steady clock
                     # during the last timed walk, summed over its workgroups;
                     # the fractions above stay against the 2.4 GHz peak
                     "clock_mhz_walk": walk_mhz},
    }
    if tuned is not None:
        rec["autotune"] = {k: v for k, v in tuned.items() if k != "cached"}
        rec["autotune"]["cached"] = tuned["cached"]
    rec["context"] = CONTEXT

    if neighbours and not batched:
        total = int(off[-1].item())
        rec["irregular"] = bench_irregular(p, inp, off, idx[:total], dev, not args.no_cpu_baseline)
    if not batched:
        rec["core"] = bench_core(p, inp, dev, not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"], rec["accuracy"] = cpu_baseline(inp, theta, prm, acc, pot)
    if args.prec == "mixed" and not batched:
        # after the accuracy check above: this leg overwrites acc and pot
        rec["fp64_walk"] = fp64_walk_leg(p, build, force, neighbours, off, idx, cap, per_step_inter,
                                         walk_avg, prm)
    p.close()
    print(json.dumps(rec))


def bench_irregular(p, inp, off, idx, dev, with_oracle, calls=10):
    """Irregular force, jerk and potential of every particle from the step's
    neighbour lists (pbh_irregular), timed with HIP events on its stream after
    the timed step region; sampled parity and the oracle's per-target cost."""
    import torch

    from paper_2110_11658_amd._lib import check
    from paper_2110_11658_amd.api import _ptr, _stream
    n = inp["n"]
    vel = torch.from_numpy(np.ascontiguousarray(inp["vel"])).to(dev)
    a = torch.empty((n, 3), dtype=torch.float64, device=dev)
    j = torch.empty((n, 3), dtype=torch.float64, device=dev)
    ph = torch.empty(n, dtype=torch.float64, device=dev)
    pairs = int(idx.shape[0])

    def call():
        check(p.ctx, p.L.pbh_irregular(p.ctx, n, _ptr(inp["pos_d"]), _ptr(vel), _ptr(inp["mass_d"]),
                                       inp["r_in"], inp["r_out"], inp["eps"], _ptr(off), _ptr(idx),
                                       pairs, 0, None, _ptr(a), _ptr(j), _ptr(ph), 0, _stream()))
    for _ in range(2):
        call()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(calls):
        call()
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / calls
    flops = FLOPS_IRR * pairs
    tflops = flops / (ms * 1e-3) / 1e12
    # algorithmic bytes: lists and offsets once, positions/velocities/masses
    # read once, records and ranks written once, outputs written once
    nbytes = 4 * pairs + 8 * (n + 1) + 56 * n + (64 + 4) * n + 56 * n
    out = {"ms": ms, "pairs": pairs, "pairs_per_s": pairs / (ms * 1e-3),
           "targets_per_s": n / (ms * 1e-3), "calls": calls,
           "roofline": {"bound": "alu", "achieved": tflops, "peak": PEAK_FP64_TFLOPS,
                        "unit": "TFLOP/s", "frac": tflops / PEAK_FP64_TFLOPS,
                        "flops_per_launch": flops, "kernel": "k_irregular (+ k_irr_pack)",
                        "hbm_bytes": nbytes,
                        "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    if with_oracle:
        import oracle
        rng = np.random.default_rng(4321)
        tg = np.sort(rng.choice(n, size=64, replace=False))
        t = time.perf_counter()
        ra, rj, rp, sc = oracle.irregular(inp["pos"], inp["vel"], inp["mass"], inp["r_in"],
                                          inp["r_out"], inp["eps"], targets=tg)
        dt = time.perf_counter() - t
        ga, gj, gp = a.cpu().numpy()[tg], j.cpu().numpy()[tg], ph.cpu().numpy()[tg]
        live = sc[:, 0] > 0

        def worst(g, r, scale):
            d = np.linalg.norm((g - r).reshape(len(tg), -1), axis=1)
            return float(np.max(d[live] / scale[live])) if live.any() else 0.0
        out["cpu_baseline"] = {"value": len(tg) / dt, "unit": "targets/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"{len(tg)} sampled targets, each summed over all {n} "
                                         f"particles (the O(N) definition)"}
        out["accuracy"] = {"vs": f"oracle on {len(tg)} sampled targets, error / magnitude sum",
                           "acc": worst(ga, ra, sc[:, 0]), "jerk": worst(gj, rj, sc[:, 1]),
                           "pot": worst(gp, rp, sc[:, 2])}
    return out


def bench_core(p, inp, dev, with_oracle, calls=5):
    """Core quantities (pbh_core) on the step's tree with the paper's sample
    size min(N, sqrt(5000 N)); each call waits for its result. The oracle's
    brute-force search is timed on a few targets and checks their densities."""
    import torch

    from paper_2110_11658_amd import ic
    n = inp["n"]
    smp = ic.core_sample(n, 2021)
    smp_d = torch.from_numpy(smp).to(dev)
    p.core(inp["pos_d"], inp["mass_d"], smp_d)
    t = time.perf_counter()
    for _ in range(calls):
        rho, res = p.core(inp["pos_d"], inp["mass_d"], smp_d)
    ms = 1e3 * (time.perf_counter() - t) / calls
    out = {"ms": ms, "samples": int(smp.size), "samples_per_s": smp.size / (ms * 1e-3),
           "brute_force_pairs_per_s": smp.size * n / (ms * 1e-3),
           "r_core": res["r_core"], "rho_core": res["rho_core"], "n_core": res["n_core"],
           "r_half": res["r_half"], "r_min": res["r_min"], "dt_min": res["dt_min"]}
    if with_oracle:
        import oracle
        sel = np.random.default_rng(5).choice(smp.size, 64, replace=False)
        t = time.perf_counter()
        ro, _ = oracle.core(inp["pos"], inp["mass"], smp[sel].astype(np.int64))
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {"value": len(sel) / dt, "unit": "samples/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"{len(sel)} of the sampled particles, 6 nearest neighbours by "
                                         f"brute force over all {n} (the paper's search)"}
        out["densities_bit_exact"] = bool(np.array_equal(rho.cpu().numpy()[sel], ro))
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def fp64_walk_leg(p, build, force, neighbours, off, idx, cap, per_step_inter, mixed_walk_ms, prm):
    """The same step with every interaction in FP64 (same tree, groups and
    opening rule): the walk's HIP-event time against the mixed walk's."""
    import ctypes as C  # noqa: F401
    from paper_2110_11658_amd.api import _ptr
    from paper_2110_11658_amd._lib import check
    p.set_params(leaf_size=prm["leaf_size"], n_crit=prm["n_crit"], walk_tile=prm["walk_tile"],
                 prec="fp64")
    ms = []
    for r in range(4):
        build()
        check(p.ctx, force(_ptr(off) if neighbours else None, _ptr(idx) if neighbours else None,
                           cap if neighbours else 0, None))
        s = p.stats()
        if r > 0:
            ms.append(s["ms_walk"])
    p.set_params(leaf_size=prm["leaf_size"], n_crit=prm["n_crit"], walk_tile=prm["walk_tile"],
                 prec=prm["prec"])
    w = float(np.median(ms))
    return {"ms_walk": w, "interactions_per_s_walk_only": per_step_inter / (w * 1e-3),
            "mixed_walk_speedup": w / mixed_walk_ms,
            "note": "FP64 walk (k_walk<false, tile>) on the same tree, groups and interactions"}


def cpu_baseline(inp, theta, prm, acc, pot):
    """CPU oracle on the same workload: tree walk over all particles (timed; for
    the ensemble each cluster in turn), plus FP64 direct sums on 512 sampled
    particles for the GPU result's error."""
    import oracle
    acc_h = acc.cpu().numpy()
    pot_h = pot.cpu().numpy()
    pos, mass = inp["pos"], inp["mass"]
    offsets = inp["offsets"] if inp["offsets"] is not None else np.array([0, inp["n"]])
    nc = offsets.size - 1
    r_in = np.broadcast_to(np.asarray(inp["r_in"], dtype=float), (nc,))
    r_out = np.broadcast_to(np.asarray(inp["r_out"], dtype=float), (nc,))
    t = time.perf_counter()
    inter = 0
    for k in range(nc):
        s = slice(offsets[k], offsets[k + 1])
        _, _, st = oracle.tree(pos[s], mass[s], r_in[k], r_out[k], theta, inp["eps"],
                               n_leaf=prm["leaf_size"], n_crit=prm["n_crit"])
        inter += st["pn"] + st["pp_far"] + st["pp_near"]
    dt = time.perf_counter() - t
    base = {"value": inter / dt, "unit": "interactions/s", "cores": oracle.num_threads(),
            "kind": "oracle", "seconds": dt,
            "sample": f"full workload ({inp['n']} particles, {nc} cluster(s)) through the CPU FP64 "
                      f"tree walk (tree build + walk), {oracle.num_threads()} OpenMP threads",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}
    # the same on one core, for a bounded sample: the first cluster, or the
    # first 2^17 particles of a single cluster (the walk over that subset)
    nthreads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        s = slice(offsets[0], min(offsets[1], offsets[0] + (1 << 17)))
        t = time.perf_counter()
        _, _, st = oracle.tree(pos[s], mass[s], r_in[0], r_out[0], theta, inp["eps"],
                               n_leaf=prm["leaf_size"], n_crit=prm["n_crit"])
        d1 = time.perf_counter() - t
    finally:
        oracle.set_num_threads(nthreads)
    base["one_core"] = {"value": (st["pn"] + st["pp_far"] + st["pp_near"]) / d1, "unit": "interactions/s",
                        "seconds": d1, "particles": int(s.stop - s.start),
                        "sample": "the first min(N, 2^17) particles of the first cluster as a system of "
                                  "their own, CPU FP64 tree walk on 1 thread"}
    rng = np.random.default_rng(12345)
    ea, ep = [], []
    per = max(1, 512 // nc)
    t_direct, pairs_direct = 0.0, 0
    for k in range(nc):
        s = slice(offsets[k], offsets[k + 1])
        nk = offsets[k + 1] - offsets[k]
        tg = rng.choice(nk, min(per, nk), replace=False)
        t = time.perf_counter()
        ra, rp = oracle.direct(pos[s], mass[s], r_in[k], r_out[k], inp["eps"], targets=tg)
        t_direct += time.perf_counter() - t
        pairs_direct += len(tg) * nk
        ga = acc_h[s][tg]
        gp = pot_h[s][tg]
        ea.append(np.linalg.norm(ga - ra, axis=1) / np.linalg.norm(ra, axis=1))
        ep.append(np.abs(gp - rp) / np.abs(rp))
    accuracy = {"vs": f"FP64 direct summation on {sum(len(e) for e in ea)} sampled particles",
                "force_rel": q(np.concatenate(ea)), "pot_rel": q(np.concatenate(ep))}
    # the O(N^2) definition itself (direct summation), on all cores and on one
    base["direct"] = {"value": pairs_direct / t_direct, "unit": "pairs/s", "cores": nthreads,
                      "seconds": t_direct, "sample": f"{sum(len(e) for e in ea)} sampled targets, each "
                                                     f"summed over every particle of its cluster"}
    oracle.set_num_threads(1)
    try:
        tg = np.arange(min(32, offsets[1] - offsets[0]))
        s = slice(offsets[0], offsets[1])
        t = time.perf_counter()
        oracle.direct(pos[s], mass[s], r_in[0], r_out[0], inp["eps"], targets=tg)
        d1 = time.perf_counter() - t
    finally:
        oracle.set_num_threads(nthreads)
    base["direct"]["one_core"] = {"value": len(tg) * (offsets[1] - offsets[0]) / d1, "unit": "pairs/s",
                                  "seconds": d1,
                                  "sample": f"{len(tg)} targets over all {offsets[1] - offsets[0]} "
                                            f"particles of the first cluster, 1 thread"}
    return base, accuracy


def bench_kdk(args):
    import torch

    from paper_2110_11658_amd.api import Pbh

    inp, dev = _setup(args, torch)
    n = inp["n"]
    dt, steps = 1.0 / 1024.0, 32
    leaf = args.leaf or 16
    ncrit = args.ncrit or 64
    out = {}
    for prec in ("mixed", "fp64") if args.prec == "mixed" else ("fp64",):
        p = Pbh(0, leaf_size=leaf, n_crit=ncrit, prec=prec)
        pos = inp["pos_d"].clone()
        vel = torch.from_numpy(inp["vel"]).to(dev)
        # warm-up on copies: sizes the buffers and captures the one-step graph
        p.kdk(pos.clone(), vel.clone(), inp["mass_d"], dt, 1, inp["r_in"], inp["r_out"], args.theta,
              inp["eps"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e = p.kdk(pos, vel, inp["mass_d"], dt, steps, inp["r_in"], inp["r_out"], args.theta, inp["eps"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        e = e.cpu().numpy()
        out[prec] = {"seconds": t1 - t0, "energy": e,
                     "drift": float(np.max(np.abs(e - e[0]) / abs(e[0])))}
        p.close()
    main_prec = args.prec
    secs = out[main_prec]["seconds"]
    rec = {
        "metric": "KDK leapfrog steps with full tree rebuild (hipGraph) at N=2^22",
        "value": n * steps / secs,
        "unit": "particle-steps/s",
        "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": 1e3 * secs / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if main_prec == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": f"{inp['name']}: {inp['desc']} theta={args.theta} dt=1/1024 32 KDK steps",
                   "n": n, "leaf_size": leaf, "n_crit": ncrit},
        "energy_drift": {k: v["drift"] for k, v in out.items()},
        "energy_first_last": {k: [float(v["energy"][0]), float(v["energy"][-1])] for k, v in out.items()},
        "ms_per_step_by_precision": {k: 1e3 * v["seconds"] / steps for k, v in out.items()},
    }
    if "fp64" in out and "mixed" in out:
        rec["energy_diff_mixed_vs_fp64"] = float(np.max(np.abs(out["mixed"]["energy"] - out["fp64"]["energy"])
                                                         / abs(out["fp64"]["energy"][0])))
    # the oracle's leapfrog of the same workload (CPU FP64 tree walk, written to
    # tests/golden by make_kdk4m_oracle.py): energies and the drift curve
    gold_path = os.path.join(ROOT, "tests", "golden", "kdk4m_oracle.json")
    if os.path.exists(gold_path) and leaf == 16 and ncrit == 64 and args.theta == 0.5:
        gold = json.load(open(gold_path))
        oe = np.array(gold["energy"])
        d_orc = (oe - oe[0]) / abs(oe[0])
        acc = {"vs": "oracle leapfrog (CPU FP64 tree walk, same workload), tests/golden/kdk4m_oracle.json",
               "oracle_drift_max": float(np.max(np.abs(d_orc)))}
        for k, v in out.items():
            e = v["energy"]
            acc[f"{k}_energy_max_rel_diff"] = float(np.max(np.abs(e - oe)) / abs(oe[0]))
            acc[f"{k}_drift_max_abs_diff"] = float(np.max(np.abs((e - e[0]) / abs(e[0]) - d_orc)))
        rec["accuracy"] = acc
    if not args.no_cpu_baseline:
        # one force evaluation of the oracle leapfrog (tree build + walk) on the
        # host cores: one step's worth of the oracle's run
        import oracle
        t = time.perf_counter()
        oracle.tree(inp["pos"], inp["mass"], inp["r_in"], inp["r_out"], args.theta, inp["eps"],
                    n_leaf=leaf, n_crit=ncrit)
        d = time.perf_counter() - t
        rec["cpu_baseline"] = {"value": n / d, "unit": "particle-steps/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "seconds": d,
                               "sample": "one regular-force evaluation of the oracle leapfrog (CPU FP64 "
                                         "tree build + walk over all particles), i.e. one of its steps",
                               "cpu_model": _cpu_model()}
    print(json.dumps(rec))


def bench_p3t(args):
    """The P3T loop with the paper's run parameters at N = 2^20."""
    import torch

    from paper_2110_11658_amd import ic
    from paper_2110_11658_amd.api import Pbh

    inp, dev = _setup(args, torch)
    n = inp["n"]
    pr = ic.paper_radii(n)
    r_out, r_buff, T = pr["r_cut"], pr["r_buff"], pr["dt_reg"]
    r_in, eps, eta = 0.1 * r_out, inp["eps"], 0.02
    steps = args.steps if args.steps != 10 else 4
    p = Pbh(0, leaf_size=args.leaf or 8, n_crit=args.ncrit, prec=args.prec)
    vel0 = torch.from_numpy(inp["vel"]).to(dev)
    pos, vel = inp["pos_d"].clone(), vel0.clone()
    p.p3t(pos.clone(), vel.clone(), inp["mass_d"], r_in, r_out, r_buff, args.theta, eps, T, eta, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e, st = p.p3t(pos, vel, inp["mass_d"], r_in, r_out, r_buff, args.theta, eps, T, eta, steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    e = e.cpu().numpy()
    rec = {
        "metric": "P3T regular steps (regular force + buffered lists + kicks + block-step Hermite F_I) at N=2^20",
        "value": n * steps / secs, "unit": "particle regular-steps/s",
        "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": 1e3 * secs / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if args.prec == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": f"{inp['name']}: {inp['desc'].split(' r_out')[0]} paper rule: "
                               f"r_cut={r_out:.6f} r_in={r_in:.6f} r_buff={r_buff:.6f} dt_reg={T} "
                               f"eta={eta} theta={args.theta}", "n": n},
        "hermite": {"blocks_per_step": st["blocks"] / steps, "particle_steps_per_step": st["steps"] / steps,
                    "deepest_level": st["kmax"]},
        "energy_drift": float(np.max(np.abs(e - e[0]) / abs(e[0]))),
    }
    p.close()
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
