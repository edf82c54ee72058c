#!/usr/bin/env python3
"""Gamma-point periodic J+K build throughput on one MI355X.

One step = one full build (density prep, short-range J/K, reciprocal J/K,
self term, back-transform, energies) through pbc_jk_build_device with the
density already resident in HBM.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload cfg2|cfg1]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Fock J+K builds/s & screened quartets/s, FP64 vs mixed; p50/p99 latency"
FP64_MFMA_PEAK_TFLOPS = 78.6
# FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA) x 2.4 GHz
FP64_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

CLASSES = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]
CLASS_NAMES = ["ss", "ps", "pp", "ds", "dp", "dd"]
SLOTS = [(cb, ck) for cb in range(6) for ck in range(cb, 6)]
# class pairs run by the cooperative (one wavefront per group pair) kernel
COOP_SLOTS = {(0, 5), (1, 5), (2, 4), (2, 5), (3, 4), (3, 5), (4, 4), (4, 5), (5, 5)}
CSRC = os.path.join(ROOT, "paper_2410_22278_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def _sha256(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_for(name):
    """HBM bytes per launch of `name` from the committed counter summary, or
    None when there is none or the kernel's source changed since."""
    import json as _json
    try:
        with open(TRAFFIC_FILE) as f:
            rec = _json.load(f)
    except (OSError, ValueError):
        return None
    for r in rec.get("kernels", []):
        if r.get("name") != name:
            continue
        srcs = r.get("sources", {})
        if srcs and all(os.path.exists(os.path.join(CSRC, k)) and _sha256(os.path.join(CSRC, k)) == v
                        for k, v in srcs.items()):
            return r.get("bytes_per_launch")
    return None


def _nh(l):
    return (l + 1) * (l + 2) * (l + 3) // 6


def _nc(l):
    return (l + 1) * (l + 2) // 2


def sr_flops_per_term(cb, ck):
    """Canonical McMurchie-Davidson count for one (primitive quartet, R1)
    term: geometry 30, two Boys evaluations and the short-range combination
    68 + 10L, R recurrence 2 N_R(L) with N_R = (L+1)(L+2)(L+3)(L+4)/24, ket
    transform 2 n_h(ab) n_h(cd) n_c(cd), bra transform 2 n_h(ab) n_c(ab) n_c(cd)."""
    la, lb = CLASSES[cb]
    lc, ld = CLASSES[ck]
    L = la + lb + lc + ld
    nr = (L + 1) * (L + 2) * (L + 3) * (L + 4) // 24
    nab, ncd = _nc(la) * _nc(lb), _nc(lc) * _nc(ld)
    return (30 + 68 + 10 * L + 2 * nr + 2 * _nh(la + lb) * _nh(lc + ld) * ncd
            + 2 * _nh(la + lb) * nab * ncd)


WORKLOADS = {
    "cfg1": "cubic a=5.0 A, 8 atoms, 2s+1p per atom (3 prims, exps 0.1-20), nbf 40, "
            "omega 0.3, delta 1e-10, image cap 10 A, |G| <= 3, D = C C^T (40x8), FP64",
    "cfg2": "64 rigid H2O in a cubic a=12.4 A cell, O 3s+2p, H 2s (3 prims, exps 0.1-50), "
            "nbf 832, omega 0.3, delta 1e-10, D = C C^T (832x320), FP64",
    "cfg3": "the 64-water cell of cfg2 in mixed precision: FP32 short-range quartets below a "
            "density-weighted bound of 1e-6, FP64 accumulation and reciprocal sum",
    "cfg4": "diamond 4x4x4 supercell (512 atoms, a=21.72 A, N(0, 0.05 A) displacements), 2s+2p+1d (spherical) "
            "per atom, 3 prims in [0.08, 10], nbf 6656, omega 0.2, delta 1e-11, D = C C^T (6656x1024), FP64",
    "cfg4m": "the diamond cell of cfg4 in mixed precision (FP32 short-range quartets below 1e-6)",
    "cfg5": "serving stream: cubic H/C/O cells of 8-216 atoms (log-uniform) at 0.1 atoms/A^3, mixed precision, "
            "D = C C^T with nbf/4 orbitals, Poisson arrivals at 0.8x the measured saturated rate, through the "
            "library's request server (4 slots, HBM arena admission)",
}


def cpu_baseline(system, name):
    """The oracle as it stands, on a bounded sample of the same workload,
    scaled to one full build."""
    import numpy as np

    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    if name == "cfg3":
        name = "cfg2"    # the oracle is FP64 only: same workload
    if name in ("cfg4", "cfg4m"):
        return None      # the oracle needs ~20 min for three bra shells of this cell
    if name == "cfg1":
        t0 = time.perf_counter()
        oracle.jk(system)
        t = time.perf_counter() - t0
        return {"value": 1.0 / t, "unit": "builds/s", "cores": threads, "kind": "oracle",
                "sample": "one full cfg1 build"}
    shells = [0, 3, 7]    # O s, O p, H s of the first water
    pl = oracle.pair_list(system)
    frac = float(np.isin(pl["sa"], shells).sum()) / len(pl["sa"])
    t0 = time.perf_counter()
    oracle.jk(system, bra_shells=shells, parts="sr")
    t_sr = (time.perf_counter() - t0) / frac
    G, _ = oracle.glist(system)
    ng_s = min(64, len(G))
    t0 = time.perf_counter()
    oracle.jk(system, parts="lr", g_range=(0, ng_s))
    t_lr = (time.perf_counter() - t0) * len(G) / ng_s
    t0 = time.perf_counter()
    oracle.jk(system, parts="self")
    t_self = time.perf_counter() - t0
    total = t_sr + t_lr + t_self
    return {"value": 1.0 / total, "unit": "builds/s", "cores": threads, "kind": "oracle",
            "sample": (f"short-range rows of shells {shells} ({100 * frac:.2f}% of the bra pairs) "
                       f"scaled by 1/fraction; reciprocal part over {ng_s} of {len(G)} G vectors scaled "
                       f"by {len(G)}/{ng_s}; self term in full; est. full build {total:.0f} s")}


def serve(args, np, torch, inputs, pbcjk):
    """cfg5: a stream of requests through the library's request server."""
    import threading
    reqs = [inputs.serving_request(i) for i in range(args.requests)]
    print(f"cfg5: {len(reqs)} requests, natom {min(r.natom for r in reqs)}-{max(r.natom for r in reqs)}, "
          f"nbf {min(r.nbf for r in reqs)}-{max(r.nbf for r in reqs)}", file=sys.stderr, flush=True)

    def run(arrivals):
        with pbcjk.Server(slots=4, cache_cells=False) as srv:
            t0 = time.perf_counter()
            tickets = [None] * len(reqs)

            def feeder():
                for i, r in enumerate(reqs):
                    dt = t0 + arrivals[i] - time.perf_counter()
                    if dt > 0:
                        time.sleep(dt)
                    tickets[i] = srv.submit(r)
            th = threading.Thread(target=feeder)
            th.start()
            th.join()
            res = [srv.wait(t) for t in tickets]
            wall = time.perf_counter() - t0
            st = srv.stats()
        bad = [r["error"] for r in res if r["status"] != 0]
        if bad:
            raise RuntimeError(f"cfg5: {len(bad)} requests failed: {bad[:3]}")
        return res, wall, st

    # saturated: every request queued at t = 0
    res_sat, wall_sat, _ = run(np.zeros(len(reqs)))
    sat = len(reqs) / wall_sat
    print(f"saturated: {sat:.3f} builds/s ({wall_sat:.1f} s)", file=sys.stderr, flush=True)
    rate = args.rate_factor * sat
    arr = inputs.serving_arrivals(len(reqs), rate=rate)
    res, wall, st = run(arr - arr[0])
    lat = np.array([r["latency_ms"] for r in res])
    build = np.array([r["build_ms"] for r in res])
    out = {
        "metric": METRIC, "value": len(reqs) / wall, "unit": "builds/s", "n_gpus": 1,
        "steps": len(reqs), "warmup": 0, "ms_per_step": 1000.0 * wall / len(reqs), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"cfg5: {WORKLOADS['cfg5']}", "requests": len(reqs),
                   "arrival_rate_per_s": rate, "saturated_builds_per_s": sat,
                   "precision": "mixed (fp32 below 1e-06)"},
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "build_ms_p50": float(np.percentile(build, 50)), "build_ms_max": float(build.max()),
        "server": {k: st[k] for k in ("peak_running", "peak_in_use", "budget", "retries")},
        "roofline": None, "cpu_baseline": None,
        "note": "roofline and cpu_baseline are reported on the single-cell workloads (cfg1-cfg3)",
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--requests", type=int, default=32, help="cfg5: requests of the stream to run")
    ap.add_argument("--rate-factor", type=float, default=0.8, help="cfg5: arrival rate / saturated rate")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized float64 buffer 3 times on the GPU (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the J/K build runs on one GPU; --gpus above 1 is not supported "
              "(no multi-GPU path is implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2410_22278_amd import inputs, pbcjk

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        n = args.copy_probe * 1048576 // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 3}))
        return
    if args.workload == "cfg5":
        serve(args, np, torch, inputs, pbcjk)
        return
    system = inputs.CONFIGS[args.workload]()
    h = pbcjk.Handle(system)
    dD = torch.from_numpy(system.D).cuda()
    dJ = torch.empty_like(dD)
    dK = torch.empty_like(dD)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        h.build_device(dD, dJ, dK, energies=True, stream=stream)
    torch.cuda.synchronize()
    print(f"warmup done ({args.warmup} builds)", file=sys.stderr, flush=True)

    lat, gemm_ms, gemm_fl, sfac_ms, n_gemm = [], 0.0, 0.0, 0.0, 0
    y_ms, y_fl, n_y = 0.0, 0.0, 0
    sr_class_ms, sr_terms_class = [0.0] * 21, [0.0] * 21
    stage = {"sr": 0.0, "lr": 0.0, "other": 0.0}
    quartets = terms = 0.0
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t_start.record(stream)
    for k in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        EJ, EK = h.build_device(dD, dJ, dK, energies=True, stream=stream)
        e1.record(stream)
        st = h.stats()
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
        gemm_ms += st["t_gemm_ms"]
        y_ms += st["t_y_ms"]
        y_fl += st["y_flops"]
        n_y += st["n_y"]
        gemm_fl += st["gemm_flops"]
        n_gemm += st["n_gemm"]
        sfac_ms += st["t_sfac_ms"]
        stage["sr"] += st["t_sr_ms"]
        stage["lr"] += st["t_lr_ms"]
        stage["other"] += st["t_other_ms"]
        quartets, terms = st["quartets"], st["terms"]
        for k in range(21):
            sr_class_ms[k] += st["t_sr_class_ms"][k]
            sr_terms_class[k] += st["terms_class"][k]
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)
    ms_per_step = total_ms / args.steps
    print(f"timed {args.steps} builds: {ms_per_step:.2f} ms/build (wall {wall:.2f} s)",
          file=sys.stderr, flush=True)

    lat = np.array(lat)
    steps = args.steps
    # GEMM instantiation that formed the reciprocal exchange
    gk = st["gemm_kernel"]
    gemm_name = f"k_dgemm<{gk}>"
    gemm_role = {0: "dense exchange T_G = F_G D, K += W_G T_G F_G, and the self term",
                 3: "low-rank exchange accumulation K += sum_G Y_G Y_G^T on the upper tiles (D = L L^T, "
                    "FLOPs counted on the upper triangle)"}[gk]
    cands = [{
        "kernel": f"{gemm_name}: {gemm_role}", "name": gemm_name, "bound": "mfma",
        "ms_per_build": gemm_ms / steps, "flops_per_build": gemm_fl / steps,
        "launches_per_build": n_gemm / steps, "peak": FP64_MFMA_PEAK_TFLOPS,
    }]
    if y_ms > 0:
        cands.append({
            "kernel": "k_dgemm<2>: low-rank exchange products Y_G^T = L^T F_G", "name": "k_dgemm<2>",
            "bound": "mfma", "ms_per_build": y_ms / steps, "flops_per_build": y_fl / steps,
            "launches_per_build": n_y / steps, "peak": FP64_MFMA_PEAK_TFLOPS,
        })
    for k in range(21):
        t = sr_class_ms[k] / steps
        if t <= 0:
            continue
        cb, ck = SLOTS[k]
        la, lb = CLASSES[cb]
        lc, ld = CLASSES[ck]
        fold = "true" if (st["sr_fold_mask"] >> k) & 1 else "false"
        if (st["sr_kernel_mask"] >> k) & 1:
            name = f"k_sr_coop<{la}, {lb}, {lc}, {ld}> (or k_sr_coop2)"
        elif (cb, ck) in COOP_SLOTS:
            name = f"k_sr_jk<{la}, {lb}, {lc}, {ld}, double, {fold}, *> (component slices)"
        else:
            name = f"k_sr_jk<{la}, {lb}, {lc}, {ld}, double, {fold}, 0, {_nc(lc)}>"
        cands.append({
            "kernel": f"{name}: short-range J/K, class pair ({CLASS_NAMES[cb]}|{CLASS_NAMES[ck]})", "name": name,
            "bound": "alu", "ms_per_build": t, "flops_per_build": sr_terms_class[k] / steps * sr_flops_per_term(cb, ck),
            "launches_per_build": 1.0, "peak": FP64_VALU_PEAK_TFLOPS,
        })

    def roof(c):
        ach = c["flops_per_build"] / (c["ms_per_build"] * 1e-3) / 1e12 if c["ms_per_build"] > 0 else 0.0
        return {"kernel": c["kernel"], "bound": c["bound"], "achieved": ach, "peak": c["peak"], "unit": "TFLOP/s",
                "frac": ach / c["peak"], "traffic": traffic_for(c["name"]),
                "launches_per_build": c["launches_per_build"],
                "avg_launch_ms": c["ms_per_build"] / max(1e-9, c["launches_per_build"]),
                "ms_per_build": c["ms_per_build"], "flops_per_build": c["flops_per_build"]}

    cands.sort(key=lambda c: -c["ms_per_build"])
    roof_main = roof(cands[0])
    roof2 = roof(next((c for c in cands[1:] if c["bound"] != cands[0]["bound"]), cands[min(1, len(cands) - 1)]))
    sr_total_ms = sum(sr_class_ms) / steps
    sr_total_fl = sum(c["flops_per_build"] for c in cands if c["bound"] == "alu")
    out = {
        "metric": METRIC,
        "value": 1000.0 / ms_per_step,
        "unit": "builds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if system.thr.fp32_below == 0 else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "nbf": system.nbf,
                   "natom": system.natom,
                   "precision": "fp64" if system.thr.fp32_below == 0 else f"mixed (fp32 below {system.thr.fp32_below:g})"},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "screened_quartets_per_s": quartets * 1000.0 / ms_per_step,
        "screened_terms_per_s": terms * 1000.0 / ms_per_step,
        "quartets_per_build": quartets,
        "terms_per_build": terms,
        "terms_fp32_per_build": st["terms_fp32"],
        "group_pairs": st["n_group_pairs"],
        "lr_exchange": {"form": "low-rank" if st["lr_rank"] >= 0 else "dense",
                        "density_rank": st["lr_rank"], "factor_ms": st["t_chol_ms"]},
        "stage_ms_per_build": {k: v / args.steps for k, v in stage.items()},
        "E_J": EJ,
        "E_K": EK,
        "roofline": roof_main,
        "roofline_secondary": roof2,
        "sr_classes": [{"class_pair": f"({CLASS_NAMES[SLOTS[k][0]]}|{CLASS_NAMES[SLOTS[k][1]]})",
                        "ms_per_build": sr_class_ms[k] / steps, "terms_per_build": sr_terms_class[k] / steps}
                       for k in range(21) if sr_class_ms[k] > 0],
        "sr_all_classes": {"ms_per_build": sr_total_ms,
                           "achieved_tflops": sr_total_fl / (sr_total_ms * 1e-3) / 1e12 if sr_total_ms > 0 else 0.0,
                           "frac_fp64_valu": (sr_total_fl / (sr_total_ms * 1e-3) / 1e12 / FP64_VALU_PEAK_TFLOPS
                                              if sr_total_ms > 0 else 0.0)},
    }
    h.close()
    if not args.no_cpu_baseline:
        print("cpu baseline (oracle sample) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(system, args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
