#!/usr/bin/env python3
"""Gamma-point periodic J+K build throughput on one MI355X.

One step = one full build (density prep, short-range J/K, reciprocal J/K,
self term, back-transform, energies) through pbc_jk_build_device with the
density already resident in HBM.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload headline|cfg1|cfg2|cfg3|cfg4|cfg4m|cfg5]

The default (headline) times the 64-water cell in FP64 for exactly K builds
after W warm-ups (the line's value), then in the same run the same cell in
mixed precision (same K and W), a J-only build (the J-engine), and the
512-atom diamond cell in FP64 and in mixed precision (one warm-up and one
timed build each: at about a minute a build, K of them would not fit the
run's time limit), each with its error against the stored oracle results.
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
T_START = time.perf_counter()
BUDGET_S = 480.0    # the optional legs stop before this many seconds of the run
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
    model = cpu_info()
    if name == "cfg3":
        name = "cfg2"    # the oracle is FP64 only: same workload
    if name in ("cfg4", "cfg4m"):
        return None      # the oracle needs ~20 min for three bra shells of this cell
    if name == "cfg1":
        t0 = time.perf_counter()
        oracle.jk(system)
        t = time.perf_counter() - t0
        return {"value": 1.0 / t, "unit": "builds/s", "cores": threads, "cpu": model, "kind": "oracle",
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
    return {"value": 1.0 / total, "unit": "builds/s", "cores": threads, "cpu": model, "kind": "oracle",
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
        with pbcjk.Server(slots=4, cache_cells=False, policy=args.policy) as srv:
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
            # wait in the order the requests are expected to finish (the
            # server's queue order), so that progress is reported as it happens
            if args.policy == "deadline":
                order = sorted(range(len(reqs)), key=lambda i: arrivals[i] + 6.8e-6 * reqs[i].nbf ** 2)
            else:
                order = list(range(len(reqs)))
            res = [None] * len(reqs)
            last = time.perf_counter()
            for done, i in enumerate(order, 1):
                while tickets[i] is None:
                    time.sleep(0.01)
                res[i] = srv.wait(tickets[i])
                if done % 16 == 0 or time.perf_counter() - last > 30.0:
                    last = time.perf_counter()
                    print(f"  {done}/{len(reqs)} requests done, {last - t0:.1f} s", file=sys.stderr, flush=True)
            th.join()
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
                   "arrival_rate_per_s": rate, "saturated_builds_per_s": sat, "queue_policy": args.policy,
                   "precision": "mixed (fp32 below 1e-06)"},
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "build_ms_p50": float(np.percentile(build, 50)), "build_ms_max": float(build.max()),
        "server": {k: st[k] for k in ("peak_running", "peak_in_use", "budget", "retries")},
        "roofline": None, "cpu_baseline": None,
        "note": "roofline and cpu_baseline are reported on the single-cell workloads (cfg1-cfg3)",
    }
    print(json.dumps(out), flush=True)




def oracle_counts(name):
    """Screened ordered primitive quartets and (quartet, R1) terms of the FP64
    oracle's full build of the 64-water cell (stored with its J and K)."""
    if name not in ("cfg2", "cfg3"):
        return None
    try:
        import numpy as np
        g = np.load(os.path.join(ROOT, "tests", "golden", "cfg2_full.npz"))
        return {"ordered_quartets": float(g["n_quartets"]), "terms": float(g["n_terms"]),
                "definition": "ordered primitive quartets kept by the density-weighted Schwarz screen and "
                              "their (quartet, R1) terms, counted by the oracle (each unordered quartet twice)"}
    except (OSError, KeyError):
        return None


BECKE_FLOPS_PER_FACTOR = 35.0


def time_becke(steps, np, torch, inputs, pbcjk, cpu_sample=True):
    """Periodic Becke weights (the paper's Sec. 2.8 grid partition) of
    atom-centred product grids on the diamond cell's 512 atoms: 20 radial x
    8 x 16 angular points per atom (1.31 M points, grouped by atom), 17 bohr
    sphere, delta 1e-14; points resident in HBM, `steps` timed launches on
    one stream (HIP events).  The CPU oracle runs a bounded sample."""
    s4 = inputs.cfg4()
    pts, wq, org = inputs.atom_grid(s4.xyz, 20, 8, 16, 1.0)
    with pbcjk.Becke(s4.cell, s4.xyz, rcut=17.0, delta=1e-14) as b:
        dp = torch.from_numpy(pts).cuda()
        do = torch.from_numpy(org.astype(np.int32)).cuda()
        dw = torch.empty(len(pts), dtype=torch.float64, device="cuda")
        st = torch.cuda.current_stream()
        b.weights(dp, do, out=dw, stream=st)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            b.weights(dp, do, out=dw, stream=st)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        w = dw.cpu().numpy()
        info = b.info()
        evals = b.evaluations()
    V = abs(float(np.linalg.det(s4.cell)))
    out = {"workload": "Becke weights: diamond cell (512 atoms, a = 41.05 bohr), 20 x 8 x 16 product grid per atom "
                       "(1,310,720 points), 17 bohr sphere, delta 1e-14",
           "steps": steps, "ms_per_launch": ms, "points_per_s": len(pts) / (ms * 1e-3),
           "images_per_atom": info["max_images"], "sum_w_over_V": float((wq * w).sum()) / V,
           "switching_factors_per_launch": evals}
    # FP64 VALU roofline: ~35 FLOP per switching factor (|X - Y|^2, an rsqrt with two
    # Newton steps, u, the three-fold polynomial, the product)
    ach = evals * BECKE_FLOPS_PER_FACTOR / (ms * 1e-3) / 1e12
    out["roofline"] = {"kernel": "k_becke: periodic Becke weights, one lane per grid point", "bound": "alu",
                       "achieved": ach, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": ach / FP64_VALU_PEAK_TFLOPS, "traffic": None, "launches_per_build": 1.0,
                       "avg_launch_ms": ms, "flops_per_launch": evals * BECKE_FLOPS_PER_FACTOR}
    if cpu_sample:
        from oracle import becke as obk
        sel = np.sort(np.random.default_rng(7).choice(len(pts), 512, replace=False))
        t0 = time.perf_counter()
        ref = obk.becke_weights(s4.cell, s4.xyz, pts[sel], org[sel], rcut=17.0, delta=1e-14)
        t = time.perf_counter() - t0
        out["max_abs_dw_vs_oracle_sample"] = float(np.abs(w[sel] - ref).max())
        out["cpu_baseline"] = {"value": len(sel) / t, "unit": "points/s", "cores": os.cpu_count(), "kind": "oracle",
                               "sample": f"{len(sel)} points drawn at random from the grid"}
    return out


def time_workload(system, steps, warmup, np, torch, pbcjk, want_K=True, tag="", parts=None):
    """W untimed builds, then exactly `steps` timed builds through
    pbc_jk_build_device with D resident in HBM.  Returns the timings, the
    per-kernel accounting of the handle's counters, the last J, K (host) and
    energies.  `parts`: a PART_* mask to build only those parts (profiling)."""
    t_create = time.perf_counter()
    h = pbcjk.Handle(system)
    t_create = time.perf_counter() - t_create
    if parts is not None:
        h.set_parts(parts)
    dD = torch.from_numpy(system.D).cuda()
    dJ = torch.empty_like(dD)
    dK = torch.empty_like(dD) if want_K else None
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        h.build_device(dD, dJ, dK, energies=True, stream=stream)
    torch.cuda.synchronize()
    print(f"{tag}: setup {t_create:.1f} s, warmup done ({warmup} builds)", file=sys.stderr, flush=True)
    acc = {"lat": [], "gemm_ms": 0.0, "gemm_fl": 0.0, "n_gemm": 0, "y_ms": 0.0, "y_fl": 0.0, "n_y": 0,
           "sfac_ms": 0.0, "sr_class_ms": [0.0] * 21, "sr_terms_class": [0.0] * 21,
           "stage": {"sr": 0.0, "lr": 0.0, "other": 0.0}}
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    EJ = EK = None
    st = None
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        EJ, EK = h.build_device(dD, dJ, dK, energies=True, stream=stream)
        e1.record(stream)
        st = h.stats()
        e1.synchronize()
        acc["lat"].append(e0.elapsed_time(e1))
        for k, f in (("gemm_ms", "t_gemm_ms"), ("gemm_fl", "gemm_flops"), ("n_gemm", "n_gemm"), ("y_ms", "t_y_ms"),
                     ("y_fl", "y_flops"), ("n_y", "n_y"), ("sfac_ms", "t_sfac_ms")):
            acc[k] += st[f]
        for k, f in (("sr", "t_sr_ms"), ("lr", "t_lr_ms"), ("other", "t_other_ms")):
            acc["stage"][k] += st[f]
        for k in range(21):
            acc["sr_class_ms"][k] += st["t_sr_class_ms"][k]
            acc["sr_terms_class"][k] += st["terms_class"][k]
    t_end.record(stream)
    torch.cuda.synchronize()
    acc["ms_per_step"] = t_start.elapsed_time(t_end) / steps
    acc["st"] = st
    acc["E_J"], acc["E_K"] = EJ, EK
    acc["J"] = dJ.cpu().numpy()
    acc["K"] = dK.cpu().numpy() if want_K else None
    acc["setup_s"] = t_create
    h.close()
    print(f"{tag}: timed {steps} builds: {acc['ms_per_step']:.2f} ms/build", file=sys.stderr, flush=True)
    return acc


def kernel_candidates(acc, steps):
    """Per-kernel device time and algorithmic FLOPs per build: the exchange
    GEMMs (FP64 MFMA) and each short-range class pair (FP64 VALU)."""
    st = acc["st"]
    gk = st["gemm_kernel"]
    gemm_name = f"k_dgemm<{gk}>"
    gemm_role = {0: "dense exchange T_G = F_G D, K += W_G T_G F_G, and the self term",
                 3: "low-rank exchange accumulation K += sum_G Y_G Y_G^T on the upper tiles (D = L L^T, "
                    "FLOPs counted on the upper triangle)"}[gk]
    cands = [{"kernel": f"{gemm_name}: {gemm_role}", "name": gemm_name, "bound": "mfma",
              "ms_per_build": acc["gemm_ms"] / steps, "flops_per_build": acc["gemm_fl"] / steps,
              "launches_per_build": acc["n_gemm"] / steps, "peak": FP64_MFMA_PEAK_TFLOPS}]
    if acc["y_ms"] > 0:
        yname = "k_ygemm" if st.get("y_kernel", 0) == 1 else "k_dgemm<2>"
        cands.append({"kernel": f"{yname}: low-rank exchange products Y_G^T = L^T F_G", "name": yname,
                      "bound": "mfma", "ms_per_build": acc["y_ms"] / steps, "flops_per_build": acc["y_fl"] / steps,
                      "launches_per_build": acc["n_y"] / steps, "peak": FP64_MFMA_PEAK_TFLOPS})
    for k in range(21):
        t = acc["sr_class_ms"][k] / steps
        if t <= 0:
            continue
        cb, ck = SLOTS[k]
        la, lb = CLASSES[cb]
        lc, ld = CLASSES[ck]
        if (st["sr_jengine_mask"] >> k) & 1:
            name = f"k_sr_j<{la}, {lb}, {lc}, {ld}>"
        elif (st["sr_kernel_mask"] >> k) & 1:
            name = f"k_sr_coop<{la}, {lb}, {lc}, {ld}> (or k_sr_coop2)"
        elif (cb, ck) in COOP_SLOTS:
            name = f"k_sr_jk<{la}, {lb}, {lc}, {ld}, double, *> (component slices)"
        else:
            fold = "true" if (st["sr_fold_mask"] >> k) & 1 else "false"
            name = f"k_sr_jk<{la}, {lb}, {lc}, {ld}, double, {fold}, 0, {_nc(lc)}>"
        cands.append({"kernel": f"{name}: short-range, class pair ({CLASS_NAMES[cb]}|{CLASS_NAMES[ck]})",
                      "name": name, "bound": "alu", "ms_per_build": t,
                      "flops_per_build": acc["sr_terms_class"][k] / steps * sr_flops_per_term(cb, ck),
                      "launches_per_build": 1.0, "peak": FP64_VALU_PEAK_TFLOPS})
    cands.sort(key=lambda c: -c["ms_per_build"])
    return cands


def roof(c, workload):
    """The roofline object of one kernel; `traffic` only for the workload whose
    counters profiles/traffic.json holds (the 64-water cell, FP64 or mixed)."""
    ach = c["flops_per_build"] / (c["ms_per_build"] * 1e-3) / 1e12 if c["ms_per_build"] > 0 else 0.0
    return {"kernel": c["kernel"], "bound": c["bound"], "achieved": ach, "peak": c["peak"], "unit": "TFLOP/s",
            "frac": ach / c["peak"], "traffic": traffic_for(c["name"]) if workload in ("cfg2", "cfg3") else None,
            "launches_per_build": c["launches_per_build"],
            "avg_launch_ms": c["ms_per_build"] / max(1e-9, c["launches_per_build"]),
            "ms_per_build": c["ms_per_build"], "flops_per_build": c["flops_per_build"]}


def sr_summary(acc, steps, cands):
    ms = sum(acc["sr_class_ms"]) / steps
    fl = sum(c["flops_per_build"] for c in cands if c["bound"] == "alu")
    tf = fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    return {"ms_per_build": ms, "achieved_tflops": tf, "frac_fp64_valu": tf / FP64_VALU_PEAK_TFLOPS}


def errors_vs_golden(name, system, acc, np):
    """Errors against the stored FP64 oracle results (tests/golden), when the
    file for this workload exists: max|dJ|, max|dK| and dE_J, dE_K per atom
    (full matrices), or max|dJ|, max|dK| on the stored rows."""
    gdir = os.path.join(ROOT, "tests", "golden")
    try:
        if name in ("cfg2", "cfg3"):
            g = np.load(os.path.join(gdir, "cfg2_full.npz"))
            n = int(g["n"])
            iu = np.triu_indices(n)
            out = {"reference": "tests/golden/cfg2_full.npz (FP64 oracle, full build)",
                   "max_abs_dJ": float(np.abs(acc["J"][iu] - g["J"]).max())}
            if acc["K"] is not None:
                out["max_abs_dK"] = float(np.abs(acc["K"][iu] - g["K"]).max())
                out["dE_K_per_atom"] = float((acc["E_K"] - float(g["E_K"])) / system.natom)
            out["dE_J_per_atom"] = float((acc["E_J"] - float(g["E_J"])) / system.natom)
            return out
        if name in ("cfg4", "cfg4m"):
            g = np.load(os.path.join(gdir, "cfg4_rows.npz"))
            rows = g["rows"]
            J = g["J_sr"] + g["J_lrself"]
            K = g["K_sr"] + g["K_lrself"]
            out = {"reference": "tests/golden/cfg4_rows.npz (FP64 oracle rows of 3 shells)",
                   "rows": int(len(rows)), "max_abs_dJ": float(np.abs(acc["J"][rows] - J).max())}
            if acc["K"] is not None:
                out["max_abs_dK"] = float(np.abs(acc["K"][rows] - K).max())
            return out
    except (OSError, KeyError):
        return None
    return None


def cpu_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="headline", choices=["headline", "becke"] + sorted(WORKLOADS),
                    help="headline (default): cfg2 FP64 timed as the line's value, with the cfg3 mixed, "
                         "cfg2 J-only and cfg4 FP64/mixed legs in the same line; or one workload alone")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cfg4", action="store_true", help="headline: leave out the cfg4 legs")
    ap.add_argument("--requests", type=int, default=256, help="cfg5: requests of the stream to run")
    ap.add_argument("--rate-factor", type=float, default=0.8, help="cfg5: arrival rate / saturated rate")
    ap.add_argument("--policy", default="deadline", choices=["arrival", "deadline"],
                    help="cfg5: the request server's queue order")
    ap.add_argument("--parts", default="all", choices=["all", "sr", "lr", "self", "lr+self"],
                    help="build only these parts of J and K (profiling one stream alone); the line then "
                         "reports that partial build and no legs")
    ap.add_argument("--j-only", action="store_true",
                    help="build J alone (the J-engine path; profiling); the line then reports that build")
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
    if args.workload == "becke":
        r = time_becke(args.steps, np, torch, inputs, pbcjk, cpu_sample=not args.no_cpu_baseline)
        print(json.dumps({"metric": "Becke weights points/s", "value": r["points_per_s"], "unit": "points/s",
                          "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": r["ms_per_launch"],
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic", "config": {"workload": r["workload"]}, "roofline": r["roofline"],
                          "cpu_baseline": r.get("cpu_baseline"), "detail": r}), flush=True)
        return
    name = "cfg2" if args.workload == "headline" else args.workload
    system = inputs.CONFIGS[name]()
    parts = {"all": None, "sr": pbcjk.PART_SR, "lr": pbcjk.PART_LR, "self": pbcjk.PART_SELF,
             "lr+self": pbcjk.PART_LR | pbcjk.PART_SELF}[args.parts]
    acc = time_workload(system, args.steps, args.warmup, np, torch, pbcjk, want_K=not args.j_only, tag=name,
                        parts=parts)
    steps = args.steps
    cands = kernel_candidates(acc, steps)
    roof_main = roof(cands[0], name)
    roof2 = roof(next((c for c in cands[1:] if c["bound"] != cands[0]["bound"]), cands[min(1, len(cands) - 1)]),
                 name)
    st = acc["st"]
    lat = np.array(acc["lat"])
    ms = acc["ms_per_step"]
    out = {
        "metric": METRIC,
        "value": 1000.0 / ms,
        "unit": "builds/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if system.thr.fp32_below == 0 else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{name}: {WORKLOADS[name]}", "nbf": system.nbf, "natom": system.natom,
                   "precision": "fp64" if system.thr.fp32_below == 0 else f"mixed (fp32 below {system.thr.fp32_below:g})"},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "latency_samples": int(len(lat)),
        "setup_s": acc["setup_s"],
        "screened_quartets_per_s": st["quartets"] * 1000.0 / ms,
        "screened_terms_per_s": st["terms"] * 1000.0 / ms,
        "quartets_per_build": st["quartets"],
        "terms_per_build": st["terms"],
        "terms_fp32_per_build": st["terms_fp32"],
        "group_pairs": st["n_group_pairs"],
        "lr_exchange": {"form": "low-rank" if st["lr_rank"] >= 0 else "dense", "density_rank": st["lr_rank"],
                        "factor_ms": st["t_chol_ms"]},
        "stage_ms_per_build": {k: v / steps for k, v in acc["stage"].items()},
        "E_J": acc["E_J"],
        "E_K": acc["E_K"],
        "vs_oracle": errors_vs_golden(name, system, acc, np),
        "roofline": roof_main,
        "roofline_secondary": roof2,
        "sr_classes": [{"class_pair": f"({CLASS_NAMES[SLOTS[k][0]]}|{CLASS_NAMES[SLOTS[k][1]]})",
                        "ms_per_build": acc["sr_class_ms"][k] / steps, "terms_per_build": acc["sr_terms_class"][k] / steps}
                       for k in range(21) if acc["sr_class_ms"][k] > 0],
        "sr_all_classes": sr_summary(acc, steps, cands),
    }
    if args.j_only:
        out["j_only"] = True
        out["config"]["workload"] += " (J only)"
    if parts is not None:
        out["parts"] = args.parts
        out["vs_oracle"] = None
        out["config"]["workload"] += f" (only the {args.parts} part)"
    oc = oracle_counts(name)
    if oc:
        out["oracle_screened_terms_per_s"] = oc["terms"] * 1000.0 / ms
        out["oracle_counts"] = oc
    if args.workload == "headline" and parts is None and not args.j_only:
        del acc
        legs = {}
        # mixed precision on the same cell, same steps
        s3 = inputs.cfg3()
        a3 = time_workload(s3, steps, args.warmup, np, torch, pbcjk, tag="cfg3")
        legs["mixed"] = {"workload": f"cfg3: {WORKLOADS['cfg3']}", "steps": steps, "warmup": args.warmup,
                         "ms_per_step": a3["ms_per_step"], "builds_per_s": 1000.0 / a3["ms_per_step"],
                         "speedup_vs_fp64": ms / a3["ms_per_step"],
                         "terms_fp32_fraction": a3["st"]["terms_fp32"] / max(1.0, a3["st"]["terms"]),
                         "stage_ms_per_build": {k: v / steps for k, v in a3["stage"].items()},
                         "vs_oracle": errors_vs_golden("cfg3", s3, a3, np)}
        del a3
        # J alone (J-engine) on the same cell
        nj = max(1, min(steps, 5))
        aj = time_workload(system, nj, 1, np, torch, pbcjk, want_K=False, tag="cfg2 J-only")
        legs["j_only"] = {"workload": "cfg2 without K (J-engine)", "steps": nj, "warmup": 1,
                          "ms_per_step": aj["ms_per_step"], "fraction_of_jk_build": aj["ms_per_step"] / ms,
                          "vs_oracle": errors_vs_golden("cfg2", system, aj, np)}
        del aj
        try:
            legs["becke"] = time_becke(10, np, torch, inputs, pbcjk, cpu_sample=not args.no_cpu_baseline)
        except Exception as e:   # the J/K line stands without this leg
            legs["becke"] = {"error": str(e)}
        if not args.no_cfg4:
            est = 200.0     # s: setup, one warm-up and one timed build of the diamond cell
            for key, cname in (("cfg4_fp64", "cfg4"), ("cfg4_mixed", "cfg4m")):
                if time.perf_counter() - T_START + est > BUDGET_S:
                    legs[key] = {"workload": f"{cname}: {WORKLOADS[cname]}",
                                 "skipped": f"would not finish within the run's {BUDGET_S:.0f} s budget"}
                    continue
                t_leg = time.perf_counter()
                s4 = inputs.CONFIGS[cname]()
                a4 = time_workload(s4, 1, 1, np, torch, pbcjk, tag=cname)
                c4 = kernel_candidates(a4, 1)
                legs[key] = {"workload": f"{cname}: {WORKLOADS[cname]}", "steps": 1, "warmup": 1,
                             "ms_per_step": a4["ms_per_step"], "builds_per_s": 1000.0 / a4["ms_per_step"],
                             "setup_s": a4["setup_s"],
                             "stage_ms_per_build": a4["stage"], "terms_per_build": a4["st"]["terms"],
                             "terms_fp32_fraction": a4["st"]["terms_fp32"] / max(1.0, a4["st"]["terms"]),
                             "roofline": roof(c4[0], cname),
                             "roofline_secondary": roof(next((c for c in c4[1:] if c["bound"] != c4[0]["bound"]),
                                                            c4[min(1, len(c4) - 1)]), cname),
                             "sr_all_classes": sr_summary(a4, 1, c4),
                             "vs_oracle": errors_vs_golden(cname, s4, a4, np)}
                del a4
                est = 1.1 * (time.perf_counter() - t_leg)
            if "ms_per_step" in legs["cfg4_fp64"] and "ms_per_step" in legs["cfg4_mixed"]:
                legs["cfg4_mixed"]["speedup_vs_fp64"] = legs["cfg4_fp64"]["ms_per_step"] / legs["cfg4_mixed"]["ms_per_step"]
        out["legs"] = legs
    if not args.no_cpu_baseline and parts is None and not args.j_only:
        print("cpu baseline (oracle sample) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(system, name)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
