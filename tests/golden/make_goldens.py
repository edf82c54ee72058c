#!/usr/bin/env python3
"""Writes the stored oracle results that the GPU parity tests compare with.
Every value comes from the CPU oracle alone (FP64) on the seeded workloads
of paper_2410_22278_amd.inputs; nothing is read from the GPU library.

    python3 tests/golden/make_goldens.py cfg4rows   # ~40 min on 8 cores
    python3 tests/golden/make_goldens.py serve      # ~10 min
    python3 tests/golden/make_goldens.py cfg2       # ~90 min

Files (symmetric matrices are stored as their upper triangles, row-major):
  cfg4_rows.npz   diamond workload (nbf 6656, delta 1e-11): rows of three
                  bra shells of atom 0 (an s, a p and the d shell) of the
                  real-space part and of the reciprocal + self parts of J, K
  cfg2_full.npz   64-water workload (nbf 832, delta 1e-10): J, K, E_J, E_K
  serve_reqs.npz  serving requests 4 and 7 (H/C/O with d shells, nbf 45 and
                  63) in full (J, K, E_J, E_K) and request 1 (nbf 304, the
                  largest of the first thirteen) on the rows of three shells
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2410_22278_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
CFG4_SHELLS = [0, 2, 4]
# serving requests: the two smallest with a C atom (d shells) in full, and the
# largest of the first thirteen on the rows of an H s, an O p and a C d shell
SERVE = [(4, None), (7, None), (1, [0, 7, 17])]


def upper(M):
    return M[np.triu_indices(M.shape[0])]


def unpack_upper(v, n):
    """Inverse of upper(): the full symmetric matrix."""
    M = np.zeros((n, n))
    M[np.triu_indices(n)] = v
    return M + np.triu(M, 1).T


def cfg4rows():
    s = inputs.cfg4()
    t0 = time.time()
    sr = oracle.jk(s, bra_shells=CFG4_SHELLS, parts="sr")
    print(f"cfg4 short-range rows: {time.time() - t0:.0f} s", flush=True)
    t0 = time.time()
    lr = oracle.jk(s, bra_shells=CFG4_SHELLS, parts="lr,self", g_chunk=2)
    print(f"cfg4 reciprocal + self rows: {time.time() - t0:.0f} s", flush=True)
    rows = np.asarray(sr["rows"], dtype=np.int64)
    out = os.path.join(HERE, "cfg4_rows.npz")
    np.savez_compressed(out, shells=np.array(CFG4_SHELLS), rows=rows,
                        J_sr=sr["J"][rows], K_sr=sr["K"][rows],
                        J_lrself=lr["J"][rows], K_lrself=lr["K"][rows],
                        n_quartets=sr["n_quartets"], n_terms=sr["n_terms"], n_G=lr["n_G"])
    print(f"wrote {out}", flush=True)


def cfg2():
    s = inputs.cfg2()
    t0 = time.time()
    r = oracle.jk(s)
    print(f"cfg2 full build: {time.time() - t0:.0f} s", flush=True)
    out = os.path.join(HERE, "cfg2_full.npz")
    np.savez_compressed(out, n=s.nbf, J=upper(r["J"]), K=upper(r["K"]), E_J=r["E_J"], E_K=r["E_K"],
                        n_quartets=r["n_quartets"], n_terms=r["n_terms"])
    print(f"wrote {out}", flush=True)


def serve():
    rec = {}
    done = []
    out = os.path.join(HERE, "serve_reqs.npz")
    for i, shells in SERVE:
        s = inputs.serving_request(i)
        t0 = time.time()
        # FP64 oracle of the same cell (the request itself runs mixed precision)
        r = oracle.jk(s, bra_shells=shells)
        print(f"request {i}: natom {s.natom} nbf {s.nbf} {'rows of shells %s' % shells if shells else 'full'}: "
              f"{time.time() - t0:.0f} s", flush=True)
        rec[f"n_{i}"] = s.nbf
        if shells is None:
            rec[f"J_{i}"] = upper(r["J"])
            rec[f"K_{i}"] = upper(r["K"])
            rec[f"E_J_{i}"] = r["E_J"]
            rec[f"E_K_{i}"] = r["E_K"]
        else:
            rows = np.asarray(r["rows"], dtype=np.int64)
            rec[f"rows_{i}"] = rows
            rec[f"J_{i}"] = r["J"][rows]
            rec[f"K_{i}"] = r["K"][rows]
        done.append(i)
        # written after every request, so that a long run leaves the finished ones
        np.savez_compressed(out, ids=np.array(done), **rec)
        print(f"wrote {out} (requests {done})", flush=True)


if __name__ == "__main__":
    oracle.build(force=False)
    jobs = {"cfg4rows": cfg4rows, "cfg2": cfg2, "serve": serve}
    for name in sys.argv[1:] or ["cfg4rows", "serve", "cfg2"]:
        jobs[name]()
