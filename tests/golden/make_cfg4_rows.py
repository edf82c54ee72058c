#!/usr/bin/env python3
"""Writes tests/golden/cfg4_sr_rows.npz: rows of the real-space (erfc) parts
of J and K of the diamond workload (512 atoms, nbf 6656, omega 0.2, delta
1e-11, FP64) for three bra shells of atom 0 (an s, a p and the d shell),
computed by the CPU oracle alone.  Run once; takes about 20 minutes on 8
cores.

    python3 tests/golden/make_cfg4_rows.py
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2410_22278_amd import inputs  # noqa: E402

SHELLS = [0, 2, 4]


def main():
    oracle.build()
    s = inputs.cfg4()
    t0 = time.time()
    r = oracle.jk(s, bra_shells=SHELLS, parts="sr")
    rows = np.asarray(r["rows"], dtype=np.int64)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg4_sr_rows.npz")
    np.savez_compressed(out, shells=np.array(SHELLS), rows=rows, J=r["J"][rows], K=r["K"][rows],
                        n_quartets=r["n_quartets"], n_terms=r["n_terms"])
    print(f"wrote {out}: rows {rows.tolist()} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
