#!/usr/bin/env python3
"""Write mixed1m_oracle_nu300.json: the FP64 oracle on 8 seeds of the 262144-atom
mixed sp2/sp3 lattice (M = 1048576) at nu = 300, kT = 0.1 eV, mu = -0.45 eV.

The seeds are every 2048th entry of the sorted 16384-seed sample of that
lattice (the seed sample the large-instance runs use). mu is a fixed input near
half filling (the method takes mu as given; both sides receive the same double).
Calls only the oracle and the seeded input generator. A run takes several
minutes and about 5 GB of host memory per worker.

    python tests/golden/make_mixed1m_oracle.py [--workers 4]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import mar_oracle as O  # noqa: E402
from paper_1307_3218_amd import lattice  # noqa: E402

WORKLOAD, NU, MU, KT = "mixed_32x32x32", 300, -0.45, 0.1
OUT = os.path.join(HERE, "mixed1m_oracle_nu300.json")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=4)
    args = ap.parse_args()
    system = lattice.workload(WORKLOAD)
    sample = lattice.sample_seeds(system.M, 16384, seed=0)
    seeds = [int(s) for s in sample[::2048]]
    t0 = time.perf_counter()
    res = O.solve(system.H, system.S, seeds, NU, MU, KT, workers=args.workers)
    dt = time.perf_counter() - t0
    H = system.H
    rows = {}
    for j in seeds:
        lo, hi = H.indptr[j], H.indptr[j + 1]
        rows[str(j)] = {"cols": [int(c) for c in H.indices[lo:hi]], "rho": [float(v) for v in res.rho[lo:hi]]}
    doc = {
        "what": "FP64 oracle (CGS2 mArnoldi, Sec. 2) on sampled seeds of the M=1048576 mixed lattice",
        "workload": WORKLOAD, "M": int(system.M), "nnz": int(H.nnz), "nu": NU, "mu": MU, "kT": KT,
        "seeds": seeds, "nu_eff": [int(v) for v in res.nu_eff],
        "e_seed": [float(v) for v in res.e_seed], "n_seed": [float(v) for v in res.n_seed],
        "e_band": float(res.e_band), "rho_rows": rows,
        "eps": [[float(v) for v in e] for e in res.eps],
        "weight": [[float(v) for v in w] for w in res.weight],
        "oracle_seconds": round(dt, 1), "workers": args.workers,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {OUT}: {len(seeds)} seeds in {dt:.0f} s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
