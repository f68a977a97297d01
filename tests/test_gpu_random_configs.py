"""Seeded random configurations against the oracle: lattice shape and kind, seed set (ragged, unsorted),
subspace dimension, precision, form, schedule, block size, projection variant, support tracking, stream
mode and local regions, drawn from a fixed generator so that every run checks the same cases.

Bars: every listed rho column and every E_j, N_j against the oracle (the full one, or the local-region
one) at 1e-10 in FP64 and 1e-5 in FP32; nu_eff equal. The subspace dimension stays below the point where
a seed's Krylov space (or region) is exhausted, where the breakdown step depends on the precision.
"""
import numpy as np
import pytest

from oracle import mar_local as OL
from oracle import mar_oracle as O
from paper_1307_3218_amd import lattice, mar

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}
SHAPES = [(2, 2, 2), (3, 2, 2), (2, 3, 2), (2, 2, 3), (3, 3, 2)]
N_CASES = 40


def _cases():
    rng = np.random.default_rng(20261203)
    out = []
    for i in range(N_CASES):
        shape = SHAPES[rng.integers(len(SHAPES))]
        mixed = bool(rng.integers(2))
        prec = ["fp64", "fp32"][rng.integers(2)]
        form = "plain" if rng.random() < 0.2 else "batched"
        local = form == "batched" and rng.random() < 0.35
        bmax = 128 if prec == "fp64" else 256
        bmin = (2 if prec == "fp64" else 4) if local else 1
        B = 1 if form == "plain" else int(2 ** rng.integers(int(np.log2(bmin)), int(np.log2(bmax)) + 1))
        r = int(rng.integers(2, 5)) if local else None
        nu = int(rng.integers(1, 25 if local else 61))
        variant = int(rng.integers(7))
        support = bool(rng.random() < 0.8)
        two = [None, True, False][rng.integers(3)]
        schedule = "auto" if form == "plain" else ("textbook" if rng.random() < 0.25 and not local else "delayed")
        kT = [0.1, 0.05][rng.integers(2)]
        out.append(dict(i=i, shape=shape, mixed=mixed, prec=prec, form=form, B=B, r=r, nu=nu, variant=variant,
                        support=support, two=two, schedule=schedule, kT=kT, draw=int(rng.integers(1 << 30))))
    return out


CASES = _cases()


@pytest.mark.parametrize("case", CASES, ids=[f"case{c['i']}" for c in CASES])
def test_random_configuration(case):
    s = lattice.generate(*case["shape"], mixed=case["mixed"], seed=case["draw"] % 7)
    rng = np.random.default_rng(case["draw"])
    n = int(rng.integers(1, min(s.M, 3 * case["B"] + 8) + 1))
    seeds = rng.choice(s.M, size=n, replace=False).astype(np.int32)
    mu = float(rng.uniform(-2.0, 1.0))
    label = (f"case {case['i']}: M={s.M} {'mixed' if case['mixed'] else 'diamond'} {case['prec']} {case['form']} "
             f"{case['schedule']} B={case['B']} nu={case['nu']} r={case['r']} variant={case['variant']} "
             f"support={case['support']} two_streams={case['two']} n={n} mu={mu:.3f} kT={case['kT']}")
    print(label, flush=True)
    c = mar.Context(s.H, s.S)
    try:
        if case["r"] is not None:
            c.set_local_region(case["r"])
        c.set_tuning(seed_block=case["B"] if case["form"] == "batched" else 0, schedule=case["schedule"],
                     proj_variant=case["variant"], support=case["support"], two_streams=case["two"])
        g = c.solve(seeds, case["nu"], mu, case["kT"], precision=case["prec"], form=case["form"], levels=True)
    finally:
        c.close()
    if case["r"] is None:
        ref = O.solve(s.H, s.S, seeds, case["nu"], mu, case["kT"])
    else:
        ref = OL.solve_local(s.H, s.S, seeds, case["nu"], case["r"], mu, case["kT"])
    assert np.array_equal(g.nu_eff, ref.nu_eff), label
    tol = TOL[case["prec"]]
    worst = 0.0
    for j in seeds:
        lo, hi = s.H.indptr[j], s.H.indptr[j + 1]
        d = np.linalg.norm(g.rho[lo:hi] - ref.rho[lo:hi]) / max(np.linalg.norm(ref.rho[lo:hi]), 1e-300)
        worst = max(worst, d)
    e_err = np.abs(g.e_seed - ref.e_seed) / np.maximum(np.abs(ref.e_seed), 1e-2 * np.abs(ref.e_seed).max())
    n_err = np.abs(g.n_seed - ref.n_seed) / np.maximum(np.abs(ref.n_seed), 2e-2)
    print(f"  worst rho column {worst:.2e}, E_j {e_err.max():.2e}, N_j {n_err.max():.2e}", flush=True)
    assert worst <= tol and e_err.max() <= tol and n_err.max() <= tol, label
