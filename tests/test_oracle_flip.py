"""Pins of the local flipping oracle (Appendix: sign-flip refinement of an eigenvector), on the CPU.

The pins tie the oracle to things other than itself: brute-force distance-2
reachability by dense matrix powers (validity and greedy minimality of the
colouring), R recomputed from scratch with sparse products (descent at every
logged flip, with and without the orthogonality penalty; local minimality;
tracked residual), and the exact eigenvector of LAPACK's generalized solver
(sign errors on first-colour rows are undone in the first colour). Planted
mistakes in the penalty term (its sign, a dropped square term, a p frozen at
the colour's start, a wrong update of p) must each break one of the pins.
"""
import importlib.util
import pathlib
import sys

import numpy as np
import pytest
import scipy.linalg

from oracle import mar_flip as F
from paper_1307_3218_amd import lattice


@pytest.fixture(scope="module")
def cell():
    s = lattice.generate(2, 2, 1, mixed=True, seed=1)           # 32 atoms, M = 128
    H, S = s.H.tocsr(), s.S.tocsr()
    ev, V = scipy.linalg.eigh(H.toarray(), S.toarray())
    return H, S, ev, V, F.distance2_colouring(H)


def test_colouring_is_valid_and_greedy(cell):
    H, S, ev, V, col = cell
    P = (H.toarray() != 0).astype(np.int64)
    reach = ((P @ P + P) > 0)
    M = H.shape[0]
    for l in range(M):
        near = np.nonzero(reach[l])[0]
        assert all(col[m] != col[l] for m in near if m != l)
        earlier = {int(col[m]) for m in near if m < l}
        assert all(c in earlier for c in range(col[l]))      # nothing smaller was free


def test_first_colour_sign_errors_are_undone(cell):
    H, S, ev, V, col = cell
    k = H.shape[0] // 2
    phi = V[:, k]
    bad = np.nonzero(col == 0)[0][::2]
    x = phi.copy()
    x[bad] *= -1.0
    res = F.local_flip(H, S, x, ev[k], max_sweeps=10, colour=col)
    assert np.array_equal(res.phi, phi)
    assert res.flips == len(bad) and res.sweeps == 2
    assert res.R[-1] <= 1e-20 * res.R[0]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_descent_local_minimum_and_residual(cell, seed):
    H, S, ev, V, col = cell
    rng = np.random.default_rng(seed)
    k = H.shape[0] // 2 + seed
    x = V[:, k] + 0.05 * rng.standard_normal(H.shape[0]) * np.abs(V[:, k]).max()
    x[rng.random(H.shape[0]) < 0.3] *= -1.0
    res = F.local_flip(H, S, x, ev[k], max_sweeps=200, colour=col)
    assert all(b <= a for a, b in zip(res.R, res.R[1:]))              # no penalty: R never grows
    assert res.R[-1] < res.R[0]
    r = H @ res.phi - ev[k] * (S @ res.phi)
    assert np.abs(res.r - r).max() <= 1e-12 * np.abs(r).max()
    assert abs(res.R[-1] - float(r @ r)) <= 1e-12 * res.R[-1]
    base = F.residual_norm(H, S, res.phi, ev[k])
    for l in range(H.shape[0]):                                       # no single flip lowers R
        y = res.phi.copy()
        y[l] = -y[l]
        assert F.residual_norm(H, S, y, ev[k]) >= base * (1.0 - 1e-12)


def test_penalty_tracks_the_definition(cell):
    H, S, ev, V, col = cell
    rng = np.random.default_rng(7)
    k = H.shape[0] // 2
    ref = V[:, k - 1]
    x = V[:, k].copy()
    x[rng.choice(H.shape[0], 12, replace=False)] *= -1.0
    res = F.local_flip(H, S, x, ev[k], phi_ref=ref, c=F.C_PAPER_EV2, max_sweeps=100, colour=col)
    want = F.residual_norm(H, S, res.phi, ev[k], ref, F.C_PAPER_EV2)
    assert abs(res.R[-1] - want) <= 1e-10 * max(want, 1e-300)
    assert res.R[-1] < res.R[0]
    # without the penalty term the same start is refined differently only through the penalty
    plain = F.local_flip(H, S, x, ev[k], max_sweeps=100, colour=col)
    assert plain.R[-1] == pytest.approx(F.residual_norm(H, S, plain.phi, ev[k]), rel=1e-10)


def test_paper_constant():
    assert F.C_PAPER_EV2 == pytest.approx(5.0 * 27.211386245988 ** 2)


def _penalised_start(V, k, seed, noise=0.02, frac=0.15):
    rng = np.random.default_rng(seed)
    x = V[:, k] + noise * rng.standard_normal(V.shape[0]) * np.abs(V[:, k]).max()
    x[rng.random(V.shape[0]) < frac] *= -1.0
    return x


def _penalised_checks(Fm, H, S, ev, V, col, cases):
    """Failed pin names for a flip oracle module on (seed, c) cases with the penalty of V[:, k-1]."""
    failed = []
    for seed, cpen in cases:
        k = H.shape[0] // 2 + seed % 3
        ref = V[:, k - 1]
        x = _penalised_start(V, k, seed)
        log = []
        try:
            res = Fm.local_flip(H, S, x, ev[k], phi_ref=ref, c=cpen, max_sweeps=200, colour=col, log=log)
        except Exception:
            return ["raised"]
        # replay the logged flips one at a time, R of the definition from scratch
        y = x.copy()
        prev = F.residual_norm(H, S, y, ev[k], ref, cpen)
        scale = prev
        rose = False
        for l in log:
            y[l] = -y[l]
            now = F.residual_norm(H, S, y, ev[k], ref, cpen)
            if now > prev + 1e-12 * scale:
                failed.append(f"rise seed={seed} c={cpen:.3g}")
                rose = True
                break
            prev = now
        if not rose and not np.array_equal(y, res.phi):
            failed.append(f"log seed={seed}")
        want = F.residual_norm(H, S, res.phi, ev[k], ref, cpen)
        if not abs(res.R[-1] - want) <= 1e-10 * max(want, 1e-300):
            failed.append(f"R tracked seed={seed}")
        if res.sweeps < 200:                           # converged: no single flip lowers R
            for l in range(H.shape[0]):
                z = res.phi.copy()
                z[l] = -z[l]
                if F.residual_norm(H, S, z, ev[k], ref, cpen) < want * (1.0 - 1e-12):
                    failed.append(f"not a local minimum seed={seed} row={l}")
                    break
    return failed


PEN_CASES = [(seed, cpen) for seed in range(6) for cpen in (F.C_PAPER_EV2, 50.0 * F.C_PAPER_EV2)]


def test_penalised_descent_per_flip_and_local_minimum(cell):
    H, S, ev, V, col = cell
    assert _penalised_checks(F, H, S, ev, V, col, PEN_CASES) == []


def test_unpenalised_descent_per_flip(cell):
    H, S, ev, V, col = cell
    for seed in range(3):
        k = H.shape[0] // 2 + seed
        x = _penalised_start(V, k, seed, noise=0.05, frac=0.3)
        log = []
        res = F.local_flip(H, S, x, ev[k], max_sweeps=200, colour=col, log=log)
        assert len(log) == res.flips
        y = x.copy()
        prev = F.residual_norm(H, S, y, ev[k])
        for l in log:
            y[l] = -y[l]
            now = F.residual_norm(H, S, y, ev[k])
            assert now <= prev + 1e-12 * res.R[0]
            prev = now
        assert np.array_equal(y, res.phi)


FLIP_SRC = pathlib.Path(__file__).resolve().parent.parent / "oracle" / "mar_flip.py"
PENALTY_MUTANTS = {
    "penalty_cross_sign": ("- 4.0 * a * s[l] * p)", "+ 4.0 * a * s[l] * p)"),
    "penalty_no_square_term": ("d += c * (4.0 * a * a * s[l] * s[l] - 4.0 * a * s[l] * p)",
                               "d += c * (- 4.0 * a * s[l] * p)"),
    "penalty_p_update_sign": ("p = p - (2.0 * a) * s[l]", "p = p + (2.0 * a) * s[l]"),
    "penalty_p_stale_in_colour": (
        "                for l in rows:                        # index order, p as left by the flips before\n",
        "                p_start = p\n"
        "                for l in rows:                        # index order, p as left by the flips before\n"),
    "penalty_p_never_updated": ("p = p - (2.0 * a) * s[l]", "p = p"),
}


def _load(src, name):
    spec = importlib.util.spec_from_loader(name, loader=None)
    mod = importlib.util.module_from_spec(spec)
    sys.modules[name] = mod
    exec(compile(src, f"<{name}>", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(PENALTY_MUTANTS))
def test_penalty_mutant_is_caught(cell, name):
    H, S, ev, V, col = cell
    old, new = PENALTY_MUTANTS[name]
    src = FLIP_SRC.read_text()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    src = src.replace(old, new)
    if name == "penalty_p_stale_in_colour":        # decide on the colour's starting p
        src = src.replace("- 4.0 * a * s[l] * p)", "- 4.0 * a * s[l] * p_start)")
    Fm = _load(src, f"flip_mutant_{name}")
    assert _penalised_checks(Fm, H, S, ev, V, col, PEN_CASES), f"mutant {name} passed every pin"
