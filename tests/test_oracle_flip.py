"""Pins of the local flipping oracle (Appendix: sign-flip refinement of an eigenvector), on the CPU.

The pins tie the oracle to things other than itself: brute-force distance-2
reachability by dense matrix powers (validity and greedy minimality of the
colouring), R recomputed from scratch with sparse products (monotone descent,
local minimality, tracked residual, the penalty term), and the exact
eigenvector of LAPACK's generalized solver (sign errors on first-colour rows
are undone in the first colour).
"""
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
