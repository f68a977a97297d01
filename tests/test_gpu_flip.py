"""Local flipping refinement (Appendix) on the GPU against the flip oracle.

The decisions are comparisons of FP64 sums taken in the same order on both
sides with separately rounded products, so the refined vector, the sweep and
flip counts must agree exactly and the residual history to rounding. With the
orthogonality penalty the rows of a colour decide one after the other on the
current p, so the penalised R never rises from sweep to sweep.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import mar_flip as OF
from paper_1307_3218_amd import lattice, mar

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[(2, 2, 1), (4, 4, 4)], ids=["M128", "M2048"])
def case(request):
    s = lattice.generate(*request.param, mixed=True, seed=1)
    H, S = s.H.tocsr(), s.S.tocsr()
    ev, V = scipy.linalg.eigh(H.toarray(), S.toarray())
    ctx = mar.Context(H, S)
    yield H, S, ev, V, ctx
    ctx.close()


def _start(V, k, seed, noise=0.05, frac=0.3):
    rng = np.random.default_rng(seed)
    x = V[:, k] + noise * rng.standard_normal(V.shape[0]) * np.abs(V[:, k]).max()
    x[rng.random(V.shape[0]) < frac] *= -1.0
    return x


def test_colouring_matches(case):
    H, S, ev, V, ctx = case
    assert ctx.flip_colours() == int(OF.distance2_colouring(H).max()) + 1


@pytest.mark.parametrize("seed", [0, 1])
def test_flip_matches_oracle(case, seed):
    H, S, ev, V, ctx = case
    k = H.shape[0] // 2 + seed
    x = _start(V, k, seed)
    ref = OF.local_flip(H, S, x, ev[k], max_sweeps=60)
    g = ctx.local_flip(x, ev[k], max_sweeps=60)
    print(f"[flip M={H.shape[0]}] sweeps {g['sweeps']} flips {g['flips']} R {g['R'][0]:.3e} -> {g['R'][-1]:.3e}",
          flush=True)
    assert g["sweeps"] == ref.sweeps and g["flips"] == ref.flips
    assert np.array_equal(g["phi"], ref.phi)
    np.testing.assert_allclose(g["R"], ref.R, rtol=1e-10, atol=1e-14 * ref.R[0])
    assert g["R"][-1] < g["R"][0]


@pytest.mark.parametrize("seed,cscale", [(5, 1.0), (2, 50.0), (7, 50.0)])
def test_flip_with_penalty_matches_oracle(case, seed, cscale):
    """With the orthogonality penalty every row decides on the p left by the flips before it (a sequential
    descent): the penalised R never rises, on the device as in the oracle."""
    H, S, ev, V, ctx = case
    k = H.shape[0] // 2
    x = _start(V, k, seed, noise=0.02, frac=0.1 if seed == 5 else 0.2)
    c = cscale * OF.C_PAPER_EV2
    ref = OF.local_flip(H, S, x, ev[k], phi_ref=V[:, k - 1], c=c, max_sweeps=60)
    g = ctx.local_flip(x, ev[k], phi_ref=V[:, k - 1], c=c, max_sweeps=60)
    print(f"[flip penalty M={H.shape[0]} c={c:.3g}] sweeps {g['sweeps']} flips {g['flips']} "
          f"R {g['R'][0]:.3e} -> {g['R'][-1]:.3e}", flush=True)
    assert g["sweeps"] == ref.sweeps and g["flips"] == ref.flips
    assert np.array_equal(g["phi"], ref.phi)
    np.testing.assert_allclose(g["R"], ref.R, rtol=1e-10)
    assert all(b <= a * (1.0 + 1e-12) for a, b in zip(g["R"], g["R"][1:]))
    assert g["R"][-1] == pytest.approx(OF.residual_norm(H, S, g["phi"], ev[k], V[:, k - 1], c), rel=1e-10)


def test_first_colour_errors_undone(case):
    H, S, ev, V, ctx = case
    k = H.shape[0] // 3
    col = OF.distance2_colouring(H)
    x = V[:, k].copy()
    x[np.nonzero(col == 0)[0][::3]] *= -1.0
    g = ctx.local_flip(x, ev[k], max_sweeps=10)
    assert np.array_equal(g["phi"], V[:, k]) and g["sweeps"] == 2


def test_zero_sweeps_and_errors(case):
    H, S, ev, V, ctx = case
    x = _start(V, 3, 9)
    g = ctx.local_flip(x, ev[3], max_sweeps=0)
    assert np.array_equal(g["phi"], x) and g["sweeps"] == 0 and len(g["R"]) == 1
    assert g["R"][0] == pytest.approx(OF.residual_norm(H, S, x, ev[3]), rel=1e-12)
    with pytest.raises(mar.MarError):
        ctx.local_flip(x, ev[3], c=-1.0)
    with pytest.raises(mar.MarError):
        ctx.local_flip(x, float("nan"))
    with pytest.raises(mar.MarError):
        ctx.local_flip(x, ev[3], max_sweeps=-1)
    assert mar.mar_local_flip(ctx.handle, None, 0.0, None, 0.0, 1, None, None, None) == mar.MAR_ERR_ARG


def test_refines_an_eigen_state():
    """Eq. 3 output (nu < M, every seed) refined by flips: R drops, as the oracle's does on the same input."""
    s = lattice.workload("diamond_2x2x2")
    H, S = s.H.tocsr(), s.S.tocsr()
    ctx = mar.Context(H, S)
    try:
        st = ctx.eigen_state(np.arange(s.M), 16, s.M // 2, 0.002, precision="fp64")
        phi = st["phi"]
        eps = st["eps_k"]
        ref = OF.local_flip(H, S, phi, eps, max_sweeps=50)
        g = ctx.local_flip(phi, eps, max_sweeps=50)
        assert np.array_equal(g["phi"], ref.phi) and g["flips"] == ref.flips
        assert g["R"][-1] <= g["R"][0]
    finally:
        ctx.close()
