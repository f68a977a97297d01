"""Eigen states on the GPU (mar_eigen_state): the k-th level eps_k = eta(k - 1/2)
and the components e_j^T phi_k of Eq. 3 with the inner-product sign method.

At nu = M (every subspace is the whole space) the result must be the exact
generalized eigenpair (LAPACK) up to one global sign, the vector at the FP64 bar
(the levels tested lie 0.5-9 % of the spectral scale from their neighbours, so two
eigensolvers agree on the vector to about 1e-13); at nu < M it must match the
eigen-state oracle (oracle/mar_eigenstate.py) on the same seeds, at the bars of the
two forms (FP64 1e-10, FP32 1e-5): phi relative to its norm (up to one global sign),
the level eps_k relative to the spectral scale max |eps|. The bisection points
eta(k - 1) and eta(k) lie in gaps of the integrated density of states, where it is
flat to within the smoothing, so they are compared with the oracle's to 1e-3 of the
spectral scale in FP32 (FP64: 1e-10); they enter phi only through the window, which
is flat there too.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import mar_eigenstate as ES
from paper_1307_3218_amd import lattice, mar

pytestmark = pytest.mark.gpu


def _sign_free(a, b):
    return min(np.linalg.norm(a - b), np.linalg.norm(a + b)) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def small():
    s = lattice.generate(2, 1, 1)
    ev, V = scipy.linalg.eigh(s.H.toarray(), s.S.toarray())
    ctx = mar.Context(s.H, s.S)
    yield s, ev, V, ctx
    ctx.close()


@pytest.mark.parametrize("form", ["batched", "plain"])
@pytest.mark.parametrize("k", [1, 32, 33, 64])
def test_exact_state_at_nu_M(small, form, k):
    s, ev, V, ctx = small
    seeds = np.arange(s.M, dtype=np.int32)
    out = ctx.eigen_state(seeds, s.M, k, 1e-6, "fp64", form)
    err = _sign_free(out["phi"], V[:, k - 1])
    print(f"[es exact {form} k={k}] eps_k {out['eps_k']:.12f} exact {ev[k - 1]:.12f} phi err {err:.2e} "
          f"ref {out['ref']}", flush=True)
    assert abs(out["eps_k"] - ev[k - 1]) <= 1e-9
    assert out["eta_lo"] < out["eps_k"] < out["eta_hi"]
    assert err <= 1e-10


@pytest.fixture(scope="module")
def cell256_states(cell256):
    return ES.subspace_states(cell256.H, cell256.S, np.arange(cell256.M), 30)


@pytest.mark.parametrize("k", [128, 129])
def test_cell256_state_against_oracle(cell256, cell256_states, k):
    sigma = 0.02
    ref = ES.eigen_state(cell256_states, k, sigma)
    ctx = mar.Context(cell256.H, cell256.S)
    try:
        scale = max(np.abs(st.eps).max() for st in cell256_states)
        for prec, bar in (("fp64", 1e-10), ("fp32", 1e-5)):
            out = ctx.eigen_state(np.arange(cell256.M, dtype=np.int32), 30, k, sigma, prec, "batched")
            err = _sign_free(out["phi"], ref.phi)
            print(f"[es cell256 k={k} {prec}] eps_k {out['eps_k']:.10f} oracle {ref.eps_k:.10f} phi err {err:.2e} "
                  f"ref {out['ref'][:2]} oracle ref {ref.ref}", flush=True)
            gap_bar = 1e-10 if prec == "fp64" else 1e-3
            assert abs(out["eps_k"] - ref.eps_k) <= bar * scale
            assert abs(out["eta_lo"] - ref.eta_lo) <= gap_bar * scale
            assert abs(out["eta_hi"] - ref.eta_hi) <= gap_bar * scale
            assert err <= bar
    finally:
        ctx.close()


def test_eigen_state_argument_errors(small):
    s, ev, V, ctx = small
    seeds = np.arange(8, dtype=np.int32)
    for k, sigma in ((0, 0.1), (9, 0.1), (1, -1.0)):
        with pytest.raises(mar.MarError) as e:
            ctx.eigen_state(seeds, 8, k, sigma)
        assert e.value.status == mar.MAR_ERR_ARG
