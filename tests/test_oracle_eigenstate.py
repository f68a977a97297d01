"""Pins of the eigen-state oracle (Sec. 3, Eq. 3; Appendix inner-product method).

At nu = M every subspace is the whole space, so the subspace eigenvectors are
exact eigenvectors: eps_k = eta(k - 1/2) must be the k-th generalized eigenvalue
of H phi = eps S phi and Eq. 3 with the sign method must give the S-normalized
eigenvector phi_k up to one global sign (checked against LAPACK's generalized
symmetric-definite solver). Also: n(eta) counts exact eigenvalues at nu = M,
n(+inf) = number of seeds, closed forms for one seed, invariance under flips of
non-reference subspace eigenvectors, and a mutant without the sign method.
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

from oracle import mar_eigenstate as ES
from paper_1307_3218_amd import lattice

SIGMA = 1e-6


@pytest.fixture(scope="module")
def small():
    """128-orbital periodic diamond cell (2x1x1 conventional cells); min level gap 0.047 eV."""
    s = lattice.generate(2, 1, 1)
    ev, V = scipy.linalg.eigh(s.H.toarray(), s.S.toarray())
    states = ES.subspace_states(s.H, s.S, np.arange(s.M), s.M)
    return s, ev, V, states


@pytest.mark.parametrize("k", [1, 2, 17, 32, 33, 64])
def test_exact_level_and_vector_at_nu_M(small, k):
    s, ev, V, states = small
    st = ES.eigen_state(states, k, SIGMA)
    assert abs(st.eps_k - ev[k - 1]) <= 1e-9
    assert ev[k - 2] < st.eta_lo < ev[k - 1] < st.eta_hi if k > 1 else st.eta_lo < ev[0] < st.eta_hi
    exact = V[:, k - 1]          # S-normalized by the solver
    err = min(np.linalg.norm(st.phi - exact), np.linalg.norm(st.phi + exact))
    assert err <= 1e-12, err


def test_integrated_dos_counts_exact_levels(small):
    s, ev, V, states = small
    eps = [x.eps for x in states]
    w = [x.weight for x in states]
    assert abs(ES.integrated_dos(eps, w, 1e6) - s.M) <= 1e-10
    assert abs(ES.integrated_dos(eps, w, -1e6)) == 0.0
    # between two levels n(eta) is the count of levels below
    for k in (1, 10, 40, 63):
        mid = 0.5 * (ev[k - 1] + ev[k])
        assert abs(ES.integrated_dos(eps, w, mid) - k) <= 1e-9


def test_integrated_dos_monotone_for_identity_overlap():
    s = lattice.generate(1, 1, 1)
    I = sp.identity(s.M, format="csr")
    states = ES.subspace_states(s.H, I, np.arange(s.M), 8)
    eps = [x.eps for x in states]
    w = [x.weight for x in states]
    assert all((x >= -1e-15).all() for x in w)     # w = (e_j . v)^2 when S = I
    grid = np.linspace(-25.0, 25.0, 101)
    vals = [ES.integrated_dos(eps, w, g) for g in grid]
    assert all(b >= a - 1e-12 for a, b in zip(vals, vals[1:]))
    assert abs(vals[-1] - s.M) <= 1e-10


def test_one_seed_closed_form():
    st = [ES.SubspaceStates(j=0, eps=np.array([-1.0, 2.0]), weight=np.array([0.3, 0.7]), V=np.eye(2))]
    eps, w = [st[0].eps], [st[0].weight]
    assert ES.integrated_dos(eps, w, -1.0) == pytest.approx(0.15)    # theta(0) = 1/2
    assert ES.integrated_dos(eps, w, 0.0) == pytest.approx(0.3)
    assert ES.level_of_count(eps, w, 0.15) == pytest.approx(-1.0, abs=1e-12)
    assert ES.level_of_count(eps, w, 0.5) == pytest.approx(2.0, abs=1e-12)
    # smoothed count: n(eps_1) = 0.3 F(0) + 0.7 F(-3/sigma); the count 0.3 is reached in the gap
    assert ES.integrated_dos(eps, w, -1.0, 0.01) == pytest.approx(0.15)
    mid = ES.level_of_count(eps, w, 0.3, 0.01)
    assert -1.0 + 0.2 < mid < 2.0 - 0.2
    # sharp window: half weight at an endpoint
    assert ES.window(np.array([2.0]), 0.0, 2.0, 0.0)[0] == 0.5
    assert ES.window(np.array([1.0]), 0.0, 2.0, 0.0)[0] == 1.0
    # logistic window: symmetric about the midpoint, tends to the sharp one
    a = ES.window(np.array([1.0]), 0.0, 2.0, 0.1)[0]
    assert a == pytest.approx(1.0 - 2.0 * ES.logistic(-10.0))


def test_flips_of_non_reference_vectors_do_not_change_phi(small):
    s, ev, V, states = small
    k = 33
    st = ES.eigen_state(states, k, SIGMA)
    rng = np.random.default_rng(3)
    flipped = []
    for p, x in enumerate(states):
        Vf = x.V.copy()
        for a in range(Vf.shape[1]):
            if (p, a) != st.ref and rng.random() < 0.5:
                Vf[:, a] = -Vf[:, a]
        flipped.append(ES.SubspaceStates(j=x.j, eps=x.eps, weight=x.weight, V=Vf))
    st2 = ES.eigen_state(flipped, k, SIGMA)
    assert st2.ref == st.ref
    assert np.abs(st2.phi - st.phi).max() <= 1e-14


def test_mutant_without_sign_method_misses_the_vector(small):
    """Without the inner-product method the per-seed signs are arbitrary."""
    s, ev, V, states = small
    rng = np.random.default_rng(5)
    flipped = [ES.SubspaceStates(j=x.j, eps=x.eps, weight=x.weight,
                                 V=x.V * np.where(rng.random(x.V.shape[1]) < 0.5, -1.0, 1.0)[None, :])
               for x in states]
    k = 33
    exact = V[:, k - 1]
    good = ES.eigen_state(flipped, k, SIGMA)
    bad = ES.eigen_state(flipped, k, SIGMA, sign_method=False)
    err = lambda phi: min(np.linalg.norm(phi - exact), np.linalg.norm(phi + exact))
    assert err(good.phi) <= 1e-12
    assert err(bad.phi) > 0.1
