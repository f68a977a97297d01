"""Pins of the local-region oracle (order-N form of the method), on the CPU.

Each pin ties the oracle to something other than itself: the full-method
oracle where the truncation cannot act (r >= nu - 1), LAPACK's dense
generalized eigensolver where the subspace exhausts the region, brute-force
reachability by matrix powers for the region, and invariance / sensitivity to
entries outside / inside the region.
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

from oracle import mar_local as L
from oracle import mar_oracle as O
from paper_1307_3218_amd import lattice

KT = 0.1


@pytest.fixture(scope="module")
def sysm():
    return lattice.generate(3, 3, 3, mixed=True, seed=5)      # 216 atoms, M = 864


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_region_matches_matrix_powers(sysm):
    """Blocks within r hops = nonzero pattern of (A + I)^r applied to the seed's block."""
    G = L.block_graph(sysm.H)
    A = (G != 0).astype(np.int64).toarray()
    for j, r in ((0, 0), (5, 1), (400, 2), (863, 3)):
        x = np.zeros(A.shape[0], dtype=np.int64)
        x[j // 4] = 1
        for _ in range(r):
            x = np.minimum(A @ x, 1)
        blocks = np.nonzero(x)[0]
        rows = (blocks[:, None] * 4 + np.arange(4)).ravel()
        assert np.array_equal(L.region(G, sysm.M, j, r), rows)


@pytest.mark.parametrize("nu", [3, 6, 9])
def test_wide_region_is_the_full_method(sysm, nu):
    """The first nu Krylov vectors stay within nu - 1 hops: r >= nu - 1 changes nothing."""
    seeds = [0, 17, 301, 862]
    full = O.solve(sysm.H, sysm.S, seeds, nu, -0.3, KT)
    for r in (nu - 1, nu + 2):
        loc = L.solve_local(sysm.H, sysm.S, seeds, nu, r, -0.3, KT)
        assert np.array_equal(loc.nu_eff, full.nu_eff)
        assert _rel(loc.rho, full.rho) < 1e-12
        assert abs(loc.e_band - full.e_band) < 1e-12 * abs(full.e_band)


def test_narrow_region_truncates(sysm):
    """r < nu - 1 is a different (truncated) subspace: the result must move."""
    seeds = [0, 17, 301, 862]
    full = O.solve(sysm.H, sysm.S, seeds, 8, -0.3, KT)
    loc = L.solve_local(sysm.H, sysm.S, seeds, 8, 2, -0.3, KT)
    assert _rel(loc.rho, full.rho) > 1e-6


@pytest.mark.parametrize("r", [0, 1])
def test_exhausted_region_is_exact(sysm, r):
    """nu >= |R|: rho_ij equals the dense density matrix of the region's pair (H_R, S_R)."""
    H, S = sp.csr_matrix(sysm.H), sp.csr_matrix(sysm.S)
    G = L.block_graph(H)
    for j in (2, 333, 700):
        R = L.region(G, sysm.M, j, r)
        loc = L.solve_local(H, S, [j], len(R) + 5, r, -0.3, KT)
        Hd, Sd = H[R][:, R].toarray(), S[R][:, R].toarray()
        eps, phi = scipy.linalg.eigh(Hd, Sd)
        f = O.fermi(eps, -0.3, KT)
        rho_d = 2.0 * (phi * f[None, :]) @ phi.T
        jl = int(np.searchsorted(R, j))
        lo, hi = H.indptr[j], H.indptr[j + 1]
        want = np.array([rho_d[int(np.searchsorted(R, i)), jl] if i in set(R.tolist()) else 0.0
                         for i in H.indices[lo:hi]])
        assert np.abs(loc.rho[lo:hi] - want).max() < 1e-9 * max(1.0, np.abs(want).max())


def test_entries_outside_region_do_not_matter(sysm):
    H, S = sp.csr_matrix(sysm.H).copy(), sp.csr_matrix(sysm.S).copy()
    j, r, nu = 100, 2, 12
    G = L.block_graph(H)
    R = set(L.region(G, sysm.M, j, r).tolist())
    base = L.solve_local(H, S, [j], nu, r, -0.3, KT)
    # scale every stored entry with both ends outside the region (keeps symmetry and S positive definite)
    Hc, Sc = H.tocoo(), S.tocoo()
    out_h = np.array([(a not in R) and (b not in R) for a, b in zip(Hc.row, Hc.col)])
    out_s = np.array([(a not in R) and (b not in R) for a, b in zip(Sc.row, Sc.col)])
    H2 = sp.csr_matrix((np.where(out_h, 3.0 * Hc.data, Hc.data), (Hc.row, Hc.col)), shape=H.shape)
    S2 = sp.csr_matrix((np.where(out_s, 0.5 * Sc.data, Sc.data), (Sc.row, Sc.col)), shape=S.shape)
    moved = L.solve_local(H2, S2, [j], nu, r, -0.3, KT)
    assert np.array_equal(moved.rho, base.rho) and moved.e_band == base.e_band
    # and an entry inside the region does
    ins = np.array([(a in R) and (b in R) and a != b for a, b in zip(Hc.row, Hc.col)])
    H3 = sp.csr_matrix((np.where(ins, 1.1 * Hc.data, Hc.data), (Hc.row, Hc.col)), shape=H.shape)
    inside = L.solve_local(H3, S, [j], nu, r, -0.3, KT)
    assert _rel(inside.rho, base.rho) > 1e-6
