"""FP64 CPU oracle of the local-region (order-N) form of the mArnoldi method.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test suite,
the smoke check and the bench's CPU-baseline leg may import or run it. It shares
no code with the HIP library.

What it restates. The paper gives the cost of the method as proportional to the
number of atoms (Sec. 1, which points to the scaling figure of the mArnoldi
paper it cites), so the work of one seed must not grow with the system. How the
subspace is kept local is left to the cited paper. Reading taken here (listed in
the design notes):
  * the local region R_j of seed j is the set of rows whose 4-row block lies
    within r hops of j's block in the graph of H's 4x4 block pattern (a block is
    its own neighbour; r = 0 keeps j's block alone);
  * the method of Sec. 2 then runs unchanged on the principal submatrices
    H[R_j, R_j] and S[R_j, R_j] (Krylov subspace from e_j, S-orthonormal CGS2
    basis, nu x nu subspace eigenproblem, Fermi-weighted residues);
  * rho_ij for i in P(j) outside R_j is zero, and E_j, N_j sum over P(j) as in
    the full method.
Pins (tests/test_oracle_local.py): r >= nu - 1 gives the full method (the first
nu Krylov vectors never leave r hops); nu >= |R_j| gives the exact density
matrix of the submatrix pair (dense generalized eigensolve); entries of H and S
outside R_j do not matter and entries inside do; the region equals the rows
reached by r products with the block pattern plus the identity.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from oracle import mar_oracle as O


def block_graph(H) -> sp.csr_matrix:
    """Adjacency of the 4-row blocks of H's pattern (block I ~ J if some H_ij, i in I, j in J, is stored)."""
    H = sp.csr_matrix(H)
    M = H.shape[0]
    nb = (M + 3) // 4
    C = H.tocoo()
    G = sp.csr_matrix((np.ones(len(C.row)), (C.row // 4, C.col // 4)), shape=(nb, nb))
    G = G + sp.identity(nb, format="csr")
    G.sum_duplicates()
    return G


def region(G: sp.csr_matrix, M: int, j: int, r: int) -> np.ndarray:
    """Sorted rows of the blocks within r hops of row j's block (breadth-first search)."""
    seen = {j // 4}
    frontier = [j // 4]
    for _ in range(r):
        nxt = []
        for I in frontier:
            for J in G.indices[G.indptr[I]:G.indptr[I + 1]]:
                if J not in seen:
                    seen.add(int(J))
                    nxt.append(int(J))
        frontier = nxt
    blocks = np.array(sorted(seen), dtype=np.int64)
    rows = (blocks[:, None] * 4 + np.arange(4)[None, :]).ravel()
    return rows[rows < M]


def solve_seed_local(H, S, G, j: int, nu: int, r: int, mu: float, kT: float, tau: float = O.TAU_FP64):
    """One seed on its local region; rho over the full row P(j) of H (zero outside the region)."""
    M = H.shape[0]
    R = region(G, M, j, r)
    Hs = H[R][:, R]
    Ss = S[R][:, R]
    jl = int(np.searchsorted(R, j))
    res = O.solve_seed(Hs, Ss, jl, nu, mu, kT, tau)
    lo, hi = H.indptr[j], H.indptr[j + 1]
    rho_row = np.zeros(hi - lo)
    pos = {int(R[c]): v for c, v in zip(res.cols, res.rho_row)}
    for t, i in enumerate(H.indices[lo:hi]):
        rho_row[t] = pos.get(int(i), 0.0)
    hv = H.data[lo:hi]
    sv = S.getrow(j).toarray().ravel()[H.indices[lo:hi]]
    return dict(j=j, nu_eff=res.nu_eff, eps=res.eps, weight=res.weight, rho_row=rho_row,
                E=float(rho_row @ hv), N=float(rho_row @ sv), region=R)


def solve_local(H, S, seeds, nu: int, r: int, mu: float, kT: float, tau: float = O.TAU_FP64) -> O.SolveResult:
    """Every listed seed on its own region; the same result record as the full oracle."""
    H = sp.csr_matrix(H)
    S = sp.csr_matrix(S)
    G = block_graph(H)
    res = [solve_seed_local(H, S, G, int(j), nu, r, mu, kT, tau) for j in seeds]
    rho = np.zeros(H.nnz)
    for q in res:
        lo = H.indptr[q["j"]]
        rho[lo: lo + len(q["rho_row"])] = q["rho_row"]
    e_seed = np.array([q["E"] for q in res])
    return O.SolveResult(rho=rho, e_band=math.fsum(e_seed), e_seed=e_seed,
                         n_seed=np.array([q["N"] for q in res]),
                         nu_eff=np.array([q["nu_eff"] for q in res], dtype=np.int32),
                         eps=[q["eps"] for q in res], weight=[q["weight"] for q in res])
