"""FP64 CPU oracle of the local flipping refinement of an eigenvector.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test suite,
the smoke check and the bench's CPU-baseline leg may import or run it. It shares
no code with the HIP library.

What it restates (Appendix, after Eq. 3): the signs of the components a_l of a
computed eigenvector phi = (a_1, ..., a_M) of level eps are refined by flipping
single components (a_l -> -a_l), each flip lowering the residual norm
    R = r^T r,   r = (H - eps S) phi,
optionally plus c |phi_ref^T S phi|^2 for an earlier state phi_ref (an effective
orthogonality constraint; the paper uses c = 5 atomic units). The paper notes
that no matrix-vector product is needed: flipping a_l changes r by
-2 a_l (H - eps S) e_l, a column of the sparse matrix, and the penalty's inner
product p = phi_ref^T S phi by -2 a_l (S phi_ref)_l. The paper defers the order
of the flips to a later publication. Readings taken here (listed in the design
notes):
  * flipping a_l alone changes R by
        dR_l = sum_{i in P(l)} A_il (4 a_l^2 A_il - 4 a_l r_i)
               + c (4 a_l^2 s_l^2 - 4 a_l s_l p),   A = H - eps S, s = S phi_ref,
    the first sum taken in the row's column order; l flips when dR_l < 0, so
    every accepted flip lowers R;
  * the components are visited by colour of a distance-2 colouring of the
    graph of H's pattern (greedy, in index order: each row takes the smallest
    colour unused by the earlier rows within two hops), and within a colour in
    index order. Rows of one colour have disjoint column supports, so the
    first sum of dR_l does not depend on the other flips of the colour; without
    the penalty the rows of a colour therefore decide at once on the r of the
    colour's start, which is the same as deciding one after the other. The
    penalty couples every row through p, so with it each row decides on the p
    left by the flips before it (p drops by 2 a_l s_l at each flip): a
    sequential descent in (colour, index) order;
  * one sweep visits every colour once; sweeps repeat until one flips nothing
    or max_sweeps have run;
  * c = 5 atomic units of energy squared is 5 x 27.211386^2 eV^2 for matrices in eV.
Pins (tests/test_oracle_flip.py): the colouring is a valid and greedy-minimal
distance-2 colouring (brute force by matrix powers); replaying the logged flips
one at a time, R recomputed from scratch never rises, with and without the
penalty; the returned state is a local minimum for every single flip (R
recomputed from scratch); the tracked residual equals (H - eps S) phi
recomputed; isolated sign errors on an exact eigenvector are undone exactly;
planted mistakes in the penalty term each break one of these.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

HARTREE_EV = 27.211386245988
C_PAPER_EV2 = 5.0 * HARTREE_EV ** 2     # the paper's c = 5 a.u., for H and S in eV


def distance2_colouring(H) -> np.ndarray:
    """Greedy colour of every row: the smallest colour unused by earlier rows within two hops."""
    P = sp.csr_matrix(H, dtype=np.float64)
    P.data = np.ones_like(P.data)
    P2 = (P @ P + P).tocsr()
    M = P.shape[0]
    colour = np.full(M, -1, dtype=np.int64)
    for l in range(M):
        nb = P2.indices[P2.indptr[l]:P2.indptr[l + 1]]
        used = set(colour[nb[nb < l]].tolist())
        c = 0
        while c in used:
            c += 1
        colour[l] = c
    return colour


def residual_norm(H, S, phi, eps, phi_ref=None, c: float = 0.0) -> float:
    """R = |(H - eps S) phi|^2 (+ c (phi_ref^T S phi)^2), from scratch."""
    r = H @ phi - eps * (S @ phi)
    R = float(r @ r)
    if phi_ref is not None and c:
        p = float(phi_ref @ (S @ phi))
        R += c * p * p
    return R


@dataclass
class FlipResult:
    phi: np.ndarray
    r: np.ndarray            # tracked residual (H - eps S) phi
    R: list                  # R before the first sweep and after each sweep
    sweeps: int              # sweeps run
    flips: int               # total flips


def _row_dot(indptr, indices, vals, x, l):
    """sum over the stored entries of row l, in column order, of vals * x."""
    t = 0.0
    for q in range(indptr[l], indptr[l + 1]):
        t += vals[q] * x[indices[q]]
    return t


def local_flip(H, S, phi, eps: float, phi_ref=None, c: float = 0.0, max_sweeps: int = 100,
               colour=None, log=None) -> FlipResult:
    """Sign-flip refinement of phi for level eps (Appendix), by colours of a distance-2 colouring.

    Sums are taken one term at a time in a fixed order (rows in column order,
    inner products in index order), as the readings above state. When log is
    a list, the index of every accepted flip is appended to it, in the order
    the flips are made (one colour's unpenalised flips in index order).
    """
    H = sp.csr_matrix(H)
    H.sort_indices()
    S = sp.csr_matrix(S)
    M = H.shape[0]
    ip, ix = H.indptr, H.indices
    rows_of = np.repeat(np.arange(M), np.diff(ip))
    sv = np.asarray(S[rows_of, ix]).ravel()          # S on H's pattern (zeros where S stores nothing)
    av = H.data - eps * sv                            # A = H - eps S on H's pattern
    colour = distance2_colouring(H) if colour is None else colour
    order = [np.nonzero(colour == k)[0] for k in range(int(colour.max()) + 1)]
    phi = np.array(phi, dtype=np.float64)
    r = np.array([_row_dot(ip, ix, av, phi, i) for i in range(M)])
    pen = phi_ref is not None and c != 0.0
    if pen:
        s = np.array([_row_dot(ip, ix, sv, np.asarray(phi_ref, dtype=np.float64), i) for i in range(M)])
        p = 0.0
        for l in range(M):
            p += s[l] * phi[l]
    else:
        s, p = None, 0.0
    R = [float(r @ r) + (c * p * p if pen else 0.0)]
    flips = 0
    sweeps = 0
    for _ in range(max_sweeps):
        sweeps += 1
        n_sweep = 0
        for rows in order:
            if pen:
                for l in rows:                        # index order, p as left by the flips before
                    a = phi[l]
                    d = 0.0
                    for q in range(ip[l], ip[l + 1]):
                        d += av[q] * (4.0 * a * a * av[q] - 4.0 * a * r[ix[q]])
                    d += c * (4.0 * a * a * s[l] * s[l] - 4.0 * a * s[l] * p)
                    if d < 0.0:
                        for q in range(ip[l], ip[l + 1]):
                            r[ix[q]] = r[ix[q]] - (2.0 * a) * av[q]
                        p = p - (2.0 * a) * s[l]
                        phi[l] = -a
                        n_sweep += 1
                        if log is not None:
                            log.append(int(l))
                continue
            chosen = []
            for l in rows:                            # all on the r of the colour's start
                a = phi[l]
                d = 0.0
                for q in range(ip[l], ip[l + 1]):
                    d += av[q] * (4.0 * a * a * av[q] - 4.0 * a * r[ix[q]])
                if d < 0.0:
                    chosen.append(l)
            for l in chosen:                          # disjoint supports: order immaterial
                a = phi[l]
                for q in range(ip[l], ip[l + 1]):     # A symmetric: column l = row l
                    r[ix[q]] = r[ix[q]] - (2.0 * a) * av[q]
                phi[l] = -a
                if log is not None:
                    log.append(int(l))
            n_sweep += len(chosen)
        flips += n_sweep
        R.append(float(r @ r) + (c * p * p if pen else 0.0))
        if n_sweep == 0:
            break
    return FlipResult(phi=phi, r=r, R=R, sweeps=sweeps, flips=flips)
