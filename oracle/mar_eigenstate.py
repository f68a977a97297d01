"""FP64 CPU oracle of the eigen-state extension of the mArnoldi method.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test suite,
the smoke check and the bench's CPU-baseline leg may import or run it. It shares
no code with the HIP library.

What it restates (Sec. 3, Eq. 3, and the Appendix):
  * summed over all seeds, the projected Green's functions count the states
    below an energy eta:
    n(eta) = sum_j sum_alpha w_alpha^(j) theta(eta - eps_alpha^(j)), with the
    weights w_alpha^(j) = (e_j^T S v_alpha^(j)) (v_alpha^(j)^T e_j) of the
    projected Green's function; eta(n) inverts that count;
  * level k (k = 1, 2, ...) sits where the count is k - 1/2: eps_k = eta(k - 1/2);
  * the j-th component of the k-th eigenvector is Eq. 3:
        e_j^T phi_k = sum_alpha (e_j^T v_alpha^(j)) int_{eta(k-1)}^{eta(k)} d(eps - eps_alpha^(j)) deps
    with d a smoothed delta function;
  * every subspace eigenvector may be flipped (v -> -v); the inner-product
    method (Appendix) takes as reference the subspace eigenvector that
    contributes most to phi_k and flips each v_alpha^(j) so that
    v_ref . v_alpha^(j) > 0.
Readings where the paper is silent (listed in the design notes):
  * the smoothed delta is the derivative of the logistic step of width sigma,
    so the window integral is F((b - eps)/sigma) - F((a - eps)/sigma) with
    F(x) = 1/(1 + e^-x); sigma = 0 is the sharp window (1/2 at an endpoint);
  * n(eta) uses the same smoothed step, theta(x) -> F(x/sigma): n is then
    strictly increasing where the weights are positive and eta(k) falls inside
    the gap between the k-th and (k+1)-th levels instead of anywhere on the
    plateau of the sharp count (sigma = 0: the sharp step, 1/2 at 0);
  * eta(n) is found by 200 bisection halvings of [min eps - 1 eV, max eps + 1 eV];
  * the subspace eigenvector that contributes most is the one with the largest
    |(e_j^T v_alpha^(j)) x window|; a zero inner product counts as positive.
Pins (tests/test_oracle_eigenstate.py): at nu = M the subspace eigenvectors are
exact, so eps_k must equal the k-th generalized eigenvalue and phi_k the
S-normalized eigenvector up to one global sign; n(eta) is monotone with
n(+inf) = number of seeds when S = I; flipping subspace eigenvectors other than
the reference leaves phi_k unchanged.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from oracle import mar_oracle as O


def step(x):
    """Unit step with theta(0) = 1/2."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(x > 0.0, 1.0, np.where(x < 0.0, 0.0, 0.5))


def logistic(x):
    """F(x) = 1/(1 + e^-x), evaluated without overflow."""
    x = np.asarray(x, dtype=np.float64)
    t = np.exp(-np.abs(x))
    return np.where(x >= 0.0, 1.0 / (1.0 + t), t / (1.0 + t))


def window(eps, a: float, b: float, sigma: float):
    """Integral of the smoothed delta d(e - eps) over e in [a, b]."""
    if sigma == 0.0:
        return step(b - np.asarray(eps)) - step(a - np.asarray(eps))
    return logistic((b - np.asarray(eps)) / sigma) - logistic((a - np.asarray(eps)) / sigma)


def smoothed_step(x, sigma: float):
    """theta(x) for sigma = 0 (1/2 at 0), else the logistic step F(x / sigma)."""
    return step(x) if sigma == 0.0 else logistic(np.asarray(x, dtype=np.float64) / sigma)


def integrated_dos(eps_list, w_list, eta: float, sigma: float = 0.0) -> float:
    """n(eta) = sum_j sum_alpha w_alpha^(j) theta(eta - eps_alpha^(j)), theta smoothed to width sigma."""
    return math.fsum(float(np.dot(smoothed_step(eta - e, sigma), w)) for e, w in zip(eps_list, w_list))


def level_of_count(eps_list, w_list, n: float, sigma: float = 0.0, iters: int = 200) -> float:
    """eta(n): the level below which the integrated density of states reaches n (bisection)."""
    lo = min(float(np.min(e)) for e in eps_list) - 1.0
    hi = max(float(np.max(e)) for e in eps_list) + 1.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if integrated_dos(eps_list, w_list, mid, sigma) < n:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@dataclass
class SubspaceStates:
    j: int
    eps: np.ndarray       # subspace eigen levels, ascending
    weight: np.ndarray    # w_alpha = (e_j^T S v_alpha)(v_alpha^T e_j)
    V: np.ndarray         # (M, nu_eff) subspace eigenvectors v_alpha = K y_alpha as columns


def subspace_states(H, S, seeds, nu: int, tau: float = O.TAU_FP64):
    """Every listed seed's subspace eigenpairs with the full vectors kept (small M only)."""
    H = sp.csr_matrix(H)
    S = sp.csr_matrix(S)
    out = []
    for j in seeds:
        j = int(j)
        U, h, _ = O.krylov_basis(H, S, j, nu, tau)
        A = O.subspace_matrix(h)
        eps, Y = np.linalg.eigh(A)
        V = U.T @ Y
        srow = S.getrow(j).toarray().ravel()
        out.append(SubspaceStates(j=j, eps=eps, weight=(srow @ V) * V[j], V=V))
    return out


@dataclass
class EigenState:
    k: int
    eps_k: float          # eta(k - 1/2)
    eta_lo: float         # eta(k - 1)
    eta_hi: float         # eta(k)
    phi: np.ndarray       # e_j^T phi_k for the listed seeds, in their order
    ref: tuple            # (position of the reference seed in the list, alpha)


def eigen_state(states, k: int, sigma: float, sign_method: bool = True) -> EigenState:
    """The k-th eigen level and vector components (Sec. 3, Eq. 3; Appendix)."""
    eps_list = [s.eps for s in states]
    w_list = [s.weight for s in states]
    eta_lo = level_of_count(eps_list, w_list, k - 1.0, sigma)
    eta_hi = level_of_count(eps_list, w_list, float(k), sigma)
    eps_k = level_of_count(eps_list, w_list, k - 0.5, sigma)
    contrib = [s.V[s.j] * window(s.eps, eta_lo, eta_hi, sigma) for s in states]
    best, ref = -1.0, (0, 0)
    for p, c in enumerate(contrib):
        a = int(np.argmax(np.abs(c)))
        if abs(c[a]) > best:
            best, ref = abs(c[a]), (p, a)
    vref = states[ref[0]].V[:, ref[1]]
    phi = np.zeros(len(states))
    for p, (s, c) in enumerate(zip(states, contrib)):
        sgn = np.where(vref @ s.V >= 0.0, 1.0, -1.0) if sign_method else np.ones(len(c))
        phi[p] = float(np.sum(sgn * c))
    return EigenState(k=k, eps_k=eps_k, eta_lo=eta_lo, eta_hi=eta_hi, phi=phi, ref=ref)
