"""Fermi level from the subspace eigen levels and weights returned by the GPU.

Host-side helper (not part of the timed hot path; the level mu is an input of
mar_solve). The Green's function of Sec. 2 built from the subspace levels
eps_alpha^(j) and weights w_alpha^(j) = (e_j^T S v_alpha)(v_alpha^T e_j)
gives the electron count
    N(mu) = sum_j 2 sum_alpha f((eps_alpha^(j) - mu) / kT) w_alpha^(j),
f(x) = 1/(1+e^x); mu is found by bisection so that N(mu) equals a target
(half filling: N = M for four valence electrons on four orbitals per atom).
"""
from __future__ import annotations

import numpy as np


def occupation(eps: np.ndarray, mu: float, kT: float) -> np.ndarray:
    eps = np.asarray(eps, dtype=np.float64)
    if kT == 0.0:
        return np.where(eps < mu, 1.0, np.where(eps > mu, 0.0, 0.5))
    x = (eps - mu) / kT
    t = np.exp(-np.abs(x))
    return np.where(x >= 0.0, t / (1.0 + t), 1.0 / (1.0 + t))


def electron_count(eps: np.ndarray, weight: np.ndarray, nu_eff: np.ndarray, mu: float, kT: float) -> float:
    """eps, weight: (n_seeds, nu) with entries beyond nu_eff ignored."""
    eps = np.asarray(eps)
    mask = np.arange(eps.shape[1])[None, :] < np.asarray(nu_eff)[:, None]
    return float(2.0 * np.sum(np.where(mask, occupation(eps, mu, kT) * weight, 0.0)))


def fermi_level(eps, weight, nu_eff, n_target: float, kT: float, iters: int = 200) -> float:
    eps = np.asarray(eps)
    mask = np.arange(eps.shape[1])[None, :] < np.asarray(nu_eff)[:, None]
    lo = float(eps[mask].min()) - 40.0 * kT
    hi = float(eps[mask].max()) + 40.0 * kT
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if electron_count(eps, weight, nu_eff, mid, kT) < n_target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)
