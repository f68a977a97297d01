"""Planted-mistake checks: each plausible slip in the oracle must break a pin.

A textual mutation is applied to a copy of the oracle's source, the copy is
loaded as a fresh module, and a compact set of pin checks (the same facts as in
test_oracle_pins.py: nu = M exactness against Eq. (2), nu = 1 closed form with
S_jj != 1, occupation sum rules, K^T S K = I) is run against it. The unmodified
oracle must pass every check; every mutant must fail at least one.
"""
import importlib.util
import math
import pathlib
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from paper_1307_3218_amd import lattice

ORACLE_SRC = pathlib.Path(__file__).resolve().parent.parent / "oracle" / "mar_oracle.py"
KT = 0.1


def _load(src: str, name: str):
    spec = importlib.util.spec_from_loader(name, loader=None)
    mod = importlib.util.module_from_spec(spec)
    sys.modules[name] = mod
    exec(compile(src, f"<{name}>", "exec"), mod.__dict__)
    return mod


@pytest.fixture(scope="module")
def system():
    """Small diamond cell under a diagonal congruence, so S_jj != 1 everywhere."""
    s = lattice.generate(1, 1, 2, seed=4)          # 16 atoms, M = 64
    d = np.random.default_rng(9).uniform(0.7, 1.4, s.M)
    # congruence keeps every stored slot (values scaled, zeros stay zeros)
    H = sp.csr_matrix((s.H.data * d[np.repeat(np.arange(s.M), np.diff(s.H.indptr))] * d[s.H.indices],
                       s.H.indices, s.H.indptr), shape=s.H.shape)
    S = sp.csr_matrix((s.S.data * d[np.repeat(np.arange(s.M), np.diff(s.S.indptr))] * d[s.S.indices],
                       s.S.indices, s.S.indptr), shape=s.S.shape)
    return H, S


def _checks(O, H, S):
    """Return the names of the failed pin checks (NaN counts as a failure)."""
    failed = []
    M = H.shape[0]
    mu = 0.1
    rows = np.repeat(np.arange(M), np.diff(H.indptr))
    try:
        # nu = M must be exact (Eq. 1 projected on the whole space = Eq. 2)
        r = O.solve(H, S, np.arange(M), M, mu, KT)
        Hd, Sd = H.toarray(), S.toarray()
        import scipy.linalg
        ev, phi = scipy.linalg.eigh(Hd, Sd)
        f = 1.0 / (1.0 + np.exp((ev - mu) / KT))
        rho = 2.0 * (phi * f) @ phi.T
        if not np.linalg.norm(r.rho - rho[H.indices, rows]) <= 1e-10 * np.linalg.norm(rho):
            failed.append("nu=M")
        if not abs(r.e_band - 2.0 * np.sum(f * ev)) <= 1e-10 * abs(r.e_band):
            failed.append("E nu=M")
    except Exception:
        failed.append("nu=M raised")
    try:
        # nu = 1 closed form with S_jj != 1
        j = 7
        r = O.solve_seed(H, S, j, 1, mu, KT)
        hjj, sjj = H[j, j], S[j, j]
        f = 1.0 / (1.0 + math.exp((hjj / sjj - mu) / KT))
        expect = np.where(r.cols == j, 2.0 * f / sjj, 0.0)
        if not np.allclose(r.rho_row, expect, rtol=1e-12, atol=1e-300):
            failed.append("nu=1")
    except Exception:
        failed.append("nu=1 raised")
    try:
        # full occupation: N_j = 2 for every seed and nu (e_j in L, K^T S K = I)
        full = O.solve(H, S, [0, 5, 33], 6, 1e6, KT)
        if not np.allclose(full.n_seed, 2.0, atol=1e-12):
            failed.append("f=1")
        empty = O.solve(H, S, [0, 5, 33], 6, -1e6, KT)
        if np.any(empty.rho != 0.0):
            failed.append("f=0")
    except Exception:
        failed.append("occupation raised")
    try:
        # K^T S K = I through the full space of the 2x2x2 cell (CGS2 keeps it ~1e-15)
        H2, S2 = _big()
        r = O.solve_seed(H2, S2, 11, H2.shape[0], mu, KT, keep=True)
        G = r.K @ (S2 @ r.K.T)
        if not np.abs(G - np.eye(r.nu_eff)).max() <= 5e-14:
            failed.append("KtSK")
    except Exception:
        failed.append("KtSK raised")
    return failed


_BIG = {}


def _big():
    if not _BIG:
        s = lattice.generate(2, 2, 2, seed=0)
        _BIG["hs"] = (s.H, s.S)
    return _BIG["hs"]


MUTANTS = {
    "one_gs_pass": ("        c2 = SU[: n + 1] @ w\n        w = w - U[: n + 1].T @ c2\n",
                    "        c2 = 0.0 * c1\n"),
    "update_sign": ("w = w - U[: n + 1].T @ c1", "w = w + U[: n + 1].T @ c1"),
    "h_in_S_product": ("h[: n + 1, n] = U[: n + 1] @ w", "h[: n + 1, n] = SU[: n + 1] @ w"),
    "h_transposed": ("h[: n + 1, n] = U[: n + 1] @ w", "h[n, : n + 1] = U[: n + 1] @ w"),
    "no_start_normalization": ("U[0, j] = 1.0 / math.sqrt(sjj)", "U[0, j] = 1.0"),
    "start_norm_wrong_power": ("U[0, j] = 1.0 / math.sqrt(sjj)", "U[0, j] = 1.0 / sjj"),
    "fermi_sign": ("return np.where(x >= 0.0, t / (1.0 + t), 1.0 / (1.0 + t))",
                   "return np.where(x >= 0.0, 1.0 / (1.0 + t), t / (1.0 + t))"),
    "no_spin_factor": ("rho_row = 2.0 * (V[cols]", "rho_row = 1.0 * (V[cols]"),
    "beta_not_sqrt": ("U[n + 1] = w / beta\n", "U[n + 1] = w / beta2\n"),
    "sk_not_scaled": ("SU[n + 1] = z / beta", "SU[n + 1] = z"),
    "rho_uses_row_i_only": ("(f * vj)[None, :]", "(f * V[cols[0]])[None, :]"),
    "mirror_lower": ("return up + np.triu(h, 1).T", "return up + np.triu(h, 0).T"),
}


def test_unmodified_oracle_passes(system):
    O = _load(ORACLE_SRC.read_text(), "oracle_copy_clean")
    assert _checks(O, *system) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(system, name):
    old, new = MUTANTS[name]
    src = ORACLE_SRC.read_text()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    O = _load(src.replace(old, new), f"oracle_mutant_{name}")
    assert _checks(O, *system), f"mutant {name} passed every pin"
