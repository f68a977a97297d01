"""FP64 CPU oracle of the multiple-Arnoldi (mArnoldi) per-seed hot path.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the bench's
CPU-baseline leg may import or run this module. The product path (the HIP
library and its Python binding) never calls it, and it shares no code with the
product: it is a plain, slow, step-by-step restatement of the method.

What the paper fixes (Sec. 2):
  * Eq. (1): the generalized shifted equations (zS - H) x = b with H, S sparse
    real symmetric and S positive definite. With b = e_j the solution is column
    j of the Green's function G(z) = (zS - H)^-1.
  * mArnoldi reduces the problem to M small nu x nu *standard* eigenproblems,
    one in each Krylov subspace L_nu^(j) that contains e_j; the subspace eigen
    levels eps_alpha^(j) and vectors v_alpha^(j) define the Green's function,
    which gives the energy.
Readings taken where the paper is silent (all listed in the design notes):
  * the subspace is span{e_j, H e_j, ..., H^(nu-1) e_j};
  * a standard (not generalized) subspace problem needs an S-orthonormal
    basis K (K^T S K = I), built by classical Gram-Schmidt with two passes
    (CGS2) in the S-inner product, starting from u_1 = e_j / sqrt(S_jj);
  * the subspace matrix is A = K^T H K from explicit dot products
    h_kn = u_k . (H u_n), symmetrized from its upper triangle;
  * projecting Eq. (1) with b = e_j onto L gives
    G_ij(z) ~ sum_alpha (e_i . v_alpha)(v_alpha . e_j) / (z - eps_alpha),
    v_alpha = K y_alpha; the spin-summed density-matrix column is the Fermi-
    weighted residue sum rho_ij = 2 sum_alpha f_alpha (e_i.v_alpha)(e_j.v_alpha)
    kept on the pattern P(j) of H's row j, E_j = sum_{i in P(j)} rho_ij H_ij and
    N_j = sum_{i in P(j)} rho_ij S_ij;
  * f(x) = 1 / (1 + e^x), x = (eps - mu) / kT, with kT = 0 the step function
    (1/2 at eps = mu); breakdown when beta <= tau * eta (tau = 1e-12), the
    subspace is then truncated to nu_eff = n.
Pins (tests/test_oracle_pins.py): nu = M against the dense generalized
eigensolve; S = I Lanczos moments; nu = 1 and nu = 2 closed forms; occupation
sum rules; the E_j / N_j / weight identities; K^T S K = I; an explicit-Krylov
Cholesky formulation; scale and permutation covariance; rho symmetry at nu = M;
the electron count at the bisected Fermi level.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg
import scipy.sparse as sp

TAU_FP64 = 1e-12


class NotSPDError(ArithmeticError):
    """w^T S w <= 0 for a nonzero residual: S is not positive definite."""


# --------------------------------------------------------------------------
# Fermi function (the occupation used to turn subspace levels into rho, E)
# --------------------------------------------------------------------------
def fermi(eps, mu: float, kT: float):
    """f = 1/(1+exp(x)), x = (eps-mu)/kT; kT = 0 gives the step (1/2 at eps = mu).

    Written as exp(-x)/(1+exp(-x)) for x >= 0 so that neither branch overflows
    and small occupations keep full relative accuracy.
    """
    eps = np.asarray(eps, dtype=np.float64)
    if kT == 0.0:
        return np.where(eps < mu, 1.0, np.where(eps > mu, 0.0, 0.5))
    x = (eps - mu) / kT
    t = np.exp(-np.abs(x))
    return np.where(x >= 0.0, t / (1.0 + t), 1.0 / (1.0 + t))


# --------------------------------------------------------------------------
# One seed: Krylov subspace L_nu^(j), CGS2 in the S-inner product (Sec. 2)
# --------------------------------------------------------------------------
@dataclass
class SeedResult:
    j: int
    nu_eff: int
    eps: np.ndarray          # subspace eigen levels (ascending)
    weight: np.ndarray       # w_alpha = (e_j^T S v_alpha)(v_alpha^T e_j)
    cols: np.ndarray         # P(j): column indices of H row j
    rho_row: np.ndarray      # rho_ij for i in P(j) (CSR row j slot order)
    E: float
    N: float
    K: np.ndarray | None = field(default=None, repr=False)   # (nu_eff, M) basis rows
    A: np.ndarray | None = field(default=None, repr=False)   # subspace matrix


def krylov_basis(H, S, j: int, nu: int, tau: float = TAU_FP64):
    """S-orthonormal basis of span{e_j, H e_j, ...} and h_kn = u_k . (H u_n).

    Returns (U, h, nu_eff): U has the basis vectors as rows (nu_eff x M), h is
    the nu_eff x nu_eff array whose upper triangle (k <= n) holds the projections.
    """
    M = H.shape[0]
    sjj = S[j, j]
    U = np.zeros((nu, M))
    SU = np.zeros((nu, M))
    U[0, j] = 1.0 / math.sqrt(sjj)
    SU[0] = S @ U[0]
    h = np.zeros((nu, nu))
    nu_eff = nu
    for n in range(nu):
        w = H @ U[n]
        h[: n + 1, n] = U[: n + 1] @ w          # subspace Hamiltonian column
        if n + 1 == nu:
            break
        # CGS2: two classical Gram-Schmidt passes in the S-inner product
        c1 = SU[: n + 1] @ w
        w = w - U[: n + 1].T @ c1
        c2 = SU[: n + 1] @ w
        w = w - U[: n + 1].T @ c2
        z = S @ w
        beta2 = float(w @ z)
        if beta2 < 0.0:
            raise NotSPDError(f"seed {j}: w^T S w = {beta2} < 0 at step {n + 1}")
        beta = math.sqrt(beta2)
        eta = math.sqrt(float(c1 @ c1) + float(c2 @ c2) + beta2)
        if beta <= tau * eta:
            nu_eff = n + 1
            break
        U[n + 1] = w / beta
        SU[n + 1] = z / beta
    return U[:nu_eff], h[:nu_eff, :nu_eff], nu_eff


def subspace_matrix(h: np.ndarray) -> np.ndarray:
    """A = K^T H K from the computed upper triangle, mirrored."""
    up = np.triu(h)
    return up + np.triu(h, 1).T


def _row_slots(Mat: sp.csr_matrix, j: int):
    lo, hi = Mat.indptr[j], Mat.indptr[j + 1]
    return Mat.indices[lo:hi], Mat.data[lo:hi]


def assemble_seed(H, S, j, U, A, mu, kT):
    """Subspace eigenpairs -> rho_ij (i in P(j)), E_j, N_j, weights (Sec. 2 end)."""
    eps, Y = np.linalg.eigh(A)
    V = U.T @ Y                                  # v_alpha = K y_alpha, columns
    f = fermi(eps, mu, kT)
    cols, hvals = _row_slots(H, j)
    srow = S.getrow(j).toarray().ravel()
    svals = srow[cols]                           # S on H's pattern (zeros kept)
    vj = V[j]                                    # v_alpha^T e_j
    rho_row = 2.0 * (V[cols] * (f * vj)[None, :]).sum(axis=1)
    weight = (srow @ V) * vj                     # (e_j^T S v_alpha)(v_alpha^T e_j)
    E = float(rho_row @ hvals)
    N = float(rho_row @ svals)
    return eps, weight, cols, rho_row, E, N


def solve_seed(H, S, j: int, nu: int, mu: float, kT: float, tau: float = TAU_FP64,
               keep: bool = False) -> SeedResult:
    H = sp.csr_matrix(H)
    S = sp.csr_matrix(S)
    U, h, nu_eff = krylov_basis(H, S, j, nu, tau)
    A = subspace_matrix(h)
    eps, weight, cols, rho_row, E, N = assemble_seed(H, S, j, U, A, mu, kT)
    return SeedResult(j=j, nu_eff=nu_eff, eps=eps, weight=weight, cols=cols,
                      rho_row=rho_row, E=E, N=N,
                      K=U if keep else None, A=A if keep else None)


# --------------------------------------------------------------------------
# Many seeds (independent subspaces; process-parallel over seeds)
# --------------------------------------------------------------------------
_G = {}


def _init_worker(H, S, nu, mu, kT, tau):
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    _G.update(H=H, S=S, nu=nu, mu=mu, kT=kT, tau=tau)


def _work(j):
    return solve_seed(_G["H"], _G["S"], int(j), _G["nu"], _G["mu"], _G["kT"], _G["tau"])


@dataclass
class SolveResult:
    rho: np.ndarray          # nnz(H); CSR row j slots filled for listed seeds, 0 elsewhere
    e_band: float            # fsum of E_j over the listed seeds
    e_seed: np.ndarray
    n_seed: np.ndarray
    nu_eff: np.ndarray
    eps: list
    weight: list


def solve(H, S, seeds, nu: int, mu: float, kT: float, tau: float = TAU_FP64,
          workers: int = 1) -> SolveResult:
    H = sp.csr_matrix(H)
    S = sp.csr_matrix(S)
    seeds = np.asarray(seeds, dtype=np.int64)
    if workers > 1 and len(seeds) > 1:
        import multiprocessing as mp
        ctx = mp.get_context("fork")
        with ctx.Pool(workers, initializer=_init_worker, initargs=(H, S, nu, mu, kT, tau)) as pool:
            res = pool.map(_work, seeds, chunksize=max(1, len(seeds) // (8 * workers)))
    else:
        res = [solve_seed(H, S, int(j), nu, mu, kT, tau) for j in seeds]
    rho = np.zeros(H.nnz)
    for r in res:
        lo = H.indptr[r.j]
        rho[lo: lo + len(r.rho_row)] = r.rho_row
    e_seed = np.array([r.E for r in res])
    return SolveResult(rho=rho, e_band=math.fsum(e_seed), e_seed=e_seed,
                       n_seed=np.array([r.N for r in res]),
                       nu_eff=np.array([r.nu_eff for r in res], dtype=np.int32),
                       eps=[r.eps for r in res], weight=[r.weight for r in res])


# --------------------------------------------------------------------------
# Fermi level from the subspace levels (half filling by default)
# --------------------------------------------------------------------------
def electron_count(eps_list, w_list, mu: float, kT: float) -> float:
    """N(mu) = sum_j 2 sum_alpha f((eps_alpha^(j) - mu)/kT) w_alpha^(j)."""
    return math.fsum(2.0 * float(np.dot(fermi(e, mu, kT), w)) for e, w in zip(eps_list, w_list))


def fermi_level(eps_list, w_list, n_target: float, kT: float, iters: int = 200) -> float:
    lo = min(float(np.min(e)) for e in eps_list) - 40.0 * kT
    hi = max(float(np.max(e)) for e in eps_list) + 40.0 * kT
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if electron_count(eps_list, w_list, mid, kT) < n_target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


# --------------------------------------------------------------------------
# Independent cross-checks
# --------------------------------------------------------------------------
def dense(H, S, mu: float, kT: float):
    """Exact answer from the generalized eigenproblem H phi = eps S phi (Eq. 2).

    Returns (rho_dense, E, eps): rho = 2 sum_k f(eps_k) phi_k phi_k^T with
    phi^T S phi = 1, E = 2 sum_k f(eps_k) eps_k.
    """
    Hd = H.toarray() if sp.issparse(H) else np.asarray(H)
    Sd = S.toarray() if sp.issparse(S) else np.asarray(S)
    eps, phi = scipy.linalg.eigh(Hd, Sd)
    f = fermi(eps, mu, kT)
    rho = 2.0 * (phi * f[None, :]) @ phi.T
    return rho, float(2.0 * math.fsum(f * eps)), eps


def brute_seed(H, S, j: int, nu: int, mu: float, kT: float):
    """Galerkin projection on the explicit Krylov matrix (no Gram-Schmidt).

    V = [e_j, H e_j, ..., H^(nu-1) e_j] (columns scaled to unit length), then the
    nu x nu generalized problem (V^T H V) y = eps (V^T S V) y with y^T V^T S V y = 1
    is solved by LAPACK's Cholesky-based routine. Only for tiny nu: V is
    ill-conditioned. Returns (eps, rho_row over P(j), E_j, N_j).
    """
    H = sp.csr_matrix(H)
    S = sp.csr_matrix(S)
    M = H.shape[0]
    V = np.zeros((M, nu))
    x = np.zeros(M)
    x[j] = 1.0
    for k in range(nu):
        V[:, k] = x / np.linalg.norm(x)
        x = H @ V[:, k]
    a = V.T @ (H @ V)
    b = V.T @ (S @ V)
    a = 0.5 * (a + a.T)
    b = 0.5 * (b + b.T)
    eps, Y = scipy.linalg.eigh(a, b)
    Vy = V @ Y
    f = fermi(eps, mu, kT)
    cols, hvals = _row_slots(H, j)
    svals = S.getrow(j).toarray().ravel()[cols]
    rho_row = 2.0 * (Vy[cols] * (f * Vy[j])[None, :]).sum(axis=1)
    return eps, rho_row, float(rho_row @ hvals), float(rho_row @ svals)


def default_workers() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1
