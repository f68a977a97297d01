"""Seeded synthetic tight-binding matrices (H, S) for the mArnoldi hot path.

This module is the input generator shared by the GPU path's tests/bench and the
CPU oracle's tests. It holds none of the method's arithmetic: it only builds
sparse real-symmetric H and S with S positive definite (Sec. 2, the setting of
Eq. 1), in the LCAO form of a carbon-like solid with four orbitals (s, px, py,
pz) per atom.

Lattice readings (the paper gives no structure; these are stand-ins):
  * diamond: conventional cubic cell of 8 atoms, periodic n1 x n2 x n3 cells.
    Coordinates are in units of a/4; sublattice A = (0,0,0), (0,2,2), (2,0,2),
    (2,2,0); sublattice B = A + (1,1,1). Each A atom bonds to the B atoms at
    A + (+-1,+-1,+-1) with an even number of minus signs.
  * mixed sp2/sp3: start from diamond, visit the bonds in a seeded random
    permutation and delete a bond when both ends still have four bonds, until
    N_at/4 bonds are gone: exactly half of the atoms become 3-coordinated.
Atom order: cell index cx + n1*(cy + n2*cz), then the 8 basis atoms. Orbital
index = 4*atom + {0: s, 1: px, 2: py, 3: pz}.

Values (eV): on-site H = diag(-5, 1, 1, 1) + diag(N(0, 0.1)) with its
off-diagonal zeros stored; each bond a<b draws one 4x4 block X ~ N(0,1)*2 with
H_ab = X, H_ba = X^T; S on-site = I_4, S bond blocks N(0,1)*0.05 likewise.
If lambda_min(S) < 0.05 all off-diagonal S blocks are scaled by t so that
lambda_min >= 0.05 (recorded as ``s_scale``).

Draw order from numpy.random.default_rng(seed): bond-removal permutation (mixed
only), on-site noise (M values), H bond blocks (n_bonds x 4 x 4), S bond blocks
(n_bonds x 4 x 4).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

_BASIS = np.array([[0, 0, 0], [0, 2, 2], [2, 0, 2], [2, 2, 0],
                   [1, 1, 1], [1, 3, 3], [3, 1, 3], [3, 3, 1]], dtype=np.int64)
_BOND_DIRS = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.int64)

SPD_FLOOR = 0.05


@dataclasses.dataclass
class TBSystem:
    """A generated system: CSR H and S on one shared pattern of full 4x4 blocks."""
    H: sp.csr_matrix
    S: sp.csr_matrix
    n_atoms: int
    degree: np.ndarray          # bonds per atom
    bonds: np.ndarray           # (n_bonds, 2) atom pairs a < b
    s_scale: float              # factor applied to off-diagonal S blocks (1.0 = none)
    lam_min_S: float            # smallest eigenvalue of S after scaling (estimate for big M)
    name: str = ""

    @property
    def M(self) -> int:
        return self.H.shape[0]


def diamond_bonds(n1: int, n2: int, n3: int) -> np.ndarray:
    """Nearest-neighbour bonds (a, b), a < b, of a periodic n1 x n2 x n3 diamond cell."""
    dims = np.array([n1, n2, n3], dtype=np.int64)
    n_cells = int(n1 * n2 * n3)
    cidx = np.arange(n_cells, dtype=np.int64)
    cx = cidx % n1
    cy = (cidx // n1) % n2
    cz = cidx // (n1 * n2)
    cell_xyz = np.stack([cx, cy, cz], axis=1)
    pairs = []
    for ba in range(4):                      # sublattice A atoms
        pos = cell_xyz * 4 + _BASIS[ba]      # (n_cells, 3) in a/4 units
        a = cidx * 8 + ba
        for d in _BOND_DIRS:
            q = pos + d
            qc = np.floor_divide(q, 4)
            qr = q - qc * 4
            qc = np.mod(qc, dims)
            # which B basis atom sits at remainder qr
            match = np.all(qr[:, None, :] == _BASIS[None, 4:, :], axis=2)
            bb = 4 + np.argmax(match, axis=1)
            assert match.any(axis=1).all()
            b = (qc[:, 0] + n1 * (qc[:, 1] + n2 * qc[:, 2])) * 8 + bb
            pairs.append(np.stack([a, b], axis=1))
    bonds = np.concatenate(pairs, axis=0)
    bonds = np.sort(bonds, axis=1)
    bonds = np.unique(bonds, axis=0)
    return bonds


def _remove_half_coordination(bonds: np.ndarray, n_atoms: int, rng) -> np.ndarray:
    perm = rng.permutation(len(bonds))
    deg = np.bincount(bonds.ravel(), minlength=n_atoms)
    keep = np.ones(len(bonds), dtype=bool)
    target = n_atoms // 4
    removed = 0
    for e in perm:
        a, b = bonds[e]
        if deg[a] == 4 and deg[b] == 4:
            keep[e] = False
            deg[a] -= 1
            deg[b] -= 1
            removed += 1
            if removed == target:
                break
    if removed != target:
        raise RuntimeError("bond removal did not reach N_at/4 removals")
    return bonds[keep]


def _assemble(n_atoms, bonds, onsite_H, bond_H, bond_S):
    nb = len(bonds)
    rows = np.concatenate([np.arange(n_atoms), bonds[:, 0], bonds[:, 1]])
    cols = np.concatenate([np.arange(n_atoms), bonds[:, 1], bonds[:, 0]])
    eye = np.broadcast_to(np.eye(4), (n_atoms, 4, 4))
    hblk = np.concatenate([onsite_H, bond_H, np.transpose(bond_H, (0, 2, 1))])
    sblk = np.concatenate([eye, bond_S, np.transpose(bond_S, (0, 2, 1))])
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    hblk, sblk = hblk[order], sblk[order]
    indptr = np.zeros(n_atoms + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr)
    Hb = sp.bsr_matrix((np.ascontiguousarray(hblk), cols, indptr), shape=(4 * n_atoms, 4 * n_atoms))
    Sb = sp.bsr_matrix((np.ascontiguousarray(sblk), cols, indptr), shape=(4 * n_atoms, 4 * n_atoms))
    H = Hb.tocsr()
    S = Sb.tocsr()
    H.sort_indices()
    S.sort_indices()
    del nb
    return H, S


def lambda_min(S: sp.spmatrix) -> float:
    """Smallest eigenvalue of symmetric S (dense for small M, Lanczos otherwise)."""
    M = S.shape[0]
    if M <= 4096:
        return float(np.linalg.eigvalsh(S.toarray())[0])
    import scipy.sparse.linalg as sla
    val = sla.eigsh(S.tocsr(), k=1, which="SA", tol=1e-6, ncv=64, maxiter=20000,
                    v0=np.ones(M), return_eigenvectors=False)
    return float(val[0])


def generate(n1: int, n2: int, n3: int, mixed: bool = False, seed: int = 0,
             check_spd: bool = True) -> TBSystem:
    """Build H, S for a periodic n1 x n2 x n3 diamond (or mixed sp2/sp3) lattice."""
    rng = np.random.default_rng(seed)
    n_atoms = 8 * n1 * n2 * n3
    bonds = diamond_bonds(n1, n2, n3)
    if mixed:
        bonds = _remove_half_coordination(bonds, n_atoms, rng)
    M = 4 * n_atoms
    noise = rng.normal(0.0, 0.1, size=M)
    onsite = np.zeros((n_atoms, 4, 4))
    base = np.array([-5.0, 1.0, 1.0, 1.0])
    d = base[None, :] + noise.reshape(n_atoms, 4)
    onsite[:, np.arange(4), np.arange(4)] = d
    bond_H = rng.normal(0.0, 1.0, size=(len(bonds), 4, 4)) * 2.0
    bond_S = rng.normal(0.0, 1.0, size=(len(bonds), 4, 4)) * 0.05
    H, S = _assemble(n_atoms, bonds, onsite, bond_H, bond_S)
    s_scale = 1.0
    lam = float("nan")
    if check_spd:
        lam = lambda_min(S)
        if lam < SPD_FLOOR:
            # lambda_min(I + t*X) >= 1 + t*lambda_min(X); pick t for the floor
            s_scale = (1.0 - SPD_FLOOR) / (1.0 - lam)
            H, S = _assemble(n_atoms, bonds, onsite, bond_H, bond_S * s_scale)
            lam = lambda_min(S)
    degree = np.bincount(bonds.ravel(), minlength=n_atoms)
    name = f"{'mixed' if mixed else 'diamond'}_{n1}x{n2}x{n3}"
    return TBSystem(H=H, S=S, n_atoms=n_atoms, degree=degree, bonds=bonds,
                    s_scale=s_scale, lam_min_S=lam, name=name)


# Workloads of the study (name -> (cells, mixed)); M = 32 * n1 * n2 * n3.
WORKLOADS = {
    "diamond_2x2x2": ((2, 2, 2), False),     # M = 256
    "diamond_8x8x8": ((8, 8, 8), False),     # M = 16384
    "mixed_16x16x16": ((16, 16, 16), True),  # M = 131072
    "mixed_32x32x32": ((32, 32, 32), True),  # M = 1048576
}
# Eight uneven systems batched together (M = 1024 ... 65536).
UNEVEN_SYSTEMS = [(4, 4, 2), (4, 4, 4), (8, 4, 4), (8, 8, 4), (8, 8, 8), (16, 8, 8), (16, 12, 8), (16, 16, 8)]


def workload(name: str, seed: int = 0, check_spd: bool = True) -> TBSystem:
    cells, mixed = WORKLOADS[name]
    return generate(*cells, mixed=mixed, seed=seed, check_spd=check_spd)


def sample_seeds(M: int, n: int, seed: int = 0) -> np.ndarray:
    """n distinct basis indices in [0, M), sorted (uniform sample, rng seed)."""
    if n >= M:
        return np.arange(M, dtype=np.int32)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(M, n, replace=False)).astype(np.int32)
