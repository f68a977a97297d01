"""Input generator: symmetric sparse H, S with S positive definite (Sec. 2, Eq. 1 setting)."""
import numpy as np
import pytest

from paper_1307_3218_amd import lattice


def _block_pattern_ok(A, n_atoms):
    """Every stored entry sits in a full 4x4 block; block rows share one pattern."""
    A = A.tocsr()
    for I in range(n_atoms):
        pats = [tuple(A.indices[A.indptr[4 * I + r]:A.indptr[4 * I + r + 1]]) for r in range(4)]
        if len(set(pats)) != 1:
            return False
        cols = np.array(pats[0])
        if len(cols) % 4 or not np.all(cols.reshape(-1, 4) == (cols.reshape(-1, 4)[:, :1] + np.arange(4))):
            return False
    return True


def test_diamond_small(cell256):
    s = cell256
    assert s.M == 256 and s.n_atoms == 64
    assert s.H.nnz == 16 * 64 * 5 == s.S.nnz
    assert np.all(s.degree == 4)
    assert abs(s.H - s.H.T).max() == 0.0
    assert abs(s.S - s.S.T).max() == 0.0
    assert np.array_equal(s.H.indptr, s.S.indptr) and np.array_equal(s.H.indices, s.S.indices)
    assert _block_pattern_ok(s.H, s.n_atoms)
    lam = np.linalg.eigvalsh(s.S.toarray())
    assert lam[0] >= lattice.SPD_FLOOR and s.s_scale == 1.0
    # on-site blocks: H diag near (-5, 1, 1, 1), S diag exactly 1
    d = s.H.diagonal().reshape(-1, 4)
    assert np.allclose(d.mean(axis=0), [-5, 1, 1, 1], atol=0.1)
    assert np.all(s.S.diagonal() == 1.0)


def test_determinism():
    a = lattice.generate(2, 2, 2, seed=0)
    b = lattice.generate(2, 2, 2, seed=0)
    c = lattice.generate(2, 2, 2, seed=1)
    assert (a.H != b.H).nnz == 0 and (a.S != b.S).nnz == 0
    assert (a.H != c.H).nnz > 0


def test_mixed_coordination():
    s = lattice.generate(2, 2, 2, mixed=True)
    assert np.sum(s.degree == 3) == s.n_atoms // 2
    assert np.sum(s.degree == 4) == s.n_atoms // 2
    assert s.degree.mean() == 3.5
    assert s.H.nnz == 16 * (s.n_atoms + 2 * len(s.bonds))
    assert abs(s.H - s.H.T).max() == 0.0
    assert _block_pattern_ok(s.S, s.n_atoms)


@pytest.mark.parametrize("cells", [(4, 4, 2), (1, 1, 1), (3, 2, 2)])
def test_diamond_bonds_geometry(cells):
    b = lattice.diamond_bonds(*cells)
    n_atoms = 8 * np.prod(cells)
    deg = np.bincount(b.ravel(), minlength=n_atoms)
    if min(cells) >= 2:
        assert len(b) == 2 * n_atoms and np.all(deg == 4)
    assert np.all(b[:, 0] < b[:, 1])


def test_spd_scaling_path():
    # an overlap with huge neighbour blocks must be scaled back to lambda_min >= floor
    s = lattice.generate(2, 2, 2, seed=3)
    assert s.lam_min_S >= lattice.SPD_FLOOR


def test_sample_seeds():
    a = lattice.sample_seeds(1000, 10, seed=0)
    assert len(np.unique(a)) == 10 and np.all(np.diff(a) > 0) and a.max() < 1000
    assert np.array_equal(lattice.sample_seeds(8, 20), np.arange(8))
