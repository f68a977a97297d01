"""C-ABI library: loads, exports every declared symbol, validates inputs before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from paper_1307_3218_amd import mar

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mar.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mar_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["mar_create", "mar_destroy", "mar_solve", "mar_solve_async", "mar_set_tuning", "mar_last_error",
              "mar_profile_collect"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    L = mar.lib()
    for n in _declared():
        assert hasattr(L, n), n
        assert ctypes.cast(getattr(L, n), ctypes.c_void_p).value


def _csr_arrays(A):
    A = sp.csr_matrix(A)
    A.sort_indices()
    return (np.ascontiguousarray(A.indptr, np.int64), np.ascontiguousarray(A.indices, np.int32),
            np.ascontiguousarray(A.data, np.float64))


def _create(M, H, S):
    hp, hc, hv = H
    sp_, sc, sv = S
    out = ctypes.c_void_p()
    st = mar.lib().mar_create(M, hp.ctypes.data, hc.ctypes.data, hv.ctypes.data, sp_.ctypes.data,
                              sc.ctypes.data, sv.ctypes.data, ctypes.byref(out))
    if st == 0:
        mar.mar_destroy(out)
    return st, mar.mar_last_error(None)


@pytest.fixture
def small():
    H = sp.csr_matrix(np.array([[1.0, 0.5, 0.0], [0.5, -1.0, 0.2], [0.0, 0.2, 2.0]]))
    S = sp.csr_matrix(np.array([[1.0, 0.1, 0.0], [0.1, 1.0, 0.0], [0.0, 0.0, 1.0]]))
    return H, S


def test_rowptr_not_starting_at_zero(small):
    H, S = small
    hp, hc, hv = _csr_arrays(H)
    hp = hp.copy()
    hp[0] = 1
    st, msg = _create(3, (hp, hc, hv), _csr_arrays(S))
    assert st == mar.MAR_ERR_PATTERN and "rowptr[0]" in msg


def test_unsorted_columns(small):
    H, S = small
    hp, hc, hv = _csr_arrays(H)
    hc = hc.copy()
    hc[0], hc[1] = hc[1], hc[0]
    st, msg = _create(3, (hp, hc, hv), _csr_arrays(S))
    assert st == mar.MAR_ERR_PATTERN and "sorted" in msg


def test_column_out_of_range(small):
    H, S = small
    hp, hc, hv = _csr_arrays(H)
    hc = hc.copy()
    hc[-1] = 7
    st, _ = _create(3, (hp, hc, hv), _csr_arrays(S))
    assert st == mar.MAR_ERR_PATTERN


def test_asymmetric_value(small):
    H, S = small
    H = H.tolil()
    H[0, 1] = 0.6
    st, msg = _create(3, _csr_arrays(H.tocsr()), _csr_arrays(S))
    assert st == mar.MAR_ERR_PATTERN and "symmetric" in msg


def test_asymmetric_pattern(small):
    H, S = small
    H = H.tolil()
    H[0, 2] = 0.3
    st, msg = _create(3, _csr_arrays(H.tocsr()), _csr_arrays(S))
    assert st == mar.MAR_ERR_PATTERN


def test_overlap_outside_hamiltonian_pattern(small):
    H, S = small
    S = S.tolil()
    S[0, 2] = S[2, 0] = 0.05
    st, msg = _create(3, _csr_arrays(H), _csr_arrays(S.tocsr()))
    assert st == mar.MAR_ERR_PATTERN and "S stores" in msg


def test_nonpositive_overlap_diagonal(small):
    H, S = small
    S = S.tolil()
    S[1, 1] = -1.0
    st, msg = _create(3, _csr_arrays(H), _csr_arrays(S.tocsr()))
    assert st == mar.MAR_ERR_NOT_SPD


def test_nonfinite_value(small):
    H, S = small
    hp, hc, hv = _csr_arrays(H)
    hv = hv.copy()
    hv[0] = np.nan
    st, msg = _create(3, (hp, hc, hv), _csr_arrays(S))
    assert st == mar.MAR_ERR_ARG and "non-finite" in msg


def test_row_too_long():
    M = 80
    H = sp.csr_matrix(np.ones((M, M)) + np.eye(M))
    S = sp.identity(M, format="csr")
    st, msg = _create(M, _csr_arrays(H), _csr_arrays(S))
    assert st == mar.MAR_ERR_ARG and "entries" in msg


def test_bad_size():
    z = np.zeros(1, np.int64)
    out = ctypes.c_void_p()
    st = mar.lib().mar_create(0, z.ctypes.data, None, None, z.ctypes.data, None, None, ctypes.byref(out))
    assert st == mar.MAR_ERR_ARG


def _gpu_present():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def test_valid_input_without_gpu_reports_hip_error(small):
    H, S = small
    st, msg = _create(3, _csr_arrays(H), _csr_arrays(S))
    if _gpu_present():
        assert st == mar.MAR_OK
    else:
        assert st == mar.MAR_ERR_HIP and "device" in msg


def test_null_context_calls():
    L = mar.lib()
    assert L.mar_solve(None, None, 0, 1, 0.0, 0.1, 0, 0, None, None, None, None, None, None, None) == mar.MAR_ERR_STATE
    assert L.mar_set_tuning(None, None) == mar.MAR_ERR_STATE
    assert L.mar_profile_enable(None, 1) == mar.MAR_ERR_STATE
    assert isinstance(mar.mar_last_error(None), str)


def test_loaded_library_is_built_from_these_sources():
    """mar_build_id() carries the hash of the sources the library was compiled from: a library built from
    other sources (an older tree, a stale copy) fails here."""
    from paper_1307_3218_amd import build_lib
    assert mar.mar_build_id() == build_lib.source_hash()


@pytest.mark.gpu
def test_library_on_the_gpu_box_is_built_from_these_sources():
    from paper_1307_3218_amd import build_lib
    print(f"[abi] libmar.so build id {mar.mar_build_id()}", flush=True)
    assert mar.mar_build_id() == build_lib.source_hash()


def test_design_boundary_table_names_every_declaration():
    """The design notes' entry-point table (each entry point against the originally proposed boundary) lists
    exactly the header's declarations, so that every departure from that boundary is recorded there."""
    text = open(os.path.join(ROOT, "DESIGN.md")).read()
    start = text.index("<!-- entry points: first column, one per row -->")
    rows = []
    for line in text[start:].splitlines()[1:]:
        if not line.startswith("|"):
            if rows:
                break
            continue
        cell = line.split("|")[1].strip()
        m = re.fullmatch(r"`(mar_[a-z_]+)`", cell)
        if m:
            rows.append(m.group(1))
    assert sorted(rows) == _declared()
