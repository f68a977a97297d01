"""The largest single-GPU instance: the 262144-atom mixed sp2/sp3 lattice
(M = 1048576) at nu = 300, seed blocks of 64, against the FP64 oracle on 8
sampled seeds (stored by tests/golden/make_mixed1m_oracle.py, which calls only the
oracle; mu = -0.45 eV, kT = 0.1 eV).

Bars: FP64 form 1e-10, FP32 form 1e-5, on rho (Frobenius norm over the listed
rows and every listed rho column), on the summed E, on every E_j and N_j (floors
as in the other parity tests); nu_eff equal.

At this size the FP32 form's update keeps its running sums over the slabs in
FP64 (nu > 128). With FP32 sums the worst columns (seeds 14 and 786929) sat at
1.7e-5 to 3.3e-5 over seven block sizes and projection variants, and the
Frobenius norm at 5.7e-6 to 1.2e-5; with FP64 sums the same seven give a worst
column of 4.8e-6 to 1.0e-5 and a Frobenius norm of 2.2e-6 to 4.2e-6 (9.55e-6 and
4.2e-6 in the configuration tested here). Over twelve block sizes and projection
partitions the worst column spans 4.8e-6 to 2.8e-5 (three of the twelve above 1e-5),
and 2.9e-5 with 8 slabs per projection workgroup: the per-column bar holds in the
default configuration, not in every equivalent rounding order. The remaining error is that of the FP32
basis and the FP32 sparse products and projections: a numpy emulation of the
textbook CGS2 in FP32 puts seed 14 at 1.6e-5, of which FP32 storage alone is 9e-7,
and a Rayleigh-Ritz step against the FP64 Gram matrix of the FP32 basis does not
change it (the FP32 sums perturb the subspace itself).
"""
import json
import os

import numpy as np
import pytest

from paper_1307_3218_amd import lattice, mar

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mixed1m_oracle_nu300.json")
TOL = {"fp64": 1e-10, "fp32": 1e-5}


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def mixed1m(golden):
    s = lattice.workload(golden["workload"])
    assert s.M == golden["M"] and s.H.nnz == golden["nnz"]
    return s


@pytest.fixture(scope="module")
def mixed1m_ctx(mixed1m):
    ctx = mar.Context(mixed1m.H, mixed1m.S)
    yield ctx
    ctx.close()


def _check(g, out, prec, label, columns=True):
    """Assert the stated bars (every rho column too when columns is set) and print the errors."""
    tol = TOL[prec]
    seeds = g["seeds"]
    assert list(out.nu_eff) == g["nu_eff"], label
    num = den = 0.0
    cols = []
    for j in seeds:
        row = g["rho_rows"][str(j)]
        ref = np.array(row["rho"])
        got = out.rho_rows[j]
        num += float(np.sum((got - ref) ** 2))
        den += float(np.sum(ref ** 2))
        cols.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    rho_rel = (num / den) ** 0.5
    e_ref = float(np.sum(g["e_seed"]))
    e_rel = abs(float(np.sum(out.e_seed)) - e_ref) / abs(e_ref)
    worst = max(cols)
    print(f"[mixed1m {label} {prec}] rho {rho_rel:.2e} E {e_rel:.2e} worst column {worst:.2e}; columns "
          + " ".join(f"{j}:{c:.1e}" for j, c in zip(seeds, cols)), flush=True)
    assert rho_rel <= tol and e_rel <= tol
    if columns:
        assert worst <= tol
    e_ref_j, n_ref_j = np.array(g["e_seed"]), np.array(g["n_seed"])
    e_err = np.abs(np.array(out.e_seed) - e_ref_j) / np.maximum(np.abs(e_ref_j), 1e-2 * np.abs(e_ref_j).max())
    n_err = np.abs(np.array(out.n_seed) - n_ref_j) / np.maximum(np.abs(n_ref_j), 2e-2)
    assert e_err.max() <= tol and n_err.max() <= tol, (e_err.max(), n_err.max())
    # individual Ritz levels at nu = 300 are ill-conditioned (interior, unconverged,
    # near-degenerate: they move by ~1e-8 eV in FP64 and ~1e-2 eV in FP32 with the
    # rounding order), so the levels are compared through their weighted moments
    # sum_a w_a eps_a^k, k = 0..3 (the quadrature of the seed's local spectrum)
    scale = max(max(abs(v) for v in e) for e in g["eps"])
    mtol = tol
    for s in range(len(seeds)):
        m = out.nu_eff[s]
        ge, gw = out.eps[s, :m], out.weight[s, :m]
        re, rw = np.array(g["eps"][s]), np.array(g["weight"][s])
        for k in range(4):
            got, ref = float(np.sum(gw * ge ** k)), float(np.sum(rw * re ** k))
            assert abs(got - ref) <= mtol * scale ** k, (s, k, got, ref)


class _Rows:
    def __init__(self, H, seeds, o):
        self.rho_rows = {j: o.rho[H.indptr[j]:H.indptr[j + 1]] for j in seeds}
        self.e_seed, self.n_seed, self.nu_eff, self.eps, self.weight = o.e_seed, o.n_seed, o.nu_eff, o.eps, o.weight


def _solve(ctx, mixed1m, g, prec, form, block=0):
    ctx.set_tuning(seed_block=block)
    try:
        o = ctx.solve(np.array(g["seeds"], dtype=np.int32), g["nu"], g["mu"], g["kT"], prec, form, levels=True)
    finally:
        ctx.set_tuning()
    return _Rows(mixed1m.H, g["seeds"], o)


def test_mixed1m_block_size(mixed1m_ctx, golden):
    """The widest block that keeps the FP32 basis within 128 GB is the configured 64."""
    assert mixed1m_ctx.seed_block(golden["nu"], "fp32") == 64


@pytest.fixture(scope="module")
def fp32_batched(mixed1m_ctx, mixed1m, golden):
    return _solve(mixed1m_ctx, mixed1m, golden, "fp32", "batched", block=64)


def test_mixed1m_fp32_batched(fp32_batched, golden):
    _check(golden, fp32_batched, "fp32", "batched B=64", columns=False)


def test_mixed1m_fp32_batched_every_column(fp32_batched, golden):
    _check(golden, fp32_batched, "fp32", "batched B=64 per column", columns=True)


def test_mixed1m_fp64_plain(mixed1m_ctx, mixed1m, golden):
    _check(golden, _solve(mixed1m_ctx, mixed1m, golden, "fp64", "plain"), "fp64", "plain")


def test_mixed1m_fp64_batched(mixed1m_ctx, mixed1m, golden):
    _check(golden, _solve(mixed1m_ctx, mixed1m, golden, "fp64", "batched", block=8), "fp64", "batched B=8")


def test_mixed1m_blocks_in_sequence(mixed1m_ctx, golden):
    """A block of neighbouring seeds solved after another block equals that block solved alone.

    Between blocks the whole 80 GB basis is zeroed (support tracking reads tiles the block has not
    written yet as zeros); a fill of more than 2^32 work-items in one launch covers only part of it and
    leaves later slabs holding the previous block's vectors.
    """
    fill = np.arange(0, 64, dtype=np.int32)
    x = np.arange(500000, 500064, dtype=np.int32)
    mixed1m_ctx.set_tuning(seed_block=64)
    try:
        both = mixed1m_ctx.solve(np.concatenate([fill, x]), golden["nu"], golden["mu"], golden["kT"], "fp32")
        alone = mixed1m_ctx.solve(x, golden["nu"], golden["mu"], golden["kT"], "fp32")
    finally:
        mixed1m_ctx.set_tuning()
    assert np.array_equal(both.nu_eff[64:], alone.nu_eff)
    assert np.array_equal(both.e_seed[64:], alone.e_seed)
