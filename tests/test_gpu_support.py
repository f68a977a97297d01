"""Support tracking of the batched delayed schedule on the GPU.

Basis vector k of a seed is exactly zero on rows more than k hops (in H's
pattern) from the seed, so the kernels skip the row tiles farther than the
step from every seed of a block. These tests compare that path with the full
sweep (support_off) and with the FP64 oracle: blocks of neighbouring seeds
(small support, growing for many steps) and of scattered seeds (support filling
the cell at once), ragged blocks, nu = 1 and 2, every projection variant, and
the profiler's restricted byte counts.
"""
import numpy as np
import pytest

from oracle import mar_oracle as O
from paper_1307_3218_amd import lattice, mar

pytestmark = pytest.mark.gpu

KT = 0.1
TOL = {"fp64": 1e-10, "fp32": 1e-5}


def _slots(H, seeds):
    return np.concatenate([np.arange(H.indptr[j], H.indptr[j + 1]) for j in seeds])


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def sysm():
    """Mixed sp2/sp3 cell of 6x6x6 conventional cells (1728 atoms, M = 6912)."""
    return lattice.generate(6, 6, 6, mixed=True, seed=3)


@pytest.fixture(scope="module")
def ctx(sysm):
    c = mar.Context(sysm.H, sysm.S)
    assert c.info()["H_bsr"]
    yield c
    c.close()


def _solve(ctx, seeds, nu, prec, support, B=0, variant=0):
    ctx.set_tuning(seed_block=B, schedule="delayed", proj_variant=variant, support=support)
    try:
        return ctx.solve(seeds, nu, -0.3, KT, precision=prec, form="batched", levels=True)
    finally:
        ctx.set_tuning()


@pytest.mark.parametrize("prec,B", [("fp64", 8), ("fp64", 64), ("fp32", 16), ("fp32", 64), ("fp32", 256)])
@pytest.mark.parametrize("layout", ["neighbours", "scattered"])
def test_support_equals_full_sweep(sysm, ctx, prec, B, layout):
    n = 2 * B + 37                                   # ragged last block
    if layout == "neighbours":
        seeds = np.arange(1000, 1000 + n, dtype=np.int32)
    else:
        seeds = lattice.sample_seeds(sysm.M, n, seed=B).astype(np.int32)
    a = _solve(ctx, seeds, 30, prec, True, B)
    b = _solve(ctx, seeds, 30, prec, False, B)
    idx = _slots(sysm.H, seeds)
    r_rho, r_e = _rel(a.rho[idx], b.rho[idx]), abs(a.e_band - b.e_band) / abs(b.e_band)
    print(f"[support {prec} B={B} {layout}] rho {r_rho:.2e} E_band {r_e:.2e}", flush=True)
    assert np.array_equal(a.nu_eff, b.nu_eff)
    assert r_rho <= TOL[prec] and r_e <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_support_against_oracle(sysm, ctx, prec):
    seeds = np.arange(3000, 3000 + 150, dtype=np.int32)
    ref = O.solve(sysm.H, sysm.S, seeds, 40, -0.3, KT, workers=max(1, min(16, O.default_workers())))
    g = _solve(ctx, seeds, 40, prec, True, 64)
    idx = _slots(sysm.H, seeds)
    r_rho, r_e = _rel(g.rho[idx], ref.rho[idx]), abs(g.e_band - ref.e_band) / abs(ref.e_band)
    print(f"[support vs oracle {prec}] rho {r_rho:.2e} E_band {r_e:.2e}", flush=True)
    assert np.array_equal(g.nu_eff, ref.nu_eff)
    assert r_rho <= TOL[prec] and r_e <= TOL[prec]


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7])
def test_support_projection_variants(sysm, ctx, variant):
    seeds = np.arange(500, 500 + 300, dtype=np.int32)
    a = _solve(ctx, seeds, 30, "fp32", True, 128, variant)
    b = _solve(ctx, seeds, 30, "fp32", False, 128, variant)
    idx = _slots(sysm.H, seeds)
    assert np.array_equal(a.nu_eff, b.nu_eff)
    assert _rel(a.rho[idx], b.rho[idx]) <= TOL["fp32"]


@pytest.mark.parametrize("support", [True, False])
def test_fp32_update_fp64_sums_against_oracle(sysm, ctx, support):
    """nu = 140 (> 128): the FP32 form's update keeps its running sums in FP64, over the tile list with support
    tracking and over whole slabs without; every rho column, E_j and N_j against the oracle at 1e-5."""
    seeds = np.arange(2500, 2500 + 40, dtype=np.int32)
    ref = O.solve(sysm.H, sysm.S, seeds, 140, -0.3, KT, workers=max(1, min(16, O.default_workers())))
    g = _solve(ctx, seeds, 140, "fp32", support, 64)
    assert np.array_equal(g.nu_eff, ref.nu_eff)
    worst = 0.0
    for j in seeds:
        lo, hi = sysm.H.indptr[j], sysm.H.indptr[j + 1]
        worst = max(worst, _rel(g.rho[lo:hi], ref.rho[lo:hi]))
    e_err = np.abs(g.e_seed - ref.e_seed) / np.maximum(np.abs(ref.e_seed), 1e-2 * np.abs(ref.e_seed).max())
    n_err = np.abs(g.n_seed - ref.n_seed) / np.maximum(np.abs(ref.n_seed), 2e-2)
    print(f"[fp64 update sums, support={support}] worst rho column {worst:.2e} E_j {e_err.max():.2e} "
          f"N_j {n_err.max():.2e}", flush=True)
    assert worst <= TOL["fp32"] and e_err.max() <= TOL["fp32"] and n_err.max() <= TOL["fp32"]


@pytest.mark.parametrize("B", [2, 4])
def test_fp32_update_fp64_sums_narrow_blocks(sysm, ctx, B):
    """The FP64 update sums with blocks narrower than a 16-byte vector (B = 2: whole-slab update, scalar
    coefficient loads) and exactly one vector wide (B = 4), nu = 140, against the oracle per rho column."""
    seeds = np.array([5, 900, 1801, 3333, 5000, 6911, 77], dtype=np.int32)   # ragged last block
    ref = O.solve(sysm.H, sysm.S, seeds, 140, -0.3, KT, workers=max(1, min(16, O.default_workers())))
    g = _solve(ctx, seeds, 140, "fp32", True, B)
    assert np.array_equal(g.nu_eff, ref.nu_eff)
    worst = max(_rel(g.rho[sysm.H.indptr[j]:sysm.H.indptr[j + 1]], ref.rho[sysm.H.indptr[j]:sysm.H.indptr[j + 1]])
                for j in seeds)
    print(f"[fp64 update sums, B={B}] worst rho column {worst:.2e}", flush=True)
    assert worst <= TOL["fp32"]


@pytest.mark.parametrize("nu", [1, 2, 3])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_support_short_subspaces(sysm, ctx, prec, nu):
    seeds = np.arange(0, 77, dtype=np.int32)
    ref = O.solve(sysm.H, sysm.S, seeds, nu, -0.3, KT)
    g = _solve(ctx, seeds, nu, prec, True, 32)
    idx = _slots(sysm.H, seeds)
    assert np.array_equal(g.nu_eff, ref.nu_eff)
    assert _rel(g.rho[idx], ref.rho[idx]) <= TOL[prec]


def test_support_blocks_in_sequence(sysm, ctx):
    """A block far from the previous one: nothing of the earlier block's vectors may leak into it."""
    s1 = np.arange(0, 64, dtype=np.int32)
    s2 = np.arange(sysm.M - 64, sysm.M, dtype=np.int32)
    s3 = np.arange(sysm.M // 2, sysm.M // 2 + 64, dtype=np.int32)
    seq = _solve(ctx, np.concatenate([s1, s2, s3]), 30, "fp32", True, 64)
    for k, blk in enumerate((s1, s2, s3)):
        alone = _solve(ctx, blk, 30, "fp32", True, 64)
        assert np.array_equal(seq.nu_eff[64 * k:64 * (k + 1)], alone.nu_eff)
        assert np.array_equal(seq.e_seed[64 * k:64 * (k + 1)], alone.e_seed)


def test_support_profile_bytes(sysm, ctx):
    """Profiled restricted byte counts: below the full sweep for neighbouring seeds, equal for the full sweep."""
    seeds = np.arange(2000, 2000 + 256, dtype=np.int32)
    out = {}
    for support in (True, False):
        ctx.set_tuning(seed_block=64, schedule="delayed", support=support)
        ctx.profile(True)
        ctx.profile_reset()
        try:
            ctx.solve(seeds, 40, -0.3, KT, precision="fp32", form="batched")
            out[support] = ctx.profile_collect()
        finally:
            ctx.profile(False)
            ctx.set_tuning()
    on, off = out[True]["dcgs_proj"], out[False]["dcgs_proj"]
    print(f"[support bytes] proj {on['bytes'] / off['bytes']:.3f} upd "
          f"{out[True]['dcgs_upd']['bytes'] / out[False]['dcgs_upd']['bytes']:.3f}", flush=True)
    assert on["launches"] == off["launches"]
    assert 0.05 * off["bytes"] < on["bytes"] < 0.95 * off["bytes"]
    assert out[True]["dcgs_upd"]["bytes"] < out[False]["dcgs_upd"]["bytes"]
    # per block of 64: one support build and one launch that plans the projections of all steps
    assert out[True]["support"]["launches"] == 4 * (1 + 1)
    assert out[False]["support"]["launches"] == 0


@pytest.mark.parametrize("prec,form,B", [("fp64", "plain", 0), ("fp32", "plain", 0), ("fp32", "batched", 16)])
def test_textbook_eig_overlap_bit_equal(sysm, ctx, prec, form, B):
    """The plain form (and the textbook schedule of the batched form): each block's eigensolve on the second
    stream gives the same results as everything on one stream."""
    seeds = np.arange(300, 300 + (9 if form == "plain" else 3 * B + 5), dtype=np.int32)
    out = []
    for ovl in (True, False):
        ctx.set_tuning(seed_block=B, schedule="textbook", two_streams=False, overlap_eig=ovl)
        try:
            out.append(ctx.solve(seeds, 30, -0.3, KT, precision=prec, form=form, levels=True))
        finally:
            ctx.set_tuning()
    o, ref = out
    assert np.array_equal(o.rho, ref.rho) and o.e_band == ref.e_band
    assert np.array_equal(o.nu_eff, ref.nu_eff) and np.array_equal(o.eps, ref.eps)
    assert np.array_equal(o.weight, ref.weight) and np.array_equal(o.e_seed, ref.e_seed)


@pytest.mark.parametrize("prec,B", [("fp32", 64), ("fp64", 32)])
def test_two_streams_bit_equal(sysm, ctx, prec, B):
    """Alternating seed blocks between two workspaces and streams, or running each block's eigensolve on
    the second stream (the default), changes nothing in the results."""
    seeds = np.arange(100, 100 + 5 * B + 11, dtype=np.int32)
    out = []
    for two, ovl in ((True, True), (False, True), (False, False)):
        ctx.set_tuning(seed_block=B, schedule="delayed", two_streams=two, overlap_eig=ovl)
        try:
            out.append(ctx.solve(seeds, 30, -0.3, KT, precision=prec, form="batched", levels=True))
        finally:
            ctx.set_tuning()
    ref = out[2]
    for o in out[:2]:
        assert np.array_equal(o.rho, ref.rho) and o.e_band == ref.e_band
        assert np.array_equal(o.nu_eff, ref.nu_eff) and np.array_equal(o.eps, ref.eps)
        assert np.array_equal(o.weight, ref.weight) and np.array_equal(o.e_seed, ref.e_seed)
