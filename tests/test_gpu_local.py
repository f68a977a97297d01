"""Local regions (order-N form) on the GPU against the local-region oracle.

Each seed's Krylov subspace is generated on the rows within r block hops of it
(the method on the principal submatrices); the library applies per-seed region
masks to the H and S products and skips the tiles outside every region of a
block. Checked: parity with the oracle in FP64 and FP32, the exact exhausted
region, r >= nu - 1 equal to the full solve, independence of block size and
seed order, the graph-launched path, and the refusals.
"""
import numpy as np
import pytest

from oracle import mar_local as OL
from paper_1307_3218_amd import lattice, mar

pytestmark = pytest.mark.gpu

KT = 0.1
MU = -0.3
TOL = {"fp64": 1e-10, "fp32": 1e-5}


def _slots(H, seeds):
    return np.concatenate([np.arange(H.indptr[j], H.indptr[j + 1]) for j in seeds])


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def sysm():
    return lattice.generate(6, 6, 6, mixed=True, seed=3)     # M = 6912


@pytest.fixture(scope="module")
def ctx(sysm):
    c = mar.Context(sysm.H, sysm.S)
    yield c
    c.close()


def _solve(ctx, seeds, nu, r, prec, B=0, form="batched"):
    ctx.set_local_region(r)
    ctx.set_tuning(seed_block=B)
    try:
        return ctx.solve(np.asarray(seeds, dtype=np.int32), nu, MU, KT, precision=prec, form=form, levels=True)
    finally:
        ctx.set_tuning()
        ctx.set_local_region(None)


def _check(sysm, seeds, g, ref, prec, label):
    idx = _slots(sysm.H, seeds)
    r_rho, r_e = _rel(g.rho[idx], ref.rho[idx]), abs(g.e_band - ref.e_band) / abs(ref.e_band)
    print(f"[local {label} {prec}] rho {r_rho:.2e} E_band {r_e:.2e}", flush=True)
    assert np.array_equal(g.nu_eff, ref.nu_eff)
    assert r_rho <= TOL[prec] and r_e <= TOL[prec]


# 6 and 7 hops run two seed blocks in flight by default (three and four blocks here)
@pytest.mark.parametrize("prec,B,r", [("fp64", 8, 2), ("fp64", 32, 3), ("fp32", 64, 2), ("fp32", 256, 4),
                                      ("fp32", 32, 6), ("fp64", 16, 7)])
def test_local_against_oracle(sysm, ctx, prec, B, r):
    seeds = np.arange(2000, 2000 + 2 * B + 19)
    ref = OL.solve_local(sysm.H, sysm.S, seeds, 30, r, MU, KT)
    g = _solve(ctx, seeds, 30, r, prec, B)
    _check(sysm, seeds, g, ref, prec, f"r={r} B={B}")


@pytest.mark.parametrize("r", [0, 1])
def test_local_exhausted_region(sysm, ctx, r):
    """nu beyond the region's size: breakdown where the region is exhausted, exact submatrix answer."""
    seeds = np.arange(100, 140)
    ref = OL.solve_local(sysm.H, sysm.S, seeds, 40, r, MU, KT)
    assert ref.nu_eff.max() < 40
    g = _solve(ctx, seeds, 40, r, "fp64", 8)
    _check(sysm, seeds, g, ref, "fp64", f"exhausted r={r}")


def test_wide_region_is_full_solve(sysm, ctx):
    seeds = np.arange(500, 600)
    loc = _solve(ctx, seeds, 12, 11, "fp64", 32)
    ctx.set_tuning(seed_block=32)
    try:
        full = ctx.solve(seeds.astype(np.int32), 12, MU, KT, precision="fp64")
    finally:
        ctx.set_tuning()
    idx = _slots(sysm.H, seeds)
    assert np.array_equal(loc.nu_eff, full.nu_eff)
    assert _rel(loc.rho[idx], full.rho[idx]) <= 1e-12


def test_local_independent_of_blocking(sysm, ctx):
    seeds = np.arange(3000, 3200)
    a = _solve(ctx, seeds, 25, 3, "fp64", 16)
    perm = np.random.default_rng(1).permutation(len(seeds))
    b = _solve(ctx, seeds[perm], 25, 3, "fp64", 128)
    inv = np.argsort(perm)
    assert np.array_equal(a.nu_eff, b.nu_eff[inv])
    assert np.abs(a.e_seed - b.e_seed[inv]).max() <= 1e-12 * np.abs(a.e_seed).max()


def test_local_graph_launch(sysm):
    """Two local radii through one graph launch, on fresh contexts (mar_solve_many refuses a context that
    ran two seed blocks in flight, as the module's context has at 6 and 7 hops)."""
    import torch
    dev = torch.device("cuda:0")
    ctx = mar.Context(sysm.H, sysm.S)
    other = mar.Context(sysm.H, sysm.S)
    try:
        ctx.set_local_region(2)
        other.set_local_region(5)
        seeds = torch.arange(0, 300, dtype=torch.int32, device=dev)
        reqs = [dict(d_seeds=seeds, nu=20, mu=MU, kT=KT, precision="fp32", form="batched",
                     d_rho=torch.zeros(sysm.H.nnz, dtype=torch.float64, device=dev),
                     d_e_band=torch.zeros(1, dtype=torch.float64, device=dev)) for _ in range(2)]
        out = []
        for _ in range(3):
            mar.solve_many([ctx, other], reqs)
            torch.cuda.synchronize()
            out.append([float(r["d_e_band"]) for r in reqs])
        for c, r in zip((ctx, other), reqs):
            e = torch.zeros(1, dtype=torch.float64, device=dev)
            c.solve_async(seeds, 20, MU, KT, "fp32", "batched", d_rho=torch.zeros_like(r["d_rho"]), d_e_band=e)
            torch.cuda.synchronize()
            for rep in out:
                assert rep[[ctx, other].index(c)] == float(e)
        ref = OL.solve_local(sysm.H, sysm.S, np.arange(300), 20, 2, MU, KT)
        assert abs(out[0][0] - ref.e_band) <= TOL["fp32"] * abs(ref.e_band)
    finally:
        ctx.close()
        other.close()


def test_local_stream_modes_bit_equal(sysm, ctx):
    """Local regions of 6 hops: the library's default (two blocks in flight), one block at a time with the
    eigensolve on the second stream, and everything on one stream give identical results."""
    seeds = np.arange(40, 40 + 5 * 32 + 7, dtype=np.int32)
    out = []
    ctx.set_local_region(6)
    try:
        for two, ovl in ((None, True), (True, True), (False, True), (False, False)):
            ctx.set_tuning(seed_block=32, two_streams=two, overlap_eig=ovl)
            out.append(ctx.solve(seeds, 24, MU, KT, precision="fp32", form="batched", levels=True))
    finally:
        ctx.set_tuning()
        ctx.set_local_region(None)
    ref = out[3]
    for o in out[:3]:
        assert np.array_equal(o.rho, ref.rho) and o.e_band == ref.e_band
        assert np.array_equal(o.nu_eff, ref.nu_eff) and np.array_equal(o.eps, ref.eps)
        assert np.array_equal(o.weight, ref.weight) and np.array_equal(o.e_seed, ref.e_seed)


def test_local_refusals(sysm, ctx):
    seeds = np.arange(10, dtype=np.int32)
    ctx.set_local_region(2)
    try:
        with pytest.raises(mar.MarError):
            ctx.solve(seeds, 10, MU, KT, precision="fp64", form="plain")
        ctx.set_tuning(seed_block=2)
        with pytest.raises(mar.MarError):
            ctx.solve(seeds, 10, MU, KT, precision="fp32")
        ctx.set_tuning()
        with pytest.raises(mar.MarError):
            ctx.eigen_state(seeds, 10, 3, 0.01)
        assert ctx.local_region() == 2
    finally:
        ctx.set_tuning()
        ctx.set_local_region(None)
    assert ctx.local_region() == -1
    # a pattern without 4x4 blocks cannot take a local region
    cell256 = lattice.workload("diamond_2x2x2")
    import scipy.sparse as sp
    H = sp.csr_matrix(cell256.H)[:255, :255]
    S = sp.csr_matrix(cell256.S)[:255, :255]
    c = mar.Context(H, S)
    try:
        with pytest.raises(mar.MarError):
            c.set_local_region(1)
    finally:
        c.close()


def test_solve_many_refuses_after_two_blocks_in_flight(sysm):
    """A context that ran two seed blocks in flight (the default at 6 hops) is refused by mar_solve_many before
    any capture: host crashes followed that sequence and their cause is not known."""
    import torch
    dev = torch.device("cuda:0")
    c = mar.Context(sysm.H, sysm.S)
    try:
        c.set_local_region(6)
        c.set_tuning(seed_block=32)
        seeds = np.arange(40, 40 + 3 * 32, dtype=np.int32)
        c.solve(seeds, 24, MU, KT, precision="fp32")                 # three blocks: two in flight
        req = dict(d_seeds=torch.from_numpy(seeds).to(dev), nu=24, mu=MU, kT=KT, precision="fp32",
                   form="batched", d_rho=torch.zeros(sysm.H.nnz, dtype=torch.float64, device=dev),
                   d_e_band=torch.zeros(1, dtype=torch.float64, device=dev))
        with pytest.raises(mar.MarError) as e:
            mar.solve_many([c], [req])
        assert e.value.status == mar.MAR_ERR_STATE
        assert "two seed blocks in flight" in mar.mar_last_error(c.handle)
        c.set_tuning(seed_block=32, two_streams=False)                # still refused: the context ran them
        with pytest.raises(mar.MarError):
            mar.solve_many([c], [req])
    finally:
        c.close()
