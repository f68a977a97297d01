#!/usr/bin/env python3
"""Throughput of the mArnoldi per-seed hot path on one MI355X.

Workload: the 32768-atom mixed sp2/sp3 lattice (M = 131072, 4 orbitals per
atom, seeded synthetic H and S), nu = 100, kT = 0.1 eV, mu at half filling.
A step is one pass of the whole hot path (Krylov subspace + CGS2 + subspace
eigensolve + Fermi-weighted assembly + band-energy sum) over one batch of
seeds, in the batched FP32 form, with seeds, outputs and H/S resident in HBM.
Seeds go in their natural order (a block holds orbitals of neighbouring atoms,
whose early Krylov vectors are zero on most rows); --seed-order random or
sampled changes that, --no-support streams every row of every slab.
Reported: seed-subspaces/s of that form; beside it the plain FP64 form on the
same GPU (one seed at a time), the per-kernel roofline from HIP events on the
solve stream, and the FP64 CPU oracle on a bounded seed sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Other workloads (not the headline line):
    --workload uneven8   the eight uneven diamond systems (M = 1024 ... 65536,
                         nu alternating 30/100), every seed of every system,
                         FP32 batched through mar_solve_many (one graph launch
                         per call, autotuned block sizes), beside the same work
                         issued eagerly system after system.
    --workload mixed_32x32x32 --nu 300 --seed-order sampled   the M = 1048576
                         lattice (seed blocks of 64) over its 16384 sampled seeds.
    --workload eigenstate  the k-th eigen state (Sec. 3, Eq. 3) of the 4096-atom
                         diamond cell (M = 16384, nu = 30, every seed, FP32
                         batched): two passes over all seeds plus the reference.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "seed-subspaces/s at ν=100, M=131072: FP32-batched vs FP64 plain; SpMM HBM %"
# the same measurement on another workload or subspace dimension names its own
METRIC_OTHER = "seed-subspaces/s at ν={nu}, M={M}: FP32-batched vs FP64 plain; SpMM HBM %"
METRIC_LOCAL = "seed-subspaces/s, local regions of {r} block hops (order-N form), FP32 batched"
HBM_PEAK_GBPS = 8000.0
KT = 0.1


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter summary, or None.

    The summary records a hash of the kernel sources it was measured on; when the
    sources have changed since, the figure no longer describes the current kernels (None).
    """
    import glob
    import hashlib
    src = b"".join(open(os.path.join(ROOT, "paper_1307_3218_amd", "csrc", f), "rb").read()
                   for f in ("mar_launch_impl.h", "mar_device.h", "mar_support.hip"))
    sha = hashlib.sha256(src).hexdigest()[:16]
    for path in glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md")):
        text = open(path).read()
        for block in text.split("```json")[1:]:
            try:
                rec = json.loads(block.split("```")[0])
            except ValueError:
                continue
            if rec.get("kernel") == kernel and rec.get("workload") == workload and \
                    rec.get("kernel_source_sha256_16") == sha:
                return float(rec["traffic_bytes_per_launch"])
    return None


def cpu_baseline(system, nu, mu, n_seeds, workers):
    """The oracle as it stands, on a bounded seed sample, process-parallel over host cores."""
    from oracle import mar_oracle as O
    from paper_1307_3218_amd import lattice
    seeds = lattice.sample_seeds(system.M, n_seeds, seed=99)
    t0 = time.perf_counter()
    ref = O.solve(system.H, system.S, seeds, nu, mu, KT, workers=workers)
    dt = time.perf_counter() - t0
    return dict(value=n_seeds / dt, unit="seed-subspaces/s", cores=workers, kind="oracle",
                sample=f"{n_seeds} uniformly sampled seeds of the same workload (nu={nu}), "
                       f"FP64 NumPy/SciPy, one process per core, {dt:.1f} s wall"), seeds, ref


def copy_rate(torch, dev, mib=1024, reps=3):
    """Bytes read + written per second by a 1 GiB device-to-device copy (best of reps)."""
    a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
    c = torch.empty_like(a)
    best = float("inf")
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t = time.perf_counter()
        c.copy_(a)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    del a, c
    return 2.0 * mib * (1 << 20) / best / 1e9


def errors_vs_oracle(ctx, system, seeds, ref, nu, mu):
    """Per-result error of the device forms against the oracle on the oracle's seeds."""
    H = system.H
    idx = np.concatenate([np.arange(H.indptr[j], H.indptr[j + 1]) for j in seeds])
    from oracle import mar_oracle as O
    out = {}
    for prec, form in (("fp32", "batched"), ("fp64", "batched"), ("fp64", "plain")):
        g = ctx.solve(np.asarray(seeds, dtype=np.int32), nu, mu, KT, precision=prec, form=form, levels=True)
        # invariants of the device outputs alone: sum_a w_a = 1, N_j = 2 sum f w, E_j = 2 sum f eps w
        mask = np.arange(nu)[None, :] < g.nu_eff[:, None]
        w = np.where(mask, g.weight, 0.0)
        fw = np.where(mask, O.fermi(g.eps, mu, KT), 0.0) * w
        out[f"{prec}_{form}"] = dict(
            e_band_rel=float(abs(g.e_band - ref.e_band) / abs(ref.e_band)),
            rho_rel=float(np.linalg.norm(g.rho[idx] - ref.rho[idx]) / np.linalg.norm(ref.rho[idx])),
            e_seed_max_abs=float(np.abs(g.e_seed - ref.e_seed).max()),
            n_seed_max_abs=float(np.abs(g.n_seed - ref.n_seed).max()),
            nu_eff_equal=bool(np.array_equal(g.nu_eff, ref.nu_eff)),
            weight_sum_minus_1_max=float(np.abs(w.sum(axis=1) - 1.0).max()),
            n_seed_vs_levels_max=float(np.abs(g.n_seed - 2.0 * fw.sum(axis=1)).max()),
            e_seed_vs_levels_max=float(np.abs(g.e_seed - 2.0 * (fw * np.where(mask, g.eps, 0.0)).sum(axis=1)).max()))
    return out


def cpu_baseline_local(system, nu, mu, r, budget_s=12.0):
    """The local-region oracle, serial, on neighbouring seeds until about budget_s of CPU work."""
    from oracle import mar_local as OL
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s and n < system.M:
        OL.solve_local(system.H, system.S, np.arange(n, min(n + 8, system.M)), nu, r, mu, KT)
        n = min(n + 8, system.M)
    dt = time.perf_counter() - t0
    return dict(value=n / dt, unit="seed-subspaces/s", cores=1, kind="oracle",
                sample=f"seeds 0..{n - 1} of the same workload (nu={nu}, regions of {r} hops), FP64 NumPy/SciPy, "
                       f"one process, {dt:.1f} s wall")


def run_uneven(args) -> int:
    """All seeds of the eight uneven systems: graph-launched batches vs eager per-system solves."""
    import torch
    from paper_1307_3218_amd import lattice, mar
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    calls = max(1, args.uneven_calls)
    mu = -0.45
    systems, ctxs, reqs, seeds_all = [], [], [], []
    t = time.perf_counter()
    for i, cells in enumerate(lattice.UNEVEN_SYSTEMS):
        s = lattice.generate(*cells, mixed=False, seed=0)
        nu = 30 if i % 2 == 0 else 100
        systems.append((s, nu))
        ctxs.append(mar.Context(s.H, s.S))
    log(f"8 systems built ({time.perf_counter() - t:.1f} s): M = {[s.M for s, _ in systems]}")
    tuned = []
    for (s, nu), c in zip(systems, ctxs):
        perm = np.arange(s.M) if args.seed_order != "random" else np.random.default_rng(0).permutation(s.M)
        order = torch.from_numpy(perm.astype(np.int32)).to(dev)
        seeds_all.append(order)
        tuned.append(c.autotune(order[: min(256, s.M)], nu, mu, KT, "fp32"))
        n = s.M // calls
        reqs.append(dict(d_seeds=torch.empty(n, dtype=torch.int32, device=dev), nu=nu, mu=mu, kT=KT,
                         precision="fp32", form="batched",
                         d_rho=torch.zeros(s.H.nnz, dtype=torch.float64, device=dev),
                         d_e_band=torch.zeros(1, dtype=torch.float64, device=dev)))
    log("autotuned (B, variant): " + ", ".join(f"M={s.M}:{t_['seed_block']}/{t_['proj_variant']}"
                                                for (s, _), t_ in zip(systems, tuned)))
    total = sum(s.M for s, _ in systems)

    def graph_pass():
        e = 0.0
        for k in range(calls):
            for (s, _), r, order in zip(systems, reqs, seeds_all):
                n = r["d_seeds"].numel()
                r["d_seeds"].copy_(order[k * n:(k + 1) * n])
            mar.solve_many(ctxs, reqs)
            e += float(sum(r["d_e_band"] for r in reqs))   # synchronizes; E summed over calls
        return e

    def eager_pass():
        e = 0.0
        for (s, nu), c, r, order in zip(systems, ctxs, reqs, seeds_all):
            c.solve_async(order, nu, mu, KT, "fp32", "batched", d_rho=r["d_rho"], d_e_band=r["d_e_band"])
            e += float(r["d_e_band"])
        return e

    t = time.perf_counter()
    graph_pass()            # captures the graph once (identical shapes on every call)
    torch.cuda.synchronize()
    log(f"warmup pass (with capture): {time.perf_counter() - t:.1f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_graph = graph_pass()
    torch.cuda.synchronize()
    dt_graph = time.perf_counter() - t0
    t0 = time.perf_counter()
    e_eager = eager_pass()
    torch.cuda.synchronize()
    dt_eager = time.perf_counter() - t0
    log(f"graph: {total} seeds in {dt_graph:.2f} s; eager: {dt_eager:.2f} s; E_band {e_graph:.6f} / {e_eager:.6f}")
    out = {
        "metric": "seed-subspaces/s, 8 uneven diamond systems, FP32 batched, graph-launched",
        "value": round(total / dt_graph, 3), "unit": "seed-subspaces/s", "n_gpus": 1, "steps": calls, "warmup": calls,
        "ms_per_step": round(1e3 * dt_graph / calls, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "8 diamond systems M=1024..65536, nu 30/100 alternating, all seeds",
                   "M": [s.M for s, _ in systems], "nu": [nu for _, nu in systems], "seeds": total,
                   "calls_per_pass": calls, "mu": mu,
                   "autotuned": [dict(M=s.M, B=t_["seed_block"], variant=t_["proj_variant"])
                                 for (s, _), t_ in zip(systems, tuned)]},
        "eager_sequential": {"value": round(total / dt_eager, 3), "unit": "seed-subspaces/s"},
        "e_band_graph_minus_eager": e_graph - e_eager,
    }
    print(json.dumps(out), flush=True)
    for c in ctxs:
        c.close()
    return 0


def run_eigenstate(args) -> int:
    """Time the eigen-state extension (HO level, k = M/2) over every seed of the M = 16384 cell."""
    import torch
    from paper_1307_3218_amd import lattice, mar
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    s = lattice.workload("diamond_8x8x8")
    nu, k, sigma = 30, s.M // 2, 0.002
    ctx = mar.Context(s.H, s.S)
    seeds = torch.arange(s.M, dtype=torch.int32, device=dev)
    d_phi = torch.zeros(s.M, dtype=torch.float64, device=dev)
    d_lv = torch.zeros(3, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream().cuda_stream

    def once():
        st = mar.mar_eigen_state_async(ctx.handle, seeds, s.M, nu, k, sigma, mar.PRECISION["fp32"],
                                       mar.FORM["batched"], d_phi, d_lv, None, stream)
        if st != mar.MAR_OK:
            raise mar.MarError(st, mar.mar_last_error(ctx.handle))
        torch.cuda.synchronize()

    once()
    times = []
    for _ in range(max(1, args.steps)):
        t0 = time.perf_counter()
        once()
        times.append(time.perf_counter() - t0)
    dt = sorted(times)[len(times) // 2]
    lv = d_lv.cpu().numpy()
    phi = d_phi.cpu().numpy()
    log(f"eigen state k={k}: eps_k {lv[0]:.6f} eV in [{lv[1]:.6f}, {lv[2]:.6f}]; {dt:.3f} s; |phi| {np.linalg.norm(phi):.4f}")
    # local flipping refinement of that vector (Appendix), up to 100 sweeps
    flip = None
    if not args.no_flip:
        d_x = d_phi.clone()
        d_R = torch.zeros(101, dtype=torch.float64, device=dev)
        d_info = torch.zeros(2, dtype=torch.int32, device=dev)
        ctx.flip_colours()                                   # the colouring is built once, outside the timing
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = mar.mar_local_flip(ctx.handle, d_x, float(lv[0]), None, 0.0, 100, d_R, d_info, stream)
        if st != mar.MAR_OK:
            raise mar.MarError(st, mar.mar_last_error(ctx.handle))
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        info = d_info.cpu().numpy()
        R = d_R.cpu().numpy()[: int(info[0]) + 1]
        flip = dict(seconds=round(tf, 4), sweeps=int(info[0]), flips=int(info[1]), colours=ctx.flip_colours(),
                    R_before=float(R[0]), R_after=float(R[-1]))
        log(f"local flipping: {info[0]} sweeps, {info[1]} flips, R {R[0]:.4e} -> {R[-1]:.4e} in {tf * 1e3:.1f} ms")
        if not args.no_cpu_baseline:
            # the flip oracle on the same vector, on one host core: its time, and the same refined vector
            from oracle import mar_flip as OF
            col = OF.distance2_colouring(s.H)
            t0 = time.perf_counter()
            ref = OF.local_flip(s.H, s.S, phi, float(lv[0]), max_sweeps=100, colour=col)
            tc = time.perf_counter() - t0
            same = bool(np.array_equal(ref.phi, d_x.cpu().numpy())) and ref.flips == flip["flips"]
            flip["cpu_baseline"] = dict(value=round(tc, 3), unit="s", cores=1, kind="oracle",
                                        sample="the same eigen-state vector (all 16384 components), 100 sweeps max")
            flip["equal_to_oracle"] = same
            log(f"flip oracle: {tc:.2f} s on one core; refined vector equal to the device's: {same}")
    out = {
        "metric": "eigen state (Sec. 3, Eq. 3): time for one level and vector over every seed",
        "value": round(dt, 4), "unit": "s", "n_gpus": 1, "steps": len(times), "warmup": 1,
        "ms_per_step": round(1e3 * dt, 3), "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "diamond 8x8x8 cell, M=16384, nu=30, all seeds, k=M/2, sigma=0.002 eV",
                   "M": s.M, "nu": nu, "k": k, "sigma": sigma},
        "eps_k": float(lv[0]), "eta_lo": float(lv[1]), "eta_hi": float(lv[2]),
        "seed_subspaces_per_s": round(2 * s.M / dt, 1),
        "local_flip": flip,
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mixed_16x16x16")
    ap.add_argument("--nu", type=int, default=100)
    ap.add_argument("--seeds-per-step", type=int, default=1024)
    ap.add_argument("--plain-seeds", type=int, default=256)
    ap.add_argument("--fp64-batched-seeds", type=int, default=256)
    ap.add_argument("--cpu-seeds", type=int, default=0, help="oracle sample size (0 = about 20 s of CPU work)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--seed-block", type=int, default=0)
    ap.add_argument("--seed-order", choices=["natural", "random", "sampled"], default="natural",
                    help="natural: consecutive seeds (neighbouring atoms) share a block; random: a permutation of "
                         "all seeds; sampled: a sorted uniform sample of min(M, 16384) seeds")
    ap.add_argument("--no-support", action="store_true", help="stream every row of every slab")
    ap.add_argument("--proj-variant", type=int, default=0,
                    help="projection variant of the delayed schedule (0 = the autotuned or default choice)")
    ap.add_argument("--two-streams", action="store_true",
                    help="two seed blocks in flight on two streams (default: the library's choice, which is "
                         "two blocks for local regions of 6 hops or more and one block at a time otherwise)")
    ap.add_argument("--one-block", action="store_true",
                    help="one seed block at a time, each block's eigensolve on the second stream")
    ap.add_argument("--no-flip", action="store_true", help="eigenstate: skip the local flipping refinement")
    ap.add_argument("--r-cut", type=int, default=-1, metavar="HOPS",
                    help="local regions of HOPS block hops (the order-N form; a different computation from the "
                         "headline line, reported under its own metric); the seed block is autotuned unless given")
    ap.add_argument("--uneven-calls", type=int, default=8,
                    help="uneven8: mar_solve_many calls per pass over all seeds (each takes M/calls seeds per system)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="first run a plain device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the per-seed subspaces are independent, and a multi-GPU run "
              "would shard the seed list (no collective on the hot path). Run with --gpus 1.", file=sys.stderr)
        return 2

    if args.workload == "uneven8":
        return run_uneven(args)
    if args.workload == "eigenstate":
        return run_eigenstate(args)
    from oracle import mar_oracle as O
    from paper_1307_3218_amd import lattice, mar
    t = time.perf_counter()
    system = lattice.workload(args.workload)
    M, nu = system.M, args.nu
    log(f"workload {system.name}: M={M} nnz={system.H.nnz} lambda_min(S)={system.lam_min_S:.3f} "
        f"({time.perf_counter() - t:.1f} s)")

    import torch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        c = torch.empty_like(a)
        c.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + {args.copy_calibration} MiB written")
        del a, c
    ctx = mar.Context(system.H, system.S)
    ctx.set_tuning(args.seed_block, support=not args.no_support, proj_variant=args.proj_variant,
                   two_streams=True if args.two_streams else (False if args.one_block else None))
    local = args.r_cut >= 0
    if local:
        ctx.set_local_region(args.r_cut)
        args.no_plain = True                       # the plain form has no local regions
        if not args.seed_block:
            tn = ctx.autotune(torch.from_numpy(np.arange(min(M, 1024), dtype=np.int32)).to(dev), nu, 0.0, KT, "fp32")
            log(f"local regions of {args.r_cut} hops: autotuned block {tn['seed_block']}, variant {tn['proj_variant']}")
    B = ctx.seed_block(nu, "fp32")
    S_step = args.seeds_per_step
    stream = torch.cuda.current_stream().cuda_stream
    if args.seed_order == "natural":
        order = np.arange(M, dtype=np.int32)
    elif args.seed_order == "sampled":
        order = lattice.sample_seeds(M, min(M, 16384), seed=0).astype(np.int32)
    else:
        order = np.random.default_rng(0).permutation(M).astype(np.int32)
    n_steps = args.warmup + args.steps
    d_order = torch.from_numpy(order).to(dev)

    def seeds_for(k):
        lo = (k * S_step) % len(order)
        return d_order[lo: lo + S_step]

    d_rho = torch.zeros(system.H.nnz, dtype=torch.float64, device=dev)
    d_eb = torch.zeros(1, dtype=torch.float64, device=dev)
    d_e = torch.zeros(S_step, dtype=torch.float64, device=dev)
    d_n = torch.zeros(S_step, dtype=torch.float64, device=dev)
    d_nu = torch.zeros(S_step, dtype=torch.int32, device=dev)
    d_eps = torch.zeros((S_step, nu), dtype=torch.float64, device=dev)
    d_w = torch.zeros((S_step, nu), dtype=torch.float64, device=dev)

    # warmup: the first pass finds the half-filling Fermi level of its seeds on the device
    # (levels kept, mu bisected, then assembled); later passes reuse that mu
    mu = 0.0
    fermi_info = None
    d_mu = torch.zeros(1, dtype=torch.float64, device=dev)
    for k in range(args.warmup):
        t = time.perf_counter()
        if k == 0:
            ctx.profile(True)
            ctx.profile_reset()
            ctx.solve_fermi_async(seeds_for(k), nu, float(S_step), KT, "fp32", "batched", d_rho=d_rho, d_e_band=d_eb,
                                  d_mu=d_mu, d_e_seed=d_e, d_n_seed=d_n, d_nu_eff=d_nu, d_eps=d_eps, d_weight=d_w,
                                  stream=stream)
            torch.cuda.synchronize()
            fs = ctx.profile_collect().get("fermi_search")
            ctx.profile(False)
            mu = float(d_mu.cpu()[0])
            nue = d_nu.cpu().numpy()
            # the oracle's bisection on the device's levels and weights, as a check of the device search
            h_eps, h_w = d_eps.cpu().numpy(), d_w.cpu().numpy()
            eps_l = [h_eps[i, :m] for i, m in enumerate(nue) if m > 0]
            w_l = [h_w[i, :m] for i, m in enumerate(nue) if m > 0]
            mu_host = O.fermi_level(eps_l, w_l, float(S_step), KT)
            # sum rule: the seeds' electron count at the device's mu equals the target (half filling)
            n_at_mu = O.electron_count(eps_l, w_l, mu, KT)
            fermi_info = dict(mu=mu, seeds=S_step, search_ms=round(fs["ms"], 3) if fs else None,
                              host_bisection_mu=mu_host, electron_count_at_mu=n_at_mu,
                              electron_count_rel_error=abs(n_at_mu - float(S_step)) / float(S_step))
            log(f"half-filling Fermi level from {S_step} seeds on the device: mu = {mu:.6f} eV "
                f"(host bisection {mu_host:.6f}); search {fermi_info['search_ms']} ms; nu_eff min {nue.min()}")
        else:
            ctx.solve_async(seeds_for(k), nu, mu, KT, "fp32", "batched", d_rho=d_rho, d_e_band=d_eb, d_e_seed=d_e,
                            d_n_seed=d_n, d_nu_eff=d_nu, stream=stream)
            torch.cuda.synchronize()
        log(f"warmup step {k}: {time.perf_counter() - t:.2f} s")

    # timed region: the batched FP32 form (no per-kernel events: with --two-streams the library alternates
    # seed blocks between two streams, which its profiling mode does not)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, n_steps):
        ctx.solve_async(seeds_for(k), nu, mu, KT, "fp32", "batched", d_rho=d_rho, d_e_band=d_eb, d_e_seed=d_e,
                        d_n_seed=d_n, d_nu_eff=d_nu, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = args.steps * S_step / elapsed
    log(f"timed {args.steps} steps x {S_step} seeds: {elapsed:.3f} s -> {value:.1f} seed-subspaces/s")
    nue = d_nu.cpu().numpy()
    # per-kernel HIP-event durations: one more step of new seeds, profiled (one block at a time)
    prof, prof_elapsed = {}, None
    if not args.no_profile:
        ctx.profile(True)
        ctx.profile_reset()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.solve_async(seeds_for(n_steps), nu, mu, KT, "fp32", "batched", d_rho=d_rho, d_e_band=d_eb,
                        d_e_seed=d_e, d_n_seed=d_n, d_nu_eff=d_nu, stream=stream)
        torch.cuda.synchronize()
        prof_elapsed = time.perf_counter() - t1
        prof = ctx.profile_collect()
        ctx.profile(False)
        log(f"profiled step ({S_step} seeds, one block at a time): {prof_elapsed:.3f} s")
    if (nue < 0).any():
        log("error: a seed reported a non-positive-definite overlap")
        return 1

    kernels = {}
    for name, e in prof.items():
        if e["launches"] == 0:
            continue
        kernels[name] = dict(launches=int(e["launches"]), ms=round(e["ms"], 3),
                             share=round(e["ms"] / (prof_elapsed * 1e3), 4),
                             GBps=round(e["bytes"] / (e["ms"] * 1e-3) / 1e9, 1) if e["ms"] > 0 else None)
    roofline = None
    spmm = None
    if prof:
        dom = max(prof, key=lambda n: prof[n]["ms"])
        e = prof[dom]
        ach = e["bytes"] / (e["ms"] * 1e-3) / 1e9
        kind, cells = system.name.split("_", 1)          # e.g. mixed, 16x16x16
        wl = f"{kind}{cells.split('x')[0]}_nu{nu}_fp32_b{B}_{args.seed_order}" + ("_full" if args.no_support else "") \
            + (f"_r{args.r_cut}" if local else "") + (f"_v{args.proj_variant}" if args.proj_variant else "")
        traffic = measured_traffic(dom, wl) if S_step % B == 0 else None
        roofline = dict(kernel=dom, bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                        frac=round(ach / HBM_PEAK_GBPS, 4), traffic=traffic,
                        bytes_per_launch=e["bytes"] / e["launches"], avg_launch_us=1e3 * e["ms"] / e["launches"])
        s = prof.get("spmm")
        if s and s["ms"] > 0:
            sa = s["bytes"] / (s["ms"] * 1e-3) / 1e9
            cp = copy_rate(torch, dev)
            spmm = dict(achieved=round(sa, 1), peak=HBM_PEAK_GBPS, unit="GB/s", frac=round(sa / HBM_PEAK_GBPS, 4),
                        avg_launch_us=1e3 * s["ms"] / s["launches"], device_copy_GBps=round(cp, 1),
                        frac_of_copy=round(sa / cp, 4))

    # the plain FP64 form on the same GPU (one seed per block, one launch per phase)
    plain = None
    if not args.no_plain and args.plain_seeds > 0:
        n_p = args.plain_seeds
        d_sp = d_order[-n_p:]
        ctx.solve_async(d_sp[:1], nu, mu, KT, "fp64", "plain", d_rho=d_rho, d_e_band=d_eb, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.solve_async(d_sp, nu, mu, KT, "fp64", "plain", d_rho=d_rho, d_e_band=d_eb, stream=stream)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t1
        plain = dict(value=n_p / dtp, unit="seed-subspaces/s", seeds=n_p, seconds=round(dtp, 3))
        log(f"plain FP64: {n_p} seeds in {dtp:.3f} s -> {n_p / dtp:.2f} seed-subspaces/s")

    # the two other corners, splitting the precision gain from the batching gain
    split = {}
    if not args.no_plain and args.plain_seeds > 0:
        for prec, form, n_x in (("fp32", "plain", args.plain_seeds), ("fp64", "batched", args.fp64_batched_seeds)):
            if n_x <= 0:
                continue
            d_sx = d_order[-n_x:]
            ctx.solve_async(d_sx[: min(n_x, 4)], nu, mu, KT, prec, form, d_rho=d_rho, d_e_band=d_eb, stream=stream)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ctx.solve_async(d_sx, nu, mu, KT, prec, form, d_rho=d_rho, d_e_band=d_eb, stream=stream)
            torch.cuda.synchronize()
            dtx = time.perf_counter() - t1
            split[f"{prec}_{form}"] = dict(value=round(n_x / dtx, 3), unit="seed-subspaces/s", seeds=n_x,
                                           seed_block=1 if form == "plain" else ctx.seed_block(nu, prec))
            log(f"{prec} {form}: {n_x} seeds in {dtx:.3f} s -> {n_x / dtx:.2f} seed-subspaces/s")

    cpu = None
    errors = None
    if not args.no_cpu_baseline and local:
        cpu = cpu_baseline_local(system, nu, mu, args.r_cut)
        log(f"cpu oracle (local regions): {cpu['value']:.2f} seed-subspaces/s on 1 core")
    elif not args.no_cpu_baseline:
        from oracle import mar_oracle as O
        workers = min(16, O.default_workers())
        n_cpu = args.cpu_seeds or max(workers, int(round(20.0 / 1.3)))
        n_cpu = max(n_cpu, workers)
        cpu, cpu_seeds, cpu_ref = cpu_baseline(system, nu, mu, n_cpu, workers)
        log(f"cpu oracle: {cpu['value']:.2f} seed-subspaces/s on {workers} cores")
        errors = errors_vs_oracle(ctx, system, cpu_seeds, cpu_ref, nu, mu)
        for k, e in errors.items():
            log(f"error vs oracle, {k}: E_band {e['e_band_rel']:.2e}, rho {e['rho_rel']:.2e}, "
                f"nu_eff equal {e['nu_eff_equal']}")

    out = {
        "metric": METRIC_LOCAL.format(r=args.r_cut) if local else
                  (METRIC if (M, nu) == (131072, 100) else METRIC_OTHER.format(nu=nu, M=M)),
        "value": round(value, 3),
        "unit": "seed-subspaces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{system.name} {'mixed sp2/sp3' if system.name.startswith('mixed') else 'diamond'} "
                               f"lattice, M={M}, nu={nu}, kT={KT}, FP32 batched",
                   "M": M, "nnz": int(system.H.nnz), "nu": nu, "seeds_per_step": S_step, "seed_block": B,
                   "precision": "fp32", "form": "batched", "mu": mu, "seed_order": args.seed_order,
                   "support_tracking": not args.no_support, "local_region_hops": args.r_cut if local else None,
                   "two_streams": True if args.two_streams else (False if args.one_block else "auto"),
                   "proj_variant": args.proj_variant or "default"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "error_vs_oracle": errors,
        "fp64_plain": plain,
        "ratio_fp32_batched_over_fp64_plain": round(value / plain["value"], 3) if plain else None,
        "precision_batching_split": split or None,
        "fermi_level": fermi_info,
        "spmm_hbm": spmm,
        "kernels": kernels,
        "kernels_step_s": round(prof_elapsed, 4) if prof_elapsed else None,
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
