"""Python binding of libmar.so (the C ABI declared in include/mar.h).

Argument marshalling only: every step of the hot path runs in the HIP
library. The module-level functions carry the C names (mar_create,
mar_solve, ...); ``Context`` is a small object wrapper around them. Device
buffers for the asynchronous entry point are torch tensors (plumbing only).
If libmar.so is missing this module raises on first use; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmar.so")

MAR_OK, MAR_ERR_ARG, MAR_ERR_PATTERN, MAR_ERR_NOT_SPD, MAR_ERR_NOMEM, MAR_ERR_HIP, MAR_ERR_STATE = 0, -1, -2, -3, -4, -5, -6
MAR_ERR_NOCONV = -7
NU_NOCONV = -3      # nu_eff of a seed whose subspace eigensolve did not converge
STATUS_NAMES = {0: "MAR_OK", -1: "MAR_ERR_ARG", -2: "MAR_ERR_PATTERN", -3: "MAR_ERR_NOT_SPD",
                -4: "MAR_ERR_NOMEM", -5: "MAR_ERR_HIP", -6: "MAR_ERR_STATE", -7: "MAR_ERR_NOCONV"}
PRECISION = {"fp64": 0, "fp32": 1}
SCHEDULE = {"auto": 0, "textbook": 1, "delayed": 2}
FORM = {"batched": 0, "plain": 1}
PROF_CLASSES = 16


class MarError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class mar_tuning(C.Structure):
    _fields_ = [("seed_block", C.c_int32), ("schedule", C.c_int32), ("proj_wgs", C.c_int32),
                ("slab_pad_kb", C.c_int32), ("proj_variant", C.c_int32), ("upd_q", C.c_int32),
                ("support_off", C.c_int32), ("two_streams", C.c_int32), ("eig_max_sweeps", C.c_int32)]


class mar_request(C.Structure):
    _fields_ = [("d_seeds", C.c_void_p), ("n_seeds", C.c_int64), ("nu", C.c_int32), ("mu", C.c_double),
                ("kT", C.c_double), ("prec", C.c_int), ("form", C.c_int), ("d_rho", C.c_void_p),
                ("d_e_band", C.c_void_p), ("d_e_seed", C.c_void_p), ("d_n_seed", C.c_void_p),
                ("d_nu_eff", C.c_void_p), ("d_eps", C.c_void_p), ("d_weight", C.c_void_p)]


class mar_prof_entry(C.Structure):
    _fields_ = [("name", C.c_char * 24), ("launches", C.c_int64), ("ms", C.c_double),
                ("bytes", C.c_double), ("flops", C.c_double)]


_lib = None
_P = C.c_void_p


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1307_3218_amd.build_lib`")
    # torch ships its own HIP runtime. Loading torch first makes libmar bind to
    # that same runtime (one runtime per process), so torch's streams and device
    # pointers are valid handles inside libmar and torch can still use the GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    i32, i64, f64 = C.c_int32, C.c_int64, C.c_double
    L.mar_create.argtypes = [i64, _P, _P, _P, _P, _P, _P, C.POINTER(_P)]
    L.mar_create.restype = C.c_int
    L.mar_destroy.argtypes = [_P]
    L.mar_destroy.restype = None
    L.mar_solve.argtypes = [_P, _P, i64, i32, f64, f64, C.c_int, C.c_int, _P, _P, _P, _P, _P, _P, _P]
    L.mar_solve.restype = C.c_int
    L.mar_solve_async.argtypes = [_P, _P, i64, i32, f64, f64, C.c_int, C.c_int, _P, _P, _P, _P, _P, _P, _P, _P]
    L.mar_solve_async.restype = C.c_int
    L.mar_solve_async_noalloc.argtypes = L.mar_solve_async.argtypes
    L.mar_solve_async_noalloc.restype = C.c_int
    L.mar_solve_fermi.argtypes = [_P, _P, i64, i32, f64, f64, C.c_int, C.c_int, _P, _P, _P, _P, _P, _P, _P, _P]
    L.mar_solve_fermi.restype = C.c_int
    L.mar_solve_fermi_async.argtypes = [_P, _P, i64, i32, f64, f64, C.c_int, C.c_int, _P, _P, _P, _P, _P, _P, _P,
                                        _P, _P]
    L.mar_solve_fermi_async.restype = C.c_int
    L.mar_eigen_state.argtypes = [_P, _P, i64, i32, i32, f64, C.c_int, C.c_int, _P, _P, _P]
    L.mar_eigen_state.restype = C.c_int
    L.mar_eigen_state_async.argtypes = [_P, _P, i64, i32, i32, f64, C.c_int, C.c_int, _P, _P, _P, _P]
    L.mar_eigen_state_async.restype = C.c_int
    L.mar_solve_many.argtypes = [i32, C.POINTER(_P), C.POINTER(mar_request), _P]
    L.mar_solve_many.restype = C.c_int
    L.mar_autotune.argtypes = [_P, i32, C.c_int, _P, i64, f64, f64, _P, C.POINTER(i32), C.POINTER(i32),
                               C.POINTER(f64)]
    L.mar_autotune.restype = C.c_int
    L.mar_set_tuning.argtypes = [_P, C.POINTER(mar_tuning)]
    L.mar_set_tuning.restype = C.c_int
    L.mar_get_tuning.argtypes = [_P, C.POINTER(mar_tuning)]
    L.mar_get_tuning.restype = C.c_int
    L.mar_local_flip.argtypes = [_P, _P, f64, _P, f64, i32, _P, _P, _P]
    L.mar_local_flip.restype = C.c_int
    L.mar_flip_colours.argtypes = [_P]
    L.mar_flip_colours.restype = i32
    L.mar_set_local_region.argtypes = [_P, i32]
    L.mar_set_local_region.restype = C.c_int
    L.mar_local_region.argtypes = [_P]
    L.mar_local_region.restype = i32
    L.mar_seed_block.argtypes = [_P, i32, C.c_int]
    L.mar_seed_block.restype = i32
    L.mar_last_error.argtypes = [_P]
    L.mar_last_error.restype = C.c_char_p
    L.mar_profile_enable.argtypes = [_P, i32]
    L.mar_profile_enable.restype = C.c_int
    L.mar_profile_reset.argtypes = [_P]
    L.mar_profile_reset.restype = C.c_int
    L.mar_profile_collect.argtypes = [_P, C.POINTER(mar_prof_entry), C.POINTER(i32)]
    L.mar_profile_collect.restype = C.c_int
    L.mar_ctx_info.argtypes = [_P, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    L.mar_ctx_info.restype = i32
    L.mar_build_id.argtypes = []
    L.mar_build_id.restype = C.c_char_p
    _lib = L
    return L


def _ptr(a) -> int | None:
    return None if a is None else a.ctypes.data


def _check(ctx, st: int):
    if st != MAR_OK:
        raise MarError(st, mar_last_error(ctx))


# ---------------------------------------------------------------- C-named API
def mar_last_error(ctx=None) -> str:
    return (lib().mar_last_error(ctx) or b"").decode()


def _csr(A) -> tuple:
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sort_indices()
    return (np.ascontiguousarray(A.indptr, dtype=np.int64), np.ascontiguousarray(A.indices, dtype=np.int32),
            np.ascontiguousarray(A.data, dtype=np.float64), A)


def mar_create(H, S):
    """Create a context from scipy CSR H and S (copied to the device). Returns the handle."""
    hp, hc, hv, H = _csr(H)
    spp, sc, sv, S = _csr(S)
    if H.shape != S.shape or H.shape[0] != H.shape[1]:
        raise MarError(MAR_ERR_ARG, "H and S must be square and of one size")
    out = _P()
    st = lib().mar_create(H.shape[0], _ptr(hp), _ptr(hc), _ptr(hv), _ptr(spp), _ptr(sc), _ptr(sv), C.byref(out))
    _check(None, st)
    return out


def mar_destroy(ctx) -> None:
    lib().mar_destroy(ctx)


def mar_solve(ctx, seeds, nu, mu, kT, prec, form, rho, e_band, e_seed=None, n_seed=None, nu_eff=None,
              eps=None, weight=None) -> int:
    """Blocking solve on host numpy arrays (rho is updated in place)."""
    return lib().mar_solve(ctx, _ptr(seeds), len(seeds), int(nu), float(mu), float(kT), int(prec), int(form),
                           _ptr(rho), _ptr(e_band), _ptr(e_seed), _ptr(n_seed), _ptr(nu_eff), _ptr(eps), _ptr(weight))


def _tptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def mar_solve_async(ctx, d_seeds, n_seeds, nu, mu, kT, prec, form, d_rho, d_e_band, d_e_seed=None, d_n_seed=None,
                    d_nu_eff=None, d_eps=None, d_weight=None, stream=None) -> int:
    """Enqueue a solve on device tensors (torch) on ``stream`` (a hipStream_t handle as int)."""
    return lib().mar_solve_async(ctx, _tptr(d_seeds), int(n_seeds), int(nu), float(mu), float(kT), int(prec),
                                 int(form), _tptr(d_rho), _tptr(d_e_band), _tptr(d_e_seed), _tptr(d_n_seed),
                                 _tptr(d_nu_eff), _tptr(d_eps), _tptr(d_weight), stream)


def mar_solve_async_noalloc(ctx, d_seeds, n_seeds, nu, mu, kT, prec, form, d_rho, d_e_band, d_e_seed=None,
                            d_n_seed=None, d_nu_eff=None, d_eps=None, d_weight=None, stream=None) -> int:
    """As mar_solve_async, on the library's static scratch array: no device allocation."""
    return lib().mar_solve_async_noalloc(ctx, _tptr(d_seeds), int(n_seeds), int(nu), float(mu), float(kT),
                                         int(prec), int(form), _tptr(d_rho), _tptr(d_e_band), _tptr(d_e_seed),
                                         _tptr(d_n_seed), _tptr(d_nu_eff), _tptr(d_eps), _tptr(d_weight), stream)


def mar_solve_fermi(ctx, seeds, nu, n_target, kT, prec, form, rho, e_band, mu, e_seed=None, n_seed=None,
                    nu_eff=None, eps=None, weight=None) -> int:
    """Blocking solve with the Fermi level found on the device (mu: 1-element array, output)."""
    return lib().mar_solve_fermi(ctx, _ptr(seeds), len(seeds), int(nu), float(n_target), float(kT), int(prec),
                                 int(form), _ptr(rho), _ptr(e_band), _ptr(mu), _ptr(e_seed), _ptr(n_seed),
                                 _ptr(nu_eff), _ptr(eps), _ptr(weight))


def mar_solve_fermi_async(ctx, d_seeds, n_seeds, nu, n_target, kT, prec, form, d_rho, d_e_band, d_e_seed=None,
                          d_n_seed=None, d_nu_eff=None, d_eps=None, d_weight=None, d_mu=None, stream=None) -> int:
    return lib().mar_solve_fermi_async(ctx, _tptr(d_seeds), int(n_seeds), int(nu), float(n_target), float(kT),
                                       int(prec), int(form), _tptr(d_rho), _tptr(d_e_band), _tptr(d_e_seed),
                                       _tptr(d_n_seed), _tptr(d_nu_eff), _tptr(d_eps), _tptr(d_weight), _tptr(d_mu),
                                       stream)


def mar_eigen_state(ctx, seeds, nu, k, sigma, prec, form, phi, levels, ref=None) -> int:
    """Blocking k-th eigen state over the listed seeds (phi [n], levels [3], ref [3] int32 or None)."""
    return lib().mar_eigen_state(ctx, _ptr(seeds), len(seeds), int(nu), int(k), float(sigma), int(prec), int(form),
                                 _ptr(phi), _ptr(levels), _ptr(ref))


def mar_eigen_state_async(ctx, d_seeds, n_seeds, nu, k, sigma, prec, form, d_phi, d_levels, d_ref=None,
                          stream=None) -> int:
    return lib().mar_eigen_state_async(ctx, _tptr(d_seeds), int(n_seeds), int(nu), int(k), float(sigma), int(prec),
                                       int(form), _tptr(d_phi), _tptr(d_levels), _tptr(d_ref), stream)


def mar_request_of(d_seeds, nu, mu, kT, prec, form, d_rho, d_e_band, d_e_seed=None, d_n_seed=None,
                   d_nu_eff=None, d_eps=None, d_weight=None) -> mar_request:
    """A request struct for mar_solve_many from device tensors (torch)."""
    return mar_request(_tptr(d_seeds), int(d_seeds.numel()), int(nu), float(mu), float(kT), int(prec), int(form),
                       _tptr(d_rho), _tptr(d_e_band), _tptr(d_e_seed), _tptr(d_n_seed), _tptr(d_nu_eff),
                       _tptr(d_eps), _tptr(d_weight))


def mar_solve_many(ctxs, requests, stream=None) -> int:
    """One graph launch solving every (context, request) pair; returns the status."""
    n = len(ctxs)
    arr_c = (_P * n)(*[c.value if isinstance(c, _P) else c for c in ctxs])
    arr_r = (mar_request * n)(*requests)
    return lib().mar_solve_many(n, arr_c, arr_r, stream)


def mar_autotune(ctx, nu, prec, d_seeds, mu, kT, stream=None) -> tuple:
    """Returns (status, seed_block, proj_variant, probe seed-subspaces/s)."""
    b, v, r = C.c_int32(), C.c_int32(), C.c_double()
    st = lib().mar_autotune(ctx, int(nu), int(prec), _tptr(d_seeds), int(d_seeds.numel()), float(mu), float(kT),
                            stream, C.byref(b), C.byref(v), C.byref(r))
    return st, b.value, v.value, r.value


def mar_set_tuning(ctx, seed_block: int = 0, schedule: int = 0, proj_wgs: int = 0, slab_pad_kb: int = 0,
                   proj_variant: int = 0, upd_q: int = 0, support_off: int = 0, two_streams: int = 0,
                   eig_max_sweeps: int = 0) -> int:
    t = mar_tuning(seed_block, schedule, proj_wgs, slab_pad_kb, proj_variant, upd_q, support_off, two_streams,
                   eig_max_sweeps)
    return lib().mar_set_tuning(ctx, C.byref(t))


def mar_local_flip(ctx, d_phi, eps, d_phi_ref, c, max_sweeps, d_R, d_info, stream) -> int:
    return lib().mar_local_flip(ctx, _tptr(d_phi), float(eps), _tptr(d_phi_ref), float(c), int(max_sweeps),
                                _tptr(d_R), _tptr(d_info), stream)


def mar_flip_colours(ctx) -> int:
    return lib().mar_flip_colours(ctx)


def mar_set_local_region(ctx, hops: int) -> int:
    return lib().mar_set_local_region(ctx, int(hops))


def mar_local_region(ctx) -> int:
    return lib().mar_local_region(ctx)


def mar_seed_block(ctx, nu: int, prec: int) -> int:
    return lib().mar_seed_block(ctx, int(nu), int(prec))


def mar_profile_enable(ctx, on: bool) -> int:
    return lib().mar_profile_enable(ctx, 1 if on else 0)


def mar_profile_reset(ctx) -> int:
    return lib().mar_profile_reset(ctx)


def mar_profile_collect(ctx) -> dict:
    arr = (mar_prof_entry * PROF_CLASSES)()
    n = C.c_int32(0)
    _check(ctx, lib().mar_profile_collect(ctx, arr, C.byref(n)))
    return {arr[k].name.decode(): dict(launches=arr[k].launches, ms=arr[k].ms, bytes=arr[k].bytes,
                                       flops=arr[k].flops) for k in range(n.value)}


def mar_build_id() -> str:
    """The source hash the loaded library was built from (build_lib.source_hash() at build time)."""
    return lib().mar_build_id().decode()


def mar_ctx_info(ctx) -> dict:
    M, nh, ns = C.c_int64(), C.c_int64(), C.c_int64()
    flags = lib().mar_ctx_info(ctx, C.byref(M), C.byref(nh), C.byref(ns))
    return dict(M=M.value, nnz_H=nh.value, nnz_S=ns.value, H_bsr=bool(flags & 1), S_bsr=bool(flags & 2))


# ---------------------------------------------------------------- object wrapper
@dataclasses.dataclass
class SolveOutput:
    rho: np.ndarray
    e_band: float
    e_seed: np.ndarray
    n_seed: np.ndarray
    nu_eff: np.ndarray
    eps: np.ndarray | None       # (n_seeds, nu); entries >= nu_eff are 0
    weight: np.ndarray | None


class Context:
    """One (H, S) pair resident on the GPU."""

    def __init__(self, H, S):
        self.H = sp.csr_matrix(H)
        self.H.sort_indices()
        self.M = self.H.shape[0]
        self.handle = mar_create(self.H, S)

    def close(self):
        if getattr(self, "handle", None):
            mar_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, seeds, nu, mu, kT, precision="fp64", form="batched", rho=None, levels=False) -> SolveOutput:
        seeds = np.ascontiguousarray(seeds, dtype=np.int32)
        n = len(seeds)
        rho = np.zeros(self.H.nnz) if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
        e_band = np.zeros(1)
        e_seed, n_seed = np.zeros(n), np.zeros(n)
        nu_eff = np.zeros(n, dtype=np.int32)
        eps = np.zeros((n, nu)) if levels else None
        weight = np.zeros((n, nu)) if levels else None
        st = mar_solve(self.handle, seeds, nu, mu, kT, PRECISION[precision], FORM[form], rho, e_band, e_seed,
                       n_seed, nu_eff, eps, weight)
        _check(self.handle, st)
        return SolveOutput(rho, float(e_band[0]), e_seed, n_seed, nu_eff, eps, weight)

    def solve_fermi(self, seeds, nu, n_target, kT, precision="fp64", form="batched", rho=None, levels=False):
        """Solve with mu bisected on the device so that N(mu) = n_target; returns (SolveOutput, mu)."""
        seeds = np.ascontiguousarray(seeds, dtype=np.int32)
        n = len(seeds)
        rho = np.zeros(self.H.nnz) if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
        e_band, mu = np.zeros(1), np.zeros(1)
        e_seed, n_seed = np.zeros(n), np.zeros(n)
        nu_eff = np.zeros(n, dtype=np.int32)
        eps = np.zeros((n, nu)) if levels else None
        weight = np.zeros((n, nu)) if levels else None
        st = mar_solve_fermi(self.handle, seeds, nu, n_target, kT, PRECISION[precision], FORM[form], rho, e_band, mu,
                             e_seed, n_seed, nu_eff, eps, weight)
        _check(self.handle, st)
        return SolveOutput(rho, float(e_band[0]), e_seed, n_seed, nu_eff, eps, weight), float(mu[0])

    def solve_fermi_async(self, d_seeds, nu, n_target, kT, precision="fp32", form="batched", *, d_rho, d_e_band,
                          d_mu, d_e_seed=None, d_n_seed=None, d_nu_eff=None, d_eps=None, d_weight=None, stream=None):
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        st = mar_solve_fermi_async(self.handle, d_seeds, d_seeds.numel(), nu, n_target, kT, PRECISION[precision],
                                   FORM[form], d_rho, d_e_band, d_e_seed, d_n_seed, d_nu_eff, d_eps, d_weight, d_mu,
                                   stream)
        _check(self.handle, st)

    def eigen_state(self, seeds, nu, k, sigma, precision="fp64", form="batched") -> dict:
        """The k-th eigen level and eigenvector components over the listed seeds (Sec. 3, Eq. 3)."""
        seeds = np.ascontiguousarray(seeds, dtype=np.int32)
        phi = np.zeros(len(seeds))
        levels = np.zeros(3)
        ref = np.zeros(3, dtype=np.int32)
        st = mar_eigen_state(self.handle, seeds, nu, k, sigma, PRECISION[precision], FORM[form], phi, levels, ref)
        _check(self.handle, st)
        return dict(phi=phi, eps_k=float(levels[0]), eta_lo=float(levels[1]), eta_hi=float(levels[2]),
                    ref=(int(ref[0]), int(ref[1]), int(ref[2])))

    def solve_async(self, d_seeds, nu, mu, kT, precision="fp64", form="batched", *, d_rho, d_e_band,
                    d_e_seed=None, d_n_seed=None, d_nu_eff=None, d_eps=None, d_weight=None, stream=None):
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        st = mar_solve_async(self.handle, d_seeds, d_seeds.numel(), nu, mu, kT, PRECISION[precision], FORM[form],
                             d_rho, d_e_band, d_e_seed, d_n_seed, d_nu_eff, d_eps, d_weight, stream)
        _check(self.handle, st)

    def local_flip(self, phi, eps, phi_ref=None, c=0.0, max_sweeps=100, stream=None) -> dict:
        """Sign-flip refinement of the eigenvector phi of level eps (Appendix); phi: host array of M values.

        Returns dict(phi, R, sweeps, flips): the refined vector, R before the first and after every sweep.
        """
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        d_phi = torch.as_tensor(np.ascontiguousarray(phi, dtype=np.float64)).to(dev)
        d_ref = None if phi_ref is None else torch.as_tensor(np.ascontiguousarray(phi_ref, dtype=np.float64)).to(dev)
        d_R = torch.full((max_sweeps + 1,), float("nan"), dtype=torch.float64, device=dev)
        d_info = torch.zeros(2, dtype=torch.int32, device=dev)
        _check(self.handle, mar_local_flip(self.handle, d_phi, eps, d_ref, c, max_sweeps, d_R, d_info, stream))
        torch.cuda.synchronize()
        info = d_info.cpu().numpy()
        return dict(phi=d_phi.cpu().numpy(), R=d_R.cpu().numpy()[: int(info[0]) + 1], sweeps=int(info[0]),
                    flips=int(info[1]))

    def flip_colours(self) -> int:
        return mar_flip_colours(self.handle)

    def set_local_region(self, hops: int | None):
        """Later solves run each seed on the rows within `hops` block hops of it (None or < 0: the full system)."""
        _check(self.handle, mar_set_local_region(self.handle, -1 if hops is None else hops))

    def local_region(self) -> int:
        return mar_local_region(self.handle)

    def set_tuning(self, seed_block: int = 0, schedule: str = "auto", proj_wgs: int = 0, slab_pad_kb: int = 0,
                   proj_variant: int = 0, upd_q: int = 0, support: bool = True, two_streams: bool | None = None,
                   overlap_eig: bool = True, eig_max_sweeps: int = 0):
        """two_streams: None lets the library choose (two blocks in flight for local regions of 6 hops or
        more, else one block at a time); True alternates two blocks; False runs one block at a time, with
        each block's eigensolve on the second stream when overlap_eig, else everything on one stream.
        eig_max_sweeps: Jacobi sweeps allowed to the subspace eigensolve (0 = 40)."""
        _check(self.handle, mar_set_tuning(self.handle, seed_block, SCHEDULE[schedule], proj_wgs, slab_pad_kb,
                                           proj_variant, upd_q, 0 if support else 1,
                                           (0 if overlap_eig else 2) if two_streams is None else
                                           1 if two_streams else (3 if overlap_eig else 2), eig_max_sweeps))

    def autotune(self, d_seeds, nu, mu, kT, precision="fp32", stream=None) -> dict:
        """Pick the seed block and projection tiles for (nu, precision) by timing probe solves."""
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        st, b, v, r = mar_autotune(self.handle, nu, PRECISION[precision], d_seeds, mu, kT, stream)
        _check(self.handle, st)
        return dict(seed_block=b, proj_variant=v, probe_rate=r)

    def seed_block(self, nu: int, precision: str = "fp32") -> int:
        return mar_seed_block(self.handle, nu, PRECISION[precision])

    def profile(self, on: bool = True):
        _check(self.handle, mar_profile_enable(self.handle, on))

    def profile_reset(self):
        _check(self.handle, mar_profile_reset(self.handle))

    def profile_collect(self) -> dict:
        return mar_profile_collect(self.handle)

    def info(self) -> dict:
        return mar_ctx_info(self.handle)


def solve_many(contexts, requests, stream=None):
    """Solve several systems with one graph launch.

    contexts: Context objects (distinct); requests: dicts with the keyword
    arguments of Context.solve_async (d_seeds, nu, mu, kT, precision, form,
    d_rho, d_e_band, optional d_e_seed, d_n_seed, d_nu_eff, d_eps, d_weight).
    """
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    reqs = []
    for r in requests:
        reqs.append(mar_request_of(r["d_seeds"], r["nu"], r["mu"], r["kT"], PRECISION[r.get("precision", "fp32")],
                                   FORM[r.get("form", "batched")], r["d_rho"], r["d_e_band"], r.get("d_e_seed"),
                                   r.get("d_n_seed"), r.get("d_nu_eff"), r.get("d_eps"), r.get("d_weight")))
    handles = [c.handle for c in contexts]
    st = mar_solve_many(handles, reqs, stream)
    if st != MAR_OK:
        msgs = "; ".join(m for m in (mar_last_error(h) for h in handles) if m)
        raise MarError(st, msgs)
