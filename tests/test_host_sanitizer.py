"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The library's sources are compiled for the host only (no device code) with the sanitizers, linked against
a stand-in for the HIP runtime (hostcheck/hip_stub.cpp: device memory is host memory in a checked registry;
streams, events and graph capture are bookkeeping; kernels do nothing) and driven through the C ABI by
hostcheck/driver.cpp. Results are meaningless; what is checked is the host side: allocations, copies,
streams, events, graph capture and the workspace and graph caches.

Mode 0 replays the sequence that preceded the two host crashes of mar_solve_many on the GPU: autotune and
eager solves with two seed blocks in flight, then graph captures on the same contexts (repeated requests,
new seed pointers, new shapes), then the other entry points and mar_destroy. The library refuses that
sequence (MAR_ERR_STATE); this check builds a copy of the host API with the refusal taken out, so that the
capture path behind it runs. Mode 1 runs one block at a time with the eigensolves on the second stream.
A sanitizer report, a misuse of the runtime that the stand-in detects (out-of-range copies, frees of
unknown pointers, allocation or synchronization under capture, forks not joined before a capture ends),
a failed call or a leaked allocation fails the test.
"""
import concurrent.futures
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1307_3218_amd import lattice

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1307_3218_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")
REFUSAL = "if (ctx[i]->ran_two_sets)"


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}")
    return r


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc / clang++ of the ROCm toolchain not found")
    tmp = tmp_path_factory.mktemp("hostcheck")
    src = tmp / "lib" / "csrc"
    shutil.copytree(CSRC, src, ignore=shutil.ignore_patterns("*.o", "*.so"))
    shutil.copytree(os.path.join(ROOT, "include"), tmp / "include")
    api = (src / "mar_api.cpp").read_text()
    assert api.count(REFUSAL) == 1, "the refusal this check takes out has changed"
    # the refused statement stays, behind if (false); a context that would have been refused is named
    (src / "mar_api.cpp").write_text(api.replace(
        REFUSAL, 'if (ctx[i]->ran_two_sets) printf("[hostcheck] ctx %d ran two seed blocks in flight\\n", i);\n'
                 '        if (false)'))
    # host-only objects; each -fsanitize= goes right after -Xarch_host, so no device code is instrumented
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "--cuda-host-only", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", str(tmp / "include"), "-I", str(src),
             "-Wno-unused-function", "-Wno-unused-variable", '-DMAR_BUILD_ID="hostcheck"'] + san
    jobs = []
    for f in sorted(os.listdir(src)):
        if f.endswith(".hip"):
            jobs.append([HIPCC] + flags + ["-x", "hip", "-c", str(src / f), "-o", str(tmp / (f + ".o"))])
    jobs.append([HIPCC] + flags + ["-c", str(src / "mar_api.cpp"), "-o", str(tmp / "mar_api.o")])
    host = ["-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
            "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"), "-I", str(tmp / "include")]
    for f in ("hip_stub.cpp", "driver.cpp"):
        jobs.append([CLANG] + host + ["-c", os.path.join(HERE, "hostcheck", f), "-o", str(tmp / (f + ".o"))])
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(lambda c: _run(c, str(tmp)), jobs))
    objs = sorted(str(tmp / f) for f in os.listdir(tmp) if f.endswith(".o"))
    exe = str(tmp / "driver")
    # the host-only objects still name their (absent) device code images; nothing reads them here
    _run([CLANG, "-fsanitize=address,undefined", "-o", exe] + objs +
         ["-lpthread", "-Wl,--unresolved-symbols=ignore-in-object-files"], str(tmp))
    # four small systems: two cubic diamond cells, a mixed cell and a longer one
    for i, (cells, mixed) in enumerate((((2, 2, 2), False), ((2, 2, 4), False), ((4, 2, 2), True),
                                        ((4, 4, 2), False))):
        s = lattice.generate(*cells, mixed=mixed, seed=0)
        H, S = s.H.tocsr(), s.S.tocsr()
        with open(tmp / f"sys_{i}.bin", "wb") as f:
            np.array([s.M, H.nnz, S.nnz], dtype=np.int64).tofile(f)
            for A in (H, S):
                A.indptr.astype(np.int64).tofile(f)
                A.indices.astype(np.int32).tofile(f)
                A.data.astype(np.float64).tofile(f)
    return exe, str(tmp)


@pytest.mark.parametrize("mode", [0, 1])
def test_host_code_under_sanitizers(harness, mode):
    exe, d = harness
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, d, str(mode)], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    print(out[-2000:])
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "0 call failures, 0 stub errors" in out
    # the graph path really ran: four new request sets captured, each launched twice
    assert "captures 4, instantiations 4, graph launches 8" in out
    # and in mode 0 on contexts that had run two seed blocks in flight (the refused sequence)
    assert ("ran two seed blocks in flight" in out) == (mode == 0)
