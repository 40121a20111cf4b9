"""The library's host code under AddressSanitizer + UndefinedBehaviorSanitizer, on the CPU.

gs_host.cpp and gs_server.cpp (validation, the posting layout, the fixed-point plan,
batch and server bookkeeping, every error path) are compiled with host-only sanitizers
(-Xarch_host: the GPU code is built as usual) and linked with tests/asan/host_paths.cpp,
which drives them without a GPU: the device calls fail, so their cleanup paths run. Any
out-of-bounds access, use after free, leak or undefined behaviour aborts the program.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_26441_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, "%s\n%s" % (" ".join(cmd), r.stderr[-3000:])
    return r


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc is not installed")
def test_host_paths_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    objs = []
    host_flags = ["-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer"] + SAN
    for src in ("gs_host.cpp", "gs_server.cpp"):
        o = str(tmp_path / (src + ".o"))
        _run([HIPCC, *host_flags, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    drv = str(tmp_path / "host_paths.o")
    _run([HIPCC, *host_flags, "-c", os.path.join(ROOT, "tests", "asan", "host_paths.cpp"), "-o", drv])
    # the GPU sources, built as for the library (their host stubs are not instrumented)
    dev_flags = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-munsafe-fp-atomics",
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    for src in ("gs_score.hip", "gs_topk.hip", "gs_yardstick.hip", "gs_noalloc.hip"):
        o = str(tmp_path / (src + ".o"))
        _run([HIPCC, *dev_flags, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    exe = str(tmp_path / "host_paths")
    _run([HIPCC, "--offload-arch=gfx950", *SAN, drv, *objs, "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 failures" in r.stdout
