"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only). A host-only build of every source (hipcc --cuda-host-only with
relocatable device code, so the empty device link resolves the fat binary;
no device code, no GPU touched), with the sanitizers on the host pass, is
linked with tests/native/host_check.c, which drives argument validation,
error reporting and the CMA-ES search through the C-ABI."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2112_03851_amd", "csrc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _hipcc():
    return shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)


@pytest.mark.timeout(900)
@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
def test_host_code_clean_under_asan_and_ubsan(tmp_path):
    hipcc = _hipcc()
    units = [("sos_kernels.hip", []), ("sos_api.hip", []), ("sos_cmaes.cpp", [])] + \
            [("sos_fused.hip", [f"-DSOS_FUSED_CPT={c}"]) for c in (1, 2, 3, 4)]

    def compile_unit(i):
        src, defs = units[i]
        obj = str(tmp_path / f"u{i}.o")
        cmd = [hipcc, "--offload-arch=gfx950", "-fgpu-rdc", "--cuda-host-only", "-O1", "-g", "-std=c++17", "-fPIC",
               *SAN,
               "-I", os.path.join(ROOT, "include"), *defs, "-c", os.path.join(CSRC, src), "-o", obj]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-3000:]
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_unit, range(len(units))))
    exe = str(tmp_path / "host_check")
    cmd = [hipcc, "--offload-arch=gfx950", "-fgpu-rdc", "--hip-link", *SAN, "-g", "-I", os.path.join(ROOT, "include"),
           "-x", "c",
           os.path.join(ROOT, "tests", "native", "host_check.c"), "-x", "none", *objs,
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES=os.environ.get(
                   "HIP_VISIBLE_DEVICES", ""))
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = run.stdout + run.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert run.returncode == 0 and "host checks passed" in run.stdout, out[-4000:]
