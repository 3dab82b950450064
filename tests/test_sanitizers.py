"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU: the runtime behind the C ABI (validation, layout, stability analysis
and admission, batch work plans, the autotuner's cache files, error paths
without a device; the kernel launches are stubbed out) and the oracle
(steps of small solves with every boundary kind and flag)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1010_4135_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")
HOST_SOURCES = ["lbm3d_layout.cpp", "lbm3d_api.cpp", "lbm3d_batch.cpp", "lbm3d_server.cpp", "lbm3d_tune.cpp",
                "lbm3d_stability.cpp"]
# sanitizers on the host code only; the device side of each translation unit
# is compiled as usual
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _device_visible():
    from paper_1010_4135_amd import lbm3d
    return lbm3d.lbm3d_device_count() > 0


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs hipcc and clang++")
def test_host_runtime_under_sanitizers(tmp_path):
    if _device_visible():
        pytest.skip("checks the no-device error paths: run where no GPU is visible")
    objs, jobs = [], []
    for path in [os.path.join(CSRC, s) for s in HOST_SOURCES] + [os.path.join(HERE, "host_checks.cpp")]:
        src = path
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-O1", "-g"] + SAN + ["-c", path, "-o", obj]
        jobs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    for j in jobs:
        out, _ = j.communicate()
        assert j.returncode == 0, out.decode()[-3000:]
    exe = str(tmp_path / "host_checks")
    link = [CLANG] + objs + ["-fsanitize=address,undefined", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
                             "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", exe]
    r = subprocess.run(link, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    supp = tmp_path / "lsan.supp"
    # allocations the HIP and HSA runtimes keep for the life of the process
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:librocprofiler\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               LSAN_OPTIONS=f"suppressions={supp}", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "host checks passed" in r.stdout, (r.stdout[-2000:], r.stderr[-6000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-6000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_checks")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-ffp-contract=off", os.path.join(ROOT, "oracle", "lbm3d_oracle.c"),
           os.path.join(HERE, "oracle_checks.c"), "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0 and "oracle checks passed" in r.stdout, (r.stdout, r.stderr[-6000:])
    assert "runtime error" not in r.stderr, r.stderr[-6000:]
