"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle's brute-force ray march (``oracle/bruteforce.c``) built with gcc
  and both sanitizers, driven by ``tests/sanitize/bruteforce_driver.c``: it must
  run clean, and its fluence must equal the regular build's on the same scene.
* The library's host logic (``hrc_api.cpp``, ``hrc_batch.cpp`` and the host part
  of ``hrc_kernels.hip``) built with hipcc, the sanitizers on the host side only
  (device code is built as usual and never runs here), driven by
  ``tests/sanitize/host_driver.cpp``: the C ABI's argument checks and workspace
  layouts, and the batch planner's arrangements of 18 scenes over queues and
  workspace slots on fake device addresses, checked for step hazards.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2505_02041_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")


def _clean(res):
    text = res.stderr + res.stdout
    assert "AddressSanitizer" not in text and "runtime error" not in text, text[-4000:]
    assert res.returncode == 0, text[-4000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_bruteforce_under_sanitizers(tmp_path):
    exe = tmp_path / "bruteforce_driver"
    subprocess.run(["gcc", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
                    "-fno-omit-frame-pointer", "-o", str(exe),
                    os.path.join(SAN, "bruteforce_driver.c"),
                    os.path.join(ROOT, "oracle", "bruteforce.c"), "-lm"], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=ENV, timeout=300)
    _clean(res)
    rows = [line.split() for line in res.stdout.splitlines()]
    S = 12
    inp = np.array([[float(r[2]), float(r[3])] for r in rows if r[0] == "in"])
    eps, sig = inp[:, 0].reshape(S, S), inp[:, 1].reshape(S, S)
    plain = np.array([float(r[2]) for r in rows if r[0] == "plain"]).reshape(S, S)
    env = np.array([float(r[2]) for r in rows if r[0] == "env"]).reshape(5, 8)
    from oracle import bruteforce
    assert np.array_equal(plain, bruteforce.fluence(eps, sig, M=96, crop=(0, S, 0, S)))
    want = bruteforce.fluence(eps, sig, M=96, crop=(2, 7, 3, 11),
                              environment=[0.5, 1.0, 1.5, 0.25, 2.0])
    assert np.array_equal(env, want)


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)),
                    reason="needs hipcc and the ROCm clang++")
def test_host_logic_under_sanitizers(tmp_path):
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    common = ["-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
              "-packed-fp32-ops", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off"]
    objs = []
    for src in (os.path.join(CSRC, "hrc_kernels.hip"), os.path.join(CSRC, "hrc_api.cpp"),
                os.path.join(SAN, "host_driver.cpp")):
        obj = tmp_path / (os.path.basename(src) + ".o")
        subprocess.run([HIPCC, *common, *san, "-c", src, "-o", str(obj)], check=True,
                       capture_output=True)
        objs.append(str(obj))
    exe = tmp_path / "host_driver"
    subprocess.run([CLANGXX, "-fsanitize=address,undefined", "-o", str(exe), *objs,
                    "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=ENV, timeout=300)
    _clean(res)
    assert "0 failures" in res.stdout, res.stdout
