"""The oracle and the host-only paths of the C ABI built with AddressSanitizer
and UndefinedBehaviorSanitizer, run on the CPU:

  * the oracle library (g++ -fsanitize=address,undefined) under a set of its
    calls on small grids: forward steps, right-hand side, c_max, div B, the
    JVP, the reverse mode (fixed faces included), LIM03, GLM, Hall MHD and the
    operation counter;
  * the runtime's block-list validation and activation safety belt
    (amrvac_validate_blocks, amrvac_activation_flags) from a small driver,
    with sanitizers on the host code only.

Any sanitizer report fails the test."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

from conftest import ROOT

GXX = shutil.which("g++")
HIPCC = "/opt/rocm/bin/hipcc"


def libasan():
    out = subprocess.run([GXX, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.skipif(GXX is None, reason="needs g++")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan = libasan()
    if asan is None:
        pytest.skip("libasan not found")
    lib = tmp_path / "liborc_san.so"
    subprocess.run([GXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC",
                    "-shared", os.path.join(ROOT, "oracle", "amrvac_oracle.cpp"), "-o", str(lib)], check=True)
    script = textwrap.dedent(f"""
        import sys
        sys.path.insert(0, {ROOT!r}); sys.path.insert(0, {os.path.join(ROOT, 'tests')!r})
        import numpy as np, oracle
        from paper_1407_2052_amd import inputs
        from test_oracle_vjp import sod_like, mhd2d_mixed_faces, random_interior
        oracle.set_threads(1)
        bs = inputs.orszag_tang_2d(32, 16)
        oracle.run(bs, oracle.SSPRK54, 2); oracle.rhs(bs); oracle.cmax(bs); oracle.divb(bs)
        for gen in (sod_like, mhd2d_mixed_faces):
            b = gen(); dt = 1e-3
            lam = oracle.run_vjp(b, random_interior(b, 1), oracle.SSPRK54, 2, dt)
            oracle.run_jvp(b, inputs.random_tangent(b, 2), oracle.RK3, 2, dt)
        with oracle.use_recon(oracle.LIM03):
            oracle.run(inputs.brio_wu(64), oracle.RK3, 3)
        oracle.run(inputs.as_glm(inputs.orszag_tang_2d(32, 16), psi=0.01), oracle.SSPRK54, 2)
        hall = inputs.alfven_whistler(1, 32, 0.1)
        hall = hall[0] if isinstance(hall, tuple) else hall
        with oracle.use_hall(0.1):
            oracle.run(hall, oracle.SSPRK54, 2)
        oracle.count_ops(inputs.density_wave_1d(64, nblocks=2), oracle.SSPRK54, median_form=True)
        print("oracle calls done")
    """)
    env = dict(os.environ, AMRVAC_ORACLE_LIB=str(lib), LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "oracle calls done" in r.stdout, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_host_paths_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = tmp_path / "host_paths"
    csrc = os.path.join(ROOT, "paper_1407_2052_amd", "csrc")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined"]
    subprocess.run([HIPCC, "-std=c++17", "-O1", "-g", "--offload-arch=gfx950", *san,
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I", os.path.join(ROOT, "include"), "-I", csrc,
                    "-x", "hip", os.path.join(csrc, "runtime.cpp"),
                    "-x", "hip", os.path.join(ROOT, "tests", "sanitize", "host_paths.cpp"),
                    "-o", str(exe)], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (r.stdout, r.stderr[-4000:])
    assert "0 failure(s)" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
