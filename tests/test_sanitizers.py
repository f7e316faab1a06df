"""Host sanitizer runs (address + undefined behaviour): the C oracle through a driver
that calls each of its entry points on small inputs, and the library's C ABI (its host
code built with the sanitizers) through a driver that needs no device here; the same
driver runs real solves of every kind on the GPU in tests/test_gpu_sanitize.py."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, env):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, env=env, timeout=300)
    out = p.stdout.decode(errors="replace")
    assert p.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           os.path.join(ROOT, "oracle", "ipt_oracle.c"),
                           os.path.join(ROOT, "oracle", "sanitize_driver.c"), "-o", exe, "-lm"])
    out = _run([exe], SAN_ENV)
    assert "all oracle entry points ran" in out


def test_c_abi_host_code_under_sanitizers():
    from paper_2012_14702_amd import build as b
    if not os.path.exists(b.SAN_DRIVER):
        b.build_hostsan()
    # the HIP runtime's own allocations are not ours to account for: leak checks off
    env = dict(SAN_ENV, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
    out = _run([b.SAN_DRIVER], env)
    assert "abi_sanitize_driver: ok" in out
