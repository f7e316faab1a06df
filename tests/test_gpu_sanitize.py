"""The C ABI under the host address and undefined-behaviour sanitizers on the GPU: the
driver (tests/abi_sanitize_driver.cpp, linked against the library built with host
sanitizers) creates a handle, checks rejected arguments and runs a small solve of every
kind in a child process."""
import os
import subprocess

import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def test_every_entry_point_under_host_sanitizers():
    from paper_2012_14702_amd import build as b
    if not os.path.exists(b.SAN_DRIVER):
        pytest.skip("host-sanitizer build not present (paper_2012_14702_amd.build.build_hostsan)")
    say("abi sanitize driver gpu")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([b.SAN_DRIVER, "gpu"], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, env=env,
                       timeout=240)
    out = p.stdout.decode(errors="replace")
    assert p.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "abi_sanitize_driver: ok (gpu)" in out
