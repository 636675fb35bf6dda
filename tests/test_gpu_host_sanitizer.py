"""The host code of the library under AddressSanitizer and
UndefinedBehaviorSanitizer: the ABI driver tests/native/abi_sanitizer.cpp,
built with both sanitizers against hostsan/libmderi_hostsan.so (host.hip
compiled with them on its host side; build.build_hostsan), calls every entry
point through its success path and its argument checks on the GPU.  Any
out-of-bounds access, use after free or undefined operation in host code
aborts it with a report, and so does a host allocation of the library left
unfreed at exit; a failed status check makes it exit 1."""
import os
import subprocess

import pytest

from paper_2405_01834_amd import build

pytestmark = pytest.mark.gpu

EXE = os.path.join(build.HOSTSAN, "abi_sanitizer")


def test_abi_under_host_sanitizers(need_gpu):
    if not os.path.exists(EXE):
        pytest.skip("host-sanitizer driver not built (paper_2405_01834_amd.build.build_hostsan)")
    env = dict(os.environ)
    # leaks are checked, except those of the ROCm runtime's own allocations,
    # which it keeps until exit (tests/native/lsan.supp)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1:verify_asan_link_order=0"
    env["LSAN_OPTIONS"] = "suppressions=" + os.path.join(os.path.dirname(__file__), "native", "lsan.supp")
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-4000:])
    print(r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-2000:]
    assert "0 failure(s)" in r.stdout
