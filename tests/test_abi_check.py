"""The C-ABI checker (csrc/abi_check.cpp) run against the host layer built with host-side
AddressSanitizer and UndefinedBehaviorSanitizer: argument checking and error paths on a
host-only context (CPU), and every frame path on the device (GPU).  A sanitizer report or a
failed status check ends the run with a non-zero exit status."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "paper_2405_10565_amd", "bin")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _checker(name):
    exe = os.path.join(BIN, name)
    if not os.path.exists(exe):
        from paper_2405_10565_amd import build as B
        B.build_checks()
    return exe


def _run(name, *args, timeout=300):
    r = subprocess.run([_checker(name), *args], env=ENV, capture_output=True, text=True, timeout=timeout)
    print(r.stdout[-2000:], r.stderr[-4000:], flush=True)
    return r


def test_host_only_under_sanitizers():
    r = _run("abi_check_asan", "--host-only", timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "0 failed (host-only)" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["abi_check", "abi_check_asan"])
def test_device_paths(name):
    print(f"case: {name} --device 0", flush=True)
    r = _run(name, "--device", "0")
    assert r.returncode == 0, r.stderr[-2000:]
    assert "0 failed (device)" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
