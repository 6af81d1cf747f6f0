"""Sanitized native checks (tests/native): the oracle under AddressSanitizer
and UndefinedBehaviorSanitizer against brute force and closed forms, and the
C ABI driven by a sanitized host program linked with a library built with
its device-side invariant checks on.
"""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
NATIVE = os.path.join(HERE, "native")
ABI_CHECK = os.path.join(NATIVE, "abi_check")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _native_build():
    import importlib.util

    spec = importlib.util.spec_from_file_location("_native_build", os.path.join(NATIVE, "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_oracle_under_sanitizers(tmp_path):
    exe = _native_build().build_oracle_check(str(tmp_path / "oracle_check"))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    print(r.stdout, r.stderr, file=sys.stderr)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "0 failed" in r.stdout


def test_abi_check_reports_a_missing_device():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a device is present: the GPU test runs the checks")
    if not os.path.exists(ABI_CHECK):
        pytest.skip("abi_check not built (python tests/native/build.py)")
    r = subprocess.run([ABI_CHECK], capture_output=True, text=True, timeout=120, env=ENV)
    assert r.returncode == 77, (r.stdout, r.stderr[-4000:])
    assert "no device" in r.stdout


@pytest.mark.gpu
def test_abi_check_on_the_device():
    assert os.path.exists(ABI_CHECK), "abi_check not built (python tests/native/build.py)"
    print("[native] abi_check (checked device build, sanitized host)", flush=True)
    r = subprocess.run([ABI_CHECK], capture_output=True, text=True, timeout=300, env=ENV)
    print(r.stdout[-2000:], r.stderr[-6000:], flush=True)
    assert r.returncode == 0, r.stderr[-6000:]
    assert " 0 failed" in r.stdout
