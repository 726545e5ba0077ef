"""The host-side ABI tests (plan validation, device layout, argument checks;
no GPU) run once more against the AddressSanitizer build of the library's host
code.  Runs when that build exists (python -m paper_2605_21828_amd.build --asan);
the sanitizer aborts the child process on the first invalid access."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_ASAN = os.path.join(ROOT, "paper_2605_21828_amd", "libbfmht_asan.so")
SOURCES = [os.path.join(ROOT, "paper_2605_21828_amd", "csrc", f)
           for f in os.listdir(os.path.join(ROOT, "paper_2605_21828_amd", "csrc"))] + \
    [os.path.join(ROOT, "include", "bfmht.h")]


def _asan_build_current():
    """The sanitizer build exists and is newer than every source it is built from."""
    if not os.path.exists(LIB_ASAN):
        return False
    t = os.path.getmtime(LIB_ASAN)
    return all(os.path.getmtime(s) <= t for s in SOURCES if os.path.isfile(s))


@pytest.mark.skipif(not _asan_build_current(), reason="no current AddressSanitizer build "
                    "(python -m paper_2605_21828_amd.build --asan)")
def test_abi_tests_are_clean_under_address_sanitizer():
    sys.path.insert(0, ROOT)
    from paper_2605_21828_amd.build import asan_runtime
    env = dict(os.environ, BFMHT_LIB=LIB_ASAN, LD_PRELOAD=asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "AddressSanitizer" not in r.stderr
