"""The host-side CPU tests again, against the AddressSanitizer +
UndefinedBehaviorSanitizer build of the library's host code (build.py's
sanitize option; the GPU code is not instrumented).  Any report aborts the
child run."""
import shutil

import pytest

from paper_2104_04582_amd import build


@pytest.mark.skipif(shutil.which("/opt/rocm/bin/hipcc") is None, reason="needs hipcc")
def test_host_core_under_address_and_ub_sanitizers():
    assert build.run_host_tests_sanitized(("tests/test_host_core.py", "-q", "-x")) == 0
