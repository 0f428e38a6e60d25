"""Address/undefined-behaviour sanitizer builds, run on the CPU: the oracle
(every entry point on small cases of each code path) and the host side of the
library's C ABI (argument checks of every entry point, and the basis and
neighbour-table construction of dg_init, which without a GPU then fails in the
device allocation and must release everything)."""
import shutil

import pytest

pytestmark = pytest.mark.slow


def _clean(text):
    return "ERROR: AddressSanitizer" not in text and "runtime error:" not in text


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_oracle_under_sanitizers(orc):
    rc, text = orc.sanitize_check()
    assert rc == 0 and _clean(text) and "sanitize_check: ok" in text, text[-3000:]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_abi_host_checks_under_sanitizers():
    from paper_2306_12891_amd.csrc import sanitize
    rc, text = sanitize.build_and_run()
    assert rc == 0 and _clean(text) and "abi_check: ok" in text, text[-3000:]
