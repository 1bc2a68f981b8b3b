"""The oracle, and the host side of the HIP library, built with AddressSanitizer and
UndefinedBehaviorSanitizer and run on the CPU (paper_2604_07980_amd.sanitize): each driver
must finish without a report. No GPU."""
import shutil

import pytest

from paper_2604_07980_amd import sanitize


@pytest.fixture(scope="module")
def outdir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("sanitized"))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(outdir):
    assert "sanitize_driver: ok" in sanitize.run(sanitize.build_oracle(outdir))


@pytest.mark.timeout(900)
def test_library_host_side_under_sanitizers(outdir):
    assert "host_abi_driver: ok" in sanitize.run(sanitize.build_host(outdir))
