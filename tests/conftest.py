import os
import shutil
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the tests measure launch shapes afresh and write no shape file; the test of
# the file and the full-size tests (bench_shapes) name their own
os.environ["ENS_TUNE_CACHE"] = "off"
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    return oracle.lib()


@pytest.fixture
def bench_shapes(tmp_path, monkeypatch):
    """Launch shapes from a copy of the library's committed shape file, as the
    benchmark takes them (a device the file has no line for measures its
    shapes into the copy)."""
    dst = tmp_path / "ens_tune_cache.txt"
    shutil.copyfile(os.path.join(ROOT, "paper_2304_11399_amd", "ens_tune_cache.txt"), dst)
    monkeypatch.setenv("ENS_TUNE_CACHE", str(dst))
