import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# torch ships its own HIP runtime.  Loading it before libctm.so lets the
# library bind to that same runtime; the other order leaves two runtimes in
# the process and torch then finds no device.  (Importing is enough; it does
# not touch the GPU.)
try:
    import torch  # noqa: F401
except Exception:
    pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU oracle case")


@pytest.fixture(autouse=True)
def _guard_bands(request):
    """With poisoned allocations on (CTM_POISON_ALLOC), a GPU test fails if a
    library buffer freed during it had a damaged guard band (a kernel wrote
    past the end of a buffer)."""
    poison = os.environ.get("CTM_POISON_ALLOC", "")
    if request.node.get_closest_marker("gpu") is None or poison in ("", "0"):
        yield
        return
    from paper_1906_02220_amd import ctm
    before = ctm.guard_violations()
    yield
    import gc
    gc.collect()
    after = ctm.guard_violations()
    assert after == before, "%d guard band(s) damaged during this test" % (after - before)
