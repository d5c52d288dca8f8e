import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: large CPU-side case")


@pytest.fixture
def forced():
    """Setter of launch-variant overrides (ssm_set_variant); every override
    is cleared when the test ends."""
    from paper_1608_08909_amd import ssm
    yield ssm.set_variant
    ssm.set_variant(None)
