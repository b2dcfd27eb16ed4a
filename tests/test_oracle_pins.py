"""The CPU oracle against what the paper and mathematics fix (CPU only)."""
import pytest

from tests import _pins


@pytest.mark.parametrize("check", _pins.ALL, ids=lambda f: f.__name__)
def test_pin(orc, check):
    check(orc)
