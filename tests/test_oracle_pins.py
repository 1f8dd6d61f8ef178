"""The FP64 oracle against independent pins (CPU only)."""
import pytest

import pins


@pytest.mark.parametrize("name", sorted(pins.ALL_PINS))
def test_pin(name):
    ok, detail = pins.ALL_PINS[name]()
    assert ok, f"{name}: {detail}"
