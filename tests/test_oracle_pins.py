"""The FP64 oracle against its pins (CPU only)."""
import pytest

from oracle import oracle as O
from tests import oracle_pins as pins


@pytest.fixture(scope="module")
def ora():
    return O.get()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(ora, pin):
    assert ora.mutant == 0
    pin(ora)


def test_oracle_rejects_bad_arguments(ora):
    import numpy as np
    X = np.zeros((5, 2), np.float32)
    with pytest.raises(ValueError):
        ora.knn(X, 5)  # K > N - 1
    with pytest.raises(ValueError):
        ora.calibrate(np.ones((1, 10)), 10.0)  # mu must be < K
    with pytest.raises(ValueError):
        ora.calibrate(np.ones((1, 10)), 0.5)  # mu must be >= 1
