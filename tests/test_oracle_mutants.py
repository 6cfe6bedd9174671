"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each mutant is the oracle compiled with -DORACLE_MUTANT=n, which plants one
plausible bug (tie rule reversed, self not excluded, a coordinate dropped, L1
instead of squared L2, kernel width off by two, a term missing from the
normaliser, the shift sign flipped, normaliser N instead of 2N, mirrored
term dropped, distance for squared distance in the attraction kernel, force
direction reversed).  The test passes only if some pin fails on every mutant.
"""
import pytest

from oracle import oracle as O
from tests import oracle_pins as pins

MUTANTS = {
    1: pins.KNN_PINS, 2: pins.KNN_PINS, 3: pins.KNN_PINS, 4: pins.KNN_PINS,
    5: pins.CAL_PINS, 6: pins.CAL_PINS, 7: pins.CAL_PINS,
    8: pins.SYM_PINS, 9: pins.SYM_PINS,
    10: pins.ATTR_PINS, 11: pins.ATTR_PINS,
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_planted_mistake(mutant, tmp_path):
    lib = O.build(mutant=mutant, out=tmp_path / ("liboracle_m%d.so" % mutant))
    o = O.Oracle(lib)
    assert o.mutant == mutant
    caught = []
    for pin in MUTANTS[mutant]:
        try:
            pin(o)
        except (AssertionError, ValueError, FloatingPointError, ZeroDivisionError):
            caught.append(pin.__name__)
    assert caught, "mutant %d slipped past every pin" % mutant
