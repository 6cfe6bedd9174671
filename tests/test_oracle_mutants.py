"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each mutant is the oracle compiled with -DORACLE_MUTANT=n, which plants one
plausible bug (tie rule reversed, self not excluded, a coordinate dropped, L1
instead of squared L2, kernel width off by two, a term missing from the
normaliser, the shift sign flipped, normaliser N instead of 2N, mirrored
term dropped, distance for squared distance in the attraction kernel, force
direction reversed).  The test passes only if some pin fails on every mutant.
"""
import numpy as np
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


def _recall_counting_duplicates(approx, exact, query_ids=None, n=None):
    # plausible mistake: intersect the raw lists, each repeated id a hit
    M, K = np.asarray(exact).shape
    return sum(len(np.intersect1d(a, b, assume_unique=True)) for a, b in zip(approx, exact)) / float(M * K)


def _recall_counting_absent(approx, exact, query_ids=None, n=None):
    # plausible mistake: no validation, and -1 entries matched as ids
    M, K = np.asarray(exact).shape
    return sum(len(set(a.tolist()) & set(b.tolist())) for a, b in zip(approx, exact)) / float(M * K)


def _recall_over_listed(approx, exact, query_ids=None, n=None):
    # plausible mistake: divide by the approximate row's listed count
    tot = 0.0
    for a, b in zip(approx, exact):
        a = [v for v in a.tolist() if v >= 0]
        if len(set(a)) != len(a) or (query_ids is not None) or (n is not None and max(a) >= n):
            raise ValueError("invalid")
        tot += len(set(a) & set(b.tolist())) / max(1, len(a))
    return tot / len(exact)


@pytest.mark.parametrize("mutant", [_recall_counting_duplicates, _recall_counting_absent, _recall_over_listed])
def test_recall_pin_catches_planted_mistake(mutant):
    with pytest.raises(AssertionError):
        pins.pin_recall(None, recall=mutant)
