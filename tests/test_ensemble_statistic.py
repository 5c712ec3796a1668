"""The ensemble comparison used by the long-run GPU tests has power: two oracle
ensembles from different seeds pass it, and the same pair with the density of
one scaled by 1 + 0.01 (far below the noise of a single cell) fails it."""
import pytest

import _ensemble as E
from oracle import oracle as O
from paper_2305_12071_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def test_the_ensemble_comparison_sees_a_small_bias():
    c = I.mach3_small()
    a = E.oracle_runs(c, 16, 5005, 300, 150)
    b = E.oracle_runs(c, 16, 6006, 300, 150)
    E.compare(a, b, "oracle vs oracle")
    b2 = b.copy()
    b2[:, :, 0] *= 1.01
    with pytest.raises(AssertionError):
        E.compare(a, b2, "biased")
