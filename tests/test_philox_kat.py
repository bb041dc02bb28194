"""Philox4x32-10 against its published known-answer vectors (the generator's
definition, Salmon et al. 2011; fixture tests/golden/philox4x32_10_kat.txt).
Both the oracle's implementation and the library's (its host path, the same
function the device draws use) must reproduce every published word; the
avalanche and moment tests of the chain cannot catch a swapped multiplier or
a wrong key schedule, these vectors do.  No GPU needed."""
import os

import pytest

from paper_0910_2950_amd import fgi

HERE = os.path.dirname(os.path.abspath(__file__))


def kat_vectors():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.strip() and not line.startswith("#"):
            w = [int(x, 16) for x in line.split()]
            assert len(w) == 10
            rows.append((w[0:4], w[4:6], w[6:10]))
    assert len(rows) == 3
    return rows


@pytest.mark.parametrize("ctr,key,expect", kat_vectors())
def test_oracle_philox_known_answers(orc, ctr, key, expect):
    assert list(orc.philox(ctr, key)) == expect


@pytest.mark.parametrize("ctr,key,expect", kat_vectors())
def test_library_philox_known_answers(ctr, key, expect):
    assert list(fgi.philox4x32_10(ctr, key)) == expect
