"""The stored full-size floating-point reference values (tests/golden/
reference_values.json) come from two independent oracle evaluators that
agree: the double-double Glynn sum over row signs (Sec. 1.2 Eq. glynn) and
the double-double Ryser sum over column subsets (Eq. ryser_square) -- they
share no seeding, update or term, so a fault in either (a seeding error at
large Gray indices, a dropped sign) would show as a disagreement far beyond
their rounding."""
import json
import os

import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "reference_values.json")


def dd(v):
    return (v["hi"], v["lo"])


def val(v):
    """(re, im) of a stored value, each as an exact rational-free float pair."""
    if "hi" in v:
        return (dd(v), None)
    return (dd(v["re"]), dd(v["im"]))


def diff(a, b):
    # double-double difference without rounding the parts together first
    return abs((a[0] - b[0]) + (a[1] - b[1]))


@pytest.mark.parametrize("name", ["u32", "c32", "u36"])
def test_glynn_and_ryser_references_agree(name):
    rec = json.load(open(GOLDEN))[name]
    if "value_ryser" not in rec:
        pytest.skip(f"second evaluator not stored for {name} "
                    "(tests/golden/make_golden.py --second)")
    g_re, g_im = val(rec["value"])
    r_re, r_im = val(rec["value_ryser"])
    mag = abs(g_re[0]) if g_im is None else abs(complex(g_re[0], g_im[0]))
    # each double-double sum of 2^31..2^36 terms is within ~1e-26 of the true
    # value relative to its magnitude here (the terms cancel to a few digits);
    # 1e-22 relative leaves a wide margin and still checks ~22 digits
    assert diff(g_re, r_re) <= 1e-22 * mag, (name, g_re, r_re)
    if g_im is not None:
        assert diff(g_im, r_im) <= 1e-22 * mag, (name, g_im, r_im)
