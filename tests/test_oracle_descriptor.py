"""Pins of the oracle's descriptor, Eq. (6), against values fixed by its definition, and the tie between the
exported descriptor and the one inside the full evaluation."""
import numpy as np
import pytest

from tests import pins
from tests.helpers import small_system


@pytest.mark.parametrize("pin", pins.DESCRIPTOR_PINS, ids=lambda f: f.__name__)
def test_descriptor_closed_forms(oracle, pin):
    pin(oracle)


def test_network_one_path_closed_form(oracle):
    pins.one_path_network(oracle)


def test_evaluation_uses_the_pinned_descriptor(oracle):
    """The descriptor and normalisation inside the full AP evaluation equal, bit for bit, Eq. (6) applied to
    the evaluation's own CSP values."""
    s = small_system(nc=4, sigma=0.12)
    s["sw"]["d0"] = 0.07
    s["csp"] = oracle.csp_pairs(s["pos_ref"], s["box"], 8)
    aux = oracle.evaluate(s)["aux"]
    wbar, d = oracle.descriptor(s["pos"], s["box"], aux["g"], s["sw"]["r_w"], 0.07)
    assert np.array_equal(wbar, aux["wbar"]) and np.array_equal(d, aux["d"])
