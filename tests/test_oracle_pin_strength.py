"""The pins must catch plausible mistakes. Each case copies the oracle's source, plants one mistake by a
textual edit (on the CPU, in a temporary directory), builds it, and checks that at least one pin of the
descriptor (Eq. (6)) or of the network forward pass then fails."""
import os
import subprocess
import tempfile

import pytest

from tests import pins

MUTANTS = {
    # Eq. (6) without the self term in the numerator sum
    "self_term_numerator": ("double wsum = 1.0, gsum = g[(size_t)i * gs];", "double wsum = 1.0, gsum = 0.0;",
                            pins.DESCRIPTOR_PINS),
    # ... or in the normalisation
    "self_term_denominator": ("double wsum = 1.0, gsum = g[(size_t)i * gs];",
                              "double wsum = 0.0, gsum = g[(size_t)i * gs];", pins.DESCRIPTOR_PINS),
    # normalised by the neighbour count instead of the summed weight
    "count_normalisation": ("        wsum += w;\n", "        wsum += 1.0;\n", pins.DESCRIPTOR_PINS),
    # the reference descriptor d0 left out
    "d0_ignored": ("*d = gsum / wsum - d0;", "*d = gsum / wsum;", pins.DESCRIPTOR_PINS),
    # the first layer's weights read transposed
    "W1_transposed": ("s += P[MLP_W1 + c * MLP_NQ + f] * z[f];", "s += P[MLP_W1 + f * MLP_NH + c] * z[f];",
                      pins.MLP_PINS),
    # the second layer's weights read transposed
    "W2_transposed": ("s += P[MLP_W2 + c * MLP_NH + k] * h1[k];", "s += P[MLP_W2 + k * MLP_NH + c] * h1[k];",
                      pins.MLP_PINS),
    # ReLU in place of SiLU in the first layer
    "relu_activation": ("h1[c] = s * sigm(s);", "h1[c] = s > 0.0 ? s : 0.0;", pins.MLP_PINS),
    # the feature normalisation multiplied instead of divided
    "normalisation_multiplied": ("z[f] = (q[f] - P[MLP_MU + f]) / P[MLP_SIG + f];",
                                 "z[f] = (q[f] - P[MLP_MU + f]) * P[MLP_SIG + f];", pins.MLP_PINS),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(oracle, name):
    old, new, checks = MUTANTS[name]
    src_path = os.path.join(os.path.dirname(oracle.__file__), "ap_oracle.c")
    with open(src_path) as f:
        src = f.read()
    assert src.count(old) == 1, "the line to mutate must occur exactly once"
    with tempfile.TemporaryDirectory() as tmp:
        c_file = os.path.join(tmp, "mutant.c")
        so = os.path.join(tmp, "libmutant.so")
        with open(c_file, "w") as f:
            f.write(src.replace(old, new))
        subprocess.check_call(["gcc", "-O1", "-fopenmp", "-ffp-contract=off", "-std=c11", "-shared", "-fPIC",
                               "-o", so, c_file, "-lm"])
        lib = oracle.bind(so)
        failed = []
        for check in checks:
            try:
                check(oracle, _lib=lib)
            except (AssertionError, oracle.OracleError, FloatingPointError):
                failed.append(check.__name__)
        assert failed, "no pin fails with the mistake %r planted" % name
