"""The oracle's compensated k sum: Neumaier's addition keeps the low parts a
plain FP64 sum loses, and the loop matrix does not depend on how the fine
mesh is cut into chunks beyond rounding."""

import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import tufrg as otu  # noqa: E402
from synth import ff_shell, hubbard_hoppings, onsite_V0  # noqa: E402


def test_neumaier_recovers_what_a_plain_sum_loses():
    xs = [np.array([1e16 + 1e16j]), np.array([1.0 - 3.0j]), np.array([-1e16 - 1e16j])]
    acc, comp = np.zeros(1, complex), np.zeros(1, complex)
    plain = np.zeros(1, complex)
    for x in xs:
        acc, comp = otu._neumaier_add(acc, comp, x)
        plain = plain + x
    assert plain[0] != 1.0 - 3.0j  # rounded away without compensation (0 and -4j)
    assert acc[0] + comp[0] == 1.0 - 3.0j


def test_loop_matrix_is_independent_of_the_chunking():
    st = otu.TUSetup(*hubbard_hoppings(1.0, -0.25), -0.6, onsite_V0(3.0), ff_shell(5), 6, 3, "temperature")
    a = otu.loop_matrix(st, "pp", 5, 0.4, k_chunk=7)
    b = otu.loop_matrix(st, "pp", 5, 0.4, k_chunk=4096)
    assert np.abs(a - b).max() <= 1e-15 * np.abs(b).max()
