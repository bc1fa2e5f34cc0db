"""Exactness of truncated unity with the complete form-factor set (oracle, CPU).

With all L x L lattice vectors as form factors and no mesh refinement, the
TU right-hand side (orbital loops, cross projections, bundle products) must
reproduce the momentum-space one-loop right-hand side of Sec. 3.1, written in
the band basis and carried to the orbital basis with U(k) (Sec. 4.1), then
projected with the channel projections of Sec. 2.  The direct particle-hole
part must equal -dC with the last two indices exchanged (Sec. 3.2).

The state is built so that the reconstructed vertex is antisymmetric: P and C
are the projections of random antisymmetric vertices (then V^C + V^D = 2 W_C).
"""

import numpy as np
import pytest

from oracle import bruteforce as bf
from oracle import tufrg
from synth import hubbard_hoppings, kanamori_V0, onsite_V0, rashba_hoppings, t2g_soc_hoppings

CASES = [
    ("rashba", 4, "temperature", 0.7),
    ("rashba", 4, "omega", 0.25),
    ("hubbard", 4, "temperature", 0.4),
    ("t2g", 2, "temperature", 0.9),
]


def _model(name):
    if name == "rashba":
        return rashba_hoppings(1.0, 0.4, tp=0.1), -0.3, onsite_V0(2.0)
    if name == "hubbard":
        return hubbard_hoppings(1.0, -0.25), -0.5, onsite_V0(3.0)
    return t2g_soc_hoppings(0.3, seed=1), 0.1, kanamori_V0(2.0, 0.3)


@pytest.mark.parametrize("name,L,scheme,lam", CASES)
def test_tu_rhs_equals_momentum_space_rhs(name, L, scheme, lam):
    hop, mu, V0 = _model(name)
    S = bf.complete_ff(L)
    st = tufrg.TUSetup(*hop, mu, V0, S, L, 1, scheme)
    lat = bf.Lattice(L)
    n = st.n_o
    rng = np.random.default_rng(7)

    def rnd():
        shape = (lat.N,) * 3 + (n,) * 4
        return 0.1 * bf.antisymmetrize(lat, rng.standard_normal(shape) + 1j * rng.standard_normal(shape))

    WP, WC = rnd(), rnd()
    P = bf.project_P(lat, WP, S)
    C = bf.project_C(lat, WC, S)
    V = (np.broadcast_to(st.V0, WP.shape) + bf.expand_P(lat, P, S) + bf.expand_C(lat, C, S)
         + bf.expand_D(lat, tufrg.d_from_c(C), S))
    assert np.abs(V - bf.antisymmetrize(lat, V) / 4).max() < 1e-12  # antisymmetric
    pp, phc, phd = bf.orbital_rhs(lat, V, st.U, st.e, lam, scheme)
    dP_ref = bf.project_P(lat, pp, S)
    dC_ref = bf.project_C(lat, phc, S)
    dD_ref = bf.project_D(lat, phd, S)
    dP, dC = tufrg.rhs(st, lam, P, C)
    scale = max(np.abs(dP_ref).max(), np.abs(dC_ref).max())
    assert scale > 1e-3
    assert np.abs(dP - dP_ref).max() < 1e-12 * scale
    assert np.abs(dC - dC_ref).max() < 1e-12 * scale
    assert np.abs(tufrg.d_from_c(dC) - dD_ref).max() < 1e-12 * scale
