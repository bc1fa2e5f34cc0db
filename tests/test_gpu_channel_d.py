"""The third channel D (Sec. 3.2: D_{n1n2n3n4} = -C_{n1n2n4n3}) through the C
ABI: bit-exact against the oracle's d_from_c on random states, for two and
six spin-orbitals, and the argument checks."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import tufrg as otu  # noqa: E402
from synth import ff_shell, hubbard_hoppings, kanamori_V0, onsite_V0, random_exchange_state, t2g_soc_hoppings  # noqa: E402
from tests._layout import c_to_matrix  # noqa: E402


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_08830_amd import tufrg
    return tufrg


CASES = {
    "hub9": (hubbard_hoppings(1.0, -0.25), -0.6, onsite_V0(3.0), ff_shell(9), 6, 2),
    "t2g5": (t2g_soc_hoppings(0.2, seed=1), 0.35, kanamori_V0(2.0, 0.3), ff_shell(5), 5, 1),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_channel_d_equals_oracle_exactly(T, name):
    hop, mu, V0, ff, Lq, n_ref = CASES[name]
    ctx = T.Context(hop[0], hop[1], mu, V0, ff, Lq, n_ref, "temperature", "fp64")
    n_o = hop[1].shape[1]
    C = random_exchange_state(Lq * Lq, len(ff), n_o, seed=11)
    Cd = torch.from_numpy(c_to_matrix(C)).cuda()
    D = torch.empty_like(Cd)
    T.tufrg_channel_d(ctx, Cd, D)
    torch.cuda.synchronize()
    ref = c_to_matrix(otu.d_from_c(C))
    assert np.array_equal(D.cpu().numpy(), ref)
    ctx.close()


def test_channel_d_rejects_overlap_and_host_arrays(T):
    hop, mu, V0, ff, Lq, n_ref = CASES["hub9"]
    ctx = T.Context(hop[0], hop[1], mu, V0, ff, Lq, n_ref, "temperature", "fp64")
    X = torch.zeros((ctx.Nq, ctx.B, ctx.B), dtype=torch.complex128, device="cuda")
    with pytest.raises(T.TufrgError) as ei:
        T.tufrg_channel_d(ctx, X, X)
    assert "overlap" in str(ei.value)
    with pytest.raises(T.TufrgError):
        T.tufrg_channel_d(ctx, X, torch.zeros_like(X, device="cpu"))
    ctx.close()
