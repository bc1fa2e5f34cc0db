"""Non-local initial interactions on the GPU against the FP64 oracle, through
the C ABI: a density-density interaction beyond the onsite term enters as a
static C-channel term C0 (tufrg_set_initial_c) and reaches every projection,
right-hand side and flow.  The oracle side is pinned against the bare vertex
in tests/test_oracle_projections.py."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import tufrg as otu  # noqa: E402
from synth import (density_density_c0, ff_shell, hubbard_hoppings, kanamori_V0, onsite_V0,  # noqa: E402
                   random_exchange_state, rashba_hoppings, t2g_soc_hoppings)
from tests._layout import c_to_matrix, p_to_matrix  # noqa: E402

BONDS = [((1, 0), 0.6), ((-1, 0), 0.6), ((0, 1), 0.6), ((0, -1), 0.6), ((1, 1), -0.15), ((-1, -1), -0.15)]


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_08830_amd import tufrg
    return tufrg


def dev():
    return torch.device("cuda:0")


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


def _case(name):
    if name == "hub5":
        return dict(hop=hubbard_hoppings(1.0, -0.25), mu=-0.6, V0=onsite_V0(2.0), ff=ff_shell(5), Lq=6, n_ref=3,
                    cutoff="temperature")
    if name == "ras9":
        return dict(hop=rashba_hoppings(1.0, 0.3), mu=-0.4, V0=onsite_V0(2.5), ff=ff_shell(9), Lq=5, n_ref=6,
                    cutoff="omega")
    if name == "t2g9":
        return dict(hop=t2g_soc_hoppings(0.2, seed=1), mu=0.35, V0=kanamori_V0(2.0, 0.3), ff=ff_shell(9), Lq=6,
                    n_ref=2, cutoff="temperature")
    raise KeyError(name)


def _both(T, c, prec="fp64"):
    n_o = c["hop"][1].shape[1]
    C0 = density_density_c0(c["Lq"], n_o, c["ff"], BONDS)
    st = otu.TUSetup(*c["hop"], c["mu"], c["V0"], c["ff"], c["Lq"], c["n_ref"], c["cutoff"], C0=C0)
    ctx = T.Context(c["hop"][0], c["hop"][1], c["mu"], c["V0"], c["ff"], c["Lq"], c["n_ref"], c["cutoff"], prec)
    T.tufrg_set_initial_c(ctx, torch.from_numpy(c_to_matrix(C0)).to(dev()))
    return st, ctx


def _zeros(ctx):
    return torch.zeros((ctx.Nq, ctx.B, ctx.B), dtype=torch.complex128, device=dev())


def _state(st, seed):
    P = 0.1 * random_exchange_state(st.Nq, st.n_ff, st.n_o, seed=seed)
    C = 0.1 * random_exchange_state(st.Nq, st.n_ff, st.n_o, seed=seed + 1)
    return P, C


@pytest.mark.parametrize("name", ["hub5", "ras9", "t2g9"])
def test_projections_with_nonlocal_interaction(T, name):
    st, ctx = _both(T, _case(name))
    P, C = _state(st, 40)
    VP, VC = _zeros(ctx), _zeros(ctx)
    T.tufrg_project(ctx, torch.from_numpy(p_to_matrix(P)).to(dev()), torch.from_numpy(c_to_matrix(C)).to(dev()),
                    VP, VC)
    torch.cuda.synchronize()
    rVP, rVC = otu.projected_vertices(st, P, C)
    assert rel(VP.cpu().numpy(), p_to_matrix(rVP)) < 1e-12
    assert rel(VC.cpu().numpy(), c_to_matrix(rVC)) < 1e-12
    # removing C0 restores the onsite-only projections
    T.tufrg_set_initial_c(ctx, None)
    T.tufrg_project(ctx, torch.from_numpy(p_to_matrix(P)).to(dev()), torch.from_numpy(c_to_matrix(C)).to(dev()),
                    VP, VC)
    torch.cuda.synchronize()
    st.C0 = None
    rVP, _ = otu.projected_vertices(st, P, C)
    assert rel(VP.cpu().numpy(), p_to_matrix(rVP)) < 1e-12


@pytest.mark.parametrize("name,prec", [("hub5", "fp64"), ("hub5", "fp32"), ("ras9", "fp64"), ("t2g9", "fp32")])
def test_rhs_with_nonlocal_interaction(T, name, prec):
    st, ctx = _both(T, _case(name), prec)
    P, C = _state(st, 50)
    dP, dC = _zeros(ctx), _zeros(ctx)
    lam = 0.4
    T.tufrg_rhs(ctx, lam, torch.from_numpy(p_to_matrix(P)).to(dev()), torch.from_numpy(c_to_matrix(C)).to(dev()),
                dP, dC)
    torch.cuda.synchronize()
    rP, rC = otu.rhs(st, lam, P, C)
    tol = 1e-10 if prec == "fp64" else 3e-5
    assert rel(dP.cpu().numpy(), p_to_matrix(rP)) < tol
    assert rel(dC.cpu().numpy(), c_to_matrix(rC)) < tol


def test_euler_flow_with_nonlocal_interaction(T):
    """From P = C = 0 the non-local bare interaction alone drives the flow."""
    st, ctx = _both(T, _case("hub5"))
    Pr, Cr, rr = otu.flow_euler(st, 10.0, 0.3, 8, v_max=1e30)
    P, C = _zeros(ctx), _zeros(ctx)
    res = T.tufrg_flow(ctx, P, C, 10.0, 0.3, n_steps=8, v_max=1e30)
    torch.cuda.synchronize()
    assert res["n_steps"] == rr["n_steps"] == 8
    assert rel(P.cpu().numpy(), p_to_matrix(Pr)) < 1e-10
    assert rel(C.cpu().numpy(), c_to_matrix(Cr)) < 1e-10
    # the non-local terms feed form-factor blocks of P beyond (0,0)
    off = Pr.copy()
    off[:, 0, 0] = 0
    assert np.abs(off).max() > 1e-3 * np.abs(Pr).max()
