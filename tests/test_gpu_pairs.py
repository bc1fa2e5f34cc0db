"""Kramers-paired six-orbital loops: for six bands degenerate in pairs at
every k (time reversal with inversion) the loops sum each pair first (BF16X3
on the matrix cores, FP32 and FP64 on the vector units).  Checked against the
six-band evaluation on the same context and against the oracle; a
Zeeman-split model keeps the six bands, and so does an odd fine mesh in
BF16X3 (its kernel pairs ky points too)."""

import os
import sys

import numpy as np
import pytest
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

pytestmark = pytest.mark.gpu

from oracle import tufrg as otu  # noqa: E402
from synth import PAULI, ff_shell, kanamori_V0, t2g_soc_hoppings  # noqa: E402
from tests._layout import ph_loop_to_matrix, pp_loop_to_matrix  # noqa: E402

TOL = 1e-4  # BF16X3 loops against the FP64 oracle


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_08830_amd import tufrg
    return tufrg


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


def _case(zeeman=0.0, Lq=6, n_ref=3, cutoff="omega", n_ff=9):
    R, t = t2g_soc_hoppings(0.2, seed=1)
    t = np.array(t, copy=True)
    if zeeman:
        i0 = [i for i, r in enumerate(np.asarray(R)) if r[0] == 0 and r[1] == 0][0]
        t[i0] = t[i0] + zeeman * np.kron(np.eye(3), PAULI[2])
    return dict(hop=(R, t), mu=0.35, V0=kanamori_V0(2.0, 0.3), ff=ff_shell(n_ff), Lq=Lq, n_ref=n_ref,
                cutoff=cutoff, temperature=0.06 if cutoff == "shell" else None)


def _ctx(T, c, prec="bf16x3"):
    return T.Context(c["hop"][0], c["hop"][1], c["mu"], c["V0"], c["ff"], c["Lq"], c["n_ref"], c["cutoff"],
                     prec, temperature=c["temperature"])


def _bubbles(T, ctx, lam, deriv):
    out = []
    for ch in (T.PP, T.PH):
        L = torch.zeros((ctx.Nq, ctx.B, ctx.B), dtype=torch.complex128, device="cuda")
        T.tufrg_bubble(ctx, ch, lam, deriv, L)
        torch.cuda.synchronize()
        out.append(L.cpu().numpy())
    return out


def _oracle(c, lam, deriv):
    st = otu.TUSetup(*c["hop"], c["mu"], c["V0"], c["ff"], c["Lq"], c["n_ref"], c["cutoff"],
                     temperature=c["temperature"])
    return [pp_loop_to_matrix(otu.loops(st, "pp", lam, deriv=bool(deriv))),
            ph_loop_to_matrix(otu.loops(st, "ph", lam, deriv=bool(deriv)))]


@pytest.mark.parametrize("cutoff", ["omega", "temperature", "shell"])
def test_paired_loops_equal_the_six_band_loops_and_the_oracle(T, cutoff):
    c = _case(cutoff=cutoff)
    ctx = _ctx(T, c)
    lam, deriv = 0.35, 1
    print(f"pairs: t2g S9 6x6 refined 3x, {cutoff}", flush=True)
    assert T.tufrg_pair_bands(ctx, True) is True
    paired = _bubbles(T, ctx, lam, deriv)
    assert T.tufrg_pair_bands(ctx, False) is False
    six = _bubbles(T, ctx, lam, deriv)
    ref = _oracle(c, lam, deriv)
    for p, s, r in zip(paired, six, ref):
        print(f"paired vs six bands {rel(p, s):.2e}, paired vs oracle {rel(p, r):.2e}, six vs oracle {rel(s, r):.2e}")
        assert rel(p, s) < 1e-5
        assert rel(p, r) < TOL and rel(s, r) < TOL
    # back to the pairs: the A operand is rebuilt, the same bits come out
    assert T.tufrg_pair_bands(ctx, True) is True
    again = _bubbles(T, ctx, lam, deriv)
    for p, a in zip(paired, again):
        assert np.array_equal(p, a)
    ctx.close()


def test_ragged_paired_mesh_with_the_13_vector_shell(T):
    """L_f = 18: nine ky pairs, one partial tile; the S13 diamond."""
    c = _case(Lq=9, n_ref=2, cutoff="temperature", n_ff=13)
    ctx = _ctx(T, c)
    assert T.tufrg_pair_bands(ctx, True) is True
    for deriv in (1, 0):
        got = _bubbles(T, ctx, 0.35, deriv)
        for g, r in zip(got, _oracle(c, 0.35, deriv)):
            assert rel(g, r) < TOL
    ctx.close()


@pytest.mark.parametrize("what", ["zeeman", "odd mesh"])
def test_bands_that_are_not_paired_keep_six_bands(T, what):
    c = _case(zeeman=0.05) if what == "zeeman" else _case(Lq=5, n_ref=3)
    ctx = _ctx(T, c)
    assert T.tufrg_pair_bands(ctx, True) is False
    got = _bubbles(T, ctx, 0.35, 1)
    for g, r in zip(got, _oracle(c, 0.35, 1)):
        assert rel(g, r) < TOL
    ctx.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
@pytest.mark.parametrize("cutoff", ["temperature", "shell"])
def test_paired_vector_loops_equal_the_six_band_loops_and_the_oracle(T, prec, tol, cutoff):
    """The vector-unit kernels: an odd fine mesh (L_f = 15) pairs as well."""
    c = _case(Lq=5, n_ref=3, cutoff=cutoff)
    ctx = _ctx(T, c, prec)
    print(f"pairs: t2g S9 5x5 refined 3x, {prec}, {cutoff}", flush=True)
    assert T.tufrg_pair_bands(ctx, True) is True
    paired = _bubbles(T, ctx, 0.35, 1)
    assert T.tufrg_pair_bands(ctx, False) is False
    six = _bubbles(T, ctx, 0.35, 1)
    for p, s_, r in zip(paired, six, _oracle(c, 0.35, 1)):
        print(f"paired vs six bands {rel(p, s_):.2e}, paired vs oracle {rel(p, r):.2e}")
        assert rel(p, s_) < tol and rel(p, r) < tol and rel(s_, r) < tol
    ctx.close()


def test_zeeman_split_vector_loops_keep_six_bands(T):
    c = _case(zeeman=0.05)
    ctx = _ctx(T, c, "fp64")
    assert T.tufrg_pair_bands(ctx, True) is False
    for g, r in zip(_bubbles(T, ctx, 0.35, 1), _oracle(c, 0.35, 1)):
        assert rel(g, r) < 1e-10
    ctx.close()
