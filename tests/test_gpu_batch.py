"""Batched flows of independent instances (uneven models, form-factor sets and
meshes) through the C ABI: every instance of a lockstep batch reproduces its
own single-context flow exactly and the FP64 oracle flow."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import tufrg as otu  # noqa: E402
from synth import ff_shell, hubbard_hoppings, onsite_V0, rashba_hoppings  # noqa: E402
from synth.workloads import batch_instances  # noqa: E402
from tests._layout import c_to_matrix, p_to_matrix  # noqa: E402


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_08830_amd import tufrg
    return tufrg


def dev():
    return torch.device("cuda:0")


def _inst(hop, mu, U, n_ff, Lq, n_ref, cutoff="temperature"):
    return dict(hop_R=hop[0], hop_t=hop[1], mu=mu, V0=onsite_V0(U), ff=ff_shell(n_ff), Lq=Lq, n_ref=n_ref,
                cutoff=cutoff, n_o=2)


def _small_batch():
    return [
        _inst(hubbard_hoppings(1.0, -0.25), -0.6, 3.0, 5, 6, 3),
        _inst(rashba_hoppings(1.0, 0.3), -0.4, 2.5, 9, 5, 4, "omega"),
        _inst(rashba_hoppings(1.0, 0.45), -0.2, 2.0, 13, 9, 2),
        _inst(rashba_hoppings(1.0, 0.1), -0.8, 1.7, 5, 7, 3),
    ]


def _state(d):
    P = torch.zeros((d["Nq"], d["B"], d["B"]), dtype=torch.complex128, device=dev())
    return P, torch.zeros_like(P)


def _single(T, w, prec, n_steps, lam0=10.0, lam_end=1.0, **kw):
    ctx = T.Context(w["hop_R"], w["hop_t"], w["mu"], w["V0"], w["ff"], w["Lq"], w["n_ref"], w["cutoff"], prec)
    P, C = _state(dict(Nq=ctx.Nq, B=ctx.B))
    r = T.tufrg_flow(ctx, P, C, lam0, lam_end, n_steps=n_steps, **kw)
    torch.cuda.synchronize()
    ctx.close()
    return r, P.cpu().numpy(), C.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("fused", [False, True])
def test_batch_equals_single_flows(T, prec, fused):
    """Loop launches per instance (the default) and fused ones (one launch
    per kernel shape over all instances, S5/S9 and S13 shapes here) give every
    instance its own flow bit for bit."""
    print(f"batch: {prec} fused_loops={fused}", flush=True)
    ws = _small_batch()
    b = T.Batch(ws, precision=prec, n_streams=3)
    Ps, Cs = zip(*[_state(d) for d in b.dims])
    res = T.tufrg_batch_flow(b, Ps, Cs, 10.0, 1.0, n_steps=6, fused_loops=fused)
    torch.cuda.synchronize()
    for i, w in enumerate(ws):
        r, P, C = _single(T, w, prec, 6)
        assert res[i]["n_steps"] == r["n_steps"] == 6
        assert np.array_equal(Ps[i].cpu().numpy(), P) and np.array_equal(Cs[i].cpu().numpy(), C)
        assert res[i]["max_coupling"] == r["max_coupling"]


def test_batch_instance_matches_oracle_flow(T):
    ws = _small_batch()
    b = T.Batch(ws, precision="fp64", n_streams=2)
    Ps, Cs = zip(*[_state(d) for d in b.dims])
    T.tufrg_batch_flow(b, Ps, Cs, 10.0, 1.0, n_steps=4)
    torch.cuda.synchronize()
    for i in (0, 1):
        w = ws[i]
        st = otu.TUSetup(w["hop_R"], w["hop_t"], w["mu"], w["V0"], w["ff"], w["Lq"], w["n_ref"], w["cutoff"])
        Pt, Ct, _ = otu.flow_euler(st, 10.0, 1.0, 4, v_max=1e30)
        Pr, Cr = p_to_matrix(Pt), c_to_matrix(Ct)
        for got, ref in ((Ps[i], Pr), (Cs[i], Cr)):
            got = got.cpu().numpy()
            assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max()


def test_diverging_instance_stops_alone(T):
    ws = _small_batch()[:2]
    ws[0] = _inst(hubbard_hoppings(1.0, -0.25), -0.6, -4.0, 5, 6, 3)  # attractive: Cooper instability
    b = T.Batch(ws, precision="fp64", n_streams=2)
    Ps, Cs = zip(*[_state(d) for d in b.dims])
    res = T.tufrg_batch_flow(b, Ps, Cs, 5.0, 0.01, n_steps=30, v_max=20.0)
    r0, P0, _ = _single(T, ws[0], "fp64", 30, lam0=5.0, lam_end=0.01, v_max=20.0)
    assert r0["diverged"] == 1 and res[0]["diverged"] == 1
    assert res[0]["n_steps"] == r0["n_steps"] < 30 and res[0]["lambda_c"] == r0["lambda_c"]
    assert np.array_equal(Ps[0].cpu().numpy(), P0)
    r1, P1, _ = _single(T, ws[1], "fp64", 30, lam0=5.0, lam_end=0.01, v_max=20.0)
    assert res[1]["diverged"] == r1["diverged"] and res[1]["n_steps"] == r1["n_steps"]
    assert np.array_equal(Ps[1].cpu().numpy(), P1)


def test_rejects_what_it_does_not_do(T):
    b = T.Batch(_small_batch()[:1], precision="fp64", n_streams=1)
    Ps, Cs = zip(*[_state(d) for d in b.dims])
    with pytest.raises(T.TufrgError):
        T.tufrg_batch_flow(b, Ps, Cs, 10.0, 1.0, n_steps=0)


def test_full_batch_of_32_runs_and_matches_single_flows(T):
    ws = batch_instances(32, seed=2, n_ref=12)
    b = T.Batch(ws, precision="fp32", n_streams=4)
    assert sorted({d["B"] for d in b.dims}) == sorted({4 * len(w["ff"]) for w in ws})
    Ps, Cs = zip(*[_state(d) for d in b.dims])
    res = T.tufrg_batch_flow(b, Ps, Cs, 10.0, 1.0, n_steps=2)
    torch.cuda.synchronize()
    assert all(r["n_steps"] == 2 for r in res)
    for i in (0, 17, 31):
        r, P, C = _single(T, ws[i], "fp32", 2)
        assert np.array_equal(Ps[i].cpu().numpy(), P) and np.array_equal(Cs[i].cpu().numpy(), C)
