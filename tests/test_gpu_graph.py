"""Euler steps captured in HIP graphs (tufrg_flow_opts.graph_steps) against
direct launches (GPU).

A graph holds several steps with their step-dependent scales; the flow
launches a new graph (the executable updated in place) every graph_steps
steps, with the library's own eager work (state copies, slot readbacks) and
host synchronisations between the launches.  Every result must equal the
direct flow bit for bit: the kernels sum in a fixed order, so capturing them
changes nothing.  A flow that diverges inside a graph undoes that graph and
replays its steps one by one (same stopping step and critical scale).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth import (ff_shell, hubbard_hoppings, kanamori_V0, onsite_V0, rashba_hoppings,  # noqa: E402
                   t2g_soc_hoppings)


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_08830_amd import tufrg
    return tufrg


CASES = {
    "hub5": (hubbard_hoppings(1.0, -0.25), -0.6, onsite_V0(3.0), ff_shell(5), 6, 3, "temperature"),
    "ras9": (rashba_hoppings(1.0, 0.3), -0.4, onsite_V0(2.5), ff_shell(9), 5, 4, "omega"),
    "t2g9": (t2g_soc_hoppings(0.2, seed=1), 0.35, kanamori_V0(2.0, 0.3), ff_shell(9), 6, 3, "temperature"),
    # attractive Hubbard: diverges within the flow
    "hubneg": (hubbard_hoppings(1.0, -0.25), -0.5, onsite_V0(-4.0), ff_shell(5), 6, 2, "temperature"),
}


def _flow(T, name, prec, stream, **kw):
    hop, mu, V0, ff, Lq, n_ref, cut = CASES[name]
    ctx = T.Context(hop[0], hop[1], mu, V0, ff, Lq, n_ref, cut, prec, stream=stream)
    P = torch.zeros((ctx.Nq, ctx.B, ctx.B), dtype=torch.complex128, device="cuda")
    C = torch.zeros_like(P)
    r = T.tufrg_flow(ctx, P, C, **kw)
    torch.cuda.synchronize()
    ctx.close()
    return r, P.cpu().numpy(), C.cpu().numpy()


@pytest.mark.parametrize("name,prec", [("hub5", "fp64"), ("hub5", "fp32"), ("ras9", "fp32"), ("t2g9", "bf16x3")])
@pytest.mark.parametrize("on_stream", [False, True])
def test_graph_steps_equal_direct_launches(T, name, prec, on_stream):
    """13 steps with graphs of 4: one direct step, then graphs of 4, 4, 4 (each
    launched after eager copies and a synchronisation); on the null stream the
    library captures on a private stream, else on the context's stream."""
    print(f"graph: {name} {prec} stream={on_stream}", flush=True)
    stream = torch.cuda.Stream() if on_stream else None
    kw = dict(lambda0=10.0, lambda_end=0.5, n_steps=13, v_max=1e30)
    r0, P0, C0 = _flow(T, name, prec, stream, **kw)
    r1, P1, C1 = _flow(T, name, prec, stream, graph_steps=4, **kw)
    assert r0 == r1
    assert np.array_equal(P0, P1) and np.array_equal(C0, C1)


@pytest.mark.parametrize("G", [3, 16])
def test_divergence_inside_a_graph_is_replayed_step_by_step(T, G):
    print(f"graph divergence: G={G}", flush=True)
    kw = dict(lambda0=5.0, lambda_end=0.01, n_steps=30, v_max=20.0)
    r0, P0, C0 = _flow(T, "hubneg", "fp64", None, **kw)
    r1, P1, C1 = _flow(T, "hubneg", "fp64", None, graph_steps=G, **kw)
    assert r0["diverged"] == 1
    assert r0 == r1
    assert np.array_equal(P0, P1) and np.array_equal(C0, C1)


def test_max_steps_inside_graph_mode(T):
    kw = dict(lambda0=10.0, lambda_end=0.5, n_steps=13, v_max=1e30, max_steps=6)
    r0, P0, _ = _flow(T, "hub5", "fp64", None, **kw)
    r1, P1, _ = _flow(T, "hub5", "fp64", None, graph_steps=4, **kw)
    assert r0["n_steps"] == r1["n_steps"] == 6 and r0 == r1 and np.array_equal(P0, P1)


def _batch_ws():
    def inst(hop, mu, U, n_ff, Lq, n_ref, cutoff="temperature"):
        return dict(hop_R=hop[0], hop_t=hop[1], mu=mu, V0=onsite_V0(U), ff=ff_shell(n_ff), Lq=Lq, n_ref=n_ref,
                    cutoff=cutoff, n_o=2)
    return [
        inst(hubbard_hoppings(1.0, -0.25), -0.6, 3.0, 5, 6, 3),
        inst(rashba_hoppings(1.0, 0.3), -0.4, 2.5, 9, 5, 4, "omega"),
        inst(rashba_hoppings(1.0, 0.45), -0.2, 2.0, 13, 9, 2),
        # attractive: diverges inside a graph, the others continue
        inst(hubbard_hoppings(1.0, -0.25), -0.5, -4.0, 5, 6, 2),
    ]


@pytest.mark.parametrize("n_streams", [1, 3])
def test_batch_graph_steps_equal_lockstep_launches(T, n_streams):
    print(f"batch graph: streams={n_streams}", flush=True)
    ws = _batch_ws()
    outs = []
    for G in (0, 4):
        b = T.Batch(ws, precision="fp64", n_streams=n_streams)
        Ps, Cs = [], []
        for d in b.dims:
            Ps.append(torch.zeros((d["Nq"], d["B"], d["B"]), dtype=torch.complex128, device="cuda"))
            Cs.append(torch.zeros_like(Ps[-1]))
        res = T.tufrg_batch_flow(b, Ps, Cs, 5.0, 0.01, n_steps=30, v_max=20.0, graph_steps=G)
        torch.cuda.synchronize()
        outs.append((res, [p.cpu().numpy() for p in Ps], [c.cpu().numpy() for c in Cs]))
        b.close()
    (r0, P0, C0), (r1, P1, C1) = outs
    assert r0 == r1
    assert r0[3]["diverged"] == 1
    for a, b_ in zip(P0 + C0, P1 + C1):
        assert np.array_equal(a, b_)
