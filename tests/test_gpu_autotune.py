"""The launch-shape autotuner (tufrg_autotune) on the GPU: the shape it keeps
is the fastest it timed, the loops stay correct (two spin-orbitals: against
the FP64 oracle to the FP32 bar; BF16X3: bit for bit, the shape only regroups
the k sum), the JSON cache is written, read back by a second context and
refused when it is not a tuning cache."""

import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import tufrg as otu  # noqa: E402
from synth import ff_shell, kanamori_V0, onsite_V0, rashba_hoppings, t2g_soc_hoppings  # noqa: E402
from tests._layout import ph_loop_to_matrix, pp_loop_to_matrix  # noqa: E402


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_08830_amd import tufrg
    return tufrg


RAS = (rashba_hoppings(1.0, 0.3), -0.4, onsite_V0(2.5), ff_shell(9), 9, 8, "omega")
T2G = (t2g_soc_hoppings(0.2, seed=1), 0.35, kanamori_V0(2.0, 0.3), ff_shell(13), 9, 2, "temperature")


def _ctx(T, case, prec):
    hop, mu, V0, ff, Lq, n_ref, cut = case
    return T.Context(hop[0], hop[1], mu, V0, ff, Lq, n_ref, cut, prec)


def _bubble(T, ctx, ch, lam):
    L = torch.zeros((ctx.Nq, ctx.B, ctx.B), dtype=torch.complex128, device="cuda")
    T.tufrg_bubble(ctx, ch, lam, 1, L)
    torch.cuda.synchronize()
    return L.cpu().numpy()


def test_two_orbital_tuning_keeps_the_fastest_shape_and_oracle_parity(T, tmp_path):
    print("autotune: rashba S9 9x9 refined 8x fp32", flush=True)
    cache = tmp_path / "tune.json"
    ctx = _ctx(T, RAS, "fp32")
    r = T.tufrg_autotune(ctx, 0.3, str(cache))
    print(r)
    assert r["tunable"] == 1 and r["from_cache"] == 0 and r["n_candidates"] >= 2
    assert 0 < r["loop_ms"] <= r["default_ms"]
    hop, mu, V0, ff, Lq, n_ref, cut = RAS
    st = otu.TUSetup(hop[0], hop[1], mu, V0, ff, Lq, n_ref, cut)
    for ch, code, conv in (("pp", T.PP, pp_loop_to_matrix), ("ph", T.PH, ph_loop_to_matrix)):
        ref = conv(otu.loops(st, ch, 0.3))
        got = _bubble(T, ctx, code, 0.3)
        assert np.abs(got - ref).max() < 1e-5 * np.abs(ref).max()
    ctx.close()
    doc = json.loads(cache.read_text())
    assert doc["version"] == 1 and len(doc["entries"]) == 1
    (key, entry), = doc["entries"].items()
    assert "n_o=2" in key and "Lq=9" in key and entry["loop_kx_chunks"] == r["loop_kx_chunks"]
    # a second context of the same shape takes the cached shape without timing
    ctx2 = _ctx(T, RAS, "fp32")
    r2 = T.tufrg_autotune(ctx2, 0.3, str(cache))
    assert r2["from_cache"] == 1 and r2["n_candidates"] == 0 and r2["loop_kx_chunks"] == r["loop_kx_chunks"]
    assert r2["loop_ms"] == entry["loop_ms"]
    ctx2.close()


def test_bf16x3_tuning_changes_no_bit(T, tmp_path):
    print("autotune: t2g S13 9x9 refined 2x bf16x3", flush=True)
    ctx = _ctx(T, T2G, "bf16x3")
    before = [_bubble(T, ctx, ch, 0.35) for ch in (T.PP, T.PH)]
    r = T.tufrg_autotune(ctx, 0.35, str(tmp_path / "t.json"))
    print(r)
    assert r["tunable"] == 1 and r["mfma_kx_rows"] in (1, 2, 4) and r["n_candidates"] == 3
    after = [_bubble(T, ctx, ch, 0.35) for ch in (T.PP, T.PH)]
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    ctx.close()


def test_vector_six_orbital_loops_have_nothing_to_tune(T, tmp_path):
    ctx = _ctx(T, T2G, "fp32")
    r = T.tufrg_autotune(ctx, 0.35, str(tmp_path / "t.json"))
    assert r["tunable"] == 0 and r["n_candidates"] == 0
    assert not (tmp_path / "t.json").exists()
    ctx.close()


def test_a_file_that_is_not_a_tuning_cache_is_refused_and_kept(T, tmp_path):
    p = tmp_path / "notes.json"
    p.write_text('{"something": "else"}')
    ctx = _ctx(T, RAS, "fp32")
    with pytest.raises(T.TufrgError) as ei:
        T.tufrg_autotune(ctx, 0.3, str(p))
    assert ei.value.status == 1 and "not a tuning cache" in str(ei.value)
    assert p.read_text() == '{"something": "else"}'
    with pytest.raises(T.TufrgError):
        T.tufrg_autotune(ctx, -1.0)
    ctx.close()
