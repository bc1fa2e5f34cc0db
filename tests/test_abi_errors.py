"""Argument validation of the C ABI (CPU: every case is rejected on the host
before any device call, so no GPU is needed)."""

import numpy as np
import pytest

from synth import ff_shell, hubbard_hoppings, onsite_V0, t2g_soc_hoppings


@pytest.fixture(scope="module")
def T():
    from paper_1710_08830_amd import tufrg
    return tufrg


def _args(**over):
    hop = hubbard_hoppings(1.0, -0.25)
    kw = dict(hop_R=hop[0], hop_t=hop[1], mu=-0.5, V0=onsite_V0(2.0), ff=ff_shell(9), Lq=8, n_ref=4,
              cutoff="temperature", precision="fp64")
    kw.update(over)
    return kw


@pytest.mark.parametrize("over,status,text", [
    (dict(ff=np.array([[1, 0], [0, 0], [-1, 0]])), 1, "(0,0)"),
    (dict(ff=np.array([[0, 0], [1, 0]])), 1, "closed"),
    (dict(ff=np.array([[0, 0], [3, 0], [-3, 0]])), 1, "|R| <= 2"),
    (dict(ff=np.array([[0, 0], [1, 0], [-1, 0], [1, 0]])), 1, "duplicate"),
    (dict(ff=ff_shell(13), Lq=8), 1, "aliasing"),
    (dict(Lq=0), 1, "mesh"),
    (dict(n_ref=0), 1, "mesh"),
    (dict(Lq=64, n_ref=65), 1, "mesh"),
    (dict(cutoff=7), 1, "cutoff"),
    (dict(precision=9), 1, "precision"),
])
def test_create_rejects_bad_setups(T, over, status, text):
    with pytest.raises(T.TufrgError) as ei:
        T.Context(**_args(**over))
    assert ei.value.status == status
    assert text in str(ei.value)


@pytest.mark.parametrize("temperature", [None, 0.0, -0.1, float("inf"), float("nan")])
def test_shell_cutoff_needs_a_temperature(T, temperature):
    with pytest.raises(T.TufrgError) as ei:
        T.Context(**_args(cutoff="shell", temperature=temperature))
    assert ei.value.status == 1
    assert "temperature" in str(ei.value)


def test_bf16x3_needs_six_orbitals(T):
    with pytest.raises(T.TufrgError) as ei:
        T.Context(**_args(precision="bf16x3"))
    assert ei.value.status == 6


def test_create_rejects_unsupported_orbital_count(T):
    hop_R = np.array([[1, 0], [-1, 0]])
    hop_t = np.zeros((2, 3, 3), dtype=np.complex128)
    with pytest.raises(T.TufrgError) as ei:
        T.Context(**_args(hop_R=hop_R, hop_t=hop_t, V0=np.zeros((3,) * 4)))
    assert ei.value.status == 6  # TUFRG_E_UNSUPPORTED


def test_six_orbital_model_passes_validation_up_to_the_device(T):
    """A valid six-orbital setup gets past every host check; without a GPU the
    first device allocation fails (status E_NOMEM or E_HIP), never E_INVAL."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: creation would succeed")
    hop = t2g_soc_hoppings(0.2, seed=1)
    from synth import kanamori_V0
    with pytest.raises(T.TufrgError) as ei:
        T.Context(**_args(hop_R=hop[0], hop_t=hop[1], V0=kanamori_V0(2.0, 0.3), ff=ff_shell(13), Lq=9))
    assert ei.value.status in (2, 3)


@pytest.mark.parametrize("ff", [
    [[0, 0], [2, 2], [-2, -2], [2, -2], [-2, 2]],   # S - S holds (4, 4)
    [[0, 0], [2, 1], [-2, -1], [1, 2], [-1, -2]],   # (4, 2) and (3, 3)
    [[0, 0], [1, 2], [-1, -2], [2, -1], [-2, 1]],   # (2, 4) and (4, -2)
])
def test_six_orbital_sets_beyond_the_kernel_shape_are_rejected(T, ff):
    """The six-orbital loop kernels cover differences R1 - R2 in the 5 x 5 box
    or the diamond |dx| + |dy| <= 4; a set whose S - S leaves that shape is
    rejected on the host (no partial slot is left unwritten)."""
    hop = t2g_soc_hoppings(0.2, seed=1)
    from synth import kanamori_V0
    with pytest.raises(T.TufrgError) as ei:
        T.Context(**_args(hop_R=hop[0], hop_t=hop[1], V0=kanamori_V0(2.0, 0.3), ff=np.array(ff), Lq=9))
    assert ei.value.status == 6
    assert "outside" in str(ei.value)


@pytest.mark.parametrize("sizes", [[5], [0, 4], [4, 70000]])
def test_mlp_rejects_bad_sizes(T, sizes):
    with pytest.raises(T.TufrgError) as ei:
        T.Mlp(sizes)
    assert ei.value.status == 1


def test_batch_rejects_bad_stream_count(T):
    hop = hubbard_hoppings(1.0, 0.0)
    w = dict(hop_R=hop[0], hop_t=hop[1], mu=0.0, V0=onsite_V0(1.0), ff=ff_shell(5), Lq=6, n_ref=2,
             cutoff="temperature")
    with pytest.raises(T.TufrgError) as ei:
        T.Batch([w], n_streams=0)
    assert ei.value.status == 1


def test_basis_calls_reject_a_null_context(T):
    """The basis-change entry points check the context before any device call."""
    lib = T._lib
    assert lib.tufrg_basis_matrix(None, 0, None, None) == 1
    assert lib.tufrg_basis_apply(None, None, None, None, 0) == 1


def test_create_rejects_an_unknown_basis(T):
    with pytest.raises(T.TufrgError) as ei:
        T.Context(**_args(basis=7))
    assert ei.value.status == 1
    assert "basis" in str(ei.value)


def test_set_initial_p_rejects_a_null_context(T):
    assert T._lib.tufrg_set_initial_p(None, None) == 1


def test_pair_bands_rejects_a_null_context(T):
    import ctypes
    act = ctypes.c_int32(7)
    assert T._lib.tufrg_pair_bands(None, 1, ctypes.byref(act)) == 1
    assert act.value == 7  # untouched


def _fake_ctx():
    """Sizes of a small context without one (no device is needed: the binding
    checks dtype and size before it calls the library)."""
    from types import SimpleNamespace
    return SimpleNamespace(handle=None, Nq=4, B=8, Nf=16, n_dR=5, n_o=2, n_ff=2)


def test_binding_checks_dtype_and_size_before_the_library(T):
    import torch
    ctx = _fake_ctx()
    good = torch.zeros((ctx.Nq, ctx.B, ctx.B), dtype=torch.complex128)
    with pytest.raises(TypeError):
        T.tufrg_rhs(ctx, 0.5, good.to(torch.complex64), good, good, good)
    with pytest.raises(ValueError):
        T.tufrg_rhs(ctx, 0.5, good, good[:-1], good, good)
    with pytest.raises(ValueError):
        T.tufrg_loops_compact(ctx, 0.5, 1, torch.zeros(2 * ctx.Nq * ctx.n_dR * 16 - 1, dtype=torch.complex128))
    with pytest.raises(TypeError):
        T.tufrg_band_data(ctx, torch.zeros(ctx.n_o * ctx.Nf, dtype=torch.float32),
                          torch.zeros(ctx.n_o ** 3 * ctx.Nf, dtype=torch.complex128))
    with pytest.raises(ValueError):
        T.tufrg_sur_features(ctx, 3, 0.5, torch.zeros((3, 11 + ctx.n_dR), dtype=torch.float32),
                             torch.zeros(2, dtype=torch.int32), torch.zeros(3, dtype=torch.int32),
                             torch.zeros(3, dtype=torch.int32))
    with pytest.raises(ValueError):
        T.tufrg_ff_apply(ctx, np.eye(3), good, good)
    # correctly typed and sized: the call reaches the library, which refuses the null context
    with pytest.raises(T.TufrgError) as ei:
        T.tufrg_rhs(ctx, 0.5, good, good, good, good)
    assert ei.value.status == 1


def test_context_checks_the_model_arrays_before_the_library(T):
    hop_R, hop_t = hubbard_hoppings(1.0, -0.25)
    with pytest.raises(ValueError):
        T.Context(**_args(hop_t=hop_t[:-1]))
    with pytest.raises(ValueError):
        T.Context(**_args(V0=onsite_V0(2.0)[:1]))


@pytest.mark.parametrize("over,text", [
    (dict(precision="fp32"), "FP64"),
    (dict(cutoff="shell", temperature=0.05), "FP64"),
])
def test_one_orbital_contexts_are_fp64_plain_cutoffs(T, over, text):
    """The SU(2)-reduced path (one orbital per site) runs FP64 with the
    temperature or Omega cutoff; anything else is refused at creation."""
    hop = hubbard_hoppings(1.0, -0.25)
    kw = _args(hop_t=hop[1][:, :1, :1], V0=np.full((1, 1, 1, 1), 1.5, dtype=np.complex128))
    kw.update(over)
    with pytest.raises(T.TufrgError) as ei:
        T.Context(**kw)
    assert ei.value.status == 6 and text in str(ei.value)
