"""SU(2)-reduced flows of one orbital per site on the GPU against the oracle
(oracle/su2.py, itself pinned against the spinful equations): one-band loops,
the reduced right-hand side (dp, dc, dd) for S5 and S9 in both cutoff
schemes, Euler flows with and without divergence, the GPU's spinful
right-hand side of the embedded state, and the argument checks."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import su2  # noqa: E402
from oracle import tufrg as otu  # noqa: E402
from synth import ff_shell, hubbard_hoppings, onsite_V0  # noqa: E402
from tests._layout import c_to_matrix, p_to_matrix  # noqa: E402


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_08830_amd import tufrg
    return tufrg


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


def _one_band(n_ff, cutoff, U=3.0, Lq=6, n_ref=3, mu=-0.6):
    hop_R, hop_t = hubbard_hoppings(1.0, -0.25)
    v = np.full((1, 1, 1, 1), 0.5 * U, dtype=np.complex128)
    args = (hop_R, hop_t[:, :1, :1], mu, v, ff_shell(n_ff), Lq, n_ref, cutoff)
    return args, otu.TUSetup(*args)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _random(st, seed):
    rng = np.random.default_rng(seed)
    sh = (st.Nq, st.n_ff, st.n_ff)
    return [0.2 * (rng.normal(size=sh) + 1j * rng.normal(size=sh)) for _ in range(3)]


@pytest.mark.parametrize("n_ff", [5, 9])
@pytest.mark.parametrize("cutoff", ["temperature", "omega"])
def test_one_band_loops_match_oracle(T, n_ff, cutoff):
    args, st = _one_band(n_ff, cutoff, Lq=7, n_ref=4)
    ctx = T.Context(*args, "fp64")
    for ch, code in (("pp", T.PP), ("ph", T.PH)):
        L = torch.zeros((ctx.Nq, ctx.B, ctx.B), dtype=torch.complex128, device="cuda")
        T.tufrg_bubble(ctx, code, 0.35, 1, L)
        torch.cuda.synchronize()
        ref = otu.loops(st, ch, 0.35)[..., 0, 0, 0, 0]
        assert rel(L.cpu().numpy(), ref) < 1e-11, ch
    ctx.close()


@pytest.mark.parametrize("n_ff", [5, 9])
@pytest.mark.parametrize("cutoff", ["temperature", "omega"])
def test_reduced_rhs_matches_oracle(T, n_ff, cutoff):
    print(f"su2 rhs: S{n_ff} {cutoff}", flush=True)
    args, st = _one_band(n_ff, cutoff)
    ctx = T.Context(*args, "fp64")
    p, c, d = _random(st, 5)
    out = [torch.zeros((ctx.Nq, ctx.B, ctx.B), dtype=torch.complex128, device="cuda") for _ in range(3)]
    T.tufrg_su2_rhs(ctx, 0.4, _dev(p), _dev(c), _dev(d), *out)
    torch.cuda.synchronize()
    ref = su2.rhs(st, 0.4, p, c, d)
    for got, r, name in zip(out, ref, ("dp", "dc", "dd")):
        e = rel(got.cpu().numpy(), r)
        print(f"  {name}: rel err {e:.2e}")
        assert e < 1e-11, name
    ctx.close()


def test_reduced_rhs_is_the_spinful_gpu_rhs_of_the_embedded_state(T):
    """The spinful GPU path (two spin-orbitals) on the embedded state gives the
    embedding of the reduced GPU result, in both spin structures."""
    args, st1 = _one_band(9, "temperature")
    hop_R, hop_t = hubbard_hoppings(1.0, -0.25)
    stS = otu.TUSetup(hop_R, hop_t, -0.6, onsite_V0(3.0), ff_shell(9), 6, 3, "temperature")
    ctx1 = T.Context(*args, "fp64")
    ctxS = T.Context(hop_R, hop_t, -0.6, onsite_V0(3.0), ff_shell(9), 6, 3, "temperature", "fp64")
    p, c, d = _random(st1, 9)
    red = [torch.zeros((ctx1.Nq, ctx1.B, ctx1.B), dtype=torch.complex128, device="cuda") for _ in range(3)]
    T.tufrg_su2_rhs(ctx1, 0.4, _dev(p), _dev(c), _dev(d), *red)
    Pd, Cd = _dev(p_to_matrix(su2.embed_p(stS, p))), _dev(c_to_matrix(su2.embed_c(c, d)))
    dP, dC = torch.zeros_like(Pd), torch.zeros_like(Cd)
    T.tufrg_rhs(ctxS, 0.4, Pd, Cd, dP, dC)
    torch.cuda.synchronize()
    dp, dc, dd = (x.cpu().numpy() for x in red)
    eP = rel(dP.cpu().numpy(), p_to_matrix(su2.embed_p(stS, dp)))
    eC = rel(dC.cpu().numpy(), c_to_matrix(su2.embed_c(dc, dd)))
    print(f"su2 vs spinful gpu: rel err P {eP:.2e} C {eC:.2e}")
    assert eP < 1e-11 and eC < 1e-11
    ctx1.close()
    ctxS.close()


def _oracle_flow_with_stop(st, lam0, lam_end, n, v_max):
    """The oracle's reduced Euler steps with the spinful stop test
    (max |p|, |c|, |d| above v_max; Lambda_c interpolated in ln Lambda)."""
    grid = otu.log_grid(lam0, lam_end, n)
    p = np.zeros((st.Nq, st.n_ff, st.n_ff), dtype=np.complex128)
    c, d = p.copy(), p.copy()
    m_prev, res = 0.0, dict(diverged=0, n_steps=0, lambda_c=0.0)
    for i in range(n):
        dp, dc, dd = su2.rhs(st, grid[i], p, c, d)
        h = grid[i + 1] - grid[i]
        p, c, d = p + h * dp, c + h * dc, d + h * dd
        m = max(np.abs(p).max(), np.abs(c).max(), np.abs(d).max())
        res["n_steps"], res["max_coupling"] = i + 1, m
        if m > v_max:
            t = (v_max - m_prev) / (m - m_prev)
            res["diverged"] = 1
            res["lambda_c"] = float(np.exp(np.log(grid[i]) + t * (np.log(grid[i + 1]) - np.log(grid[i]))))
            break
        m_prev = m
    return p, c, d, res


@pytest.mark.parametrize("U,v_max,n", [(3.0, 1e30, 12), (-4.0, 20.0, 30)])
def test_reduced_euler_flow_matches_oracle(T, U, v_max, n):
    """Repulsive U: twelve steps 5 -> 0.05 without divergence; attractive U:
    the pairing instability, same stopping step and critical scale."""
    print(f"su2 flow: U={U}", flush=True)
    args, st = _one_band(5, "temperature", U=U)
    ctx = T.Context(*args, "fp64")
    pr, cr, dr, rr = _oracle_flow_with_stop(st, 5.0, 0.01 if U < 0 else 0.05, n, v_max)
    state = [torch.zeros((ctx.Nq, ctx.B, ctx.B), dtype=torch.complex128, device="cuda") for _ in range(3)]
    res = T.tufrg_su2_flow(ctx, *state, 5.0, 0.01 if U < 0 else 0.05, n, v_max=v_max)
    torch.cuda.synchronize()
    print(res, rr)
    assert res["n_steps"] == rr["n_steps"] and res["diverged"] == rr["diverged"]
    assert res["max_coupling"] == pytest.approx(rr["max_coupling"], rel=1e-10)
    if rr["diverged"]:
        assert res["lambda_c"] == pytest.approx(rr["lambda_c"], rel=1e-10)
    for got, r in zip(state, (pr, cr, dr)):
        assert rel(got.cpu().numpy(), r) < 1e-10
    ctx.close()


def test_calls_of_the_other_path_are_refused(T):
    args, st = _one_band(5, "temperature")
    ctx1 = T.Context(*args, "fp64")
    X = torch.zeros((ctx1.Nq, ctx1.B, ctx1.B), dtype=torch.complex128, device="cuda")
    with pytest.raises(T.TufrgError) as ei:
        T.tufrg_rhs(ctx1, 0.4, X, X, X.clone(), X.clone())
    assert ei.value.status == 6
    with pytest.raises(T.TufrgError) as ei:
        T.tufrg_project(ctx1, X, X, X.clone(), X.clone())
    assert ei.value.status == 6
    with pytest.raises(T.TufrgError):
        T.tufrg_su2_rhs(ctx1, -1.0, X, X, X, X.clone(), X.clone(), X.clone())
    ctx1.close()
    hop_R, hop_t = hubbard_hoppings(1.0, -0.25)
    ctxS = T.Context(hop_R, hop_t, -0.6, onsite_V0(3.0), ff_shell(5), 6, 3, "temperature", "fp64")
    Y = torch.zeros((ctxS.Nq, ctxS.B, ctxS.B), dtype=torch.complex128, device="cuda")
    with pytest.raises(T.TufrgError) as ei:
        T.tufrg_su2_rhs(ctxS, 0.4, Y, Y, Y, Y.clone(), Y.clone(), Y.clone())
    assert ei.value.status == 6
    ctxS.close()
