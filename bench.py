"""Benchmark of the TU-fRG right-hand side on one MI355X.

Default workload (the largest single-GPU configuration): three-orbital t2g
model with atomic spin-orbit coupling (six spin-orbitals, hoppings from seed
1, Kanamori U = 2, J = 0.3, four electrons per site), 13 form factors (bundle
dimension 468), 48 x 48 q-mesh refined 16x per cell (768^2 fine k-points),
temperature cutoff from 10 on the 200-step log grid; loops in BF16 split
products on the matrix cores (FP32 accumulation), projections and bundle
products FP32/FP64, state FP64.

One step = one explicit Euler step of the flow through the C ABI: regulator
values, both loop channels, the real-space transform, gathers and assembly of
the projected vertices, both bundle products, the FP64 state update and the
max-coupling readback (tufrg_flow with n_steps = K).  Inputs are resident in
HBM before the timed region.

Printed: one JSON line with the headline value (loop entries/s over the whole
step, 2 Nq B^2 per step) and compact loop entries/s, flow steps/s, the
roofline of the loop kernel (survey's algorithmic flop count, event-timed
inside the library over the timed region), the FP64-plain form over the first
steps with its relative error and the speed-up of the mixed form, the
surrogate-assisted form over the timed window, the two-orbital Rashba line
(24 x 24 refined 24x, FP32) as an extra key, and a CPU baseline of the FP64
oracle (one thread and all cores) on a bounded sample.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "loop entries/s + flow steps/s, mixed/surrogate vs FP64-plain at ≤1e-4 rel err"
WORKLOAD = "t2g_s13_L48"
PEAK_FP32_VECTOR = 157.3e12
PEAK_BF16_MFMA = 2.5e15
PEAK_FP64_VECTOR = 78.6e12


def loop_flops_per_pair(n_o, ndx, ndy, shell=False):
    """Algorithmic FP32 flops of the loop kernel per (q, k, channel).  Two
    spin-orbitals: 12 for the four divided differences, 16 for W_1 and D, 32
    for the 10 distinct block entries, 16 for the dx = 0 sums and 64 per
    further dx.  n_o > 2 (one entry of each Hermitian pair, U = (n_o^4 + n_o^2)
    / 2 of them): 8 n_o flops for sum_m Pi_m W_m, 2 + 8 ndy for the separable
    ky transform, plus 2 n_o^4 for W_m and 3 n_o^2 for the loop kernels.  The
    momentum-shell cutoff adds 4 flops per band pair for its shell factor."""
    extra = 4 * n_o * n_o if shell else 0
    if n_o == 2:
        return 12 + 16 + 32 + 16 + 64 * (ndx - 1) + extra
    u = (n_o ** 4 + n_o ** 2) // 2
    return u * (8 * n_o + 2 + 8 * ndy) + 2 * n_o ** 4 + 3 * n_o ** 2 + extra


def mfma_flops_per_pair(ndy, n_o=6, n_b=None):
    """Matrix-core flops the BF16X3 loop executes per (q, k, channel): one k
    adds K = n_b (bands summed: n_o, or 3 for Kramers pairs) to the product of
    the (2 ndy + 1) n_o^2 phase rows (phase times real-basis projector
    coordinate, padded to whole 16-row tiles) with the n_o^2 real-basis
    columns of its q, as three BF16 products (hi*hi, hi*lo, lo*hi)."""
    n_b = n_o if n_b is None else n_b
    rows = -(-(2 * ndy + 1) * n_o * n_o // 16) * 16
    return 3 * 2 * rows * (n_o * n_o) * n_b


def credited_loop_flops_per_pair(n_o, ndy, n_b=None):
    """Algorithmic flops of one loop entry set per (q, k, channel) in the
    survey's count: the form-factor contraction 8 n_dRy n_o^4 with the
    separable transform (n_dRy = 2 ndy + 1 phases of the ky sum), halved for
    the hermiticity the kernels exploit, plus the block build
    8 n_o^2 n_b (n_b + n_o^2)."""
    n_b = n_o if n_b is None else n_b
    return 8 * (2 * ndy + 1) * n_o ** 4 // 2 + 8 * n_o ** 2 * n_b * (n_b + n_o ** 2)


def _box(ff):
    m = max(max(abs(x), abs(y)) for x, y in ff)
    return (3, 2) if m <= 1 else (5, 4)


# sources of the loop kernel per precision, and the host function that sets
# its launch shape (chunking) in tufrg_host.hip
# the loop kernel of a workload: BF16X3 (six spin-orbitals, matrix cores),
# two spin-orbitals, or six on the vector units
LOOP_SOURCES = {"bf16x3": (("k_loop_rb.hip", "common.h"), ("loops_range_mfma", "ensure_apre")),
                "no2": (("k_loop.hip", "common.h"), ("loops_range",)),
                "gen": (("k_loop_gen.hip", "common.h"), ("loops_range",))}


def _loop_kind(workload, prec):
    return "bf16x3" if prec == "bf16x3" else ("gen" if workload.startswith("t2g") else "no2")


def _code_only(text):
    """Source text without comments and with whitespace runs collapsed: what
    the compiler sees, so that a comment edit keeps a profile's hash."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return re.sub(r"\s+", " ", text).strip()


def _host_function_text(name):
    """Text of one top-level function of tufrg_host.hip (signature to the
    closing brace in column 0)."""
    with open(os.path.join(ROOT, "paper_1710_08830_amd", "csrc", "tufrg_host.hip")) as fh:
        src = fh.read()
    i = src.find("static tufrg_status " + name + "(")
    if i < 0:
        raise RuntimeError(f"no function {name} in tufrg_host.hip")
    j = src.find("\n}\n", i)
    return src[i:j + 3]


def _loop_source_hash(workload, prec):
    """Hash of the loop kernel's sources and of the host functions that shape
    its launches, comments and layout aside."""
    files, fns = LOOP_SOURCES[_loop_kind(workload, prec)]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1710_08830_amd", "csrc", f)) as fh:
            h.update(_code_only(fh.read()).encode())
    for fn in fns:
        h.update(_code_only(_host_function_text(fn)).encode())
    return h.hexdigest()


def _traffic(workload, prec):
    """HBM bytes per loop-kernel launch from committed rocprofv3 counters, or
    None when the kernel source changed since they were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", f"loop_kernel_traffic_{workload}_{prec}.json")) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != _loop_source_hash(workload, prec):
        return None
    return float(t["hbm_bytes_per_launch"])


def _cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return model, n


def _oracle_rhs_time_per_q(w, n_sample, n_ref_sample):
    """FP64 oracle time of the right-hand side per coarse q, from a bounded
    sample: the loops (both channels) and bundle products at n_sample q on the
    workload's q-mesh with the fine mesh reduced to n_ref_sample per cell
    (the loop cost per q is linear in the number of fine k, so it is scaled
    by Nf / Nf_sample), and the projections of the whole state charged per q
    from a run on the smallest alias-free q-mesh (their cost per q does not
    depend on Nq)."""
    import numpy as np

    from oracle import tufrg as otu

    st = otu.TUSetup.from_workload(w, n_ref=n_ref_sample)
    Nf_full = (w["Lq"] * w["n_ref"]) ** 2
    rng = np.random.default_rng(0)
    qs = sorted(rng.choice(st.Nq, size=n_sample, replace=False).tolist())
    lam = 1.0
    # projections: per-q cost on the smallest q-mesh the form factors allow
    rmax = max(max(abs(int(x)), abs(int(y))) for x, y in w["ff"])
    stp = otu.TUSetup.from_workload(w, Lq=4 * rmax + 1, n_ref=1)
    Pp = np.zeros((stp.Nq, stp.n_ff, stp.n_ff) + (stp.n_o,) * 4, dtype=np.complex128)
    t0 = time.perf_counter()
    VPp, VCp = otu.projected_vertices(stp, Pp, Pp)
    t_proj_q = (time.perf_counter() - t0) / stp.Nq
    t0 = time.perf_counter()
    Lpp = otu.loops(st, "pp", lam, q_list=qs)
    Lph = otu.loops(st, "ph", lam, q_list=qs)
    t_loops = time.perf_counter() - t0
    t0 = time.perf_counter()
    otu.bundle_pp(VPp[:1].repeat(n_sample, axis=0), Lpp)
    otu.bundle_ph(VCp[:1].repeat(n_sample, axis=0), Lph)
    t_bundle = time.perf_counter() - t0
    t_q = t_loops * Nf_full / st.Nf / n_sample + t_bundle / n_sample + t_proj_q
    spent = t_loops + t_bundle + t_proj_q * stp.Nq
    return t_q, qs, spent


def cpu_baseline(w, n_sample=1, n_ref_sample=None):
    """The FP64 oracle on the machine's host cores, one thread and all cores, on a
    bounded sample (see _oracle_rhs_time_per_q), in the headline's unit: loop
    entries (2 B^2 per q and right-hand side) per second."""
    from threadpoolctl import threadpool_limits

    model, ncores = _cpu_info()
    B = len(w["ff"]) * w["n_o"] ** 2
    if n_ref_sample is None:
        n_ref_sample = w["n_ref"] if w["n_o"] == 2 else 2
    out = {}
    for label, lim in (("one_thread", 1), ("all_cores", ncores)):
        with threadpool_limits(limits=lim):
            t_q, qs, spent = _oracle_rhs_time_per_q(w, n_sample, n_ref_sample)
        out[label] = {"value": 2.0 * B * B / t_q, "threads": lim, "cpu_seconds_spent": spent}
    best = max(out.values(), key=lambda d: d["value"])
    return {"value": best["value"], "unit": "loop entries/s", "cores": best["threads"], "kind": "oracle",
            "cpu_model": model, "nproc": ncores,
            "one_thread": out["one_thread"], "all_cores": out["all_cores"],
            "sample": (f"right-hand side per coarse q of {w['name']}: loops and bundle products at "
                       f"{n_sample} of {w['Lq'] ** 2} q with the fine mesh reduced to {n_ref_sample}x per cell "
                       f"and scaled by the number of fine k (extrapolated), projections charged per q from the "
                       f"smallest alias-free q-mesh; NumPy oracle, BLAS threads set by threadpoolctl (only "
                       f"its matrix products use more than one core)")}


def surrogate_leg(T, torch, ctx, P, C, P64, C64, dp, w, K, t_plain_step, n_lam=24, n_rows=200000,
                  epochs=(40, 40, 40)):
    """Loop surrogate: train the network on plain loops at n_lam scales spread
    over the flow range (random blocks, at most n_rows rows), then run the
    timed Euler steps and the production Dormand-Prince flow with the surrogate
    (5 % of the q_x rows recomputed plainly per right-hand side, fallback above
    the sampled-error tolerance or coupling 20), each compared with its
    FP64-plain counterpart."""
    import numpy as np

    from synth import mlp_init, mlp_shape

    dev = torch.device("cuda:0")
    no4 = ctx.n_o ** 4
    nb = 2 * ctx.Nq * ctx.n_dR
    per = min(nb, n_rows // n_lam)
    lams = np.exp(np.linspace(np.log(w["lam0"]), np.log(w["lam_end"]), n_lam))
    sizes = mlp_shape(11 + ctx.n_dR, 256, 2 * no4)
    rng = np.random.default_rng(3)
    t0 = time.perf_counter()
    X = torch.zeros((n_lam * per, sizes[0]), dtype=torch.float32, device=dev)
    Y = torch.zeros((n_lam * per, sizes[-1]), dtype=torch.float32, device=dev)
    Lc = torch.zeros((2, ctx.Nq, ctx.n_dR, no4), dtype=torch.complex128, device=dev)
    Yall = torch.zeros((nb, sizes[-1]), dtype=torch.float32, device=dev)
    scales = []
    for i, lam in enumerate(lams):
        b = rng.choice(nb, size=per, replace=False)
        q, ch, iD = ((b // ctx.n_dR) % ctx.Nq, b // (ctx.n_dR * ctx.Nq), b % ctx.n_dR)
        q, ch, iD = (torch.from_numpy(a.astype(np.int32)).to(dev) for a in (q, ch, iD))
        T.tufrg_loops_compact(ctx, lam, 1, Lc)
        # scale of this Lambda: the largest |Lc| over all blocks
        scales.append(T.tufrg_sur_targets(ctx, nb, 1.0, Lc, Yall))
        T.tufrg_sur_features(ctx, per, lam, X[i * per:(i + 1) * per], q, ch, iD)
        T.tufrg_sur_targets(ctx, per, scales[-1], Lc, Y[i * per:(i + 1) * per], q, ch, iD)
    del Yall
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    print(f"surrogate bench: {n_lam * per} training rows in {t_data:.1f} s", file=sys.stderr, flush=True)
    net = T.Mlp(sizes, mlp_init(sizes, seed=3))
    t0 = time.perf_counter()
    loss = None
    for ep, lr in zip(epochs, (1e-3, 3e-4, 1e-4)):
        loss = T.tufrg_mlp_train(net, X, Y, batch=2048, epochs=ep, lr=lr, seed=3)
        print(f"surrogate bench: {ep} epochs at lr {lr:g}, loss {loss:.3e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    T.tufrg_sur_attach(ctx, net, lams, scales)
    res = dict(train_rows=int(n_lam * per), train_scales=int(n_lam), train_data_seconds=t_data,
               train_seconds=t_train, final_train_loss=loss, net=sizes)

    def rel_to(Pr, Cr):
        return max((P - Pr).abs().max().item() / Pr.abs().max().item(),
                   (C - Cr).abs().max().item() / Cr.abs().max().item())

    # (1) the headline step: Euler steps 10 -> 1 of the timed window, against
    # the FP64-plain Euler flow over the same grid
    ctx64 = T.Context.from_workload(w, precision="fp64")
    Pe, Ce = torch.zeros_like(P), torch.zeros_like(C)
    T.tufrg_flow(ctx64, Pe, Ce, w["lam0"], 1.0, n_steps=K, v_max=1e30)
    ctx64.close()
    for key, tol in (("euler_tol_1e-3", 1e-3), ("euler_tol_5e-2", 5e-2)):
        P.zero_()
        C.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = T.tufrg_flow(ctx, P, C, w["lam0"], 1.0, n_steps=K, v_max=1e30, surrogate=True, sample_frac=0.05,
                         sur_tol=tol, plain_above=20.0, sample_seed=3)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[key] = dict(r, seconds=dt, ms_per_step=dt / K * 1e3, rel_err_vs_fp64_plain=rel_to(Pe, Ce),
                        speedup_vs_fp32_plain_step=t_plain_step / (dt / K))
    # (2) the production Dormand-Prince flow 10 -> 1e-4 at the stated tolerance
    P.zero_()
    C.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = T.tufrg_flow(ctx, P, C, w["lam0"], w["lam_end"], n_steps=0, rtol=w["rtol"], atol=w["atol"],
                     v_max=w["v_max"], max_steps=400, surrogate=True, sample_frac=0.05, sur_tol=1e-3,
                     plain_above=20.0, sample_seed=3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    e = dict(r, seconds=dt, flow_steps_per_s=r["n_steps"] / dt, rhs_per_s=r["n_rhs"] / dt,
             speedup_vs_fp32_plain=dp["fp32"]["seconds"] / dt, speedup_vs_fp64_plain=dp["fp64"]["seconds"] / dt)
    if r["n_steps"] == dp["fp64"]["n_steps"]:
        e["rel_err_vs_fp64_plain"] = rel_to(P64, C64)
    res["dp54_tol_1e-3"] = e
    T.tufrg_sur_attach(ctx, None)
    net.close()
    return res


def basis_flops(Nq, n_o, Nf, box):
    """Algorithmic FP64 flops of one basis matrix (one channel) with separable
    phases: per coarse q, entry (a, b, c, d) and fine k one complex product
    U_ac(k) U_bd(k') (6 flops) and one complex multiply-add with e^{-i ky dy}
    per dy in [-box, box] (8 flops each); the kx phases per row are negligible."""
    return float(Nq) * n_o ** 4 * Nf * (6 + 8 * (2 * box + 1))


def basis_leg(T, torch, ctx, P, C, ff, reps=3, band_ctx=None, V0=None, steps=20):
    """Orbital -> band basis change on the FP64 context: the pp and ph basis
    matrices from seeded random unitaries, then Pb = M^H P M and Cb = M^H C M."""
    import numpy as np

    from synth import random_unitaries
    dev = P.device
    box = 2 if 2 * max(max(abs(x), abs(y)) for x, y in ff) <= 2 else 4  # D = S - S inside [-box, box]^2
    U = torch.from_numpy(random_unitaries(ctx.Nf, ctx.n_o, seed=17)).to(dev)
    Mp, Mc = torch.empty_like(P), torch.empty_like(P)
    Y = torch.empty_like(P)

    def run():
        T.tufrg_basis_matrix(ctx, T.PP, U, Mp)
        T.tufrg_basis_matrix(ctx, T.PH, U, Mc)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        T.tufrg_basis_apply(ctx, Mp, P, Y)
        T.tufrg_basis_apply(ctx, Mc, C, Y)
        torch.cuda.synchronize()
        return time.perf_counter() - t1

    run()  # first call allocates the workspaces
    tm = ta = 0.0
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ta += run()
        tm += time.perf_counter() - t0
    tm -= ta
    per_matrix = tm / (2 * reps)
    fl = basis_flops(ctx.Nq, ctx.n_o, ctx.Nf, box)
    out = {"matrix_ms_per_channel": per_matrix * 1e3, "apply_ms_per_channel": ta / (2 * reps) * 1e3,
           "matrix_flops_per_channel": fl, "achieved_tflops": fl / per_matrix / 1e12,
           "peak_tflops": PEAK_FP64_VECTOR / 1e12, "frac": fl / per_matrix / PEAK_FP64_VECTOR,
           "note": "matrix time includes its expansion to B x B; host-timed with device syncs"}
    # change to the symmetrised form factors and back (both channels' layouts alike)
    W, _ = T.tufrg_ff_symmetrize(np.asarray(ff))
    T.tufrg_ff_apply(ctx, W, P, Y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        T.tufrg_ff_apply(ctx, W, P, Y)
    torch.cuda.synchronize()
    out["ff_symmetrise_ms"] = (time.perf_counter() - t0) / reps * 1e3
    if band_ctx is not None:
        # band-basis Euler steps: the onsite interaction U^H P[V0] U as the static P term
        n_o, nff = ctx.n_o, ctx.n_ff
        P0 = torch.zeros_like(P)
        P0.view(ctx.Nq, nff, n_o, n_o, nff, n_o, n_o)[:, 0, :, :, 0] = torch.from_numpy(
            np.ascontiguousarray(V0.transpose(0, 1, 3, 2))).to(dev)
        T.tufrg_basis_apply(ctx, Mp, P0, Y)
        T.tufrg_set_initial_p(band_ctx, Y)
        Pb, Cb = torch.zeros_like(P), torch.zeros_like(P)
        T.tufrg_flow(band_ctx, Pb, Cb, 10.0, 1.0, n_steps=3, v_max=1e30)
        Pb.zero_()
        Cb.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T.tufrg_flow(band_ctx, Pb, Cb, 10.0, 1.0, n_steps=steps, v_max=1e30)
        torch.cuda.synchronize()
        out["band_flow_ms_per_step"] = (time.perf_counter() - t0) / steps * 1e3
    return out


def _tune(T, ctx, lam, on):
    """Launch-shape autotuning before the timed steps (--tune): the result, and
    whether the shape left the default the committed counters were taken at."""
    if not on:
        return None, False
    r = T.tufrg_autotune(ctx, lam, os.environ.get("TUFRG_TUNE_CACHE"))
    # the default shape is timed first and only a strictly faster one replaces it
    return r, bool(r["tunable"]) and r["loop_ms"] < r["default_ms"]


def six_orbital_line(T, torch, w, prec, K, W, fp64_steps=2, surrogate=True, n_rows=120000, six_bands=False,
                     epochs=(10, 10, 10), tune=False):
    """Headline of a six-orbital workload: K timed Euler steps (after W warmup
    steps) of the 200-step grid from Lambda0 in the mixed arithmetic, the
    loop-kernel roofline, the FP64-plain form over the first fp64_steps steps
    (matched against the mixed form over the same steps), and the
    surrogate-assisted form over the timed window."""
    import numpy as np

    dev = torch.device("cuda:0")
    lam0, n = w["lam0"], w["n_steps"]
    lam_at = lambda i: lam0 * (w["lam_end"] / lam0) ** (i / n)  # noqa: E731
    ctx = T.Context.from_workload(w, precision=prec)
    B, Nq, Nf, nD = ctx.B, ctx.Nq, ctx.Nf, ctx.n_dR
    # Kramers-paired bands (the default wherever found): the loops sum three
    # bands, and the credited work counts three
    paired = w["n_o"] == 6 and T.tufrg_pair_bands(ctx, not six_bands)
    n_b = 3 if paired else w["n_o"]
    P = torch.zeros((Nq, B, B), dtype=torch.complex128, device=dev)
    C = torch.zeros_like(P)
    tuned, moved = _tune(T, ctx, lam_at(K // 2), tune)
    if W > 0:
        T.tufrg_flow(ctx, P, C, lam0, lam_at(W), n_steps=W, v_max=1e30)
    P.zero_()
    C.zero_()
    torch.cuda.synchronize()
    T.tufrg_timing(ctx, True)
    t0 = time.perf_counter()
    res = T.tufrg_flow(ctx, P, C, lam0, lam_at(K), n_steps=K, v_max=w["v_max"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    loop_ms, loop_n = T.tufrg_timing_read(ctx, T.TIMER_LOOP)
    proj_ms, proj_n = T.tufrg_timing_read(ctx, T.TIMER_PROJECT)
    bund_ms, bund_n = T.tufrg_timing_read(ctx, T.TIMER_BUNDLE)
    T.tufrg_timing(ctx, False)
    entries = 2.0 * Nq * B * B
    compact = 2.0 * Nq * nD * ctx.n_o ** 4
    ndx, ndy = _box(w["ff"])
    # the survey's per-unit figure for the model's bands (the roofline's
    # achieved rate); the same count for the bands the kernel sums beside it
    credited = credited_loop_flops_per_pair(w["n_o"], ndy)
    credited_summed = credited_loop_flops_per_pair(w["n_o"], ndy, n_b)
    flops_step = 2.0 * Nq * Nf * credited
    launches = loop_n / K
    loop_step_s = loop_ms / K * 1e-3
    achieved = flops_step / loop_step_s  # = credited flops per launch / average launch time
    if prec == "bf16x3":
        bound, peak = "mfma", PEAK_BF16_MFMA
    else:
        bound, peak = "alu", PEAK_FP32_VECTOR
    out = {
        "metric": METRIC, "value": entries * K / dt, "unit": "loop entries/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": dt / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": w["name"], "n_orb": w["n_o"], "n_ff": len(w["ff"]), "B": B, "Lq": w["Lq"],
                   "n_ref": w["n_ref"], "Nq": Nq, "Nf": Nf, "cutoff": w["cutoff"],
                   "step": f"Euler step {1}..{K} of the {n}-step grid from Lambda = {lam0:g}: "
                           "loops + projections + bundles + update",
                   "parallelism": "single GPU"},
        "flow_steps_per_s": K / dt,
        "compact_loop_entries_per_s": compact * K / dt,
        "stage_ms_per_step": {"loop_kernel": loop_ms / K, "projections": proj_ms / K,
                              "bundle_products": bund_ms / K},
        "loop_kernel_ms": loop_ms / loop_n,
        "loop_launches_per_step": launches,
        "loop_entries_per_s_kernel": entries / loop_step_s,
        "roofline": {"bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None if moved or six_bands else _traffic(w["name"], prec),
                     "flops_per_pair": credited, "bands_summed": n_b,
                     "frac_with_bands_summed": (achieved * credited_summed / credited) / peak,
                     "executed_matrix_flops_per_pair": (mfma_flops_per_pair(ndy, w["n_o"], n_b)
                                                        if prec == "bf16x3" else None)},
        "flow_result": res,
    }
    if tuned is not None:
        out["autotune"] = tuned
    print(f"bench: {w['name']} {prec}: {dt / K * 1e3:.1f} ms per step", file=sys.stderr, flush=True)
    # FP64-plain over the first steps, against the mixed form over the same steps
    if fp64_steps > 0:
        P.zero_()
        C.zero_()
        T.tufrg_flow(ctx, P, C, lam0, lam_at(fp64_steps), n_steps=fp64_steps, v_max=w["v_max"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.zero_()
        C.zero_()
        T.tufrg_flow(ctx, P, C, lam0, lam_at(fp64_steps), n_steps=fp64_steps, v_max=w["v_max"])
        torch.cuda.synchronize()
        dt_mix = (time.perf_counter() - t0) / fp64_steps
        Pm, Cm = P.clone(), C.clone()
        ctx64 = T.Context.from_workload(w, precision="fp64")
        P.zero_()
        C.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T.tufrg_flow(ctx64, P, C, lam0, lam_at(fp64_steps), n_steps=fp64_steps, v_max=w["v_max"])
        torch.cuda.synchronize()
        dt64 = (time.perf_counter() - t0) / fp64_steps
        ctx64.close()
        err = max((Pm - P).abs().max().item() / P.abs().max().item(),
                  (Cm - C).abs().max().item() / C.abs().max().item())
        out["fp64_plain"] = {"steps": fp64_steps, "ms_per_step": dt64 * 1e3, "value": entries / dt64,
                             "flow_steps_per_s": 1.0 / dt64,
                             "note": "first steps from Lambda0 only (an FP64 step takes seconds)"}
        out["mixed_vs_fp64_plain"] = {"rel_err": err, "speedup": dt64 / dt_mix, "steps": fp64_steps,
                                      "mixed_ms_per_step": dt_mix * 1e3}
        del Pm, Cm
        print(f"bench: fp64-plain {dt64 * 1e3:.0f} ms per step, rel err {err:.2e}", file=sys.stderr, flush=True)
    if surrogate:
        out["surrogate_flow"] = surrogate_window(T, torch, ctx, w, K, dt / K, n_rows=n_rows, epochs=epochs)
    ctx.close()
    return out


def surrogate_window(T, torch, ctx, w, K, t_plain_step, n_rows=120000, epochs=(10, 10, 10)):
    """Surrogate-assisted form over the timed window: the network trained on
    n_rows random blocks of the plain loops at the scales of the K steps (the
    loops a plain flow produces), then the same K steps with the network (5 %
    of the q_x rows recomputed plainly per right-hand side, plain loops
    everywhere when the sampled error exceeds 1e-3 or the coupling 20),
    compared with the plain flow of those steps."""
    import numpy as np

    from synth import mlp_init, mlp_shape

    dev = torch.device("cuda:0")
    no4 = ctx.n_o ** 4
    nb = 2 * ctx.Nq * ctx.n_dR
    lam0, n = w["lam0"], w["n_steps"]
    lam_k = lam0 * (w["lam_end"] / lam0) ** (K / n)
    lams = lam0 * (w["lam_end"] / lam0) ** (np.arange(K) / n)
    P = torch.zeros((ctx.Nq, ctx.B, ctx.B), dtype=torch.complex128, device=dev)
    C = torch.zeros_like(P)
    T.tufrg_flow(ctx, P, C, lam0, lam_k, n_steps=K, v_max=w["v_max"])
    P0, C0 = P.clone(), C.clone()
    per = min(nb, n_rows // K)
    sizes = mlp_shape(11 + ctx.n_dR, 256, 2 * no4)
    rng = np.random.default_rng(3)
    X = torch.zeros((K * per, sizes[0]), dtype=torch.float32, device=dev)
    Y = torch.zeros((K * per, sizes[-1]), dtype=torch.float32, device=dev)
    Lc = torch.zeros((2, ctx.Nq, ctx.n_dR, no4), dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    scales = []
    for i, lam in enumerate(lams):
        b = rng.choice(nb, size=per, replace=False)
        q, ch, iD = ((b // ctx.n_dR) % ctx.Nq, b // (ctx.n_dR * ctx.Nq), b % ctx.n_dR)
        q, ch, iD = (torch.from_numpy(a.astype(np.int32)).to(dev) for a in (q, ch, iD))
        T.tufrg_loops_compact(ctx, lam, 1, Lc)
        ys = Y[i * per:(i + 1) * per]
        scales.append(T.tufrg_sur_targets(ctx, per, 1.0, Lc, ys, q, ch, iD))
        T.tufrg_sur_features(ctx, per, lam, X[i * per:(i + 1) * per], q, ch, iD)
        T.tufrg_sur_targets(ctx, per, scales[-1], Lc, ys, q, ch, iD)
    del Lc
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = T.Mlp(sizes, mlp_init(sizes, seed=3))
    t0 = time.perf_counter()
    loss = None
    for ep, lr in zip(epochs, (1e-3, 3e-4, 1e-4)):
        loss = T.tufrg_mlp_train(net, X, Y, batch=2048, epochs=ep, lr=lr, seed=3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del X, Y
    T.tufrg_sur_attach(ctx, net, lams, scales)
    out = {"training": {"rows": K * per, "scales": K, "data_seconds": t_data, "train_seconds": t_train,
                        "final_loss": loss, "net": sizes}}
    for key, tol in (("tol_1e-3", 1e-3), ("tol_5e-2", 5e-2)):
        P.zero_()
        C.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = T.tufrg_flow(ctx, P, C, lam0, lam_k, n_steps=K, v_max=w["v_max"], surrogate=True, sample_frac=0.05,
                         sur_tol=tol, plain_above=20.0, sample_seed=3)
        torch.cuda.synchronize()
        dts = time.perf_counter() - t0
        err = max((P - P0).abs().max().item() / P0.abs().max().item(),
                  (C - C0).abs().max().item() / C0.abs().max().item())
        out[key] = dict(r, seconds=dts, ms_per_step=dts / K * 1e3, speedup_vs_plain=t_plain_step / (dts / K),
                        rel_err_vs_plain=err, served_fraction=r["n_surrogate"] / max(1, r["n_rhs"]))
        print(f"bench: surrogate at tol {tol:g}: {r['n_surrogate']} of {r['n_rhs']} from the network, "
              f"rel err {err:.2e}", file=sys.stderr, flush=True)
    T.tufrg_sur_attach(ctx, None)
    net.close()
    del P0, C0
    return out


def batch_bench(T, torch, K, W):
    """32 independent Rashba/Hubbard instances of uneven size (seed 2), FP32
    loops and products, lockstep Euler steps 10 -> 1 through tufrg_batch_flow;
    the same batch on one stream for comparison."""
    from synth.workloads import batch_instances

    dev = torch.device("cuda:0")
    ws = batch_instances(32, seed=2, n_ref=12)
    out = {}
    for n_streams, G, fused in ((4, 0, False), (1, 0, False), (4, 8, False), (4, 0, True)):
        b = T.Batch(ws, precision="fp32", n_streams=n_streams)
        Ps, Cs = [], []
        for d in b.dims:
            Ps.append(torch.zeros((d["Nq"], d["B"], d["B"]), dtype=torch.complex128, device=dev))
            Cs.append(torch.zeros_like(Ps[-1]))
        if W > 0:
            T.tufrg_batch_flow(b, Ps, Cs, 10.0, 1.0, n_steps=W, v_max=1e30, graph_steps=G, fused_loops=fused)
        for x in Ps + Cs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = T.tufrg_batch_flow(b, Ps, Cs, 10.0, 1.0, n_steps=K, v_max=1e30, graph_steps=G, fused_loops=fused)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        entries = sum(2.0 * d["Nq"] * d["B"] ** 2 for d in b.dims)
        out[(n_streams, G, fused)] = dict(seconds=dt, value=entries * K / dt, ms_per_step=dt / K * 1e3,
                                   steps=min(r["n_steps"] for r in res),
                                   checksum=float(sum(x.abs().sum().item() for x in Ps)))
        b.close()
    best = max((out[(4, 0, False)], out[(4, 8, False)]), key=lambda d: d["value"])
    return {
        "metric": METRIC, "value": best["value"], "unit": "loop entries/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": best["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": "rashba_batch32", "instances": len(ws),
                   "Lq": sorted({w["Lq"] for w in ws}), "n_ff": sorted({len(w["ff"]) for w in ws}),
                   "n_ref": 12, "step": "lockstep Euler step of every instance", "parallelism": "single GPU"},
        "flow_steps_per_s": K / best["seconds"],
        "four_streams": out[(4, 0, False)], "one_stream": out[(1, 0, False)],
        "four_streams_graph_steps_8": out[(4, 8, False)], "four_streams_fused_loops": out[(4, 0, True)],
        "speedup_4_streams_vs_1": out[(1, 0, False)]["seconds"] / out[(4, 0, False)]["seconds"],
        "speedup_graph_vs_direct": out[(4, 0, False)]["seconds"] / out[(4, 8, False)]["seconds"],
        "speedup_fused_loops_vs_per_instance": out[(4, 0, False)]["seconds"] / out[(4, 0, True)]["seconds"],
        "graph_checksum_equal": out[(4, 0, False)]["checksum"] == out[(4, 8, False)]["checksum"],
        "fused_checksum_equal": out[(4, 0, False)]["checksum"] == out[(4, 0, True)]["checksum"],
        "roofline": None,
    }


def su2_leg(T, torch, w, K, W):
    """Spin-degenerate one-band workload: the same K Euler steps 10 -> 1 as the
    SU(2)-reduced flow (one orbital, B = n_ff) and as the spinful FP64 flow
    (two spin-orbitals, B = 4 n_ff); both in FP64, with the max-coupling
    agreement (max(|p|,|c|,|d|) of the reduced state is max(|P|,|C|))."""
    import numpy as np
    dev = torch.device("cuda:0")
    v = np.full((1, 1, 1, 1), w["V0"][0, 1, 0, 1], dtype=np.complex128)
    ctx1 = T.Context(w["hop_R"], w["hop_t"][:, :1, :1], w["mu"], v, w["ff"], w["Lq"], w["n_ref"], w["cutoff"], "fp64")
    st = [torch.zeros((ctx1.Nq, ctx1.B, ctx1.B), dtype=torch.complex128, device=dev) for _ in range(3)]
    if W > 0:
        T.tufrg_su2_flow(ctx1, *st, 10.0, 1.0, W, v_max=1e30)
    for x in st:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r1 = T.tufrg_su2_flow(ctx1, *st, 10.0, 1.0, K, v_max=1e30)
    torch.cuda.synchronize()
    dt1 = time.perf_counter() - t0
    ctx1.close()
    ctxS = T.Context.from_workload(w, precision="fp64")
    P = torch.zeros((ctxS.Nq, ctxS.B, ctxS.B), dtype=torch.complex128, device=dev)
    C = torch.zeros_like(P)
    if W > 0:
        T.tufrg_flow(ctxS, P, C, 10.0, 1.0, n_steps=W, v_max=1e30)
    P.zero_()
    C.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rS = T.tufrg_flow(ctxS, P, C, 10.0, 1.0, n_steps=K, v_max=1e30)
    torch.cuda.synchronize()
    dtS = time.perf_counter() - t0
    ctxS.close()
    return {"B_reduced": int(len(w["ff"])), "B_spinful": int(4 * len(w["ff"])),
            "ms_per_step": dt1 / K * 1e3, "spinful_fp64_ms_per_step": dtS / K * 1e3, "speedup": dtS / dt1,
            "max_coupling_rel_diff": abs(r1["max_coupling"] / rS["max_coupling"] - 1)}


def two_orbital_line(T, torch, w, args, K, W, extras=True, cpu=True):
    """Line of a two-orbital workload (Rashba, Hubbard): K timed Euler steps
    10 -> 1 in FP32 (or the precision asked for), the loop-kernel roofline,
    and optionally the FP64-plain form, Dormand-Prince flows, the surrogate,
    the basis change and the CPU baseline."""
    import numpy as np

    dev = torch.device("cuda:0")
    no_extras = args.no_extras or not extras
    own_cutoff = args.cutoff is None or args.cutoff == w["cutoff"]
    if not own_cutoff:
        w = dict(w, cutoff=args.cutoff, temperature=args.temperature)
    prec = args.prec or "fp32"
    lam0, lam_mid = 10.0, 1.0

    def make(prec):
        ctx = T.Context.from_workload(w, precision=prec)
        P = torch.zeros((ctx.Nq, ctx.B, ctx.B), dtype=torch.complex128, device=dev)
        return ctx, P, torch.zeros_like(P)

    def timed_steps(ctx, P, C, timing):
        # warmup: W steps of the same grid; then K steps from the start state
        if W > 0:
            T.tufrg_flow(ctx, P, C, lam0, lam_mid, n_steps=W, v_max=1e30)
        P.zero_()
        C.zero_()
        torch.cuda.synchronize()
        if timing:
            T.tufrg_timing(ctx, True)
        t0 = time.perf_counter()
        res = T.tufrg_flow(ctx, P, C, lam0, lam_mid, n_steps=K, v_max=1e30)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        loop_ms = loop_n = None
        if timing:
            loop_ms, loop_n = T.tufrg_timing_read(ctx, T.TIMER_LOOP)
            T.tufrg_timing(ctx, False)
        return dt, res, loop_ms, loop_n

    ctx32, P32, C32 = make(prec)
    tuned, moved = _tune(T, ctx32, 3.0, getattr(args, "tune", False))
    dt32, res32, loop_ms, loop_n = timed_steps(ctx32, P32, C32, timing=True)
    B, Nq, Nf = ctx32.B, ctx32.Nq, ctx32.Nf
    entries = 2.0 * Nq * B * B
    value = entries * K / dt32
    # the loop timer brackets each launch of the dominant loop kernel: one
    # per step (both channels) on the vector units, one per channel and chunk
    # of coarse q on the matrix cores
    loop_avg_s = loop_ms / loop_n * 1e-3
    launches = loop_n / K
    ndx, ndy = _box(w["ff"])
    if prec == "bf16x3":
        flops_step = 2.0 * Nq * Nf * credited_loop_flops_per_pair(w["n_o"], ndy)
        bound, peak = "mfma", PEAK_BF16_MFMA
    else:
        flops_step = 2.0 * Nq * Nf * loop_flops_per_pair(w["n_o"], ndx, ndy, w["cutoff"] == "shell")
        bound, peak = "alu", PEAK_FP32_VECTOR
    achieved = flops_step / launches / loop_avg_s
    # the committed counters were taken with the workload's own regulator
    traffic = _traffic(w["name"], prec) if own_cutoff and not moved else None
    out = {
        "metric": METRIC, "value": value, "unit": "loop entries/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": dt32 / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": w["name"], "n_orb": w["n_o"], "n_ff": len(w["ff"]), "B": B,
                   "Lq": w["Lq"], "n_ref": w["n_ref"], "Nq": Nq, "Nf": Nf, "cutoff": w["cutoff"],
                   **({"temperature": w["temperature"]} if w["cutoff"] == "shell" else {}),
                   "step": "Euler step: loops + projections + bundles + update",
                   "parallelism": "single GPU"},
        **({"autotune": tuned} if tuned is not None else {}),
        "flow_steps_per_s": K / dt32,
        "loop_kernel_ms": loop_avg_s * 1e3,
        "loop_launches_per_step": launches,
        "loop_entries_per_s_kernel": entries / (loop_avg_s * launches),
        "roofline": {"bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic},
    }
    if not no_extras:
        # the same steps with HIP graphs of 8 steps each (one host
        # synchronisation per graph instead of one per step)
        Pd, Cd = P32.clone(), C32.clone()
        P32.zero_()
        C32.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T.tufrg_flow(ctx32, P32, C32, lam0, lam_mid, n_steps=K, v_max=1e30, graph_steps=8)
        torch.cuda.synchronize()
        dtg = time.perf_counter() - t0
        out["graph_steps_8"] = {"ms_per_step": dtg / K * 1e3, "speedup_vs_direct": dt32 / dtg,
                                "bit_equal_to_direct": bool(torch.equal(Pd, P32) and torch.equal(Cd, C32))}
        del Pd, Cd
    if not no_extras and w["name"].startswith("hubbard"):
        out["su2_reduced"] = su2_leg(T, torch, w, K, W)
    if not no_extras:
        ctx64, P64, C64 = make("fp64")
        dt64, res64, l64_ms, l64_n = timed_steps(ctx64, P64, C64, timing=True)
        ref = P64.abs().max().item(), C64.abs().max().item()
        err = max((P32 - P64).abs().max().item() / ref[0], (C32 - C64).abs().max().item() / ref[1])
        out["fp64_plain"] = {"value": entries * K / dt64, "ms_per_step": dt64 / K * 1e3,
                             "loop_kernel_ms": l64_ms / l64_n, "flow_steps_per_s": K / dt64}
        out["speedup_fp32_vs_fp64"] = dt64 / dt32
        out["rel_err_fp32_vs_fp64"] = err
    if not no_extras and not args.no_dp:
        # production integrator: Dormand-Prince 5(4), rtol = atol = 1e-6, 10 -> 1e-4
        dp = {}
        for name, (ctx, P, C) in (("fp32", (ctx32, P32, C32)), ("fp64", (ctx64, P64, C64))):
            P.zero_()
            C.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = T.tufrg_flow(ctx, P, C, w["lam0"], w["lam_end"], n_steps=0, rtol=w["rtol"],
                             atol=w["atol"], v_max=w["v_max"], max_steps=400)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            dp[name] = dict(r, seconds=dt, flow_steps_per_s=r["n_steps"] / dt,
                            rhs_per_s=r["n_rhs"] / dt)
        refP, refC = P64.abs().max().item(), C64.abs().max().item()
        same_stop = dp["fp32"]["n_steps"] == dp["fp64"]["n_steps"]
        if same_stop:
            dp["rel_err_fp32_vs_fp64"] = max((P32 - P64).abs().max().item() / refP,
                                             (C32 - C64).abs().max().item() / refC)
        if dp["fp64"]["diverged"] and dp["fp32"]["diverged"]:
            dp["lambda_c_rel_err"] = abs(dp["fp32"]["lambda_c"] / dp["fp64"]["lambda_c"] - 1.0)
        out["dp54_flow"] = dp
    if not no_extras and not args.no_dp and not args.no_surrogate:
        out["surrogate_flow"] = surrogate_leg(T, torch, ctx32, P32, C32, P64, C64, dp, w, K, dt32 / K)
    if not no_extras and not args.no_basis:
        band = T.Context.from_workload(w, precision=prec, basis="band", V0=0 * w["V0"])
        out["basis_change"] = basis_leg(T, torch, ctx64, P64, C64, w["ff"], band_ctx=band,
                                        V0=np.asarray(w["V0"]), steps=K)
        band.close()
    if not no_extras:
        ctx64.close()
    if cpu and not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, n_sample=2)
    ctx32.close()
    return out




def _counter_per_dispatch(csv_path, name_part, counter):
    """Per-dispatch values of one counter for the kernels whose name contains
    name_part, from a rocprofv3 counter_collection.csv."""
    import csv
    vals = {}
    names = set()
    with open(csv_path, newline="") as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter or name_part not in r["Kernel_Name"]:
                continue
            d = r["Dispatch_Id"]
            vals[d] = vals.get(d, 0.0) + float(r["Counter_Value"])
            names.add(r["Kernel_Name"])
    if not vals:
        raise RuntimeError(f"no {counter} rows for kernels matching {name_part!r} in {csv_path}")
    return list(vals.values()), sorted(names)


def summarize_traffic(args):
    """profiles/loop_kernel_traffic_<workload>_<prec>.json from four
    rocprofv3 --pmc runs (FETCH_SIZE and WRITE_SIZE of the bench, the same of
    --calibrate-copy): KiB per dispatch of the loop kernel, each scaled by
    what the counter reads per byte of a plain 1 GiB device copy."""
    f_dir, w_dir, cf_dir, cw_dir = args.summarize_traffic
    # the main loop kernel of the precision (two orbitals: loop_no2, six: loop_gen)
    kname = "loop_rb_kernel" if args.prec == "bf16x3" else (
        "loop_gen_kernel" if args.workload.startswith("t2g") else "loop_no2_kernel")
    pick = lambda d, nm: os.path.join(d, nm + "_counter_collection.csv")
    fetch, names = _counter_per_dispatch(pick(f_dir, "fetch"), kname, "FETCH_SIZE")
    write, _ = _counter_per_dispatch(pick(w_dir, "write"), kname, "WRITE_SIZE")
    # the 1 GiB copies are the largest dispatches of the calibration run
    cf, _ = _counter_per_dispatch(pick(cf_dir, "fetch"), "", "FETCH_SIZE")
    cw, _ = _counter_per_dispatch(pick(cw_dir, "write"), "", "WRITE_SIZE")
    cf = sorted(cf)[-3:]
    cw = sorted(cw)[-3:]
    n = 1 << 30
    f_kib, w_kib = sum(fetch) / len(fetch), sum(write) / len(write)
    cf_kib, cw_kib = sum(cf) / len(cf), sum(cw) / len(cw)
    fb, wb = n / cf_kib, n / cw_kib
    run = f"python3 -u bench.py --workload {args.workload} --prec {args.prec} --steps 1 --warmup 0 --no-cpu --no-extras"
    out = {
        "kernel": names[0] if len(names) == 1 else names,
        "workload": args.workload,
        "precision": args.prec,
        "source_sha256": _loop_source_hash(args.workload, args.prec),
        "fetch_kib_per_dispatch": f_kib,
        "write_kib_per_dispatch": w_kib,
        "dispatches": len(fetch),
        "copy_calibration": {"bytes_copied": n, "fetch_kib": cf_kib, "write_kib": cw_kib,
                             "fetch_bytes_per_kib": fb, "write_bytes_per_kib": wb},
        "fetch_bytes_per_launch": f_kib * fb,
        "write_bytes_per_launch": w_kib * wb,
        "hbm_bytes_per_launch": f_kib * fb + w_kib * wb,
        "commands": [
            f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {f_dir} -o fetch -- {run}",
            f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {w_dir} -o write -- {run}",
            f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {cf_dir} -o fetch -- python3 -u bench.py --calibrate-copy",
            f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {cw_dir} -o write -- python3 -u bench.py --calibrate-copy",
            "python3 bench.py --summarize-traffic " + " ".join(args.summarize_traffic)
            + f" --workload {args.workload} --prec {args.prec}",
        ],
        "note": "FETCH_SIZE and WRITE_SIZE count L2-to-fabric traffic; each is scaled by what the same counter "
                "reads for a plain 1 GiB device copy.  Misses served by the MALL are included, so this bounds "
                "HBM bytes from above.",
    }
    path = os.path.join(ROOT, "profiles", f"loop_kernel_traffic_{args.workload}_{args.prec}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(path)


def summarize_trace(args):
    """A markdown table of a rocprofv3 --kernel-trace --stats run (the
    kernel_stats.csv it writes), the command that made it on top."""
    import csv
    stats_csv, cmd, out_path = args.summarize_trace
    rows = list(csv.DictReader(open(stats_csv, newline="")))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# Kernel trace: {args.workload} ({args.prec})", "", "Command:", "", "```", cmd, "```", "",
             "| kernel | calls | total ms | average us | min us | max us | share |", "|---|---|---|---|---|---|---|"]
    for r in rows[:20]:
        nm = r["Name"].replace("|", "\\|")
        if len(nm) > 110:
            nm = nm[:107] + "..."
        lines.append(f"| `{nm}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {100 * float(r['TotalDurationNs']) / tot:.1f} % |")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(out_path)


def summarize_counters(args):
    """A markdown table of the SQ counters of a rocprofv3 --pmc run, summed
    over the dispatches of the loop kernel and divided by their number, with
    the instruction counts per wave and tile of 16 ky (BF16X3 loop kernel)."""
    csv_path, cmd, out_path = args.summarize_counters
    kname = "loop_rb_kernel" if args.prec == "bf16x3" else (
        "loop_gen_kernel" if args.workload.startswith("t2g") else "loop_no2_kernel")
    import csv
    names, disp = set(), set()
    with open(csv_path, newline="") as fh:
        rows = [r for r in csv.DictReader(fh) if kname in r["Kernel_Name"]]
    if not rows:
        raise RuntimeError(f"no rows for kernels matching {kname!r} in {csv_path}")
    tot = {}
    for r in rows:
        tot[r["Counter_Name"]] = tot.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        disp.add(r["Dispatch_Id"])
        names.add(r["Kernel_Name"])
    n = len(disp)
    lines = [f"# SQ counters of the loop kernel: {args.workload} ({args.prec})", "", "Command:", "", "```", cmd, "```",
             "", f"Kernel: `{sorted(names)[0][:120]}`, {n} dispatches.", "",
             "| counter | per dispatch |", "|---|---|"]
    for k in sorted(tot):
        lines.append(f"| {k} | {tot[k] / n:.4g} |")
    if args.prec == "bf16x3" and "SQ_WAVES" in tot:
        from synth import workload
        w = workload(args.workload)
        lf = w["Lq"] * w["n_ref"]
        # the t2g models are Kramers-paired: 16 ky pairs per tile unless --six-bands
        paired = w["n_o"] == 6 and args.workload.startswith("t2g") and not args.six_bands and lf % 2 == 0
        tiles = ((lf // 2 if paired else lf) + 15) // 16  # tiles per kx row; one kx row per work item
        per = lambda c: tot[c] / tot["SQ_WAVES"] / tiles
        what = "16 ky pairs (paired bands)" if paired else "16 ky"
        lines += ["", f"Per wave and tile of {what} (one kx row per work item, {tiles} tiles):", ""]
        for c in ("SQ_INSTS_VALU", "SQ_INSTS_MFMA", "SQ_INSTS_LDS"):
            if c in tot:
                lines.append(f"* {c}: {per(c):.0f}")
        if "SQ_LDS_BANK_CONFLICT" in tot and "SQ_INSTS_LDS" in tot:
            lines.append(f"* bank-conflict cycles per LDS instruction: "
                         f"{tot['SQ_LDS_BANK_CONFLICT'] / tot['SQ_INSTS_LDS']:.2f}")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(out_path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="time the headline steps only (for profiler runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (scales HBM counters)")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="synthetic workload (the headline line uses the default)")
    ap.add_argument("--no-dp", action="store_true", help="skip the Dormand-Prince flows")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate-assisted flow")
    ap.add_argument("--no-basis", action="store_true", help="skip the orbital -> band basis change")
    ap.add_argument("--prec", default=None, choices=["fp32", "bf16x3", "fp64"],
                    help="arithmetic of the timed loops (default: bf16x3 for six spin-orbitals, else fp32)")
    ap.add_argument("--fp64-steps", type=int, default=1,
                    help="steps of the FP64-plain comparison of a six-orbital workload")
    ap.add_argument("--cutoff", choices=["temperature", "omega", "shell"],
                    help="regulator in place of the workload's own")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the loop kernels' launch shape before timing (cache: $TUFRG_TUNE_CACHE)")
    ap.add_argument("--six-bands", action="store_true",
                    help="six spin-orbitals: sum all six bands even where they are Kramers pairs")
    ap.add_argument("--temperature", type=float, default=0.02,
                    help="fixed temperature of the momentum-shell regulator")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write the loop kernel's HBM traffic summary under profiles/ from rocprofv3 counter runs "
                         "(CPU only)")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("KERNEL_STATS_CSV", "COMMAND", "OUT_MD"),
                    help="write a markdown summary of a rocprofv3 --stats run (CPU only)")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("COUNTER_CSV", "COMMAND", "OUT_MD"),
                    help="write a markdown summary of a rocprofv3 --pmc run of SQ counters (CPU only)")
    args = ap.parse_args()
    if args.summarize_traffic or args.summarize_trace or args.summarize_counters:
        args.prec = args.prec or ("bf16x3" if args.workload.startswith("t2g") else "fp32")
        if args.summarize_traffic:
            summarize_traffic(args)
        if args.summarize_trace:
            summarize_trace(args)
        if args.summarize_counters:
            summarize_counters(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the q-sharded multi-GPU "
              "path is a design, not implemented in this library", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1710_08830_amd import tufrg as T
    from synth import workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        n = 1 << 30
        x = torch.ones(n // 8, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 3}))
        return
    K, W = args.steps, args.warmup
    if args.workload == "rashba_batch32":
        print(json.dumps(batch_bench(T, torch, K, W)))
        return
    w = workload(args.workload)
    if w["n_o"] == 6:
        if args.cutoff and args.cutoff != w["cutoff"]:
            w = dict(w, cutoff=args.cutoff, temperature=args.temperature)
        prec = args.prec or "bf16x3"
        out = six_orbital_line(T, torch, w, prec, K, W, fp64_steps=0 if args.no_extras else args.fp64_steps,
                               six_bands=args.six_bands,
                               tune=args.tune,
                               surrogate=not (args.no_extras or args.no_surrogate))
        if not args.no_extras:
            # the two-orbital Rashba workload (24 x 24 refined 24x, FP32) as an extra key
            wr = workload("rashba_s9_L24")
            ar = argparse.Namespace(**dict(vars(args), cutoff=None, prec="fp32"))
            out["rashba_s9_L24"] = two_orbital_line(T, torch, wr, ar, min(K, 20), min(W, 3), extras=False,
                                                    cpu=False)
        if not args.no_cpu:
            out["cpu_baseline"] = cpu_baseline(w, n_sample=1)
        print(json.dumps(out))
        return
    print(json.dumps(two_orbital_line(T, torch, w, args, K, W)))


if __name__ == "__main__":
    main()
