"""Orbital-basis truncated-unity fRG, plain FP64 (oracle; test infrastructure).

State tensors use the paper's index order: an exchange propagator is stored as
``X[q, iR, iR', n1, n2, n3, n4]`` = X^{R R'}_{n1 n2 n3 n4}(q), with q running
over the coarse L_q x L_q mesh (index mx * L_q + my, q = 2 pi m / L_q) and iR,
iR' indexing the form-factor list S (plane waves f_R(k) = exp(-i k.R), Sec. 2).

What is computed, and where it comes from:

* Orbital loops (Sec. 4.2).  The paper writes the pp loop with four orbital
  indices through the U-matrix product (eq. for the orbital loop) and says the
  C and D loops follow "similarly".  Inserting the partition of unity only
  around the loop, the orbital loops are direct k-sums on the refined mesh
  (fine mesh L_f = n_ref L_q, loop average 1/N_f):

    Lpp_{t1t2t3t4}(s)_{R1R2} = 1/N_f sum_k f_R1(k) f*_R2(k)
        sum_{mn} Pi_m(s-k)_{t1t3} Pi_n(k)_{t2t4} L-(e_m(s-k), e_n(k))
    Lph_{t1t2t3t4}(u)_{R1R2} = 1/N_f sum_k f_R1(k) f*_R2(k)
        sum_{mn} Pi_m(k)_{t1t3} Pi_n(k-u)_{t4t2} L+(e_m(k), e_n(k-u))

  With U = 1 these are the band loops of Sec. 3.1 (loop matrices L-/L+), and
  with a complete form-factor set Lpp equals the U-matrix product of Sec. 4.2.
* Matrix RGE (Sec. 3.1 and the orbital form of Sec. 4.2):

    dP_{s1s2s3s4} = sum_t VP[s1 s2 t1 t2] Lpp_{t1t2t3t4} VP[t4 t3 s3 s4]
    dC_{s1s2s3s4} = 2 sum_t VC[s1 t2 s3 t1] Lph_{t1t2t3t4} VC[t3 s2 t4 s4]

  (matrix products in the form-factor indices).  D is not flowed: it equals
  -C with the last two orbital indices exchanged (Sec. 3.2).
* Projected vertices (Sec. 3.3): VP = P[V0] + P + P[V^C] + P[V^D] and
  VC = C[V0] + C[V^P] + C + C[V^D], with the four cross projections evaluated
  through the real-space transform X(R'') = 1/N_q sum_q exp(i q.R'') X(q), and
  every term whose form-factor labels leave S dropped (the truncation).  The
  projections of a momentum-independent V0 fill only the (R, R') = (0, 0)
  block.
* Band basis (Sec. 3.1, the form in which the paper derives the RGE; basis
  change of Sec. 4.1): with basis="band" the single-particle basis is the
  eigenbasis of H(k), so the loops see unit projectors and depend on two band
  indices; the projections and bundle products are the same formulas.  The
  bare vertex then enters as a static particle-particle term P0 (its band
  form, e.g. U^dagger P[V0] U with the basis matrices of ``oracle.basis``),
  projected with the flowing P; exact for a complete form-factor set, the
  truncated expansion otherwise.
* Integration of the single-channel couplings (Sec. 3.1): explicit Euler in
  Lambda on a log grid, or Dormand-Prince 5(4) in ln Lambda; the flow stops
  when max(|P|, |C|) exceeds v_max, and the critical scale is interpolated
  linearly in ln Lambda.
"""

import numpy as np

from . import bands, cutoff

_DP_C = np.array([0.0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1.0, 1.0])
_DP_A = [
    [],
    [1 / 5],
    [3 / 40, 9 / 40],
    [44 / 45, -56 / 15, 32 / 9],
    [19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729],
    [9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656],
    [35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84],
]
_DP_B5 = np.array([35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84, 0.0])
_DP_B4 = np.array([5179 / 57600, 0.0, 7571 / 16695, 393 / 640, -92097 / 339200,
                   187 / 2100, 1 / 40])


class TUSetup:
    """Meshes, form factors, band data and the initial interaction."""

    def __init__(self, hop_R, hop_t, mu, V0, ff, Lq, n_ref, scheme, temperature=None, C0=None, P0=None,
                 basis="orbital"):
        self.hop_R = np.asarray(hop_R)
        self.hop_t = np.asarray(hop_t)
        self.mu = float(mu)
        self.V0 = np.asarray(V0, dtype=np.complex128)
        # non-local part of the initial interaction in crossed particle-hole
        # form (a static term of the C channel, its D partner by antisymmetry)
        self.C0 = None if C0 is None else np.asarray(C0, dtype=np.complex128)
        # static particle-particle term of the bare vertex (its P-channel
        # expansion, projected with the flowing P): the band-basis form of a
        # bare interaction given in the orbital basis (Sec. 4.1)
        self.P0 = None if P0 is None else np.asarray(P0, dtype=np.complex128)
        if basis not in ("orbital", "band"):
            raise ValueError(basis)
        self.basis = basis
        self.S = np.asarray(ff, dtype=np.int64).reshape(-1, 2)
        self.n_ff = len(self.S)
        self.n_o = self.hop_t.shape[1]
        self.Lq = int(Lq)
        self.n_ref = int(n_ref)
        self.Lf = self.Lq * self.n_ref
        self.Nq = self.Lq ** 2
        self.Nf = self.Lf ** 2
        # "temperature", "omega", or "shell" at the fixed temperature given
        self.scheme = cutoff.Shell(temperature) if scheme == cutoff.SHELL else scheme
        self.coarse = bands.mesh(self.Lq)
        self.fine = bands.mesh(self.Lf)
        self.e, self.U = bands.band_data(self.hop_R, self.hop_t, self.mu, self.Lf)
        if basis == "band":
            # band basis (Sec. 3.1): the single-particle basis diagonalises H(k),
            # so the loops see unit projectors and depend on two band indices
            self.Pi = bands.projectors(np.broadcast_to(np.eye(self.n_o), self.U.shape))
        else:
            self.Pi = bands.projectors(self.U)
        # membership of a residue class mod L_q in S
        self._ff_of = {}
        for i, R in enumerate(self.S):
            self._ff_of[self._res(R)] = i
        # R'' range of the real-space transform: D = S - S (mod L_q)
        D = {}
        for R1 in self.S:
            for R2 in self.S:
                r = self._res(R1 - R2)
                if r not in D:
                    D[r] = R1 - R2
        self.D = D

    @classmethod
    def from_workload(cls, w, **over):
        kw = dict(hop_R=w["hop_R"], hop_t=w["hop_t"], mu=w["mu"], V0=w["V0"],
                  ff=w["ff"], Lq=w["Lq"], n_ref=w["n_ref"], scheme=w["cutoff"],
                  temperature=w.get("temperature"))
        kw.update(over)
        return cls(**kw)

    def _res(self, R):
        return (int(R[0]) % self.Lq, int(R[1]) % self.Lq)

    def ff_index(self, R):
        """Index of the form factor whose label equals R (mod L_q), or -1."""
        return self._ff_of.get(self._res(R), -1)

    def coarse_phase(self, R):
        """exp(i q.R) for every coarse q, exact reduction of m.R mod L_q."""
        mr = (self.coarse @ np.asarray(R, dtype=np.int64)) % self.Lq
        return np.exp(2j * np.pi * mr / self.Lq)

    def zero_state(self):
        n = self.n_o
        return np.zeros((self.Nq, self.n_ff, self.n_ff, n, n, n, n), dtype=np.complex128)


# ----------------------------------------------------------------------------
# loops
# ----------------------------------------------------------------------------

def _neumaier_add(acc, comp, x):
    """acc + x with the lost low part added to comp (Neumaier's compensated
    summation, applied to the real and imaginary parts alike)."""
    t = acc + x
    big = np.abs(acc.real) >= np.abs(x.real)
    cr = np.where(big, (acc.real - t.real) + x.real, (x.real - t.real) + acc.real)
    big = np.abs(acc.imag) >= np.abs(x.imag)
    ci = np.where(big, (acc.imag - t.imag) + x.imag, (x.imag - t.imag) + acc.imag)
    return t, comp + (cr + 1j * ci)


def loop_matrix(st, channel, qi, lam, deriv=True, k_chunk=4096):
    """Orbital loop matrix [iR1, iR2, t1, t2, t3, t4] at coarse q index qi.
    The k sum runs over chunks of the fine mesh; the chunk sums are added with
    Neumaier compensation."""
    n = st.n_o
    qf = st.coarse[qi] * st.n_ref
    diffs = {}
    for R1 in st.S:
        for R2 in st.S:
            d = tuple(int(x) for x in (R1 - R2))
            diffs[d] = None
    dlist = list(diffs.keys())
    dR = np.array(dlist, dtype=np.int64)
    acc = np.zeros((len(dlist), n, n, n, n), dtype=np.complex128)
    comp = np.zeros_like(acc)
    for k0 in range(0, st.Nf, k_chunk):
        kk = np.arange(k0, min(k0 + k_chunk, st.Nf))
        nk = st.fine[kk]
        if channel == "pp":
            kp = (qf[None, :] - nk) % st.Lf
        else:
            kp = (nk - qf[None, :]) % st.Lf
        kpi = kp[:, 0] * st.Lf + kp[:, 1]
        if channel == "pp":
            # L-(e_m(s-k), e_n(k)); Pi_m(s-k)_{t1t3} Pi_n(k)_{t2t4}
            Lmn = cutoff.loop_pp(st.e[kpi][:, :, None], st.e[kk][:, None, :],
                                 lam, st.scheme, deriv).reshape(len(kk), n, n)
            W = np.einsum("kmn,knbd->kmbd", Lmn, st.Pi[kk])
            M = np.einsum("kmac,kmbd->kabcd", st.Pi[kpi], W)
        else:
            # L+(e_m(k), e_n(k-u)); Pi_m(k)_{t1t3} Pi_n(k-u)_{t4t2}
            Lmn = cutoff.loop_ph(st.e[kk][:, :, None], st.e[kpi][:, None, :],
                                 lam, st.scheme, deriv).reshape(len(kk), n, n)
            W = np.einsum("kmn,kndb->kmbd", Lmn, st.Pi[kpi])
            M = np.einsum("kmac,kmbd->kabcd", st.Pi[kk], W)
        kr = (nk @ dR.T) % st.Lf
        ph = np.exp(-2j * np.pi * kr / st.Lf)  # f_R1(k) f*_R2(k) = e^{-ik.(R1-R2)}
        acc, comp = _neumaier_add(acc, comp, np.einsum("kr,kabcd->rabcd", ph, M))
    acc = (acc + comp) / st.Nf
    out = np.zeros((st.n_ff, st.n_ff, n, n, n, n), dtype=np.complex128)
    for i, R1 in enumerate(st.S):
        for j, R2 in enumerate(st.S):
            out[i, j] = acc[dlist.index(tuple(int(x) for x in (R1 - R2)))]
    return out


def loops(st, channel, lam, deriv=True, q_list=None):
    """Loop matrices at every coarse q (or at the listed q indices)."""
    q_list = range(st.Nq) if q_list is None else q_list
    return np.stack([loop_matrix(st, channel, qi, lam, deriv) for qi in q_list])


# ----------------------------------------------------------------------------
# projections
# ----------------------------------------------------------------------------

def to_real_space(st, X):
    """X(R'') = 1/N_q sum_q exp(i q.R'') X(q) for every R'' in D (dict by
    residue; Sec. 3.3), all R'' at once as one product of the phase matrix
    [R''][q] with X viewed as [q][rest]."""
    keys = list(st.D.keys())
    ph = np.stack([st.coarse_phase(st.D[r]) for r in keys])
    Xr = (ph @ X.reshape(st.Nq, -1)) / st.Nq
    return {r: Xr[i].reshape(X.shape[1:]) for i, r in enumerate(keys)}


def _swap34(X):
    return np.swapaxes(X, -1, -2)


def projected_vertices(st, P, C, q_list=None):
    """VP = P[V0] + P + P[V^C] + P[V^D];  VC = C[V0] + C[V^P] + C + C[V^D].

    A non-local initial interaction given in crossed particle-hole form (st.C0)
    is projected with the flowing C: V^C -> V^C + C0, V^D -> V^D + D0; one given
    in particle-particle form (st.P0) with the flowing P: V^P -> V^P + P0.
    q_list: evaluate the vertices at these coarse q only (the real-space
    coefficients always sum over every q)."""
    if st.C0 is not None:
        C = C + st.C0
    if st.P0 is not None:
        P = P + st.P0
    Pr = to_real_space(st, P)
    Cr = to_real_space(st, C)
    qs = np.arange(st.Nq) if q_list is None else np.asarray(q_list, dtype=np.int64)
    VP = P[qs].copy()
    VC = C[qs].copy()
    VP[:, 0, 0] += st.V0
    VC[:, 0, 0] += st.V0
    for i, R in enumerate(st.S):
        for j, Rp in enumerate(st.S):
            phRp = st.coarse_phase(Rp)[qs]
            for r, R2 in st.D.items():
                ph = st.coarse_phase(R2)[qs][:, None, None, None, None]
                # P[V^C]: sum_R'' e^{is.R''} C^{R+R'', R'-R''}_{n1n2n3n4}(R'')
                a, b = st.ff_index(R + R2), st.ff_index(Rp - R2)
                if a >= 0 and b >= 0:
                    VP[:, i, j] += ph * Cr[r][a, b][None]
                # P[V^D]: -e^{is.R'} sum_R'' e^{is.R''} C^{R+R'', -R'-R''}_{n1n2n4n3}(R'')
                a, b = st.ff_index(R + R2), st.ff_index(-Rp - R2)
                if a >= 0 and b >= 0:
                    VP[:, i, j] -= phRp[:, None, None, None, None] * ph * _swap34(Cr[r][a, b])[None]
                # C[V^P]: sum_R'' e^{iu.R''} P^{R+R'', R'-R''}_{n1n2n3n4}(R'')
                a, b = st.ff_index(R + R2), st.ff_index(Rp - R2)
                if a >= 0 and b >= 0:
                    VC[:, i, j] += ph * Pr[r][a, b][None]
            # C[V^D]: -sum_R'' e^{iu.R''} C^{R-R'+R'', R''}_{n1n2n4n3}(-R')
            rneg = st._res(-Rp)
            for b, R2 in enumerate(st.S):
                a = st.ff_index(R - Rp + R2)
                if a >= 0:
                    ph = st.coarse_phase(R2)[qs][:, None, None, None, None]
                    VC[:, i, j] -= ph * _swap34(Cr[rneg][a, b])[None]
    return VP, VC


# ----------------------------------------------------------------------------
# right-hand side
# ----------------------------------------------------------------------------

def bundle_pp(VP, Lpp):
    """dP^{RR'}_{s1s2s3s4} = sum VP^{R R1}_{s1s2t1t2} Lpp^{R1R2}_{t1t2t3t4} VP^{R2R'}_{t4t3s3s4}."""
    return np.einsum("xyzabij,xzwijkl,xwvlkcd->xyvabcd", VP, Lpp, VP, optimize="greedy")


def bundle_ph(VC, Lph):
    """dC^{RR'}_{s1s2s3s4} = 2 sum VC^{R R1}_{s1t2s3t1} Lph^{R1R2}_{t1t2t3t4} VC^{R2R'}_{t3s2t4s4}."""
    return 2.0 * np.einsum("xyzajci,xzwijkl,xwvkbld->xyvabcd", VC, Lph, VC, optimize="greedy")


def rhs(st, lam, P, C, flow_P=True, flow_C=True, q_list=None, loops_pp=None, loops_ph=None):
    """Right-hand side (dP/dLambda, dC/dLambda) of the matrix RGE, at every
    coarse q or at the listed ones (the projections still sum over every q).
    loops_pp, loops_ph: the loop matrices at those q, if already computed."""
    VP, VC = projected_vertices(st, P, C, q_list)
    if flow_P:
        Lpp = loops(st, "pp", lam, q_list=q_list) if loops_pp is None else loops_pp
        dP = bundle_pp(VP, Lpp)
    else:
        dP = np.zeros_like(VP)
    if flow_C:
        Lph = loops(st, "ph", lam, q_list=q_list) if loops_ph is None else loops_ph
        dC = bundle_ph(VC, Lph)
    else:
        dC = np.zeros_like(VC)
    return dP, dC


def d_from_c(C):
    """D_{n1n2n3n4} = -C_{n1n2n4n3} (Sec. 3.2, antisymmetry of the ph terms)."""
    return -_swap34(C)


# ----------------------------------------------------------------------------
# integration
# ----------------------------------------------------------------------------

def log_grid(lam0, lam_end, n):
    return lam0 * (lam_end / lam0) ** (np.arange(n + 1) / n)


def _maxabs(P, C):
    return max(float(np.abs(P).max()), float(np.abs(C).max()))


def _lambda_c(l0, m0, l1, m1, v_max):
    t = (v_max - m0) / (m1 - m0)
    return float(np.exp(np.log(l0) + t * (np.log(l1) - np.log(l0))))


def flow_euler(st, lam0, lam_end, n_steps, v_max=50.0, flow_P=True, flow_C=True,
               P=None, C=None):
    """Explicit Euler in Lambda on the log grid Lambda_i = Lambda0 (Lend/Lambda0)^(i/n)."""
    P = st.zero_state() if P is None else P.copy()
    C = st.zero_state() if C is None else C.copy()
    grid = log_grid(lam0, lam_end, n_steps)
    res = dict(lambda_stop=lam_end, lambda_c=0.0, diverged=0, n_steps=0, n_rhs=0,
               trajectory=[(lam0, _maxabs(P, C))])
    for i in range(n_steps):
        dP, dC = rhs(st, grid[i], P, C, flow_P, flow_C)
        res["n_rhs"] += 1
        h = grid[i + 1] - grid[i]
        P = P + h * dP
        C = C + h * dC
        m = _maxabs(P, C)
        if not np.isfinite(m):
            raise FloatingPointError(f"non-finite state after step {i}")
        res["n_steps"] += 1
        lam_prev, m_prev = res["trajectory"][-1]
        res["trajectory"].append((grid[i + 1], m))
        if m > v_max:
            res.update(diverged=1, lambda_stop=float(grid[i + 1]),
                       lambda_c=_lambda_c(lam_prev, m_prev, grid[i + 1], m, v_max))
            break
    res["max_coupling"] = res["trajectory"][-1][1]
    return P, C, res


def flow_dp54(st, lam0, lam_end, rtol=1e-6, atol=1e-6, v_max=50.0, h0=0.05,
              flow_P=True, flow_C=True, max_steps=100000):
    """Dormand-Prince 5(4) in l = ln Lambda with dX/dl = Lambda dX/dLambda.

    Error norm: max over real and imaginary parts of
    |err| / (atol + rtol max(|X|, |X_new|)); step factor
    clip(0.9 err^(-1/5), 0.2, 5); the last step is clipped to Lambda_end.
    """
    P = st.zero_state()
    C = st.zero_state()
    l, l_end = np.log(lam0), np.log(lam_end)
    h = -abs(h0) if l_end < l else abs(h0)

    def f(lv, P_, C_):
        lam = np.exp(lv)
        dP, dC = rhs(st, lam, P_, C_, flow_P, flow_C)
        return lam * dP, lam * dC

    res = dict(lambda_stop=lam_end, lambda_c=0.0, diverged=0, n_steps=0, n_rhs=0,
               n_reject=0, trajectory=[(lam0, 0.0)])
    k1 = f(l, P, C)
    res["n_rhs"] += 1
    while (l_end - l) * np.sign(h) > 1e-14:
        if (l + h - l_end) * np.sign(h) > 0:
            h = l_end - l
        ks = [k1]
        for s in range(1, 7):
            Ps = P + h * sum(a * kk[0] for a, kk in zip(_DP_A[s], ks))
            Cs = C + h * sum(a * kk[1] for a, kk in zip(_DP_A[s], ks))
            ks.append(f(l + _DP_C[s] * h, Ps, Cs))
            res["n_rhs"] += 1
        Pn, Cn = Ps, Cs  # stage 7 is the 5th-order solution (FSAL)
        eP = h * sum((b5 - b4) * kk[0] for b5, b4, kk in zip(_DP_B5, _DP_B4, ks))
        eC = h * sum((b5 - b4) * kk[1] for b5, b4, kk in zip(_DP_B5, _DP_B4, ks))
        err = 0.0
        for e_, x0, x1 in ((eP, P, Pn), (eC, C, Cn)):
            for part in (np.real, np.imag):
                sc = atol + rtol * np.maximum(np.abs(part(x0)), np.abs(part(x1)))
                err = max(err, float(np.max(np.abs(part(e_)) / sc)))
        if not np.isfinite(err):
            raise FloatingPointError("non-finite error estimate")
        fac = 5.0 if err == 0.0 else min(5.0, max(0.2, 0.9 * err ** -0.2))
        if err <= 1.0:
            lam_prev, m_prev = res["trajectory"][-1]
            l = l + h
            P, C, k1 = Pn, Cn, ks[6]
            m = _maxabs(P, C)
            res["n_steps"] += 1
            res["trajectory"].append((float(np.exp(l)), m))
            if m > v_max:
                res.update(diverged=1, lambda_stop=float(np.exp(l)),
                           lambda_c=_lambda_c(lam_prev, m_prev, float(np.exp(l)), m, v_max))
                break
        else:
            res["n_reject"] += 1
        h = h * fac
        if abs(h) < 1e-12:
            raise FloatingPointError("step size underflow")
        if res["n_steps"] + res["n_reject"] > max_steps:
            raise RuntimeError("too many steps")
    res["max_coupling"] = res["trajectory"][-1][1]
    return P, C, res
