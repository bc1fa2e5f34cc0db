"""Momentum-space vertex on a tiny lattice (oracle; test infrastructure).

A vertex is an array ``V[k1, k2, k3, n1, n2, n3, n4]`` on one L x L mesh
(index ix * L + iy); the fourth momentum is k4 = k1 + k2 - k3.  This module
writes out the paper's plain definitions:

* the channel projections P^[V], C^[V], D^[V] as double k-sums and their
  converse form-factor expansions (Sec. 2);
* the transformation between orbital and band basis with U(k) (Sec. 4.1);
* the band-basis one-loop right-hand side Phi^pp + Phi^ph,c + Phi^ph,d
  (Sec. 3.1), with the loop kernels of ``cutoff``.

With a complete form-factor set and no mesh refinement the truncated-unity
equations reproduce these exactly, which is what the tests check.
"""

import numpy as np

from . import bands, cutoff


class Lattice:
    def __init__(self, L):
        self.L = L
        self.N = L * L
        self.k = bands.mesh(L)
        kk = self.k
        self.add = np.array([[self.idx(kk[a] + kk[b]) for b in range(self.N)] for a in range(self.N)])
        self.sub = np.array([[self.idx(kk[a] - kk[b]) for b in range(self.N)] for a in range(self.N)])

    def idx(self, n):
        return int(n[0] % self.L) * self.L + int(n[1] % self.L)

    def ff(self, S):
        """f_R(k) = exp(-i k.R) as [n_ff, N]."""
        kr = (np.asarray(S, dtype=np.int64) @ self.k.T) % self.L
        return np.exp(-2j * np.pi * kr / self.L)


def complete_ff(L):
    """All L*L lattice vectors (the complete form-factor set), origin first."""
    return bands.mesh(L).astype(np.int32)


# ---------------------------------------------------------------------------
# projections and expansions (Sec. 2)
# ---------------------------------------------------------------------------

def project_P(lat, V, S):
    """P^[V]_{RR'}(s) = 1/N^2 sum_{k,k'} f_R(k) f*_R'(k') V(k, s-k, s-k', k')."""
    f = lat.ff(S)
    out = []
    for s in range(lat.N):
        sk = lat.sub[s]  # s - k
        W = V[np.arange(lat.N)[:, None], sk[:, None], sk[None, :]]  # [k, k', n...]
        out.append(np.einsum("rk,pl,kl...->rp...", f, f.conj(), W) / lat.N ** 2)
    return np.stack(out)


def project_C(lat, V, S):
    """C^[V]_{RR'}(u) = 1/N^2 sum f_R(k) f*_R'(k') V(k, k'-u, k-u, k')."""
    f = lat.ff(S)
    out = []
    for u in range(lat.N):
        ku = lat.sub[:, u]  # k - u
        W = V[np.arange(lat.N)[:, None], ku[None, :], ku[:, None]]
        out.append(np.einsum("rk,pl,kl...->rp...", f, f.conj(), W) / lat.N ** 2)
    return np.stack(out)


def project_D(lat, V, S):
    """D^[V]_{RR'}(t) = 1/N^2 sum f_R(k) f*_R'(k') V(k, k'-t, k', k-t)."""
    f = lat.ff(S)
    out = []
    for t in range(lat.N):
        kt = lat.sub[:, t]
        W = V[np.arange(lat.N)[:, None], kt[None, :], np.arange(lat.N)[None, :]]
        out.append(np.einsum("rk,pl,kl...->rp...", f, f.conj(), W) / lat.N ** 2)
    return np.stack(out)


def expand_P(lat, X, S):
    """V(k1,k2,k3) = sum_{RR'} f*_R(k1) f_R'(k4) X_{RR'}(k1+k2)."""
    f = lat.ff(S)
    N = lat.N
    V = np.zeros((N, N, N) + X.shape[3:], dtype=np.complex128)
    for k1 in range(N):
        for k2 in range(N):
            s = lat.add[k1, k2]
            k4 = lat.sub[s]  # over k3
            V[k1, k2] = np.einsum("r,pl,rp...->l...", f[:, k1].conj(), f[:, k4], X[s])
    return V


def expand_C(lat, X, S):
    """V(k1,k2,k3) = sum_{RR'} f*_R(k1) f_R'(k4) X_{RR'}(k1-k3)."""
    f = lat.ff(S)
    N = lat.N
    V = np.zeros((N, N, N) + X.shape[3:], dtype=np.complex128)
    for k1 in range(N):
        for k2 in range(N):
            k4 = lat.sub[lat.add[k1, k2]]
            u = lat.sub[k1]  # k1 - k3 over k3
            V[k1, k2] = np.einsum("r,pl,lrp...->l...", f[:, k1].conj(), f[:, k4], X[u])
    return V


def expand_D(lat, X, S):
    """V(k1,k2,k3) = sum_{RR'} f*_R(k1) f_R'(k3) X_{RR'}(k3-k2)."""
    f = lat.ff(S)
    N = lat.N
    V = np.zeros((N, N, N) + X.shape[3:], dtype=np.complex128)
    for k1 in range(N):
        for k2 in range(N):
            t = lat.sub[:, k2]  # k3 - k2 over k3
            V[k1, k2] = np.einsum("r,pl,lrp...->l...", f[:, k1].conj(), f, X[t])
    return V


# ---------------------------------------------------------------------------
# basis change (Sec. 4.1)
# ---------------------------------------------------------------------------

def _k4_table(lat):
    """k4[k1, k2, k3] = k1 + k2 - k3."""
    return lat.sub[lat.add]


def to_band(lat, V, U):
    """V_n = sum U*_{s1n1}(k1) U*_{s2n2}(k2) V_s U_{s3n3}(k3) U_{s4n4}(k4)."""
    N = lat.N
    k4 = _k4_table(lat)
    i1, i2, i3 = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    return np.einsum("xyzae,xyzbf,xyzabcd,xyzcg,xyzdh->xyzefgh",
                     U[i1].conj(), U[i2].conj(), V, U[i3], U[k4], optimize="greedy")


def to_orbital(lat, V, U):
    """Inverse of to_band."""
    N = lat.N
    k4 = _k4_table(lat)
    i1, i2, i3 = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    return np.einsum("xyzae,xyzbf,xyzefgh,xyzcg,xyzdh->xyzabcd",
                     U[i1], U[i2], V, U[i3].conj(), U[k4].conj(), optimize="greedy")


# ---------------------------------------------------------------------------
# band-basis one-loop right-hand side (Sec. 3.1)
# ---------------------------------------------------------------------------

def phi_pp(lat, Vb, e, lam, scheme):
    """-1/N sum_{l1 l2 k} V_{n1n2l1l2}(p1,p2,k) L-_{l1l2}(k, p1+p2-k) V_{l1l2n3n4}(k, p1+p2-k, p3)."""
    N = lat.N
    out = np.zeros_like(Vb)
    kk = np.arange(N)
    for p1 in range(N):
        for p2 in range(N):
            s = lat.add[p1, p2]
            sk = lat.sub[s]
            A = Vb[p1, p2]  # [k, n1, n2, l1, l2]
            Lk = cutoff.loop_pp(e[kk][:, :, None], e[sk][:, None, :], lam, scheme)
            Lk = Lk.reshape(N, e.shape[1], e.shape[1])
            Bm = Vb[kk, sk]  # [k, p3, l1, l2, n3, n4]
            out[p1, p2] = -np.einsum("kabij,kij,kpijcd->pabcd", A, Lk, Bm) / N
    return out


def phi_phc(lat, Vb, e, lam, scheme):
    """2/N sum V_{n1l2n3l1}(p1, k+p3-p1, p3) L+_{l1l2}(k, k+p3-p1) V_{l1n2l2n4}(k, p2, k+p3-p1)."""
    N = lat.N
    out = np.zeros_like(Vb)
    kk = np.arange(N)
    for p1 in range(N):
        for p3 in range(N):
            u = lat.sub[p1, p3]
            kq = lat.sub[kk, u]  # k - u = k + p3 - p1
            A = Vb[p1, kq, p3]  # [k, n1, l2, n3, l1]
            Lk = cutoff.loop_ph(e[kk][:, :, None], e[kq][:, None, :], lam, scheme)
            Lk = Lk.reshape(N, e.shape[1], e.shape[1])
            Bm = Vb[kk[:, None], np.arange(N)[None, :], kq[:, None]]  # [k, p2, l1, n2, l2, n4]
            out[p1, :, p3] = 2.0 * np.einsum("kajci,kij,kpibjd->pabcd", A, Lk, Bm) / N
    return out


def phi_phd(lat, phic):
    """Phi^ph,d_{n1n2n3n4}(p1,p2,p3) = -Phi^ph,c_{n1n2n4n3}(p1,p2,p1+p2-p3)."""
    k4 = _k4_table(lat)
    N = lat.N
    i1, i2, _ = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    return -np.swapaxes(phic[i1, i2, k4], -1, -2)


def orbital_rhs(lat, V, U, e, lam, scheme):
    """Orbital-basis (Phi^pp, Phi^ph,c, Phi^ph,d) of the orbital vertex V."""
    Vb = to_band(lat, V, U)
    pp = to_orbital(lat, phi_pp(lat, Vb, e, lam, scheme), U)
    phc_b = phi_phc(lat, Vb, e, lam, scheme)
    phc = to_orbital(lat, phc_b, U)
    phd = to_orbital(lat, phi_phd(lat, phc_b), U)
    return pp, phc, phd


def antisymmetrize(lat, X):
    """X - X(1<->2) - X(3<->4) + X(1<->2, 3<->4), exchanging momenta and indices."""
    N = lat.N
    k4 = _k4_table(lat)
    i1, i2, i3 = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    Xin = np.swapaxes(X[i2, i1, i3], 3, 4)
    Xout = np.swapaxes(X[i1, i2, k4], 5, 6)
    Xboth = np.swapaxes(np.swapaxes(X[i2, i1, k4], 3, 4), 5, 6)
    return X - Xin - Xout + Xboth
