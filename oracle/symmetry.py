"""Point-group-symmetrised form factors (oracle; test infrastructure).

The plane-wave form factors f_R(k) = exp(-i k.R) of a set S closed under the
square lattice's point group C4v can be recombined into functions that
transform under an irreducible representation: f~_i = sum_R W_iR f_R with W
unitary.  A propagator then changes by X~ = W X W^dagger in the form-factor
indices (orbital indices untouched): from V = sum_RR' f*_R(k) f_R'(k') X^{RR'}
and f_R = sum_i conj(W_iR) f~_i.

W is built here with the projection operators of C4v, P_G = (d_G / 8) sum_g
chi_G(g) D(g), acting on the orbits of S (D(g) e_R = e_{gR}, since
f_R(g^-1 k) = f_{gR}(k) for an orthogonal g), then orthonormalised.
Conventions that fix the remaining freedom: orbits in order of first
appearance in S; inside an orbit the irreducible representations in the order
A1, A2, B1, B2, E; the two partners of E as an x-like function (odd under
x -> -x, even under y -> -y) and then a y-like one; every row's first nonzero
coefficient (in the order of S) real and positive.  Orbits of eight vectors
(two E copies) are not handled.
"""

import numpy as np

A1, A2, B1, B2, EX, EY = 0, 1, 2, 3, 4, 5


def c4v():
    """The 8 operations as integer 2x2 matrices, with their class labels."""
    r = np.array([[0, -1], [1, 0]])
    mx = np.array([[-1, 0], [0, 1]])  # x -> -x
    ops, cls = [], []
    for k in range(4):
        g = np.linalg.matrix_power(r, k)
        ops.append(g)
        cls.append(["E", "C4", "C2", "C4"][k])
    for k in range(4):
        g = np.linalg.matrix_power(r, k) @ mx
        ops.append(g)
        # mirrors: x -> -x and y -> -y are sigma_v, the diagonals sigma_d
        cls.append("sv" if k % 2 == 0 else "sd")
    return ops, cls


CHAR = {  # characters per class E, C2, C4, sv, sd
    A1: {"E": 1, "C2": 1, "C4": 1, "sv": 1, "sd": 1},
    A2: {"E": 1, "C2": 1, "C4": 1, "sv": -1, "sd": -1},
    B1: {"E": 1, "C2": 1, "C4": -1, "sv": 1, "sd": -1},
    B2: {"E": 1, "C2": 1, "C4": -1, "sv": -1, "sd": 1},
    EX: {"E": 2, "C2": -2, "C4": 0, "sv": 0, "sd": 0},
}


def _index(S):
    return {tuple(int(v) for v in R): i for i, R in enumerate(S)}


def _image(idx, g, R):
    t = tuple(int(v) for v in g @ np.asarray(R))
    if t not in idx:
        raise ValueError("the set is not a union of C4v orbits")
    return idx[t]


def _D(S, g):
    """Permutation matrix of g on the plane waves of S: e_R -> e_{gR}."""
    idx = _index(S)
    n = len(S)
    D = np.zeros((n, n))
    for i, R in enumerate(S):
        D[_image(idx, g, R), i] = 1.0
    return D


def orbits(S):
    idx = _index(S)
    ops, _ = c4v()
    seen, out = set(), []
    for R in S:
        t = tuple(int(v) for v in R)
        if t in seen:
            continue
        orb = sorted({_image(idx, g, R) for g in ops})
        seen.update(tuple(int(v) for v in S[i]) for i in orb)
        out.append(orb)
    return out


def symmetric_ff(S):
    """W [n_ff, n_ff] (rows = symmetrised form factors) and the irrep label of each row."""
    S = np.asarray(S, dtype=np.int64).reshape(-1, 2)
    n = len(S)
    ops, cls = c4v()
    Ds = [_D(S, g) for g in ops]
    mirror_x = _D(S, np.array([[-1, 0], [0, 1]]))
    mirror_y = _D(S, np.array([[1, 0], [0, -1]]))
    rows, labels = [], []
    for orb in orbits(S):
        if len(orb) == 8:
            raise ValueError("orbits of eight form factors are not handled")
        basis = np.eye(n)[:, orb]
        for G in (A1, A2, B1, B2, EX):
            d = 2 if G == EX else 1
            Pg = sum(CHAR[G][c] * D for c, D in zip(cls, Ds)) * d / 8.0
            vecs = Pg @ basis
            if G == EX:
                for lab, sx, sy in ((EX, -1, 1), (EY, 1, -1)):
                    part = (np.eye(n) + sx * mirror_x) @ (np.eye(n) + sy * mirror_y) @ vecs / 4.0
                    rows, labels = _add(rows, labels, part, lab)
            else:
                rows, labels = _add(rows, labels, vecs, G)
    W = np.array(rows, dtype=np.complex128)
    if W.shape != (n, n):
        raise ValueError("the set is not a union of C4v orbits")
    return W, np.array(labels)


def _add(rows, labels, vecs, label):
    """Gram-Schmidt of the columns of vecs against the rows so far; sign fixed."""
    for v in vecs.T:
        w = v.astype(np.complex128)
        for r in rows:
            w = w - np.vdot(r, w) * r
        nrm = np.linalg.norm(w)
        if nrm < 1e-9:
            continue
        w = w / nrm
        first = w[np.flatnonzero(np.abs(w) > 1e-12)[0]]
        w = w * (abs(first) / first)
        rows = rows + [w]
        labels = labels + [label]
    return rows, labels


def to_symmetric(X, W):
    """X~[q, i, j, ...] = sum_RR' W_iR X[q, R, R', ...] conj(W_jR')."""
    return np.einsum("iR,qRP...,jP->qij...", W, X, W.conj(), optimize=True)


def from_symmetric(Xs, W):
    return np.einsum("iR,qij...,jP->qRP...", W.conj(), Xs, W, optimize=True)
