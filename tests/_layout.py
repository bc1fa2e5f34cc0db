"""Conversions between the paper's tensor order and the matrix layout of the
HIP library's exchange propagators (test helper).

Tensor order (oracle): X[q, iR, iR', n1, n2, n3, n4] = X^{RR'}_{n1n2n3n4}(q).
Matrix layout (library), B = n_ff * n_o^2, flat index r * n_o^2 + a * n_o + b:
  P[q, (R, n1, n2), (R', n4, n3)] = P^{RR'}_{n1n2n3n4}(q)
  C[q, (R, n1, n3), (R', n4, n2)] = C^{RR'}_{n1n2n3n4}(q)
In these layouts the matrix RGE is a plain product of B x B matrices per q.
"""

import numpy as np

# tensor axes: 0 q, 1 R, 2 R', 3 n1, 4 n2, 5 n3, 6 n4
_P_AXES = (0, 1, 3, 4, 2, 6, 5)
_C_AXES = (0, 1, 3, 5, 2, 6, 4)


def _inv(axes):
    inv = [0] * len(axes)
    for i, a in enumerate(axes):
        inv[a] = i
    return tuple(inv)


def p_to_matrix(P):
    nq, nf, _, n = P.shape[:3] + (P.shape[3],)
    return np.ascontiguousarray(P.transpose(_P_AXES)).reshape(nq, nf * n * n, nf * n * n)


def c_to_matrix(C):
    nq, nf, n = C.shape[0], C.shape[1], C.shape[3]
    return np.ascontiguousarray(C.transpose(_C_AXES)).reshape(nq, nf * n * n, nf * n * n)


def p_from_matrix(M, n_ff, n_o):
    nq = M.shape[0]
    T = M.reshape(nq, n_ff, n_o, n_o, n_ff, n_o, n_o)
    return np.ascontiguousarray(T.transpose(_inv(_P_AXES)))


def c_from_matrix(M, n_ff, n_o):
    nq = M.shape[0]
    T = M.reshape(nq, n_ff, n_o, n_o, n_ff, n_o, n_o)
    return np.ascontiguousarray(T.transpose(_inv(_C_AXES)))


def pp_loop_to_matrix(Lt):
    """Loop tensor [q, R1, R2, t1, t2, t3, t4] (oracle order) to the B x B matrix
    sandwiched by the P layout: rows (R1, t2, t1), columns (R2, t4, t3)."""
    nq, nf, n = Lt.shape[0], Lt.shape[1], Lt.shape[3]
    return np.ascontiguousarray(Lt.transpose(0, 1, 4, 3, 2, 6, 5)).reshape(nq, nf * n * n, nf * n * n)


def ph_loop_to_matrix(Lt):
    """Loop tensor [q, R1, R2, t1, t2, t3, t4] to the matrix sandwiched by the C
    layout: rows (R1, t1, t2), columns (R2, t3, t4)."""
    nq, nf, n = Lt.shape[0], Lt.shape[1], Lt.shape[3]
    return np.ascontiguousarray(Lt.transpose(0, 1, 3, 4, 2, 5, 6)).reshape(nq, nf * n * n, nf * n * n)


def u_to_matrix(Um):
    """U matrix [q, R, R', s1, s2, n1, n2] to the pp basis matrix of the bundle
    layout: M[(R, a, b), (R', c, d)] = U^{RR'}_{b a d c}."""
    nq, nf, n = Um.shape[0], Um.shape[1], Um.shape[3]
    return np.ascontiguousarray(Um.transpose(0, 1, 4, 3, 2, 6, 5)).reshape(nq, nf * n * n, nf * n * n)


def x_to_matrix(Xm):
    """X matrix [q, R, R', s1, s2, n1, n2] to the ph basis matrix of the bundle
    layout: M[(R, a, b), (R', c, d)] = X^{RR'}_{a b c d}."""
    nq, nf, n = Xm.shape[0], Xm.shape[1], Xm.shape[3]
    return np.ascontiguousarray(Xm.transpose(0, 1, 3, 4, 2, 5, 6)).reshape(nq, nf * n * n, nf * n * n)
