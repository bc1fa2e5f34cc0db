"""Model inputs: hopping tables, initial interactions, form-factor shells.

Conventions (fixed here once, used by every consumer):

* Lattice vectors are integer pairs (x, y) of the square lattice.
* A hopping table is a pair ``(hop_R, hop_t)`` with ``hop_R`` of shape
  ``[n_hop, 2]`` (int32) and ``hop_t`` of shape ``[n_hop, n_o, n_o]``
  (complex128), such that the Bloch Hamiltonian is
  ``H(k) = sum_R t(R) exp(i k.R)``.  Every table is closed under ``R -> -R``
  with ``t(-R) = t(R)^dagger``, so ``H(k)`` is Hermitian.
* Spin-orbital index of a multi-orbital model is ``orbital * 2 + spin``.
* Initial interactions are antisymmetric tensors ``V0[n1, n2, n3, n4]`` in the
  normalisation ``H_int = 1/2 sum V_{1234} c+_1 c+_2 c_4 c_3`` (the onsite
  Hubbard vertex of the paper's Rashba application, Sec. 5, is
  ``U/2 (d13 d24 - d14 d23)``, which gives ``U n_up n_dn`` in this form).
"""

from functools import lru_cache

import numpy as np

PAULI = np.array(
    [
        [[0, 1], [1, 0]],
        [[0, -1j], [1j, 0]],
        [[1, 0], [0, -1]],
    ],
    dtype=np.complex128,
)

# Plane-wave form-factor shells (Sec. 2: bond picture, truncation at |R_c|).
# Ordered lists, the onsite vector first, every shell closed under R -> -R.
_SHELLS = {
    5: [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)],
    9: [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1),
        (1, 1), (-1, -1), (1, -1), (-1, 1)],
    13: [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1),
         (1, 1), (-1, -1), (1, -1), (-1, 1),
         (2, 0), (-2, 0), (0, 2), (0, -2)],
}


def ff_shell(n):
    """Form-factor bond vectors of the 5-, 9- or 13-vector shell, int32 [n, 2]."""
    return np.array(_SHELLS[n], dtype=np.int32)


def _table(entries, n_o):
    hop_R = np.array([r for r, _ in entries], dtype=np.int32).reshape(-1, 2)
    hop_t = np.array([t for _, t in entries], dtype=np.complex128).reshape(-1, n_o, n_o)
    return hop_R, hop_t


def hubbard_hoppings(t=1.0, tp=-0.25):
    """Spin-degenerate square-lattice band, 2 spin-orbitals.

    Dispersion -2t(cos kx + cos ky) - 4t' cos kx cos ky.
    """
    one = np.eye(2, dtype=np.complex128)
    ent = []
    for r in [(1, 0), (-1, 0), (0, 1), (0, -1)]:
        ent.append((r, -t * one))
    for r in [(1, 1), (-1, -1), (1, -1), (-1, 1)]:
        ent.append((r, -tp * one))
    return _table(ent, 2)


def rashba_hoppings(t=1.0, alpha=0.3, tp=0.0):
    """Lattice-regularised Rashba model (Sec. 5, general two-band form).

    ``H(k) = f(k) 1 + g(k).sigma`` with ``f = -2t(cos kx + cos ky)
    - 4t' cos kx cos ky`` and ``g = alpha(-sin ky, sin kx, 0)``, which is odd
    in k as time-reversal symmetry requires.
    """
    one = np.eye(2, dtype=np.complex128)
    sx, sy = PAULI[0], PAULI[1]
    # sin(k.d) = (e^{ik.d} - e^{-ik.d}) / (2i)
    ent = [
        ((1, 0), -t * one + alpha * sy / 2j),
        ((-1, 0), -t * one - alpha * sy / 2j),
        ((0, 1), -t * one - alpha * sx / 2j),
        ((0, -1), -t * one + alpha * sx / 2j),
    ]
    if tp != 0.0:
        for r in [(1, 1), (-1, -1), (1, -1), (-1, 1)]:
            ent.append((r, -tp * one))
    return _table(ent, 2)


def t2g_soc_hoppings(lam=0.2, seed=1, nn=(0.2, 1.0), nnn=(0.0, 0.2)):
    """Three t2g orbitals (yz, xz, xy) times spin with atomic SOC, 6 spin-orbitals.

    ``h(k) = -sum_d [T(d) e^{ik.d} + T(d)^T e^{-ik.d}]`` over
    ``d in {x, y, x+y, x-y}``; every ``T(d)`` is real symmetric with its upper
    triangle drawn (d-major, row-major) from ``default_rng(seed)``: uniform in
    ``nn`` for the nearest neighbours and in ``nnn`` for the diagonal ones.
    SOC is ``lam * sum_i l_i (x) sigma_i / 2`` with ``(l_i)_{ab} = -i eps_{iab}``.
    """
    rng = np.random.default_rng(seed)
    deltas = [(1, 0), (0, 1), (1, 1), (1, -1)]
    iu = np.triu_indices(3)
    ent = []
    for j, d in enumerate(deltas):
        lo, hi = nn if j < 2 else nnn
        T = np.zeros((3, 3))
        T[iu] = rng.uniform(lo, hi, size=len(iu[0]))
        T = T + np.triu(T, 1).T
        Tf = np.kron(T, np.eye(2))
        ent.append((d, -Tf.astype(np.complex128)))
        ent.append(((-d[0], -d[1]), -Tf.T.astype(np.complex128)))
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1.0
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1.0
    hsoc = np.zeros((6, 6), dtype=np.complex128)
    for i in range(3):
        li = -1j * eps[i]
        hsoc += lam * np.kron(li, PAULI[i]) / 2.0
    ent.append(((0, 0), hsoc))
    return _table(ent, 6)


def onsite_V0(U):
    """Onsite Hubbard vertex of one orbital with spin: (U/2)(d13 d24 - d14 d23)."""
    d = np.eye(2)
    V = 0.5 * U * (np.einsum("ac,bd->abcd", d, d) - np.einsum("ad,bc->abcd", d, d))
    return V.astype(np.complex128)


def kanamori_V0(U, J, n_orb=3):
    """Antisymmetrised onsite Kanamori vertex on ``n_orb`` orbitals times spin.

    ``W_{(a1s1)(a2s2)(a3s3)(a4s4)} = I_{a1a2;a3a4} d_{s1s3} d_{s2s4}`` with
    ``I_{aa;aa}=U``, ``I_{ab;ab}=U-2J``, ``I_{ab;ba}=J``, ``I_{aa;bb}=J``
    (a != b), and ``V0 = (W_{1234} - W_{1243}) / 2``.
    """
    I = np.zeros((n_orb,) * 4)
    for a in range(n_orb):
        for b in range(n_orb):
            if a == b:
                I[a, a, a, a] = U
            else:
                I[a, b, a, b] = U - 2.0 * J
                I[a, b, b, a] = J
                I[a, a, b, b] = J
    n = 2 * n_orb
    W = np.zeros((n,) * 4)
    for i1 in range(n):
        for i2 in range(n):
            for i3 in range(n):
                for i4 in range(n):
                    a1, s1 = divmod(i1, 2)
                    a2, s2 = divmod(i2, 2)
                    a3, s3 = divmod(i3, 2)
                    a4, s4 = divmod(i4, 2)
                    if s1 == s3 and s2 == s4:
                        W[i1, i2, i3, i4] = I[a1, a2, a3, a4]
    V = 0.5 * (W - W.transpose(0, 1, 3, 2))
    return V.astype(np.complex128)


def density_density_c0(Lq, n_o, ff, bonds):
    """Non-local density-density interaction (1/2) sum_i sum_d V_d n_i n_{i+d}
    (n_i summed over all spin-orbitals of cell i) as the static crossed
    particle-hole term of the initial vertex: its antisymmetrised form is
    (1/2) Vt(k1 - k3) d13 d24 - (1/2) Vt(k1 - k4) d14 d23 (the onsite Hubbard
    tensor of ``onsite_V0`` for d = 0), whose first part has the channel form
    C^{00}(u) = (1/2) Vt(u) d13 d24 and whose second is the matching D term.
    ``bonds``: [(d, V_d)] with d != (0, 0), closed under d -> -d with equal V
    (so Vt(u) = sum_d V_d exp(-i u.d) is real).  Returns C0 in the layout
    [Nq][n_ff][n_ff][n_o]^4 of the exchange propagators (only the (0,0)
    form-factor block is nonzero)."""
    ff = np.asarray(ff, dtype=np.int64).reshape(-1, 2)
    i0 = int(np.flatnonzero((ff[:, 0] == 0) & (ff[:, 1] == 0))[0])
    table = {(int(d[0]), int(d[1])): float(v) for d, v in bonds}
    for (dx, dy), v in table.items():
        if (dx, dy) == (0, 0):
            raise ValueError("the onsite term belongs to V0")
        if table.get((-dx, -dy)) != v:
            raise ValueError("bonds must be closed under d -> -d with equal V")
    n = np.arange(Lq)
    qx, qy = np.meshgrid(n, n, indexing="ij")
    qx, qy = qx.reshape(-1), qy.reshape(-1)
    vt = np.zeros(Lq * Lq)
    for (dx, dy), v in table.items():
        vt += v * np.cos(2.0 * np.pi * (qx * dx + qy * dy) / Lq)
    d = np.eye(n_o)
    C0 = np.zeros((Lq * Lq, len(ff), len(ff)) + (n_o,) * 4, dtype=np.complex128)
    C0[:, i0, i0] = 0.5 * vt[:, None, None, None, None] * np.einsum("ac,bd->abcd", d, d)[None]
    return C0


@lru_cache(maxsize=None)
def _mu_cached(key, filling, L, T):
    hop_R, hop_t = _MU_TABLES[key]
    n_o = hop_t.shape[1]
    ks = 2.0 * np.pi * np.arange(L) / L
    kx, ky = np.meshgrid(ks, ks, indexing="ij")
    kv = np.stack([kx.ravel(), ky.ravel()], axis=1)
    ph = np.exp(1j * kv @ hop_R.T.astype(np.float64))
    H = np.einsum("kr,rab->kab", ph, hop_t)
    E = np.linalg.eigvalsh(H)
    lo, hi = E.min() - 1.0, E.max() + 1.0
    target = filling * n_o
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        x = np.clip((E - mid) / T, -700, 700)
        n = np.mean(np.sum(1.0 / (np.exp(x) + 1.0), axis=1))
        if n > target:
            hi = mid
        else:
            lo = mid
        if hi - lo < 1e-13:
            break
    return 0.5 * (lo + hi)


_MU_TABLES = {}


def chemical_potential(hop_R, hop_t, filling, L=512, T=1e-3):
    """Chemical potential at which the fraction ``filling`` of all states is
    occupied (Fermi function at temperature T, L x L k-mesh, bisection)."""
    key = (hop_R.tobytes(), hop_t.tobytes())
    _MU_TABLES[key] = (hop_R, hop_t)
    return float(_mu_cached(key, float(filling), int(L), float(T)))


def random_exchange_state(n_q, n_ff, n_o, seed, scale=1.0):
    """Seeded complex random exchange propagator in tensor form
    ``X[q, R, R', n1, n2, n3, n4]`` (standard normal real and imaginary parts)."""
    rng = np.random.default_rng(seed)
    shape = (n_q, n_ff, n_ff, n_o, n_o, n_o, n_o)
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def random_unitaries(n_k, n, seed):
    """Seeded Haar-random n x n unitaries, [n_k, n, n] (QR of complex Gaussian
    matrices with the phases of R's diagonal moved into Q): an arbitrary gauge
    of band eigenvectors for the basis-change inputs."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n_k, n, n)) + 1j * rng.standard_normal((n_k, n, n))
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=1, axis2=2)
    return Q * (d / np.abs(d))[:, None, :]


def mlp_shape(n_in, width=256, n_out=2 * 6 ** 4, n_hidden=3):
    """Layer sizes of the loop surrogate: n_in -> width (x n_hidden) -> n_out."""
    return [int(n_in)] + [int(width)] * int(n_hidden) + [int(n_out)]


def mlp_init(sizes, seed=3):
    """Seeded initial parameters of an MLP with layer sizes ``sizes``, one flat
    FP32 vector: for each layer the weight matrix W[out][in] (row-major) then
    the bias b[out].  W ~ U(-a, a) with a = sqrt(6 / (in + out)), b = 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for n_i, n_o in zip(sizes[:-1], sizes[1:]):
        a = np.sqrt(6.0 / (n_i + n_o))
        parts.append(rng.uniform(-a, a, size=n_o * n_i))
        parts.append(np.zeros(n_o))
    return np.concatenate(parts).astype(np.float32)


def mlp_batch(n, n_in, n_out, seed):
    """Seeded probe batch (inputs, targets) for surrogate parity tests."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n_in)).astype(np.float32)
    T = (0.5 * rng.standard_normal((n, n_out))).astype(np.float32)
    return X, T


def probe_vector(n, seed, scale=1.0):
    """Seeded FP32 probe vector (e.g. a gradient fed to an optimiser step)."""
    rng = np.random.default_rng(seed)
    return (scale * rng.standard_normal(n)).astype(np.float32)
