"""Band data of the single-particle Hamiltonian (oracle; test infrastructure).

e_l(k) = E_l(k) - mu are the eigenvalues of H(k) measured from the chemical
potential and U(k) the unitary that diagonalises H(k) (Sec. 4.1, the
transformation between orbital and band basis).  The orbital-basis loops only
need the band projectors Pi_l(k)_{ab} = U_{al}(k) U*_{bl}(k), whose sums over
degenerate bands do not depend on the eigenvector gauge.
"""

import numpy as np


def mesh(L):
    """Integer coordinates of the L x L Gamma-centred mesh, index ix * L + iy."""
    ix, iy = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    return np.stack([ix.ravel(), iy.ravel()], axis=1)


def bloch_hamiltonian(hop_R, hop_t, L):
    """H(k) = sum_R t(R) exp(i k.R) on the L x L mesh, [L*L, n_o, n_o]."""
    n = mesh(L)
    # k.R = 2 pi (n.R) / L, reduced mod L before the exponential
    kr = (n @ np.asarray(hop_R, dtype=np.int64).T) % L
    ph = np.exp(2j * np.pi * kr / L)
    return np.einsum("kr,rab->kab", ph, hop_t)


def band_data(hop_R, hop_t, mu, L):
    """Return e [L*L, n_b] (E - mu, ascending) and U [L*L, n_o, n_b]."""
    H = bloch_hamiltonian(hop_R, hop_t, L)
    E, U = np.linalg.eigh(H)
    return E - mu, U


def projectors(U):
    """Pi[k, l, a, b] = U[k, a, l] conj(U[k, b, l])."""
    return np.einsum("kal,kbl->klab", U, U.conj())
