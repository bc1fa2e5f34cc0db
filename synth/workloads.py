"""Named synthetic workloads: model, form factors, meshes, cutoff, flow grid.

Each workload is a plain dict; every number a consumer needs is resolved here,
so the oracle and the GPU library receive identical bytes.

* ``hubbard_s5_L8``  : single-band Hubbard (t=1, t'=-0.25, 0.9 e/site), U=3,
  5 form factors, 8x8 q-mesh refined 12x, temperature cutoff 10 -> 1e-3,
  200 explicit Euler steps on a log grid, FP64.
* ``rashba_s9_L24``  : lattice Rashba (t=1, mu=-0.4, alpha=0.3), U=2.5,
  9 form factors (bundle dimension 36), 24x24 q-mesh refined 24x,
  Omega cutoff 10 -> 1e-4, Dormand-Prince 5(4) with rtol=atol=1e-6,
  complex FP32 loops.
* ``t2g_s13_L32``    : t2g + SOC (lam=0.2, hoppings from seed 1), Kanamori
  U=2, J=0.3, 13 form factors (bundle dimension 468), 32x32 q-mesh refined 16x,
  temperature cutoff 10 -> 1e-3, 200 Euler steps, BF16-split loops.
* ``t2g_s13_L48``    : the same model on a 48x48 q-mesh (surrogate workload).
* ``rashba_batch32`` : 32 Rashba/Hubbard instances drawn from seed 2.

Small variants (suffix ``_small``) keep the structure at sizes the oracle
finishes in seconds.
"""

import numpy as np

from .models import (
    chemical_potential,
    ff_shell,
    hubbard_hoppings,
    kanamori_V0,
    onsite_V0,
    rashba_hoppings,
    t2g_soc_hoppings,
)

TEMPERATURE = "temperature"
OMEGA = "omega"


def _wl(name, hop, mu, V0, n_ff, Lq, n_ref, cutoff, lam0, lam_end, n_steps,
        prec, rtol=1e-6, atol=1e-6, v_max=50.0):
    hop_R, hop_t = hop
    return dict(
        name=name, hop_R=hop_R, hop_t=hop_t, n_o=hop_t.shape[1], mu=float(mu),
        V0=V0, ff=ff_shell(n_ff), Lq=int(Lq), n_ref=int(n_ref), cutoff=cutoff,
        lam0=float(lam0), lam_end=float(lam_end), n_steps=int(n_steps),
        prec=prec, rtol=rtol, atol=atol, v_max=v_max,
    )


def _hubbard(Lq, n_ref, n_steps=200, name="hubbard_s5_L8"):
    hop = hubbard_hoppings(1.0, -0.25)
    # filling 0.45 of the spin-degenerate band (0.9 electrons per site)
    mu = chemical_potential(*hop, filling=0.45)
    return _wl(name, hop, mu, onsite_V0(3.0), 5, Lq, n_ref, TEMPERATURE,
               10.0, 1e-3, n_steps, "fp64")


def _rashba(Lq, n_ref, name="rashba_s9_L24", prec="fp32"):
    hop = rashba_hoppings(1.0, 0.3)
    return _wl(name, hop, -0.4, onsite_V0(2.5), 9, Lq, n_ref, OMEGA,
               10.0, 1e-4, 0, prec)


def _t2g(Lq, n_ref, name, n_steps=200, prec="bf16x3"):
    hop = t2g_soc_hoppings(0.2, seed=1)
    # four electrons in the six t2g spin-orbitals
    mu = chemical_potential(*hop, filling=4.0 / 6.0, L=256)
    return _wl(name, hop, mu, kanamori_V0(2.0, 0.3), 13, Lq, n_ref,
               TEMPERATURE, 10.0, 1e-3, n_steps, prec)


def batch_instances(n=32, seed=2, n_ref=12):
    """Uneven Rashba/Hubbard instances: per instance, in this order,
    mu ~ U[-1, 0], U ~ U[1.5, 3.5], alpha ~ U[0, 0.5], L_q in {16, 24, 32},
    |S| in {5, 9, 13}; temperature cutoff 10 -> 1e-3, 200 Euler steps, FP32."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        mu = rng.uniform(-1.0, 0.0)
        U = rng.uniform(1.5, 3.5)
        alpha = rng.uniform(0.0, 0.5)
        Lq = int(rng.choice([16, 24, 32]))
        n_ff = int(rng.choice([5, 9, 13]))
        out.append(_wl(f"rashba_batch_{i}", rashba_hoppings(1.0, alpha), mu,
                       onsite_V0(U), n_ff, Lq, n_ref, TEMPERATURE, 10.0, 1e-3,
                       200, "fp32"))
    return out


WORKLOADS = {
    "hubbard_s5_L8": lambda: _hubbard(8, 12),
    "hubbard_s5_small": lambda: _hubbard(6, 3, n_steps=20, name="hubbard_s5_small"),
    "rashba_s9_L24": lambda: _rashba(24, 24),
    "rashba_s9_small": lambda: _rashba(6, 4, name="rashba_s9_small"),
    "t2g_s13_L32": lambda: _t2g(32, 16, "t2g_s13_L32"),
    "t2g_s13_small": lambda: _t2g(9, 2, "t2g_s13_small", n_steps=10),
    "t2g_s13_L48": lambda: _t2g(48, 16, "t2g_s13_L48"),
}


def workload(name):
    """Resolved workload dict by name (see the module docstring)."""
    return WORKLOADS[name]()
