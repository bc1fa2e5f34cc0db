"""Writes hubbard_s5_L8_flow.json: the oracle's 200-step explicit Euler flow
of the single-band Hubbard workload (t = 1, t' = -0.25, 0.9 electrons per
site, U = 3, five form factors, 8 x 8 coarse mesh refined 12 x, temperature
cutoff 10 -> 1e-3; Sec. 3.1 matrix RGE, Sec. 3.3 projections, Sec. 5 onsite
interaction).  Calls only oracle/ (and the seeded workload definition of
synth/); the GPU library is never imported.

Stored: the stopping step, divergence flag, critical scale and the max-coupling
trajectory; per coarse q the Frobenius norms of P, C and the third channel D
(Sec. 3.2, D_{n1n2n3n4} = -C_{n1n2n4n3}, in the layout of C); 512 entries of
each at indices drawn from default_rng(0) in the bundle layout [Nq][B][B].

    python tests/golden/make_hubbard_s5_L8_flow.py
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import tufrg as otu  # noqa: E402
from synth import workload  # noqa: E402
from tests._layout import c_to_matrix, p_to_matrix  # noqa: E402


def main():
    w = workload("hubbard_s5_L8")
    st = otu.TUSetup.from_workload(w)
    P, C, res = otu.flow_euler(st, w["lam0"], w["lam_end"], w["n_steps"], v_max=w["v_max"])
    Pm, Cm, Dm = p_to_matrix(P), c_to_matrix(C), c_to_matrix(otu.d_from_c(C))
    rng = np.random.default_rng(0)
    idx = rng.choice(Pm.size, size=512, replace=False)
    out = dict(
        workload=w["name"], n_steps_grid=w["n_steps"], lam0=w["lam0"], lam_end=w["lam_end"], v_max=w["v_max"],
        n_steps=res["n_steps"], diverged=res["diverged"], lambda_stop=res["lambda_stop"],
        lambda_c=res["lambda_c"], max_coupling=res["max_coupling"],
        trajectory=[[float(a), float(b)] for a, b in res["trajectory"]],
        index=[int(i) for i in idx],
        P=[[float(Pm.flat[i].real), float(Pm.flat[i].imag)] for i in idx],
        C=[[float(Cm.flat[i].real), float(Cm.flat[i].imag)] for i in idx],
        D=[[float(Dm.flat[i].real), float(Dm.flat[i].imag)] for i in idx],
        P_norm_q=[float(x) for x in np.linalg.norm(Pm.reshape(Pm.shape[0], -1), axis=1)],
        C_norm_q=[float(x) for x in np.linalg.norm(Cm.reshape(Cm.shape[0], -1), axis=1)],
        D_norm_q=[float(x) for x in np.linalg.norm(Dm.reshape(Dm.shape[0], -1), axis=1)],
        P_max=float(np.abs(Pm).max()), C_max=float(np.abs(Cm).max()), D_max=float(np.abs(Dm).max()),
    )
    with open(os.path.join(HERE, "hubbard_s5_L8_flow.json"), "w") as f:
        json.dump(out, f, indent=0)
    print("n_steps", res["n_steps"], "diverged", res["diverged"], "lambda_c", res["lambda_c"])


if __name__ == "__main__":
    main()
