"""Planted-mistake audit of the oracle (test infrastructure, not collected by pytest).

Each entry below plants one plausible mistake (a dropped term, a wrong sign,
index or momentum, a transposed operand, a wrong coefficient) in a copy of
``oracle/`` and runs the CPU pins of the oracle on that copy; every mistake
must make at least one pin fail (or exceed the per-test time limit, which a
broken integrator does by shrinking its steps; four copies run at once, two
BLAS threads each).  Mutations marked
"(equivalent)" change no result on any input the pins can build and are
listed for completeness.

    python tests/oracle_mutations.py            # all, about twenty minutes on 8 cores
    python tests/oracle_mutations.py 3 14       # selected entries
"""

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_TESTS = sorted(f for f in os.listdir(os.path.join(REPO, "tests")) if f.startswith("test_oracle_"))
TESTS = ORACLE_TESTS + ["test_ff_symmetry_host.py"]

MUTATIONS = [
 ("tufrg.py", "VP[:, i, j] += ph * Cr[r][a, b][None]", "VP[:, i, j] += 0 * ph * Cr[r][a, b][None]", "drop P[V^C]"),
 ("tufrg.py", "VP[:, i, j] -= phRp", "VP[:, i, j] += phRp", "sign P[V^D]"),
 ("tufrg.py", "VP[:, i, j] -= phRp[:, None, None, None, None] * ph * _swap34(Cr[r][a, b])[None]",
              "VP[:, i, j] -= phRp[:, None, None, None, None] * ph * Cr[r][a, b][None]", "no swap34 in P[V^D]"),
 ("tufrg.py", "VP[:, i, j] -= phRp[:, None, None, None, None] * ph", "VP[:, i, j] -= ph", "no e^{is.R'} in P[V^D]"),
 ("tufrg.py", "VC[:, i, j] += ph * Pr[r][a, b][None]", "VC[:, i, j] += 0 * ph * Pr[r][a, b][None]", "drop C[V^P]"),
 ("tufrg.py", "VC[:, i, j] -= ph * _swap34", "VC[:, i, j] += ph * _swap34", "sign C[V^D]"),
 ("tufrg.py", "a = st.ff_index(R - Rp + R2)", "a = st.ff_index(R + Rp + R2)", "index C[V^D]"),
 ("tufrg.py", "rneg = st._res(-Rp)", "rneg = st._res(Rp)", "residue C[V^D]"),
 ("tufrg.py", "VC[:, 0, 0] += st.V0", "VC[:, 0, 0] += 0 * st.V0", "no V0 in VC"),
 ("tufrg.py", "return 2.0 * np.einsum(\"xyzajci", "return 1.0 * np.einsum(\"xyzajci", "ph factor 2"),
 ("tufrg.py", "xwvlkcd->xyvabcd", "xwvklcd->xyvabcd", "pp index order"),
 ("tufrg.py", "ph = np.exp(-2j * np.pi * kr / st.Lf)", "ph = np.exp(2j * np.pi * kr / st.Lf)", "loop phase sign"),
 ("tufrg.py", "kp = (qf[None, :] - nk) % st.Lf", "kp = (qf[None, :] + nk) % st.Lf", "pp partner momentum"),
 ("tufrg.py", "\"kmn,kndb->kmbd\"", "\"kmn,knbd->kmbd\"", "ph projector transposed"),
 ("tufrg.py", "    [44 / 45, -56 / 15, 32 / 9],", "    [44 / 45, -56 / 15, 32 / 8],", "DP tableau entry"),
 ("tufrg.py", "187 / 2100, 1 / 40])", "187 / 2100, 1 / 41])", "DP error weight"),
 ("tufrg.py", "Xr = (ph @ X.reshape(st.Nq, -1)) / st.Nq", "Xr = (ph.conj() @ X.reshape(st.Nq, -1)) / st.Nq", "real-space phase sign"),
 ("cutoff.py", "return -e / (4.0 * lam * lam) / np.cosh(e / (2.0 * lam)) ** 2", "return -e / (4.0 * lam) / np.cosh(e / (2.0 * lam)) ** 2", "K temperature"),
 ("cutoff.py", "return e * (2.0 * a + lam) / (4.0 * (a + lam) ** 2)", "return e * (a + lam) / (4.0 * (a + lam) ** 2)", "J omega"),
 ("cutoff.py", "return -e * (3.0 * a + lam) / (4.0 * (a + lam) ** 3)", "return -e * (3.0 * a + lam) / (4.0 * (a + lam) ** 2)", "K omega"),
 ("cutoff.py", "return -2.0 * lam * e * e / (d * d)", "return -1.0 * lam * e * e / (d * d)", "dchi factor"),
 ("cutoff.py", "return 0.5 * s  # mean", "return 0.6 * s  # mean", "GL mean weight"),
 ("cutoff.py", "return -(1.0 - 2.0 * x * np.tanh(x)) / (4.0 * lam * lam) / np.cosh(x) ** 2", "return -(1.0 - x * np.tanh(x)) / (4.0 * lam * lam) / np.cosh(x) ** 2", "dK/de temperature"),
 ("basis.py", "kp = (qf[None, :] - fine) % Lf if channel", "kp = (qf[None, :] + fine) % Lf if channel", "basis partner"),
 ("basis.py", "lambda kp, k: U[kp].conj())", "lambda kp, k: U[kp])", "X matrix conj"),
 ("basis.py", "\"qABbaji,qACabcd,qCDcdkl->qBDijkl\"", "\"qABabij,qACabcd,qCDcdkl->qBDijkl\"", "p_to_band order"),
 ("basis.py", "\"qABacik,qACabcd,qCDdblj->qBDijkl\"", "\"qABacik,qACabcd,qCDbdlj->qBDijkl\"", "c_to_band order"),
 ("basis.py", "\"qABadil,qACabcd,qCDcbkj->qBDijkl\"", "\"qABadil,qACabcd,qCDbckj->qBDijkl\"", "d_to_band order"),
 ("basis.py", "return np.exp(-2j * np.pi * kr / Lf)", "return np.exp(2j * np.pi * kr / Lf)", "basis phases sign"),
 ("symmetry.py", "(EX, -1, 1), (EY, 1, -1)", "(EX, 1, -1), (EY, -1, 1)", "E partners swapped"),
 # equivalent: rows built from an orbit taken in the order of S already start positive
 ("symmetry.py", "w = w * (abs(first) / first)", "w = w", "sign convention (equivalent)"),
 ("symmetry.py", "cls.append(\"sv\" if k % 2 == 0 else \"sd\")", "cls.append(\"sd\" if k % 2 == 0 else \"sv\")", "mirror classes"),
 ("su2.py", "out[:, :, j] = st.coarse_phase(R)[:, None] * X[:, :, jm]", "out[:, :, j] = X[:, :, jm]", "exchange phase"),
 ("su2.py", "dt = d + m[\"CP_px\"] + m[\"CD_c\"]", "dt = d + m[\"CP_p\"] + m[\"CD_c\"]", "d~ uses p not p^x"),
 ("su2.py", "dd = -2.0 * _mm(_mm(dt, Lph), dt)", "dd = -1.0 * _mm(_mm(dt, Lph), dt)", "dd factor"),
 ("bands.py", "ph = np.exp(2j * np.pi * kr / L)", "ph = np.exp(-2j * np.pi * kr / L)", "Bloch phase sign"),
 ("bands.py", "\"kal,kbl->klab\", U, U.conj()", "\"kal,kbl->klab\", U.conj(), U", "projector transposed"),
 ("mlp.py", "+ x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)", "+ 0.5 * x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)", "GELU derivative"),
 ("mlp.py", "vh = v / (1.0 - beta2 ** t)", "vh = v", "Adam bias correction"),
 ("mlp.py", "d = 2.0 * (Y - T) / (n * n_out)", "d = 2.0 * (Y - T) / n", "loss gradient scale"),
 ("mlp.py", "d = d * gelu_deriv(pre[i])", "d = d * gelu(pre[i])", "backprop activation"),
 ("mlp.py", "y = np.log(np.asarray(s_tab, dtype=np.float64))", "y = np.asarray(s_tab, dtype=np.float64)", "scale table interpolation"),
 ("tufrg.py", "        C = C + st.C0\n", "        C = C\n", "initial C0 not projected"),
 ("tufrg.py", "        P = P + st.P0\n", "        P = P\n", "static P0 not projected"),
 ("tufrg.py", "t = (v_max - m0) / (m1 - m0)", "t = (v_max - m1) / (m1 - m0)", "lambda_c interpolation"),
 ("tufrg.py", "        if m > v_max:\n            res.update(diverged=1, lambda_stop=float(grid[i + 1]),",
              "        if m > 2 * v_max:\n            res.update(diverged=1, lambda_stop=float(grid[i + 1]),", "Euler stop test"),
 ("tufrg.py", "self.Pi = bands.projectors(np.broadcast_to(np.eye(self.n_o), self.U.shape))",
              "self.Pi = bands.projectors(self.U)", "band basis keeps orbital projectors"),
 ("su2.py", "            P[..., a, b, b, a] -= px", "            P[..., a, b, b, a] += px", "SU(2) embedding sign"),
 ("bruteforce.py", "out[p1, :, p3] = 2.0 * np.einsum(", "out[p1, :, p3] = 1.0 * np.einsum(", "brute-force ph factor"),
 ("bruteforce.py", "return -np.swapaxes(phic[i1, i2, k4], -1, -2)", "return np.swapaxes(phic[i1, i2, k4], -1, -2)", "brute-force D sign"),
 ("cutoff.py", "return dchi(e1, lam) * chi(e2, lam) + chi(e1, lam) * dchi(e2, lam)",
               "return dchi(e1, lam) * chi(e2, lam)", "shell product rule"),
]



def run(i):
    f, old, new, name = MUTATIONS[i]
    env = dict(os.environ, OMP_NUM_THREADS="2", OPENBLAS_NUM_THREADS="2", MKL_NUM_THREADS="2")
    with tempfile.TemporaryDirectory(prefix="oracle_mut_") as d:
        for sub in ("oracle", "synth", "tests", "paper_1710_08830_amd"):
            shutil.copytree(os.path.join(REPO, sub), os.path.join(d, sub),
                            ignore=shutil.ignore_patterns("__pycache__"))
        shutil.copy(os.path.join(REPO, "pytest.ini"), d)
        path = os.path.join(d, "oracle", f)
        src = open(path).read()
        if src.count(old) != 1:
            return name, f"NOT APPLIED (pattern found {src.count(old)} times)"
        open(path, "w").write(src.replace(old, new))
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                            "--timeout", "300"] + [f"tests/{t}" for t in TESTS],
                           cwd=d, capture_output=True, text=True, env=env)
    failed = [line[7:] for line in r.stdout.splitlines() if line.startswith("FAILED")]
    last = r.stdout.strip().splitlines()[-1] if r.stdout.strip() else r.stderr.strip()[-200:]
    if r.returncode == 0:
        return name, "SURVIVED " + last
    return name, "caught by " + (failed[0][:90] if failed else last)


def main():
    sel = range(len(MUTATIONS)) if len(sys.argv) < 2 else [int(x) for x in sys.argv[1:]]
    survived = 0
    with cf.ThreadPoolExecutor(4) as ex:
        for name, res in ex.map(run, sel):
            survived += res.startswith("SURVIVED") and "(equivalent)" not in name
            print(f"{name:32s} {res}", flush=True)
    return 1 if survived else 0


if __name__ == "__main__":
    sys.exit(main())
