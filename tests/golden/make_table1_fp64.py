"""Writes tests/golden/table1_fp64_oracle.txt: the FP64 counterpart of the paper's Table I,
computed with the oracle only.

Table I (Sec. III-C) reports eps_r = ||c_reg - c_fast||_2 / ||c_reg||_2 between the regular
implementation (every product with the explicit L x L matrix) and the fast one (2D FFTs,
eq. (23)) of ISTA, FISTA and ADMM, at the sweep geometry (51 x 16 URA, 40 elements with the
aperture preserved, L2 = 32, L1 in {64, 128, 256, 512}, 15 dB, K ~ U{1..10}), for
n_iter in {50, 100, 200, 400}, averaged over 10 trials.  Here both sides run in FP64 (numpy,
as the paper's CPU runs): regular = G x with G = D_s^H D_s formed explicitly (and, for ADMM,
the explicit (G + rho I)^-1 by the Woodbury identity), fast = eq. (23) with Omega from eq. (21).
The 10 trials share one array (drawn once) and are run as the columns of one matrix, each with
its own tau = 0.1 max |A^H y|.  ADMM uses rho = 40, the Gram's diagonal (the paper gives no
rho); its eps_r is taken on the sparse estimate z (R6).

Usage: python tests/golden/make_table1_fp64.py  (about 15 minutes on 8 cores, ~12 GB of RAM)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import bccb_oracle as O  # noqa: E402
from paper_2509_13592_amd import scenes as S  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "table1_fp64_oracle.txt")
L1S = (64, 128, 256, 512)
NITER = (50, 100, 200, 400)
RHO = 40.0


def run(L1, trials=10):
    scs = S.paper_sweep_trials(L1, trials)
    mask, L2 = scs[0].mask, scs[0].L2
    op = O.Operator(mask, L1, L2)
    Y = np.stack([sc.y.astype(np.complex64).astype(np.complex128) for sc in scs], axis=1)   # [M][n]
    Bm = np.stack([op.adjoint(Y[:, j]) for j in range(trials)], axis=1)                        # [L][n]
    tau = np.array([float(np.float32(0.1 * np.abs(Bm[:, j]).max())) for j in range(trials)])[None, :]
    mu = O.step_size(op)
    G = O.gram_dense(mask, L1, L2)
    Om = O.bccb_eigenvalues(mask, L1, L2)
    res = {}
    for name, solver in (("ISTA", O.ista), ("FISTA", O.fista)):
        got = {}
        for tag, apply in (("reg", lambda X: G @ X), ("fast", lambda X: O.fft_matvec_columns(Om, X))):
            snaps = {}
            t = [0]

            def trace(c, snaps=snaps, t=t):
                t[0] += 1
                if t[0] in NITER:
                    snaps[t[0]] = c.copy()

            solver(apply, Bm, mu, tau, max(NITER), trace=trace)
            got[tag] = snaps
        res[name] = [float(np.mean([np.linalg.norm(got["reg"][n][:, j] - got["fast"][n][:, j]) /
                                    np.linalg.norm(got["reg"][n][:, j]) for j in range(trials)])) for n in NITER]
    del G
    Minv = O.shifted_inverse_dense(op, RHO)
    spec = 1.0 / (Om + RHO)
    got = {}
    for tag, apply in (("reg", lambda X: Minv @ X), ("fast", lambda X: O.fft_matvec_columns(spec, X))):
        snaps = {}
        t = [0]

        def trace(z, c, v, snaps=snaps, t=t):
            t[0] += 1
            if t[0] in NITER:
                snaps[t[0]] = z.copy()

        O.admm(apply, Bm, RHO, tau, max(NITER), trace=trace)
        got[tag] = snaps
    res["ADMM"] = [float(np.mean([np.linalg.norm(got["reg"][n][:, j] - got["fast"][n][:, j]) /
                                  max(np.linalg.norm(got["reg"][n][:, j]), 1e-300) for j in range(trials)]))
                   for n in NITER]
    return res


def main():
    table = {}
    for L1 in L1S:
        t0 = time.time()
        table[L1] = run(L1)
        print(f"L1 = {L1}: {time.time() - t0:.0f} s", {k: [f'{v:.2e}' for v in vs] for k, vs in table[L1].items()},
              flush=True)
    with open(OUT, "w") as f:
        f.write("# FP64 eps_r = ||c_reg - c_fast|| / ||c_reg|| between the explicit-matrix and the FFT (eq. (23))\n"
                "# implementations, mean of 10 trials, written by tests/golden/make_table1_fp64.py from the oracle\n"
                "# only (Table I geometry: 51 x 16 URA, 40 kept with the aperture, L2 = 32, 15 dB, K ~ U{1..10};\n"
                "# ADMM rho = 40, eps_r on z).  Columns: solver n_iter eps(L1=64) eps(L1=128) eps(L1=256) eps(L1=512)\n")
        for name in ("ISTA", "FISTA", "ADMM"):
            for i, n in enumerate(NITER):
                f.write(f"{name:5s} {n:4d} " + " ".join(f"{table[L1][name][i]:.3e}" for L1 in L1S) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
