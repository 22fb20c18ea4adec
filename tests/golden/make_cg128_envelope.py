"""Write cg128_envelope.txt: the serial oracle's CG on the 27-point matrix at
128^3 (2,097,152 rows), right-hand side U[-1,1) from seed 1, 500 iterations,
run twice -- once with the dots summed naively in index order and once with
Neumaier-compensated dots. The two runs differ only in the rounding of the
dot products; how far their rho_k = r_k.r_k drift apart is the envelope
within which any other correct summation order (the GPU's) may drift from
the compensated run. Also records ||b - A x_500|| / ||b|| of both runs.

    python tests/golden/make_cg128_envelope.py

Calls only the oracle and the seeded input generators (about 40 s per run;
the two runs go on two threads).
"""
import os
import sys
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gf_inputs as gi  # noqa: E402
import oracle  # noqa: E402

M, ITERS, SEED = 128, 500, 1
OUT = os.path.join(HERE, "cg128_envelope.txt")


def main():
    rowptr, col, val = gi.poisson27_csr(M)
    b = gi.cg_rhs(M ** 3, seed=SEED)
    runs = {}

    def run(comp):
        runs[comp] = oracle.cg(rowptr, col, val, b, ITERS, compensated=comp)

    th = [threading.Thread(target=run, args=(c,)) for c in (False, True)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    bn = float(np.linalg.norm(b))
    true_res = {c: float(np.linalg.norm(b - oracle.spmv(rowptr, col, val, runs[c][0])) / bn) for c in runs}
    assert runs[False][4] == ITERS and runs[True][4] == ITERS
    with open(OUT, "w") as f:
        f.write("# Oracle CG, 27-point matrix at 128^3, b = U[-1,1) seed 1, x0 = 0, 500 iterations.\n")
        f.write("# Written by make_cg128_envelope.py from the serial oracle only.\n")
        f.write(f"# true_residual_naive {true_res[False]!r}\n")
        f.write(f"# true_residual_compensated {true_res[True]!r}\n")
        f.write("# k rho_naive rho_compensated (rho after iteration k+1)\n")
        for k in range(ITERS):
            f.write(f"{k} {float(runs[False][1][k])!r} {float(runs[True][1][k])!r}\n")
    print(OUT)


if __name__ == "__main__":
    main()
