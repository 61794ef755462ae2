"""Write oracle results that are too slow to recompute inside a GPU test.

Calls only ``oracle`` (and the seeded input generators).  Output:
``er4096_sweep.txt``: Algorithm 2 (Jacobi step, safeguard on) on the
Erdos-Renyi graph n=4096, M=12288, start uniform on [0,64]^2 (seed 2000),
run to res <= 1e-3 or 2000 iterations for omega in {1.0, 1.2, 1.4, 1.6}:
iterations, converged, rejected, the last two residuals and the final stress.

usage: python tests/golden/make_oracle_golden.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1711_01228_amd import inputs  # noqa: E402

OMEGAS = (1.0, 1.2, 1.4, 1.6)


def main():
    g, X0 = inputs.er4096(0)
    D = oracle.apsp(g.row_ptr, g.col_idx)
    lines = ["# Oracle (FP64, Jacobi step, safeguard on) on G(n=4096, M=12288), seed 2000,",
             "# start uniform on [0,64]^2 (seed 2500); stop at res <= 1e-3 or 2000 iterations.",
             "# Written by make_oracle_golden.py, which calls only the oracle.",
             "# columns: omega iterations converged rejected res_last res_prev final_stress"]
    for om in OMEGAS:
        t = time.time()
        X, info = oracle.layout(D, X0, omega=om, tol=1e-3, max_iter=2000)
        tr = info["trace"]
        f = oracle.stress(D, X)
        prev = tr[-2, 0] if len(tr) > 1 else float("nan")
        lines.append("%.1f %d %d %d %.17g %.17g %.17g" % (om, info["iterations"], int(info["converged"]),
                                                       info["rejected"], tr[-1, 0], prev, f))
        print(lines[-1], "(%.1f s)" % (time.time() - t), flush=True)
    with open(os.path.join(HERE, "er4096_sweep.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
