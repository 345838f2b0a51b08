"""Write c2_lambda_f.txt: the FP64 Fermi level of the 64^3 periodic workload
(synth.config(2): all 262,144 nodes, K = 100, kT = 0.001 Ha, N_e = 192) from the
oracle alone -- Lanczos bounds, moments of every node (Eq. (Chebyshev)), their
sums and the bisection of Eq. (Ne).  The uneven-region workload (synth.config(3))
has no electron count of its own and takes this level as its fixed lambda_f.

Run from the repository root: python tests/golden/make_c2_lambda_f.py
(about 20 minutes on 8 cores; the oracle parallelises over nodes)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2011_13517_amd import synth  # noqa: E402


def main():
    prob = synth.config(2)
    lmin, lmax = O.lanczos_bounds(prob)
    n = prob.n_nodes
    M = np.zeros(prob.order + 1)
    t = time.time()
    chunk = 8192
    for s in range(0, n, chunk):
        mu = O.moments(prob, lmin, lmax, nodes=np.arange(s, min(s + chunk, n), dtype=np.int64))
        M += mu.sum(axis=0)
        print(f"{min(s + chunk, n)}/{n} nodes, {time.time() - t:.0f} s", flush=True)
    lf, it, ok = O.fermi_level(M, prob.kT, lmin, lmax, prob.Ne, tol=1e-10, with_status=True)
    assert ok, "bisection did not converge"
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_lambda_f.txt")
    with open(out, "w") as f:
        f.write("# FP64 Fermi level of synth.config(2), oracle only (make_c2_lambda_f.py)\n")
        f.write(f"# bounds {lmin!r} {lmax!r}; bisection iterations {it}; "
                f"N_e(lambda_f) - 192 = {O.electron_count(M, lf, prob.kT, lmin, lmax) - prob.Ne:.3e}\n")
        f.write(f"{lf!r}\n")
    print("lambda_f", lf)


if __name__ == "__main__":
    main()
