"""Write reference eigenvalues of the full-size synthetic workloads.

Calls only the CPU oracle (ARPACK on the assembled sparse Hamiltonian) and the
seeded input generators.  Usage:
    python tests/golden/make_golden.py fin_qd_128x40x40 [--index I] [--tol T]
Output: tests/golden/<workload>[_i<I>].txt with one eigenvalue (eV) per line,
preceded by '#' comment lines stating how it was made and the largest residual.
"""

import argparse
import os
import sys
import time

import numpy as np
import scipy.sparse.linalg as spla

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import SI_MATERIAL, Grid, hamiltonian_ls, lowest_arpack, residuals  # noqa: E402
from synth import workload  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--index", type=int, default=None, help="Hamiltonian index of a sweep")
    ap.add_argument("--tol", type=float, default=1e-11)
    ap.add_argument("--nev", type=int, default=None)
    args = ap.parse_args()
    w = workload(args.name)
    V = w.V if args.index is None else w.V[args.index]
    nev = w.nev if args.nev is None else args.nev
    g = Grid(w.nx, w.ny, w.nz, w.h)
    t0 = time.time()
    H = hamiltonian_ls(g, SI_MATERIAL, V, w.strain, w.B)
    t1 = time.time()
    # count ARPACK's operator applications (the CPU solve-time extrapolation
    # of the benchmark multiplies this count by a measured matvec time)
    count = [0]

    def matvec(x):
        count[0] += 1
        return H @ x

    op = spla.LinearOperator(H.shape, matvec=matvec, dtype=H.dtype)
    E, v = lowest_arpack(op, nev, tol=args.tol, guard=max(4, nev // 2))
    t2 = time.time()
    r = residuals(H, E, v)
    tag = args.name if args.index is None else f"{args.name}_i{args.index}"
    path = os.path.join(HERE, f"{tag}.txt")
    with open(path, "w") as f:
        f.write(f"# lowest {nev} eigenvalues (eV) of the oracle Hamiltonian for {tag}\n")
        f.write(f"# made by: python tests/golden/make_golden.py {args.name}"
                + (f" --index {args.index}" if args.index is not None else "")
                + f" --tol {args.tol}\n")
        f.write(f"# oracle: scipy ARPACK eigsh(which='SA'), assembly {t1 - t0:.1f} s,"
                f" solve {t2 - t1:.1f} s, max residual {r.max():.3e} eV\n")
        f.write(f"# matvecs {count[0]}\n")
        for e in E:
            f.write(f"{e:.15e}\n")
    print(path, E, r.max(), f"{t2 - t1:.1f}s")


if __name__ == "__main__":
    main()
