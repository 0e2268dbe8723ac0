"""Writes two_drops_p32_solution.npz: the oracle's right-hand side and
Galerkin solution (GMRES to 1e-12) of the two-drop workload (degree 32, gap
0.2, viscosity ratios 1 and 5, surfactant 1 + 0.2 Y_2^0 with the linear
equation of state, Omega_1 threshold 5h, 4x upsampling).

Calls only the oracle (plain FP64 CPU implementation of Sec. 1, 1.2, 2.1-2.3);
run from the repository root:  python tests/golden/make_two_drops_p32.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "two_drops_p32_solution.npz")


def main():
    wl = W.two_drops()
    o = oracle.Options(A_tilde=wl.A_tilde, U_tilde=wl.U_tilde, U_sing=wl.U_sing, U_geom=wl.U_geom, eos=wl.eos,
                       E=wl.E, xs=wl.xs, sigma0=wl.sigma0, gmres_tol=1e-12)
    s = oracle.System([oracle.Drop(d.p, d.xc, d.lam, d.gc) for d in wl.drops], o)
    t0 = time.time()
    b = s.rhs()
    print(f"rhs {time.time() - t0:.1f} s", flush=True)
    n = [0]

    def A(v):
        n[0] += 1
        y = s.matvec(v)
        print(f"matvec {n[0]} {time.time() - t0:.1f} s", flush=True)
        return y

    x, it, hist = oracle.gmres(A, b, 1e-12, o.gmres_restart, o.gmres_maxit)
    print(f"gmres {it} iterations, relative residual estimate {hist[-1]:.2e}", flush=True)
    np.savez_compressed(OUT, b=b, u=x, iterations=it, tol=1e-12)


if __name__ == "__main__":
    main()
