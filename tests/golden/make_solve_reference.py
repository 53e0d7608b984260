"""Write the oracle's reference for a full-size FP64 solve (test data).

Runs the CPU oracle's PCG (``oracle.pcg``) on the heat equation with a
seeded Fourier forcing (``synth.fourier_g``) and either
``u0 = sin(pi x) sin(pi y)`` (the single large solves) or a seeded smooth
``u0`` (``synth.smooth_u0``, the batched right-hand sides) to the relative
tolerance 1e-8 of the stopping quantity ``sqrt(r^T K_X r)`` (Section 3.4,
eq. (13), read relative to the first residual), and stores:

  * ``iterations``: the number of S-hat applications the oracle needed;
  * ``history``: ``sqrt(r_k^T K_X r_k)`` for k = 0 .. iterations;
  * ``rows`` x ``nodes``: a fixed sample of the solution ``u = W w`` (time rows
    at both ends and at several wavelet levels, spatial nodes drawn from a
    seeded generator plus the four corners of the grid), with its values.

Only ``oracle`` and ``synth`` are called.  Usage (from the repository root)::

    python tests/golden/make_solve_reference.py J K out.json [--g-seed 2] [--u0 sin]
        [--threads 8]

``--u0 smooth`` draws ``u0`` with the forcing's seed (solve b of the 64
right-hand sides of the batched workload uses seed 1000 + b for both).

The multigrid applications K_x and K_X act on every time row separately
(they are block-diagonal in time, Section 3.1 and Theorem 3.1), so this script
hands blocks of rows to a pool of threads, each calling the oracle's own
``multigrid.apply`` and ``spatial.stiffness`` on its block: the values are the
oracle's, bit for bit (``tests/test_reference_script.py`` checks this), and
the run takes minutes instead of hours.  At J = 10, K = 9 (2.7e8 unknowns) it
needs about 40 GB of host memory.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import multigrid, spatial, wavelet  # noqa: E402
from oracle.schur import Problem  # noqa: E402

TOL = 1e-8
NODE_SEED = 4242
NODES_PER_ROW = 512


ROW_BLOCK = 2


class RowParallelProblem(Problem):
    """The oracle's Problem with its row-by-row multigrid operators spread over
    threads (NumPy releases the interpreter lock inside its array loops).
    Each block of ``ROW_BLOCK`` time rows goes through exactly the oracle's
    calls, so every value equals the oracle's."""

    def __init__(self, J: int, K: int, workers: int):
        super().__init__(J, K)
        self.pool = ThreadPoolExecutor(max_workers=workers)

    def _by_rows(self, fn, X, per_row=None):
        out = np.empty_like(X)

        def run(lo):
            hi = min(lo + ROW_BLOCK, X.shape[0])
            out[lo:hi] = fn(X[lo:hi], None if per_row is None else per_row[lo:hi])

        list(self.pool.map(run, range(0, X.shape[0], ROW_BLOCK)))
        return out

    def Kx(self, y):
        return self._by_rows(
            lambda b, _: multigrid.apply(b, self.K, 1.0, 0.0, self.cycles, self.sweeps), y)

    def KX(self, R):
        sigma = 2.0 ** wavelet.row_levels(self.J).astype(np.float64)

        def block(b, s):
            z = multigrid.apply(b, self.K, self.alpha, s, self.cycles, self.sweeps)
            return multigrid.apply(spatial.stiffness(z), self.K, self.alpha, s, self.cycles,
                                   self.sweeps)

        return self._by_rows(block, R, sigma)


def sample_rows(J: int):
    """Both ends, the middle (level 1) and rows of levels 2, J - 1 and J."""
    N = 2 ** J
    rows = {0, N, N // 2, N // 4, 3 * N // 4, 1, N - 1, 2 if N >= 4 else 1}
    return sorted(r for r in rows if 0 <= r <= N)


def sample_nodes(K: int):
    n = 2 ** K - 1
    rng = np.random.default_rng(NODE_SEED)
    count = min(NODES_PER_ROW, n * n)
    pick = rng.choice(n * n, size=count, replace=False)
    corners = [0, n - 1, n * (n - 1), n * n - 1]
    return sorted(set(int(v) for v in pick) | set(corners))


def main(J: int, K: int, out: str, g_seed: int = 2, u0_kind: str = "sin",
         workers: int = 8) -> None:
    t0 = time.time()
    P = RowParallelProblem(J, K, workers)
    print(f"# oracle reference J={J} K={K} g seed {g_seed} u0 {u0_kind}", flush=True)
    g = synth.fourier_g(J, K, g_seed)
    u0 = synth.sine_product(K, 1, 1) if u0_kind == "sin" else synth.smooth_u0(K, g_seed)
    f = P.rhs(g, u0)
    del g
    fhat = P.WT(f)
    del f
    print(f"# f-hat ready after {time.time() - t0:.0f} s", flush=True)

    def progress(k, w, r):
        print(f"# iteration {k} after {time.time() - t0:.0f} s", flush=True)

    w, its, hist = oracle.pcg.pcg(P, fhat, TOL, 200, callback=progress)
    del fhat
    u = P.W(w)
    del w
    rows = sample_rows(J)
    nodes = sample_nodes(K)
    flat = u.reshape(u.shape[0], -1)
    vals = flat[np.ix_(rows, nodes)]
    rec = {
        "what": "oracle FP64 PCG solution samples, heat equation, seeded Fourier forcing, "
                "relative tolerance 1e-8 (Section 3.4, eq. (13))",
        "J": J, "K": K, "g_seed": g_seed, "u0": u0_kind, "tol": TOL,
        "iterations": int(its),
        "history": [float(h) for h in hist],
        "rows": rows, "nodes": nodes,
        "u": [[float(v) for v in row] for row in vals],
        "u_norm_all": float(np.linalg.norm(u)),
        "seconds": round(time.time() - t0, 1),
        "script": "tests/golden/make_solve_reference.py",
    }
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=0)
    print(f"# wrote {out}: {its} iterations in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("J", type=int)
    ap.add_argument("K", type=int)
    ap.add_argument("out")
    ap.add_argument("--g-seed", type=int, default=2)
    ap.add_argument("--u0", choices=["sin", "smooth"], default="sin")
    ap.add_argument("--threads", type=int, default=8)
    a = ap.parse_args()
    main(a.J, a.K, a.out, a.g_seed, a.u0, a.threads)
