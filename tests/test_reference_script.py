"""The script that writes the stored solve references computes the oracle's
values exactly: its row-parallel K_x and K_X equal the oracle's bit for bit,
and its PCG reaches the oracle's iterate with the same iteration count."""
import importlib.util
import os

import numpy as np

import oracle
import synth
from oracle.schur import Problem

HERE = os.path.dirname(os.path.abspath(__file__))


def _script():
    path = os.path.join(HERE, "golden", "make_solve_reference.py")
    spec = importlib.util.spec_from_file_location("make_solve_reference", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_row_parallel_operators_equal_oracle():
    mod = _script()
    J, K = 3, 5
    P = Problem(J, K)
    Q = mod.RowParallelProblem(J, K, workers=3)
    X = synth.random_field(P.shape, 5)
    assert np.array_equal(Q.Kx(X), P.Kx(X))
    assert np.array_equal(Q.KX(X), P.KX(X))
    assert np.array_equal(Q.Shat(X), P.Shat(X))


def test_row_parallel_pcg_equals_oracle():
    mod = _script()
    J, K = 3, 4
    g, u0 = synth.fourier_g(J, K, 2), synth.sine_product(K, 1, 1)
    P = Problem(J, K)
    Q = mod.RowParallelProblem(J, K, workers=2)
    fhat = P.WT(P.rhs(g, u0))
    w1, k1, h1 = oracle.pcg.pcg(P, fhat, 1e-8, 100)
    w2, k2, h2 = oracle.pcg.pcg(Q, Q.WT(Q.rhs(g, u0)), 1e-8, 100)
    assert k1 == k2 and h1 == h2
    assert np.array_equal(w1, w2)


def test_stored_references_are_consistent():
    """Every stored reference names its sizes, and its history ends at or
    below the tolerance after `iterations` steps (Section 3.4)."""
    import glob
    import json

    files = glob.glob(os.path.join(HERE, "golden", "solve_*.json"))
    assert files
    for f in files:
        rec = json.load(open(f))
        h = rec["history"]
        assert len(h) == rec["iterations"] + 1
        assert h[-1] <= rec["tol"] * h[0] < h[-2]
        u = np.asarray(rec["u"])
        assert u.shape == (len(rec["rows"]), len(rec["nodes"]))
        assert np.all(np.isfinite(u)) and np.any(u)
