"""Values the paper prints, kept as text fixtures under tests/golden/ (each
file names its passage), against the oracle's kernel evaluation."""
import os

import numpy as np

import workloads as W
from oracle import kernels

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _fixture(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_yukawa_eq36_diagonal_and_off_diagonal_form():
    g = _fixture("yukawa_eq36.txt")
    p = W.yukawa_cube(n=64, leaf=16, eps=1e-6, nrhs=1)  # the workloads' Yukawa kernel
    assert p.kernel.kappa == g["kappa"]
    X = np.array([[0.0, 0.0, 0.0], [0.25, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 3.0, 0.0]])
    idx = np.arange(len(X))
    A = kernels.evaluate(p.kernel, X, X, idx, idx)
    # the printed diagonal, exactly
    assert np.all(np.diag(A) == g["diagonal"])
    # off the diagonal the regularised form differs from exp(-r)/r by the
    # factor r/(r + delta) only: it equals exp(-kappa r)/(r + delta) and stays
    # within delta/r of the printed form
    r = np.linalg.norm(X[:, None, :] - X[None, :, :], axis=2)
    off = ~np.eye(len(X), dtype=bool)
    paper = np.exp(-g["kappa"] * r[off]) / r[off]
    assert np.allclose(A[off] * (r[off] + p.kernel.delta), np.exp(-g["kappa"] * r[off]),
                       rtol=1e-15, atol=0)
    assert np.all(np.abs(A[off] - paper) / paper <= p.kernel.delta / r[off] + 1e-15)
