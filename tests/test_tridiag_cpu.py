"""The host's tridiagonal square root (csrc/tridiag.hpp) against numpy's dense eigh.

The Lanczos square roots of the Brownian terms (Section 2.5) read T^{1/2} e1 of the k x k
tridiagonal of Lanczos coefficients at every convergence check.  The host computes it by the
implicit QL method; this compiles the header into a small program with g++ and compares its
result with Q diag(sqrt(max(lambda, 0))) Q^T e1 from numpy.linalg.eigh on the dense matrix.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2607_25161_amd", "csrc")

HARNESS = r"""
#include <cstdio>
#include <vector>
#include "tridiag.hpp"
int main() {
  int k;
  while (std::scanf("%d", &k) == 1) {
    std::vector<double> a(k), b(k > 0 ? k - 1 : 0);
    for (auto& x : a) std::scanf("%lf", &x);
    for (auto& x : b) std::scanf("%lf", &x);
    const std::vector<double> o = fsd::tridiag_sqrt_e1(a, b);
    for (double x : o) std::printf("%.17g ", x);
    std::printf("\n");
  }
}
"""


@pytest.fixture(scope="module")
def root_e1(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("tridiag")
    src, exe = d / "h.cpp", d / "h"
    src.write_text(HARNESS)
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)

    def run(cases):
        text = "".join(f"{len(a)} " + " ".join(repr(float(x)) for x in a) + " " +
                       " ".join(repr(float(x)) for x in b) + "\n" for a, b in cases)
        out = subprocess.run([str(exe)], input=text, check=True, capture_output=True, text=True).stdout
        return [np.array([float(x) for x in line.split()]) for line in out.strip("\n").split("\n")]
    return run


def reference(a, b):
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    lam, Q = np.linalg.eigh(T)
    return Q @ (np.sqrt(np.clip(lam, 0.0, None)) * Q[0])


def test_positive_definite_tridiagonals(root_e1):
    rng = np.random.default_rng(7)
    cases = []
    for k in (1, 2, 3, 7, 40, 100):
        a = 2.0 + rng.uniform(0.5, 2.0, k)
        b = rng.uniform(-0.8, 0.8, k - 1)
        cases.append((a, b))
    for (a, b), got in zip(cases, root_e1(cases)):
        ref = reference(a, b)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), len(a)


def test_lanczos_like_and_split_tridiagonals(root_e1):
    """Coefficients spread over decades (as the lubrication matrix gives), a negligible
    off-diagonal entry (the matrix splits), and a singular positive semi-definite matrix."""
    rng = np.random.default_rng(8)
    k = 60
    a = 10.0 ** rng.uniform(-3, 3, k)
    b = np.sqrt(a[:-1] * a[1:]) * rng.uniform(0.05, 0.45, k - 1)
    split_a, split_b = a.copy(), b.copy()
    split_b[k // 2] = 1e-300
    lap_a = np.full(30, 2.0)
    lap_a[[0, -1]] = 1.0
    lap_b = np.full(29, -1.0)  # path-graph Laplacian: eigenvalue 0 with eigenvector of ones
    got = root_e1([(a, b), (split_a, split_b), (lap_a, lap_b)])
    for (aa, bb), g, tol in zip([(a, b), (split_a, split_b), (lap_a, lap_b)], got, (1e-11, 1e-11, 1e-7)):
        ref = reference(aa, bb)
        assert np.abs(g - ref).max() <= tol * np.abs(ref).max()
    # the square root squares back: for the Laplacian, S^2 e1 = T e1 with S from the same map
    T = np.diag(lap_a) + np.diag(lap_b, 1) + np.diag(lap_b, -1)
    lam, Q = np.linalg.eigh(T)
    S = Q @ np.diag(np.sqrt(np.clip(lam, 0, None))) @ Q.T
    assert np.abs(S @ got[2] - T[:, 0]).max() < 1e-7
