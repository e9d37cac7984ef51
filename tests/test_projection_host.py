"""The small dense solve of the projected warm start (proj_coefficients in csrc/kernels.h, the
same function the one-block device kernel calls), built for the host and checked against
numpy: the Galerkin coefficients of A x = b on the span of up to four vectors, with a vector
that is linearly dependent on the earlier ones dropped, partial histories and a zero system."""
import os
import subprocess

import numpy as np
import pytest

from paper_2608_12868_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
HARNESS = r"""
#include "kernels.h"
#include <cstdio>
int main() {
  double s[14], c[4];
  int m;
  while (scanf("%d", &m) == 1) {
    for (int k = 0; k < 14; ++k)
      if (scanf("%lf", &s[k]) != 1) return 1;
    ehd::proj_coefficients<4>(s, m, c);
    printf("%.17g %.17g %.17g %.17g\n", c[0], c[1], c[2], c[3]);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def solver(tmp_path_factory):
    d = tmp_path_factory.mktemp("proj")
    src = d / "harness.cpp"
    src.write_text(HARNESS)
    exe = d / "harness"
    r = subprocess.run([B.hipcc(), "-O2", "-std=c++17", "-I", os.path.join(B.ROOT, "include"), "-I",
                        os.path.join(B.ROOT, "paper_2608_12868_amd", "csrc"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]

    def run(cases):
        inp = "\n".join(f"{m} " + " ".join(repr(float(v)) for v in s) for m, s in cases) + "\n"
        out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
        return [np.array([float(x) for x in line.split()]) for line in out.strip().split("\n")]
    return run


def _system(rng, n=300, dependent=False):
    # a 1D Dirichlet Laplacian (SPD) as the operator
    A = np.diag(np.full(n, 2.5)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)
    H = rng.standard_normal((n, 4))
    if dependent:
        H[:, 2] = 2.0 * H[:, 0] - H[:, 1]
    b = rng.standard_normal(n)
    G, g = H.T @ A @ H, H.T @ b
    s = [G[r, c] for r in range(4) for c in range(r, 4)] + list(g)
    return A, H, b, G, g, s


def test_projection_coefficients_match_numpy(solver):
    rng = np.random.default_rng(7)
    cases, refs = [], []
    for trial in range(16):
        m = 1 + trial % 4
        dependent = trial >= 8
        A, H, b, G, g, s = _system(rng, dependent=dependent)
        keep = [j for j in range(m) if not (dependent and j == 2)]
        c = np.zeros(4)
        c[keep] = np.linalg.solve(G[np.ix_(keep, keep)], g[keep])
        cases.append((m, s))
        refs.append(c)
    for c, ref in zip(solver(cases), refs):
        assert np.abs(c - ref).max() <= 1e-10 * np.abs(ref).max()


def test_projection_minimises_energy_error(solver):
    """x0 = H c is the A-norm-closest point of the span to the solution of A x = b."""
    rng = np.random.default_rng(3)
    A, H, b, G, g, s = _system(rng)
    c = solver([(4, s)])[0]
    x = np.linalg.solve(A, b)
    e0 = H @ c - x
    best = e0 @ A @ e0
    for _ in range(50):
        e = H @ (c + 1e-3 * rng.standard_normal(4)) - x
        assert e @ A @ e >= best


def test_projection_degenerate_inputs(solver):
    zero = [0.0] * 14
    c_zero, = solver([(4, zero)])
    assert np.array_equal(c_zero, np.zeros(4))
    rng = np.random.default_rng(5)
    _, _, _, G, g, s = _system(rng)
    c0, c2 = solver([(0, s), (2, s)])
    assert np.array_equal(c0, np.zeros(4))
    assert c2[2] == 0.0 and c2[3] == 0.0
