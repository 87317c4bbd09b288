"""Pins for the oracle's diagonal power iteration (CPU only): closed forms.

* d constant c > 0: one step normalises v0 and every later step keeps it;
  lambda = c ||v|| = c.
* v0 a unit vector e_j: it stays e_j and lambda = |d_j|.
* d = (2, 1), v0 = (1, 1): after k steps v is proportional to u_k = (2^k, 1),
  and lambda_k = ||D v_(k-1)|| = sqrt(4^k + 1) / sqrt(4^(k-1) + 1) for k >= 2
  (v_(k-1) = u_(k-1) / ||u_(k-1)||), sqrt(5) for k = 1 (v_0 = u_0 itself).
"""
import math

import numpy as np

import oracle


def test_constant_diagonal():
    g = np.random.Generator(np.random.PCG64(9))
    v0 = g.standard_normal(1000)
    for iters in (1, 2, 7):
        v, lam = oracle.power_iteration(np.full(1000, 2.5), v0, iters)
        assert np.allclose(v, v0 / np.linalg.norm(v0), rtol=1e-13, atol=1e-16)
        want = 2.5 * np.linalg.norm(v0) if iters == 1 else 2.5
        assert math.isclose(lam, want, rel_tol=1e-13)


def test_unit_vector_stays():
    d = np.array([3.0, -7.0, 0.5, 2.0])
    for j in range(4):
        v0 = np.zeros(4)
        v0[j] = 1.0
        v, lam = oracle.power_iteration(d, v0, 5)
        assert np.array_equal(np.abs(v), v0) and lam == abs(d[j])


def test_two_by_two_closed_form():
    for k in (1, 2, 3, 10, 30):
        v, lam = oracle.power_iteration([2.0, 1.0], [1.0, 1.0], k)
        u = np.array([2.0 ** k, 1.0])
        assert np.allclose(v, u / np.linalg.norm(u), rtol=1e-14)
        want = math.sqrt(5.0) if k == 1 else math.sqrt(4.0 ** k + 1) / math.sqrt(4.0 ** (k - 1) + 1)
        assert math.isclose(lam, want, rel_tol=1e-14)
