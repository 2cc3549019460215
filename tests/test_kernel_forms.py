"""The rewritten cubic-spline expressions the HIP neighbour sums evaluate,
checked against the textbook piecewise form on a dense grid of q = r/h in
[0, 2] (CPU only; the kernels themselves are checked against the oracle by
the GPU parity tests):

  shape   (2-q)^3 - 4 (1-q)+^3  =  (2-q)^3 - (c (1-q))+^3,  c = 4^(1/3)
  -g q    -(4 t1^2 - t2^2)      =  min(q, 2-q) max(4-3q, 2-q)

with t1 = (1-q)+, t2 = (2-q)+ (the gradient factor of the force pass)."""
import numpy as np

CBRT4 = 1.5874010519681994


def _grid():
    q = np.linspace(0.0, 2.0, 200001)
    return np.concatenate([q, [1.0 - 1e-12, 1.0, 1.0 + 1e-12, 2.0 - 1e-12]])


def test_shape_with_cube_root_of_four():
    q = _grid()
    t1 = np.maximum(1.0 - q, 0.0)
    t2 = np.maximum(2.0 - q, 0.0)
    ref = t2 ** 3 - 4.0 * t1 ** 3
    u = np.maximum(CBRT4 * (1.0 - q), 0.0)
    got = (2.0 - q) ** 3 - u ** 3
    assert np.max(np.abs(got - ref)) <= 4e-15 * 4.0
    assert abs(CBRT4 ** 3 - 4.0) <= 1e-15


def test_gradient_factor_min_max():
    q = _grid()
    t1 = np.maximum(1.0 - q, 0.0)
    t2 = np.maximum(2.0 - q, 0.0)
    ref = -(4.0 * t1 * t1 - t2 * t2)
    got = np.minimum(q, 2.0 - q) * np.maximum(4.0 - 3.0 * q, 2.0 - q)
    assert np.max(np.abs(got - ref)) <= 1e-14
    # the piecewise closed forms: q (4 - 3q) below 1, (2 - q)^2 above
    lo, hi = q < 1.0, q >= 1.0
    assert np.allclose(got[lo], q[lo] * (4.0 - 3.0 * q[lo]), rtol=0, atol=1e-14)
    assert np.allclose(got[hi], (2.0 - q[hi]) ** 2, rtol=0, atol=1e-14)
    # zero at the self pair (q = 0) and at the support's edge (q = 2)
    assert got[0] == 0.0
    assert min(2.0, 2.0 - 2.0) * max(4.0 - 6.0, 2.0 - 2.0) == 0.0
