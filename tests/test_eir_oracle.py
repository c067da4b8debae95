"""Pins of the transducer-response oracle (oracle/eir.py): the identity and delay kernels,
the explicit Toeplitz matrix, and adjointness."""
import numpy as np

from oracle.eir import eir_adjoint, eir_apply


def test_delta_kernel_is_identity_and_shift_is_delay():
    rng = np.random.default_rng(0)
    z = rng.standard_normal((30, 4))
    assert np.array_equal(eir_apply([1.0], z), z)
    d = eir_apply([0.0, 0.0, 1.0], z)
    assert np.array_equal(d[2:], z[:-2]) and np.all(d[:2] == 0)
    a = eir_adjoint([0.0, 0.0, 1.0], z)
    assert np.array_equal(a[:-2], z[2:]) and np.all(a[-2:] == 0)


def test_matches_explicit_toeplitz_matrix():
    rng = np.random.default_rng(1)
    M, L, nh = 17, 3, 5
    h = rng.standard_normal(nh)
    T = np.zeros((M, M))
    for m in range(M):
        for k in range(nh):
            if m - k >= 0:
                T[m, m - k] = h[k]
    z = rng.standard_normal((M, L))
    assert np.allclose(eir_apply(h, z), T @ z, rtol=0, atol=1e-13)
    assert np.allclose(eir_adjoint(h, z), T.T @ z, rtol=0, atol=1e-13)


def test_kernel_longer_than_the_traces():
    rng = np.random.default_rng(2)
    h = rng.standard_normal(12)
    z = rng.standard_normal((7, 2))
    y = rng.standard_normal((7, 2))
    assert abs(np.sum(eir_apply(h, z) * y) - np.sum(z * eir_adjoint(h, y))) <= 1e-12
