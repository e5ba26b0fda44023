"""Host-side helpers of the parity tests that carry arithmetic of their own:
the change of basis between the conic gradient the oracle reports (w.r.t. the
inverse covariance entries A, B, C of Q = A dx^2 + 2 B dx dy + C dy^2) and the
one the kernels accumulate (w.r.t. the stored a = A, beta = B / A,
gamma = C - B^2 / A).  Pinned by central finite differences of a smooth test
function, not by re-deriving the chain rule."""
import numpy as np

from tests import gpu_util as U


def _conics(rng, n):
    # positive-definite conics over six decades of anisotropy
    l1 = 10.0 ** rng.uniform(-3, 0, n)
    l2 = l1 * 10.0 ** rng.uniform(0, 6, n)
    th = rng.uniform(0, np.pi, n)
    c, s = np.cos(th), np.sin(th)
    A = l1 * c * c + l2 * s * s
    B = (l1 - l2) * c * s
    C = l1 * s * s + l2 * c * c
    return np.stack([A, B, C], 1)


def _f(A, B, C, w):
    # a smooth scalar of the conic with no special structure
    return w[0] * np.sin(A) + w[1] * B * C + w[2] * np.log1p(C * C) + w[3] * A * B * B


def _grad_abc(A, B, C, w):
    return np.stack([w[0] * np.cos(A) + w[3] * B * B, w[1] * C + 2 * w[3] * A * B,
                     w[1] * B + w[2] * 2 * C / (1 + C * C)], 1)


def test_stable_conic_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    con = _conics(rng, 64)
    w = rng.normal(size=4)
    A, B, C = con.T
    a, beta, gamma = A, B / A, C - B * B / A
    got = U.dstable_from_dabc(a, beta, _grad_abc(A, B, C, w))

    def f_stable(a, beta, gamma):
        return _f(a, a * beta, gamma + a * beta * beta, w)

    fd = np.empty_like(got)
    for j in range(3):
        p = [a.copy(), beta.copy(), gamma.copy()]
        h = 1e-6 * np.maximum(np.abs(p[j]), 1e-3)
        p[j] = p[j] + h
        up = f_stable(*p)
        p[j] = p[j] - 2 * h
        dn = f_stable(*p)
        fd[:, j] = (up - dn) / (2 * h)
    scale = np.abs(fd).max(axis=1, keepdims=True) + 1e-12
    assert np.all(np.abs(got - fd) / scale < 1e-6)


def test_conic_gradient_bases_round_trip():
    rng = np.random.default_rng(6)
    con = _conics(rng, 256)
    d = rng.normal(size=(256, 3))
    A, B, C = con.T
    back = U.dabc_from_dstable(con, U.dstable_from_dabc(A, B / A, d))
    assert np.allclose(back, d, rtol=1e-9, atol=1e-9 * np.abs(d).max())
