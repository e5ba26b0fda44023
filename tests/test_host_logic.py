"""Host-side helpers of the parity tests that carry arithmetic of their own:
the change of basis between the conic gradient the oracle reports (w.r.t. the
inverse covariance entries A, B, C of Q = A dx^2 + 2 B dx dy + C dy^2) and the
one the kernels accumulate (w.r.t. the stored a = A, beta = B / A,
gamma = C - B^2 / A).  Pinned by central finite differences of a smooth test
function, not by re-deriving the chain rule.  Also the closed form of the
row interval the binning's culling evaluates, against dense sampling."""
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


def _row_interval(u, v, a, beta, gamma, cut, y0, y1):
    """x-extent of {a (ex + beta ey)^2 + gamma ey^2 <= cut} within the band
    of rows y0 <= y <= y1 (ex = x - u, ey = y - v): the rightmost point of the
    ellipse, at ey = -beta sqrt(cut a / (gamma c)) with c = gamma + a beta^2,
    clamped to the band bounds the right end, its mirror the left one.  The
    binning kernels evaluate this interval per cell row."""
    H = np.sqrt(cut / gamma)
    ey_r = -beta * np.sqrt(cut * a / (gamma * (gamma + a * beta * beta)))
    e0, e1 = max(y0 - v, -H), min(y1 - v, H)
    if e0 > e1:
        return None
    er, el = min(max(ey_r, e0), e1), min(max(-ey_r, e0), e1)
    sr = np.sqrt(max(0.0, (cut - gamma * er * er) / a))
    sl = np.sqrt(max(0.0, (cut - gamma * el * el) / a))
    return u - (sl + beta * el), u + (sr - beta * er)


def test_row_interval_bounds_the_ellipse_slice():
    """Against a dense sampling of the band: the interval holds every sampled
    point of the slice and is no wider than the sampling resolution."""
    rng = np.random.default_rng(8)
    for _ in range(300):
        l1, l2 = 10.0 ** rng.uniform(-1, 3, 2)
        th = rng.uniform(0, np.pi)
        c, s = np.cos(th), np.sin(th)
        cov = np.array([[l1 * c * c + l2 * s * s, (l1 - l2) * c * s], [(l1 - l2) * c * s, l1 * s * s + l2 * c * c]])
        A, B, C = np.linalg.inv(cov)[[0, 0, 1], [0, 1, 1]]
        u, v = rng.uniform(-50, 150, 2)
        y0 = rng.uniform(0, 100)
        y1 = y0 + rng.uniform(0, 30)
        iv = _row_interval(u, v, A, B / A, C - B * B / A, 9.0, y0, y1)
        half = 3.0 * np.sqrt(cov[0, 0]) + 5.0
        xs = np.linspace(u - half, u + half, 1500)
        ys = np.linspace(y0, y1, 80)
        X, Y = np.meshgrid(xs, ys)
        ex, ey = X - u, Y - v
        inside = A * ex * ex + 2 * B * ex * ey + C * ey * ey <= 9.0
        if not inside.any():
            continue
        assert iv is not None
        step = xs[1] - xs[0]
        xmin, xmax = X[inside].min(), X[inside].max()
        assert iv[0] <= xmin + 1e-9 * abs(xmin) and iv[1] >= xmax - 1e-9 * abs(xmax)
        span = xmax - xmin + 1.0
        assert iv[0] >= xmin - 2 * step - 0.05 * span and iv[1] <= xmax + 2 * step + 0.05 * span


def test_lambda_schedules_follow_the_experiments():
    """Sec. 4.1 (implementation details): alpha = 0.1 from iteration 19000 to
    20000, beta = 0.0005 and gamma = 0.001 throughout."""
    from paper_2412_20522_amd import prune as P
    assert P.lambda_m(18_999, "alpha") == 0.0
    assert P.lambda_m(19_000, "alpha") == 0.1 and P.lambda_m(19_999, "alpha") == 0.1
    assert P.lambda_m(20_000, "alpha") == 0.0
    for it in (0, 1, 15_000, 29_999):
        assert P.lambda_m(it, "beta") == 0.0005 and P.lambda_m(it, "gamma") == 0.001


def test_prune_cadence():
    """Sec. 3.5: pruning at every densification step and every 1000
    iterations afterwards (densification every 100 iterations in [500, 15000])."""
    from paper_2412_20522_amd import prune as P
    due = [it for it in range(0, 20_001) if P.prune_due(it)]
    assert due[:3] == [500, 600, 700]
    assert 15_000 in due and 15_100 not in due and 16_000 in due and 20_000 in due
    assert all(it % 100 == 0 for it in due)
    assert sum(1 for it in due if it > 15_000) == 5


def test_gumbel_bound_decides_pruning_draws_like_the_exact_rule():
    """The pruning draws settle most draws by comparing the uniforms with two
    per-Gaussian thresholds: g(u) = -log(-log u) increases with u and is at
    least g(2^-25) over the generator's uniforms, so u0 below
    g^-1(g_min - d) - 1e-6 forces a 0 and u1 below g^-1(g_min + d) - 1e-6
    forces a 1 (d = s0 - s1).  Over the whole 24-bit grid of one uniform and
    random partners, both never contradict the double-precision rule."""
    rng = np.random.default_rng(31)
    g = lambda u: -np.log(-np.log(u))
    g_min = g(0.5 / 16777216.0)
    u_grid = (np.arange(0, 2 ** 24, 97) + 0.5) / 16777216.0
    for d in (-12.0, -8.0, -1.5, 0.0, 0.7, 8.0, 12.0):
        s0, s1 = d / 2, -d / 2
        u_other = (rng.integers(0, 2 ** 24, u_grid.size) + 0.5) / 16777216.0
        t0 = np.exp(-np.exp(d - g_min)) - 1e-6
        t1 = np.exp(-np.exp(-d - g_min)) - 1e-6
        # u0 on the grid, u1 random: the "0" shortcut
        exact = (s0 + g(u_grid)) > (s1 + g(u_other))
        assert not np.any(exact[u_grid < t0]), d
        # u1 on the grid, u0 random: the "1" shortcut
        exact = (s0 + g(u_other)) > (s1 + g(u_grid))
        assert np.all(exact[u_grid < t1]), d
        # the extreme partner (the smallest uniform) is the worst case
        u_min = 0.5 / 16777216.0
        assert not np.any(((s0 + g(u_grid)) > (s1 + g(u_min)))[u_grid < t0]), d
