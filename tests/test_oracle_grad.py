"""Pins of the oracle's gradients (oracle/gradient.py) against finite differences of the
oracle's forward sum, translation invariance, a hand case with ties, brute-force
derivative sums and the d = 1 closed form."""
import numpy as np
import pytest

from oracle import gradient, kernels, sliced
from oracle.directions import directions


def _case(kernel, N=60, M=50, d=6, P=5, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((N, d))
    y = rng.standard_normal((M, d))
    w = rng.random(N) + 0.1
    g = rng.standard_normal(M)
    xi = directions(d, P, seed + 3)
    if kernel == "negdist":
        kw = dict(sigma=1.0, method="sort", n_coeff=0, T=0.0)
    elif kernel == "gaussian":
        kw = dict(sigma=2.0, method="ndft", n_coeff=64, T=0.045)
    elif kernel == "matern":
        kw = dict(sigma=2.0, method="nfft", n_coeff=1024, T=0.125)
    else:
        kw = dict(sigma=2.0, method="nfft", n_coeff=256, T=0.125)
    return x, y, w, g, xi, kw


def _loss(kernel, x, y, w, g, xi, kw):
    return float(g @ sliced.sliced_sum(kernel, x, y, w, xi, **kw))


def test_absdist_deriv_hand_case_with_ties():
    # sources at 0, 1, 1, 2 with weights 1, 2, 3, 4; target at 1: A_< = 1, A_> = 4
    c = 1.5
    D = gradient.absdist_deriv_sum([0.0, 1.0, 1.0, 2.0], [1.0, -1.0, 3.0], [1.0, 2.0, 3.0, 4.0], c)
    assert D[0] == pytest.approx(-c * (1.0 - 4.0), abs=0)
    assert D[1] == pytest.approx(-c * (0.0 - 10.0), abs=0)
    assert D[2] == pytest.approx(-c * (10.0 - 0.0), abs=0)


# The Laplacian's smooth part k1 keeps the |u|^3 term of the series, so its Fourier
# coefficients decay like k^-4 and the derivative of the truncated sum converges like
# n_coeff^-2.5 .. -3 (1.5e-5 relative at 256 coefficients, 5e-7 at 1024); the Matern
# counterpart (nu = 3/2) has the same |u|^3 term (4e-6 at 1024 coefficients).
@pytest.mark.parametrize("kernel,tol", [("negdist", 1e-9), ("gaussian", 1e-6), ("laplacian", 3e-5),
                                        ("matern", 1e-5)])
def test_slice_deriv_vs_brute_force(kernel, tol):
    rng = np.random.default_rng(4)
    d = 5
    zx = rng.standard_normal(80)
    zy = rng.standard_normal(70)
    w = rng.random(80)
    _, _, _, _, _, kw = _case(kernel)
    D = gradient.slice_deriv(kernel, d, zx, zy, w, kw["sigma"], kw["method"], kw["n_coeff"], kw["T"])

    def f(t):
        return kernels.counterpart_f(kernel, d, t, kw["sigma"])

    ref = gradient.direct_deriv_1d(zx, zy, w, f)
    assert np.linalg.norm(D - ref) <= tol * np.linalg.norm(ref)


@pytest.mark.parametrize("kernel", ["negdist", "gaussian", "laplacian", "matern"])
def test_gradient_vs_central_differences(kernel):
    x, y, w, g, xi, kw = _case(kernel)
    gx, gy, gw = gradient.sliced_grad(kernel, x, y, w, g, xi, **kw)
    # |.| makes the negative distance and the Laplacian's sorted part piecewise smooth:
    # a step small enough not to cross a kink keeps central differences exact there
    h = 1e-3 if kernel in ("gaussian", "matern") else 1e-6
    rng = np.random.default_rng(1)
    errs, refs = [], []
    for arr, grad in ((x, gx), (y, gy)):
        for _ in range(16):
            i, j = rng.integers(arr.shape[0]), rng.integers(arr.shape[1])
            old = arr[i, j]
            arr[i, j] = old + h
            lp = _loss(kernel, x, y, w, g, xi, kw)
            arr[i, j] = old - h
            lm = _loss(kernel, x, y, w, g, xi, kw)
            arr[i, j] = old
            fd = (lp - lm) / (2 * h)
            errs.append(fd - grad[i, j])
            refs.append(grad[i, j])
    errs, refs = np.array(errs), np.array(refs)
    tol = 5e-5 if kernel in ("laplacian", "matern") else 2e-6
    assert np.linalg.norm(errs) <= tol * np.linalg.norm(refs) + 1e-12
    # the sum is linear in w: central differences are exact up to rounding
    hw = 1e-2
    for n in rng.integers(0, w.shape[0], 4):
        old = w[n]
        w[n] = old + hw
        lp = _loss(kernel, x, y, w, g, xi, kw)
        w[n] = old - hw
        lm = _loss(kernel, x, y, w, g, xi, kw)
        w[n] = old
        assert (lp - lm) / (2 * hw) == pytest.approx(gw[n], rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("kernel", ["negdist", "gaussian", "laplacian", "matern"])
def test_gradient_translation_invariance(kernel):
    x, y, w, g, xi, kw = _case(kernel, seed=2)
    gx, gy, _ = gradient.sliced_grad(kernel, x, y, w, g, xi, **kw)
    tot = gx.sum(axis=0) + gy.sum(axis=0)
    scale = np.abs(gx).sum() + np.abs(gy).sum()
    assert np.linalg.norm(tot) <= 1e-10 * scale


def test_negdist_d1_closed_form():
    # d = 1: the sliced sum is the exact sum -sum_n w_n |x_n - y_m| (c_1 = 1), so
    # dL/dy_m = -g_m sum_n w_n sign(y_m - x_n) and dL/dx_n = -w_n sum_m g_m sign(x_n - y_m)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((40, 1))
    y = np.concatenate([rng.standard_normal((30, 1)), x[:5]])      # includes ties with sources
    w = rng.random(40)
    g = rng.standard_normal(35)
    xi = directions(1, 3, 0)
    gx, gy, gw = gradient.sliced_grad("negdist", x, y, w, g, xi)
    sgn = np.sign(y[:, 0][:, None] - x[:, 0][None, :])
    assert np.allclose(gy[:, 0], -g * (sgn @ w), rtol=1e-12, atol=1e-12)
    assert np.allclose(gx[:, 0], -w * (-sgn.T @ g), rtol=1e-12, atol=1e-12)
    assert np.allclose(gw, -(np.abs(x[:, 0][:, None] - y[:, 0][None, :]) @ g), rtol=1e-12)
