"""Host logic of the HMC driver on analytic targets (CPU): the leapfrog
integrator is time-reversible and its energy error falls as eps^2, the
box transform's Jacobian turns a flat density into a uniform one on the box,
and NUTS reproduces the mean and covariance of a correlated Gaussian."""
import numpy as np

from paper_2105_14782_amd import hmc


def _gauss(mu, cov):
    P = np.linalg.inv(cov)

    def f(z):
        d = z - mu
        return -0.5 * d @ P @ d, -P @ d
    return f


def test_leapfrog_reversible_and_second_order():
    f = _gauss(np.zeros(3), np.diag([1.0, 4.0, 0.25]))
    z0 = np.array([0.3, -1.0, 0.2])
    r0 = np.array([0.5, 0.1, -0.7])
    lp0, g0 = f(z0)
    errs = []
    for eps in (0.1, 0.05, 0.025):
        z, r, lp, g = z0, r0, lp0, g0
        for _ in range(int(round(1.0 / eps))):
            z, r, lp, g = hmc._leapfrog(f, z, r, g, eps)
        errs.append(abs((lp - 0.5 * r @ r) - (lp0 - 0.5 * r0 @ r0)))
        zb, rb, lpb, gb = z, -r, lp, g
        for _ in range(int(round(1.0 / eps))):
            zb, rb, lpb, gb = hmc._leapfrog(f, zb, rb, gb, eps)
        np.testing.assert_allclose(zb, z0, atol=1e-12)
        np.testing.assert_allclose(-rb, r0, atol=1e-12)
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_box_transform_of_flat_density_is_uniform():
    post = hmc.BoxPosterior(lambda th: (0.0, np.zeros(2)), [1.0, -3.0], [3.0, 5.0])
    res = hmc.nuts(post, np.zeros(2), 3000, 500, np.random.default_rng(1))
    m, v = res.samples.mean(axis=0), res.samples.var(axis=0)
    assert abs(m[0] - 2.0) < 0.1 and abs(m[1] - 1.0) < 0.4
    np.testing.assert_allclose(v, np.array([4.0, 64.0]) / 12.0, rtol=0.15)
    assert res.samples.min(axis=0)[0] > 1.0 and res.samples.max(axis=0)[1] < 5.0


def test_nuts_recovers_correlated_gaussian():
    mu = np.array([1.0, -2.0, 0.5])
    A = np.array([[1.0, 0.6, 0.0], [0.6, 2.0, -0.4], [0.0, -0.4, 0.5]])
    res = hmc.nuts(_gauss(mu, A), np.zeros(3), 4000, 500, np.random.default_rng(2))
    m = res.samples.mean(axis=0)
    c = np.cov(res.samples.T)
    se = np.sqrt(np.diag(A) / 400.0)          # generous: effective sample size >= 400
    assert np.all(np.abs(m - mu) < 4 * se), (m, mu)
    np.testing.assert_allclose(c, A, atol=0.15 * np.max(np.abs(A)))
    assert 0.6 < res.accept.mean() < 0.95
    assert res.divergences == 0
