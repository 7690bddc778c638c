"""The runtime predictor (iteration-number regressor, per-iteration
polynomial regressor with interaction terms, asymmetric-kernel GP
adjustment; Eq. (13)-(21)), on the CPU with synthetic runs.

Pins: runs generated from a known model in the predictor's own family are
predicted back (least squares recovers it); the adjustment after one and
after two observations equals the GP posterior mean with the asymmetric
kernel, written out here (the kernel is one-sided: an iteration is
uncorrelated with earlier ones); exact predictions leave the forecast at
the prior mean.
"""

import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def ekm():
    import paper_2412_02244_amd as m
    m.load_library()
    return m


def _true_ms(f, j):
    # per-iteration time of the synthetic workloads: in the order-2 family of
    # base features (f0, f1, 1/j): intercept, linear and pairwise terms
    return 0.5 + 0.3 * f[0] + 0.2 * f[1] + 1.5 * f[0] / j + 0.1 * f[0] * f[1]


def _true_iters(f):
    return int(round(4 + 3 * f[0] + 2 * f[1]))


def _workloads(seed, count):
    rng = np.random.default_rng(seed)
    return [rng.uniform(0.5, 3.0, 2) for _ in range(count)]


def test_recovers_a_model_of_its_own_family(ekm):
    q = 40
    p = ekm.Predictor(q, 2, order=2)
    for f in _workloads(1, 40):
        v = _true_iters(f)
        p.add_run(f, [_true_ms(f, j) for j in range(1, v + 1)])
    p.fit()
    for f in _workloads(2, 10):
        it, per, tot = p.predict(f)
        v = _true_iters(f)
        assert it == v
        want = [_true_ms(f, j) for j in range(1, q + 1)]
        np.testing.assert_allclose(per, want, rtol=1e-4, atol=1e-4)
        assert tot == pytest.approx(sum(want[:v]), rel=1e-4)


def _kernel(i, ip, sigma):
    x = ip - i
    if x <= -1:
        return 0.0
    h = math.log(x + 1) if x <= 0 else x
    return math.exp(-h * h / (2 * sigma * sigma))


def test_adjustment_matches_the_gp_closed_form(ekm):
    q, sigma, noise = 30, 3.0, 0.05
    p = ekm.Predictor(q, 2, order=2, sigma=sigma, noise=noise)
    for f in _workloads(3, 30):
        v = _true_iters(f)
        p.add_run(f, [_true_ms(f, j) for j in range(1, v + 1)])
    p.fit()
    f = np.array([1.2, 2.0])
    v, per, _ = p.predict(f)
    p.begin(f)
    # iteration 2 took twice its prediction: g = 1/2
    i, ms = 2, 2 * per[1]
    rem, tot = p.observe(i, ms)
    alpha = (0.5 - 1.0) / (_kernel(i, i, sigma) + noise)
    want = sum(per[j - 1] / (1 + alpha * _kernel(i, j, sigma)) for j in range(i + 1, v + 1))
    assert rem == pytest.approx(want, rel=1e-9)
    assert tot == pytest.approx(want + ms, rel=1e-9)
    # the adjustment raises the remaining time, most for the next iterations
    assert rem > sum(per[i:v])


def test_one_sided_kernel_and_prior(ekm):
    q = 30
    p = ekm.Predictor(q, 2, order=2, sigma=2.0, noise=0.0)
    for f in _workloads(4, 30):
        v = _true_iters(f)
        p.add_run(f, [_true_ms(f, j) for j in range(1, v + 1)])
    p.fit()
    f = np.array([2.0, 1.0])
    v, per, tot0 = p.predict(f)
    # exact predictions leave the forecast unchanged (g = 1, the prior mean)
    p.begin(f)
    for j in range(1, 4):
        rem, tot = p.observe(j, per[j - 1])
        assert rem == pytest.approx(sum(per[j:v]), rel=1e-12)
        assert tot == pytest.approx(tot0, rel=1e-12)
    # two observations: the posterior mean solves the (non-symmetric: an
    # iteration is uncorrelated with earlier ones) kernel system, written out
    p.begin(f)
    g1, g3 = per[0] / (1.1 * per[0]), per[2] / (3 * per[2])
    p.observe(1, 1.1 * per[0])
    rem, tot = p.observe(3, 3 * per[2])
    K = np.array([[_kernel(1, 1, 2.0), _kernel(1, 3, 2.0)], [_kernel(3, 1, 2.0), _kernel(3, 3, 2.0)]])
    assert K[1, 0] == 0.0 and K[0, 1] > 0.0
    alpha = np.linalg.solve(K, np.array([g1 - 1, g3 - 1]))
    want = sum(per[j - 1] / (1 + alpha[0] * _kernel(1, j, 2.0) + alpha[1] * _kernel(3, j, 2.0))
               for j in range(4, v + 1))
    assert rem == pytest.approx(want, rel=1e-9)
    assert tot == pytest.approx(1.1 * per[0] + 3 * per[2] + rem, rel=1e-12)


def test_rejects_misuse(ekm):
    with pytest.raises(ekm.EKMError):
        ekm.Predictor(0, 2)
    p = ekm.Predictor(10, 2)
    with pytest.raises(ekm.EKMError):
        p.fit()  # no runs
    with pytest.raises(ekm.EKMError):
        p.predict([1.0, 1.0])  # not fitted
    with pytest.raises(ekm.EKMError):
        p.add_run([1.0, 1.0], [1.0] * 11)  # more than q iterations
    p.add_run([1.0, 1.0], [1.0, 1.0])
    p.add_run([2.0, 1.0], [1.0, 1.0, 1.0])
    p.fit()
    p.begin([1.5, 1.0])
    p.observe(2, 1.0)
    with pytest.raises(ekm.EKMError):
        p.observe(2, 1.0)  # not increasing
