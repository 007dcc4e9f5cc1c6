"""Pins of the oracle's calibration loop: Adam (Kingma and Ba 2015, algorithm 1) on (mu, xi) with the loss
gradient of the smooth deposit from the adjoint.

* the Adam update follows torch.optim.Adam (an independent implementation) on the same gradient sequence;
* the loss is the mean squared deposit error and its raster gradient 2 (D - T) / N (numpy in binary64);
* on the calibration scene with the target made at (mu*, xi*) = (0.22, 1800) and the start at
  (0.26, 1400), the first gradient points back toward mu*, the loss falls by two orders of magnitude and
  the iterates end near (mu*, xi*).
"""
import numpy as np
import pytest
import torch

import oracle
import synth


def test_adam_matches_torch():
    rng = np.random.default_rng(3)
    grads = rng.normal(size=(60, 2)) * np.array([0.05, 3e-6])
    lr = (0.003, 30.0)
    s = oracle.adam_init(lr, 0.9, 0.999, 1e-8)
    theta = [0.26, 1400.0]
    p = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in theta]
    b1, b2, eps = (float(np.float32(v)) for v in (0.9, 0.999, 1e-8))
    opts = [torch.optim.Adam([p[i]], lr=float(np.float32(lr[i])), betas=(b1, b2), eps=eps) for i in range(2)]
    for g in grads:
        theta = oracle.adam_step(s, theta, list(g))
        for i in range(2):
            opts[i].zero_grad()
            p[i].grad = torch.tensor(g[i], dtype=torch.float64)
            opts[i].step()
        for i in range(2):
            assert abs(theta[i] - p[i].item()) <= 1e-12 * abs(p[i].item())


def test_mse_and_raster_gradient():
    rng = np.random.default_rng(4)
    d = rng.random((37, 53)).astype(np.float32)
    t = rng.random((37, 53)).astype(np.float32)
    loss, g = oracle.mse_grad(d, t)
    diff = d.astype(np.float64) - t.astype(np.float64)
    # the differences are rounded once to binary32 before squaring
    assert abs(loss - np.mean(diff ** 2)) <= 2.0 * 2.0 ** -24 * loss
    assert g.dtype == np.float32
    np.testing.assert_allclose(g, 2.0 * diff / d.size, rtol=4 * 2.0 ** -24, atol=1e-30)


def test_deposit_of_fixed_point():
    q = np.array([[0, 1, 1 << 24, 3 << 23, -(5 << 22)]], np.int64)
    np.testing.assert_array_equal(oracle.deposit_of(q), np.array([[0.0, 2.0 ** -24, 1.0, 1.5, -1.25]], np.float32))


@pytest.fixture(scope="module")
def scene():
    c = synth.make_calibration()
    base = dict(flow_height=c.flow_height, persistence=0.9, randomness=0.16)
    P = 4
    pt = oracle.make_params(**dict(base, mu=c.mu_star, xi=c.xi_star))
    fwd = oracle.smooth_forward(c.dem, c.mask, c.cell_size, pt, P, c.step_limit, c.seed, mass=c.mass)
    return c, base, P, oracle.deposit_of(fwd.dep_q)


def test_calibration_recovers_the_target_parameters(scene):
    c, base, P, target = scene
    hist, (mu, xi) = oracle.calibrate(c.dem, c.mask, c.cell_size, base, P, c.step_limit, c.seed, target, c.mu0,
                                      c.xi0, 60, lr=(0.003, 30.0), mass=c.mass)
    assert hist.shape == (60, 5)
    assert hist[0, 1] == c.mu0 and hist[0, 2] == c.xi0
    assert hist[0, 3] > 0          # too much friction: the loss grows with mu
    assert hist[:, 0].min() < 0.01 * hist[0, 0]
    assert abs(mu - c.mu_star) < 0.01 and abs(xi - c.xi_star) < 200.0
