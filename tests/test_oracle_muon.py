"""Pins of the oracle's Muon update (oracle.muon) to facts that do not come
from the oracle itself: the Newton-Schulz quintic acts on singular values
only (closed form through an SVD built by hand), the rank-one closed form,
the near-orthogonality the published coefficients are designed for, and the
parameter count of the matrices Muon takes."""
import math

import numpy as np
import pytest

from oracle import estimator, muon, network as net
from workloads import ModelConfig

A, B, C = 3.4445, -4.7750, 2.0315       # published with the Muon optimiser


def _scalar_map(x, steps):
    for _ in range(steps):
        x = A * x + B * x ** 3 + C * x ** 5
    return x


def _orthonormal(rng, n, k):
    q, r = np.linalg.qr(rng.standard_normal((n, k)))
    return q * np.sign(np.diag(r))


def _with_svd(rng, rows, cols, s):
    k = min(rows, cols)
    U, V = _orthonormal(rng, rows, k), _orthonormal(rng, cols, k)
    return U, V, (U * s) @ V.T


@pytest.mark.parametrize("rows,cols", [(16, 48), (48, 16), (32, 32), (20, 37), (37, 20), (1, 9), (128, 384)])
@pytest.mark.parametrize("steps", [1, 5])
def test_newton_schulz_acts_on_singular_values(rows, cols, steps):
    """M = U diag(s) V^T  =>  NS(M) = U diag(p^steps(s / ||s||)) V^T."""
    rng = np.random.default_rng(rows * 1000 + cols + steps)
    k = min(rows, cols)
    s = np.sort(rng.uniform(0.05, 3.0, k))[::-1] * 7.0
    U, V, M = _with_svd(rng, rows, cols, s)
    eps = 1e-7
    want = (U * _scalar_map(s / (np.linalg.norm(s) + eps), steps)) @ V.T
    got = muon.newton_schulz(M, steps, eps)
    assert got.shape == M.shape
    assert np.max(np.abs(got - want)) < 1e-12


def test_newton_schulz_rank_one_closed_form():
    """The all-ones r x c matrix has one singular value sqrt(rc) with unit
    vectors 1/sqrt(r), 1/sqrt(c): NS gives p^5(1) / sqrt(rc) everywhere (eps = 0)."""
    for r, c in [(3, 5), (8, 2), (6, 6)]:
        got = muon.newton_schulz(np.ones((r, c)), 5, 0.0)
        assert np.allclose(got, _scalar_map(1.0, 5) / math.sqrt(r * c), rtol=0, atol=1e-14)


@pytest.mark.parametrize("rows,cols", [(128, 512), (512, 128), (384, 128), (40, 100)])
def test_newton_schulz_is_nearly_orthogonal(rows, cols):
    """The published coefficients push every singular value of a well-
    conditioned matrix into roughly [0.7, 1.2] after 5 iterations."""
    M = np.random.default_rng(rows + cols).standard_normal((rows, cols))
    s = np.linalg.svd(muon.newton_schulz(M), compute_uv=False)
    assert 0.6 < s.min() and s.max() < 1.25


def _cfg():
    return ModelConfig(n_spins=6, d_model=8, n_layers=2, n_heads=1).full_causal()


def test_muon_takes_exactly_the_layer_matrices():
    """Count of Muon entries = n_layers * (3d*d + 4d*d + d*4d) = 11 d^2 n_layers;
    with an all-ones gradient, Adam entries move by lr/(1+eps) and Muon
    entries by the rank-one closed form."""
    cfg = _cfg()
    d, L = cfg.d_model, cfg.n_layers
    n = net.count(cfg)
    theta = np.zeros(n)
    lr, alr = 1e-2, 1e-3
    new, _, _ = muon.muon_update(theta, np.ones(n), np.zeros(n), np.zeros(n), 1, cfg, lr, ns_eps=0.0, adam_lr=alr)
    step = -new
    adam_moved = np.isclose(step, alr / (1 + 1e-8), rtol=1e-12, atol=0)
    assert int((~adam_moved).sum()) == 11 * d * d * L
    off = 0
    for name, shape in net.layout(cfg):
        k = int(np.prod(shape))
        if not adam_moved[off]:
            r, c = shape
            want = lr * 0.2 * math.sqrt(max(r, c)) * _scalar_map(1.0, 5) / math.sqrt(r * c)
            assert np.allclose(step[off:off + k], want, rtol=1e-12, atol=0)
        off += k


def test_muon_two_steps_closed_form():
    """Step 1 from M_0 = 0 and step 2 with momentum, on gradients built from
    known SVDs; the non-matrix entries follow Adam (pinned against
    torch.optim.Adam elsewhere)."""
    cfg = _cfg()
    rng = np.random.default_rng(5)
    n = net.count(cfg)
    theta0 = rng.standard_normal(n) * 0.1
    mu, lr, wd, eps = 0.9, 3e-2, 0.1, 1e-7
    g1, g2 = rng.standard_normal(n), rng.standard_normal(n)
    want1, want2, off = theta0.copy(), None, 0
    mats = []
    for name, shape in net.layout(cfg):
        k = int(np.prod(shape))
        if muon.is_muon_param(name):
            r, c = shape
            kk = min(r, c)
            s1 = rng.uniform(0.1, 2.0, kk)
            U1, V1, G1 = _with_svd(rng, r, c, s1)
            s2 = rng.uniform(0.1, 2.0, kk)
            U2, V2, M2 = _with_svd(rng, r, c, s2)
            g1[off:off + k] = G1.ravel()
            g2[off:off + k] = (M2 - mu * G1).ravel()       # so that M_2 = mu M_1 + G_2 = M2
            mats.append((off, k, r, c, U1, V1, s1, U2, V2, s2))
        off += k
    kw = dict(momentum=mu, weight_decay=wd, ns_eps=eps, adam_lr=1e-3)
    t1, m1, v1 = muon.muon_update(theta0, g1, np.zeros(n), np.zeros(n), 1, cfg, lr, **kw)
    t2, m2, v2 = muon.muon_update(t1, g2, m1, v1, 2, cfg, lr, **kw)
    muon_mask = muon.muon_entries(cfg)
    for off, k, r, c, U1, V1, s1, U2, V2, s2 in mats:
        scale = 0.2 * math.sqrt(max(r, c))
        O1 = (U1 * _scalar_map(s1 / (np.linalg.norm(s1) + eps), 5)) @ V1.T
        w0 = theta0[off:off + k]
        w1 = w0 - lr * (scale * O1.ravel() + wd * w0)
        O2 = (U2 * _scalar_map(s2 / (np.linalg.norm(s2) + eps), 5)) @ V2.T
        w2 = w1 - lr * (scale * O2.ravel() + wd * w1)
        assert np.max(np.abs(t1[off:off + k] - w1)) < 1e-12
        assert np.max(np.abs(t2[off:off + k] - w2)) < 1e-12
    a1, am, av = estimator.adam_update(theta0[~muon_mask], g1[~muon_mask], np.zeros((~muon_mask).sum()),
                                       np.zeros((~muon_mask).sum()), 1, 1e-3)
    a2, _, _ = estimator.adam_update(a1, g2[~muon_mask], am, av, 2, 1e-3)
    assert np.array_equal(t1[~muon_mask], a1) and np.array_equal(t2[~muon_mask], a2)
