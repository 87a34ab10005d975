"""Pins for the warm-start application and the network's training loop in the
oracle (CPU only).

The warm start is checked on a loss whose minimiser is known (a quadratic
bowl), so every outcome of the alpha = 1, 1/2, 1/4 retries and of the fallback
is fixed by arithmetic; the training loop is checked against its special cases
(one full batch = one Adam step on the full-data gradient, a zero learning
rate, a batch of one row) and against the library routines it must reduce to.
"""
import math

import numpy as np
import pytest

from oracle import alloc as A
from oracle import mlp as Mo


def _bowl(theta_star):
    return lambda th: float(np.sum((np.asarray(th) - theta_star) ** 2))


@pytest.mark.parametrize("scale,applied", [(1.0, 1), (2.5, 2), (5.0, 3), (10.0, 0), (-1.0, 0)])
def test_warmstart_picks_first_alpha_that_lowers_the_loss(scale, applied):
    """Delta = scale (theta* - theta): on the bowl L(alpha) = (1 - alpha scale)^2 L(0),
    so alpha is accepted iff |1 - alpha scale| < 1.  scale 2.5: alpha 1 gives
    2.25 L0 (rejected), 1/2 gives 0.0625 L0 (kept); scale 5: 16, 2.25, then
    0.0625; scale 10: 81, 16, 2.25 -> fallback; scale -1: 4, 2.25, 1.5625."""
    rng = np.random.default_rng(3)
    n = 7
    theta = rng.normal(size=(11, n))
    star = theta + rng.normal(size=(11, n))
    tmean = rng.normal(size=11)
    tstd = rng.uniform(0.5, 2.0, size=11)
    delta = scale * (star - theta).T                     # [n, 11]
    Y = (delta - tmean) / tstd                           # standardised network output
    got, L, th = Mo.warmstart(theta, Y, tmean, tstd, _bowl(star))
    L0 = np.sum((theta - star) ** 2)
    assert got == applied
    assert abs(L[0] - L0) <= 1e-12 * L0
    tried = applied if applied else 3
    for j in range(1, 4):
        alpha = Mo.WARM_ALPHAS[j - 1]
        if j <= tried:
            assert abs(L[j] - (1 - alpha * scale) ** 2 * L0) <= 1e-9 * L0
        else:
            assert math.isnan(L[j])
    if applied:
        alpha = Mo.WARM_ALPHAS[applied - 1]
        assert np.allclose(th, theta + alpha * scale * (star - theta), atol=1e-12)
    else:
        assert np.array_equal(th, theta)


def test_warmstart_rejects_non_finite_losses_and_destandardises():
    theta = np.zeros((11, 3))
    Y = np.zeros((3, 11))
    tmean = np.arange(11.0)
    tstd = np.full(11, 4.0)
    assert np.array_equal(Mo.destandardise(Y, tmean, tstd), np.tile(tmean, (3, 1)))
    assert np.array_equal(Mo.destandardise(np.ones((3, 11)), tmean, tstd),
                          np.tile(tmean + 4.0, (3, 1)))
    got, L, th = Mo.warmstart(theta, Y, tmean, tstd,
                              lambda t: 1.0 if not np.any(t) else math.nan)
    assert got == 0 and L[0] == 1.0 and all(math.isnan(x) for x in L[1:])
    assert np.array_equal(th, theta)


def test_column_stats_are_population_moments_with_a_floor():
    rng = np.random.default_rng(0)
    X = rng.normal(3.0, 2.0, size=(1000, 5))
    X[:, 4] = 7.0
    m, s = Mo.column_stats(X)
    assert np.allclose(m, X.mean(axis=0), rtol=1e-12)
    assert np.allclose(s[:4], X[:, :4].std(axis=0), rtol=1e-9)
    assert s[4] == 1.0 and m[4] == 7.0


def test_epoch_permutation_is_a_seeded_stable_sort_of_counter_keys():
    n = 5000
    p = Mo.epoch_permutation(n, seed=11, epoch=2)
    assert np.array_equal(np.sort(p), np.arange(n))
    keys = (A.hash_bits(11, 2, np.arange(n, dtype=np.uint64)) >> np.uint64(32)).astype(np.uint64)
    k = keys[p]
    assert np.all(k[:-1] <= k[1:])
    ties = np.nonzero(k[:-1] == k[1:])[0]
    assert np.all(p[ties] < p[ties + 1])
    assert not np.array_equal(p, Mo.epoch_permutation(n, 11, 3))
    assert not np.array_equal(p, Mo.epoch_permutation(n, 12, 2))
    # uniform: every position equally likely for row 0 (chi-square over 200 epochs)
    pos = np.array([int(np.nonzero(Mo.epoch_permutation(10, 5, e) == 0)[0][0]) for e in range(400)])
    counts = np.bincount(pos, minlength=10)
    assert np.sum((counts - 40.0) ** 2 / 40.0) < 27.9          # chi2(9) at p = 0.001


def _data(n, seed=1):
    rng = np.random.default_rng(seed)
    X = rng.normal(2.0, 3.0, size=(n, Mo.D_IN))
    T = np.tanh(X @ rng.normal(size=(Mo.D_IN, Mo.D_OUT)) / 6.0) + 0.5
    return X, T


def test_full_batch_epoch_is_one_adam_step_on_the_full_data_gradient():
    X, T = _data(64)
    p0 = Mo.init_params(4)
    p1, stats, hist = Mo.train(p0, X, T, epochs=1, batch=64, lr=1e-3, seed=9, bf16=False,
                               stats_dtype=np.float64)
    fm, fs, tm, ts = stats
    assert np.allclose(fm, X.mean(axis=0)) and np.allclose(ts, T.std(axis=0))
    L, g = Mo.loss_and_grads(p0, (X - fm) / fs, (T - tm) / ts)
    ref = Mo.adam(p0, g, {}, lr=1e-3)
    assert abs(hist[0] - L) <= 1e-12 * L
    for k in p0:
        assert np.allclose(p1[k], ref[k], rtol=0, atol=1e-12), k
        # first Adam step moves every weight with a clear gradient by -lr sign(g)
        # (|step| = lr |g| / (|g| + eps), within lr eps / |g| of lr)
        big = np.abs(g[k]) > 1e-4
        assert big.sum() > 0.5 * big.size
        assert np.allclose((p1[k] - p0[k])[big], -1e-3 * np.sign(g[k][big]), atol=1e-3 * 1e-4)


def test_zero_rate_keeps_weights_and_batch_of_one_visits_every_row_once():
    X, T = _data(12, seed=2)
    p0 = Mo.init_params(6)
    p1, stats, hist = Mo.train(p0, X, T, epochs=2, batch=1, lr=0.0, seed=3, bf16=False,
                               stats_dtype=np.float64)
    for k in p0:
        assert np.array_equal(p1[k], p0[k])
    fm, fs, tm, ts = stats
    L, _ = Mo.loss_and_grads(p0, (X - fm) / fs, (T - tm) / ts)
    # the mean of the twelve one-row losses is the full-data mean loss
    assert np.allclose(hist, L, rtol=1e-12)


def test_training_lowers_the_loss_on_a_learnable_map():
    X, T = _data(512, seed=5)
    p, _, hist = Mo.train(Mo.init_params(1), X, T, epochs=6, batch=64, lr=3e-3, seed=2,
                          bf16=True)
    assert hist[-1] < 0.5 * hist[0]


def test_flat_layout_round_trip():
    p = Mo.init_params(2)
    flat = np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"],
                           p["W3"].ravel(), p["b3"]])
    assert flat.size == 20107
    q = Mo.flat_to_params(flat)
    for k in p:
        assert np.array_equal(p[k], q[k])
