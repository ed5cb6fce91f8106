"""Pins of the oracle's probabilistic anchor update (Eq. 7): log-odds
additivity, fixed points, repeated observations and clamping (CPU only)."""
import numpy as np

from oracle.anchors import anchor_update


def logit(p):
    return np.log(p / (1 - p))


def test_log_odds_add_up():
    rng = np.random.default_rng(0)
    pp, po = rng.uniform(0.01, 0.99, 200), rng.uniform(0.01, 0.99, 200)
    for prior in (0.5, 0.3, 0.8):
        p, keep = anchor_update(pp, po, prior)
        assert np.abs(logit(p) - (logit(po) + logit(pp) - logit(prior))).max() < 1e-10
        assert keep.all()


def test_neutral_observation_and_prior():
    pp = np.array([0.1, 0.5, 0.93])
    p, _ = anchor_update(pp, np.full(3, 0.5), prior=0.5)
    assert np.abs(p - pp).max() < 1e-15
    # an observation equal to the prior leaves the estimate unchanged for any prior
    p, _ = anchor_update(pp, np.full(3, 0.3), prior=0.3)
    assert np.abs(p - pp).max() < 1e-15


def test_repeated_observations_and_clamping():
    p = np.array([0.5])
    for t in range(1, 6):
        p, _ = anchor_update(p, np.array([0.7]))
        assert abs(logit(p[0]) - t * logit(0.7)) < 1e-12
    p, keep = anchor_update(np.array([0.2, 0.9]), np.array([0.1, 0.99]), p_min=0.12, p_max=0.97, prune_below=0.15)
    # 0.2 with 0.1: odds 9 * 4 = 36 -> 1/37 = 0.027 -> clamped to 0.12 -> pruned
    assert abs(p[0] - 0.12) < 1e-15 and not keep[0]
    assert abs(p[1] - 0.97) < 1e-15 and keep[1]
