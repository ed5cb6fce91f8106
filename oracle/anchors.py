"""Probabilistic anchor update (Sec. 3.3, Eq. 7) in float64 (test
infrastructure, see the package docstring).

Each anchor n carries the probability P(n | z_1:t) that it is occupied by
static structure; a new observation z_t with P(n | z_t) updates it by Bayes'
rule with the prior P(n), in the odds form of occupancy mapping:
  P(n | z_1:t) = [1 + (1 - P(n|z_t))/P(n|z_t) * (1 - P(n|z_1:t-1))/P(n|z_1:t-1)
                    * P(n)/(1 - P(n))]^-1
(Eq. 7's garbled P(n)/P(n) factor read as the prior odds P(n)/(1 - P(n))).
The result is clamped to [p_min, p_max]; anchors below prune_below are
marked for removal. Readings: ``oracle.readings.ANCHOR_READINGS``.
"""
from __future__ import annotations

import numpy as np


def anchor_update(p_prev, p_obs, prior=0.5, p_min=0.0, p_max=1.0, prune_below=0.0):
    """Returns (p_new, keep) for arrays of previous and observation
    probabilities in (0, 1)."""
    p_prev = np.asarray(p_prev, np.float64)
    p_obs = np.asarray(p_obs, np.float64)
    odds = ((1.0 - p_obs) / p_obs) * ((1.0 - p_prev) / p_prev) * (prior / (1.0 - prior))
    p = 1.0 / (1.0 + odds)
    p = np.minimum(np.maximum(p, p_min), p_max)
    return p, p >= prune_below
