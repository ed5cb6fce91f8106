"""Pins of the oracle's tracking residual (Eq. 6) and uncertainty (Eq. 15)
against closed forms, brute force and library routines (CPU only)."""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar
from scipy.spatial.distance import cosine as scipy_cosine_distance

from oracle.uncertainty import RESIDUAL_WEIGHTS, box3, cosine, residual, uncertainty


def test_box3_brute_force_and_closed_forms():
    rng = np.random.default_rng(0)
    D = rng.uniform(0.5, 4.0, (7, 9))
    B = box3(D)
    H, W = D.shape
    for y in range(H):
        for x in range(W):
            vals = [D[yy, xx] for yy in range(y - 1, y + 2) for xx in range(x - 1, x + 2)
                    if 0 <= yy < H and 0 <= xx < W]
            assert abs(B[y, x] - sum(vals) / len(vals)) < 1e-14
    # constant map unchanged; an impulse spreads 1/9 inside, 1/6 on an edge, 1/4 in a corner
    assert np.allclose(box3(np.full((4, 5), 2.5)), 2.5)
    imp = np.zeros((5, 5))
    imp[2, 2] = 9.0
    assert abs(box3(imp)[1, 1] - 1.0) < 1e-15 and box3(imp)[0, 0] == 0.0
    edge = np.zeros((5, 5))
    edge[0, 2] = 6.0
    assert abs(box3(edge)[0, 2] - 1.0) < 1e-15
    corner = np.zeros((5, 5))
    corner[0, 0] = 4.0
    assert abs(box3(corner)[0, 0] - 1.0) < 1e-15 and abs(box3(corner)[1, 1] - 4.0 / 9.0) < 1e-15


def test_cosine_against_scipy_and_special_cases():
    rng = np.random.default_rng(1)
    F = rng.normal(size=(384, 3, 4))
    G = rng.normal(size=(384, 3, 4))
    c = cosine(F, G)
    for y in range(3):
        for x in range(4):
            assert abs(c[y, x] - (1.0 - scipy_cosine_distance(F[:, y, x], G[:, y, x]))) < 1e-13
    assert np.allclose(cosine(F, 3.0 * F), 1.0) and np.allclose(cosine(F, -F), -1.0)
    e = np.zeros((2, 1, 1))
    e[0] = 1.0
    f = np.zeros((2, 1, 1))
    f[1] = 5.0
    assert cosine(e, f)[0, 0] == 0.0
    assert cosine(np.zeros((2, 1, 1)), f)[0, 0] == 0.0  # a zero vector gives 0 (norm product floored)


def test_residual_hand_pixel():
    """One 3x3 view with every term known: colour L1 over channels, depth
    against the box-filtered observation, capped feature term, visibility."""
    rgb = np.zeros((3, 3, 3))
    obs = np.zeros((3, 3, 3))
    rgb[:, 1, 1] = (0.5, 0.2, 0.9)
    obs[:, 1, 1] = (0.4, 0.6, 0.9)          # |d| sum = 0.1 + 0.4 + 0 = 0.5
    obs_d = np.arange(9, dtype=np.float64).reshape(3, 3)  # box mean at the centre = 4
    depth = np.full((3, 3), 1.0)
    depth[1, 1] = 5.5                       # |5.5 - 4| = 1.5
    cos = np.full((3, 3), 0.25)             # 1 - cos = 0.75
    cos[0, 0] = -0.5                        # 1 - cos = 1.5, capped at 1
    alpha = np.full((3, 3), 0.95)           # 1 - alpha = 0.05 < 0.1: visible
    alpha[2, 2] = 0.85                      # 1 - alpha = 0.15: not visible
    R = residual(rgb, depth, alpha, cos, obs, obs_d)
    l1, l2, l3 = RESIDUAL_WEIGHTS
    assert abs(R[1, 1] - (l1 * 0.5 + l2 * 1.5 + l3 * 0.75)) < 1e-14
    # corner (0, 0): colour 0, depth |1 - mean(0, 1, 3, 4)| = 1, feature capped
    assert abs(R[0, 0] - (l2 * 1.0 + l3 * 1.0)) < 1e-14
    assert R[2, 2] == 0.0
    # a term's weight scales only that term
    R2 = residual(rgb, depth, alpha, cos, obs, obs_d, weights=(2 * l1, l2, l3))
    assert abs(R2[1, 1] - R[1, 1] - l1 * 0.5) < 1e-14


def test_uncertainty_minimises_eq15_per_pixel():
    R = np.array([[0.0, 1e-7, 0.01], [0.2, 0.2499, 0.2501]])
    smin = 1e-3
    sigma, xi, dyn = uncertainty(R, sigma_min=smin)
    objs = []
    for r, s in zip(R.ravel(), sigma.ravel()):
        f = lambda t: 0.5 * (r / t ** 2 + np.log(t))
        res = minimize_scalar(f, bounds=(smin, 100.0), method="bounded", options={"xatol": 1e-12})
        assert abs(res.x - s) <= 1e-5 * max(1.0, s), (r, s, res.x)
        assert f(s) <= res.fun + 1e-12
        objs.append(f(s))
    assert abs(xi - np.mean(objs)) < 1e-14
    # unconstrained pixels: sigma^2 = 2R and the objective is (1 + log 2R) / 4
    r = 0.2
    assert abs(sigma[1, 0] ** 2 - 2 * r) < 1e-15
    assert abs(0.5 * (r / sigma[1, 0] ** 2 + np.log(sigma[1, 0])) - 0.25 * (1 + np.log(2 * r))) < 1e-14
    # R = 0 and tiny R sit on the floor
    assert sigma[0, 0] == smin and sigma[0, 1] == smin
    # motion mask 2 sigma^2 > 1, i.e. 4R > 1: just below and just above the threshold
    assert dyn.tolist() == [[False, False, False], [False, False, True]]
    assert (dyn == (2 * sigma ** 2 > 1)).all()
    _, _, dyn2 = uncertainty(R, sigma_min=smin, dyn_thresh=0.5)
    assert dyn2[1, 0] and dyn2[1, 1] and not dyn2[0, 2]
    # a floor above the threshold marks every pixel dynamic
    _, _, dyn3 = uncertainty(R, sigma_min=0.8)
    assert dyn3.all()


@pytest.mark.parametrize("seed", [0, 1])
def test_residual_nonnegative_and_bounded(seed):
    rng = np.random.default_rng(seed)
    H, W = 6, 7
    rgb, obs = rng.uniform(size=(3, H, W)), rng.uniform(size=(3, H, W))
    d, od = rng.uniform(1, 4, (H, W)), rng.uniform(1, 4, (H, W))
    cos = rng.uniform(-1, 1, (H, W))
    alpha = rng.uniform(0.8, 1.0, (H, W))
    R = residual(rgb, d, alpha, cos, obs, od)
    l1, l2, l3 = RESIDUAL_WEIGHTS
    assert (R >= 0).all()
    assert (R <= l1 * 3 + l2 * 3 + l3 + 1e-12).all()
    assert (R[(1 - alpha) >= 0.1] == 0).all()
