"""Host-side pose algebra of the autograd front end (no GPU): the SE(3)
exponential against the oracle's closed form, and the defining property of
the left Jacobian, Exp(xi + d) = Exp(J_l(xi) d) Exp(xi) + O(|d|^2)."""
import numpy as np
import torch

from oracle.geometry import se3_exp as oracle_se3_exp
from paper_2505_22335_amd.autograd import se3_exp, se3_left_jacobian, camera_at, T_cw_of
import synth


def _xi(seed, rho=0.3, phi=1.2):
    rng = np.random.default_rng(seed)
    a, b = rng.normal(size=3), rng.normal(size=3)
    return np.concatenate([rho * a / np.linalg.norm(a), phi * b / np.linalg.norm(b)])


def _hat(w):
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])


def test_exp_matches_closed_form():
    """Rodrigues' formula for the rotation and the V matrix for the
    translation of Exp((rho, phi))."""
    for s in range(4):
        xi = _xi(s)
        rho, phi = xi[:3], xi[3:]
        th = np.linalg.norm(phi)
        K = _hat(phi)
        R = np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th ** 2 * K @ K
        V = np.eye(3) + (1 - np.cos(th)) / th ** 2 * K + (th - np.sin(th)) / th ** 3 * K @ K
        T = se3_exp(xi)
        assert np.abs(T[:3, :3] - R).max() < 1e-12
        assert np.abs(T[:3, 3] - V @ rho).max() < 1e-12
        assert np.abs(oracle_se3_exp(torch.as_tensor(xi)).numpy() - T).max() < 1e-12


def test_left_jacobian_property():
    for s in range(4):
        xi = _xi(10 + s)
        J = se3_left_jacobian(xi)
        E = se3_exp(xi)
        errs = []
        for eps in (1e-4, 5e-5):
            worst = 0.0
            for j in range(6):
                d = np.zeros(6)
                d[j] = eps
                lhs = se3_exp(xi + d)
                rhs = se3_exp(J @ d) @ E
                worst = max(worst, np.abs(lhs - rhs).max())
            errs.append(worst)
        assert errs[0] < 1e-6
        assert errs[1] < 0.3 * errs[0]          # second order remainder
    assert np.allclose(se3_left_jacobian(np.zeros(6)), np.eye(6))


def test_camera_placement_round_trip():
    cam = synth.camera_c2()
    T = T_cw_of(cam)
    c2 = camera_at(cam, T)
    assert np.abs(c2.T_wc - cam.T_wc).max() < 1e-6
    xi = _xi(3, 0.01, 0.02)
    c3 = camera_at(cam, se3_exp(xi) @ T)
    assert np.abs(T_cw_of(c3) - se3_exp(xi) @ T).max() < 1e-5
