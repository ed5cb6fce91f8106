"""Rigid-body and rotation helpers (float64, differentiable).

Test infrastructure (see the package docstring).
"""
from __future__ import annotations

import torch

F64 = torch.float64


def hat(w: torch.Tensor) -> torch.Tensor:
    """Skew matrix [w]x with [w]x v = w x v."""
    z = torch.zeros((), dtype=w.dtype)
    return torch.stack([
        torch.stack([z, -w[2], w[1]]),
        torch.stack([w[2], z, -w[0]]),
        torch.stack([-w[1], w[0], z]),
    ])


def se3_exp(xi: torch.Tensor) -> torch.Tensor:
    """Exp of the twist xi = (rho, phi) as a 4x4 matrix, via the matrix
    exponential of [[phi]x, rho; 0, 0]."""
    M = torch.zeros((4, 4), dtype=xi.dtype)
    M = M.index_put((torch.tensor([0, 1, 2]).repeat_interleave(3), torch.tensor([0, 1, 2] * 3)),
                    hat(xi[3:6]).reshape(-1))
    M = M.index_put((torch.tensor([0, 1, 2]), torch.tensor([3, 3, 3])), xi[0:3])
    return torch.linalg.matrix_exp(M)


def pose_cw(T_wc, xi: torch.Tensor | None = None):
    """World-to-camera rotation and translation from a 3x4 camera-to-world pose.

    R_cw is the transpose of the rotation block of T_wc and t_cw = -R_cw c,
    c = the translation column (the camera centre). With ``xi``, the pose is
    left-perturbed: T_cw <- Exp(xi) T_cw.
    """
    T = torch.as_tensor(T_wc, dtype=F64)
    R_cw = T[:, :3].T
    t_cw = -R_cw @ T[:, 3]
    if xi is not None:
        E = se3_exp(xi)
        R_cw = E[:3, :3] @ R_cw
        t_cw = E[:3, :3] @ t_cw + E[:3, 3]
    return R_cw, t_cw


def camera_center(R_cw: torch.Tensor, t_cw: torch.Tensor) -> torch.Tensor:
    """World position of the camera centre, c = -R_cw^T t_cw."""
    return -R_cw.T @ t_cw


def quat_to_rotmat(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrices (n,3,3) from unit quaternions (n,4) ordered (w,x,y,z)."""
    w, x, y, z = q.unbind(-1)
    r00 = 1 - 2 * (y * y + z * z)
    r01 = 2 * (x * y - w * z)
    r02 = 2 * (x * z + w * y)
    r10 = 2 * (x * y + w * z)
    r11 = 1 - 2 * (x * x + z * z)
    r12 = 2 * (y * z - w * x)
    r20 = 2 * (x * z - w * y)
    r21 = 2 * (y * z + w * x)
    r22 = 1 - 2 * (x * x + y * y)
    return torch.stack([
        torch.stack([r00, r01, r02], -1),
        torch.stack([r10, r11, r12], -1),
        torch.stack([r20, r21, r22], -1),
    ], -2)
