"""Seeded scene, camera and target generators (numpy PCG64, float32 outputs).

Every generator documents its draw order so that a scene is a pure function of
its seed. Arrays are laid out as the library consumes them: per-Gaussian
attributes as planes ``[c][n]`` (structure of arrays), anchor features as
``[A][32]`` rows. The workloads mirror the 640x480 RGB-D setting of the paper
(Sec. 4.1, dataset paragraph of the appendix): the datasets themselves are not
available, so these synthetic rooms stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, Optional, Tuple

import numpy as np

# Decoder heads in the fixed order used everywhere: name, values per Gaussian.
# opacity, colour, scale, rotation (quaternion w,x,y,z) and low-dim feature.
HEADS: Tuple[Tuple[str, int], ...] = (
    ("opacity", 1),
    ("rgb", 3),
    ("scale", 3),
    ("rot", 4),
    ("feat", 16),
)

ROOM_LO = np.array([-2.0, -1.5, 0.0])
ROOM_HI = np.array([2.0, 1.5, 3.0])
VOXEL = 0.02
GRID = (200, 150, 150)  # cells along x, y, z (4 m x 3 m x 3 m at 2 cm)


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    T_wc: np.ndarray  # (3, 4) float32, camera-to-world, row-major
    t: float = 0.0    # frame time (the temporal embedding of the scene-variant decoder)

    def copy_with(self, T_wc: np.ndarray) -> "Camera":
        return Camera(self.width, self.height, self.fx, self.fy, self.cx, self.cy,
                      np.ascontiguousarray(T_wc, dtype=np.float32), self.t)


@dataclass
class PlainScene:
    """Explicit Gaussians, planes [c][n] float32."""
    mean: np.ndarray
    scale: np.ndarray
    rot: np.ndarray
    opacity: np.ndarray
    rgb: np.ndarray
    feat: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])

    def arrays(self) -> Dict[str, np.ndarray]:
        d = dict(mean=self.mean, scale=self.scale, rot=self.rot,
                 opacity=self.opacity, rgb=self.rgb)
        if self.feat is not None:
            d["feat"] = self.feat
        return d


@dataclass
class AnchorScene:
    """Anchors with k offsets each, plus five two-layer head MLPs."""
    xyz: np.ndarray          # (3, A) float32
    feat: np.ndarray         # (A, 32) float32
    off: np.ndarray          # (3, A*k) float32, Gaussian n = v*k + i
    k: int
    weights: Dict[str, Dict[str, np.ndarray]] = field(default_factory=dict)
    l_o: float = 1.0         # offset scaling (metres per unit offset)
    l_s: float = VOXEL       # scale bound (metres), the voxel size
    in_dim: int = 35
    hidden: int = 32

    @property
    def n_anchors(self) -> int:
        return int(self.xyz.shape[1])

    @property
    def n_gauss(self) -> int:
        return self.n_anchors * self.k


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def look_at(eye, target, up) -> np.ndarray:
    """Camera-to-world 3x4 (x right, y down, z forward), centre = eye."""
    eye = np.asarray(eye, np.float64)
    zc = np.asarray(target, np.float64) - eye
    zc /= np.linalg.norm(zc)
    xc = np.cross(zc, np.asarray(up, np.float64))
    xc /= np.linalg.norm(xc)
    yc = np.cross(zc, xc)
    T = np.zeros((3, 4))
    T[:, 0], T[:, 1], T[:, 2], T[:, 3] = xc, yc, zc, eye
    return _f32(T)


def camera_c1() -> Camera:
    return Camera(160, 120, 150.0, 150.0, 79.5, 59.5, _f32(np.eye(3, 4)))


C2_EYE = (-1.6, -1.1, 0.2)
C2_TARGET = (1.0, 0.6, 3.0)
C2_UP = (0.0, -1.0, 0.0)


def camera_c2(T_wc: Optional[np.ndarray] = None) -> Camera:
    if T_wc is None:
        T_wc = look_at(C2_EYE, C2_TARGET, C2_UP)
    return Camera(640, 480, 525.0, 525.0, 319.5, 239.5, _f32(T_wc))


def camera_half(T_wc: np.ndarray) -> Camera:
    """320x240 keyframe camera with the same field of view as camera_c2."""
    return Camera(320, 240, 262.5, 262.5, 159.5, 119.5, _f32(T_wc))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def plain_scene(seed: int = 0, n: int = 10_000, n_feat: int = 0) -> PlainScene:
    """Explicit Gaussians in a box in front of an identity camera.

    Draw order: xy ~ U[-1,1]^2 (n,2); z ~ U[1,5] (n); log-scale ~ N(-3,0.5)
    (n,3); quaternion ~ N(0,I4) (n,4) then unit-normalised; opacity logit
    ~ N(0,1) (n); rgb ~ U[0,1] (n,3); [feat ~ N(0,1) (n,n_feat)].
    """
    rng = np.random.default_rng(seed)
    xy = rng.uniform(-1.0, 1.0, (n, 2))
    z = rng.uniform(1.0, 5.0, n)
    logs = rng.normal(-3.0, 0.5, (n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    o = _sigmoid(rng.normal(size=n))
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    feat = rng.normal(size=(n, n_feat)) if n_feat else None
    mean = np.stack([xy[:, 0], xy[:, 1], z])
    return PlainScene(mean=_f32(mean), scale=_f32(np.exp(logs).T), rot=_f32(q.T),
                      opacity=_f32(o), rgb=_f32(rgb.T),
                      feat=None if feat is None else _f32(feat.T))


def tiny_scene(seed: int, n: int, n_feat: int = 0, logs_mu: float = -2.3,
               logs_sd: float = 0.4, zrange=(1.5, 4.0), spread: float = 0.8) -> PlainScene:
    """Small scenes for brute-force and finite-difference checks.

    Same draw order as plain_scene, with adjustable spread, depth range and
    log-scale distribution so that a few dozen Gaussians cover a small image.
    """
    rng = np.random.default_rng(seed)
    xy = rng.uniform(-spread, spread, (n, 2))
    z = rng.uniform(zrange[0], zrange[1], n)
    logs = rng.normal(logs_mu, logs_sd, (n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    o = _sigmoid(rng.normal(size=n))
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    feat = rng.normal(size=(n, n_feat)) if n_feat else None
    mean = np.stack([xy[:, 0] * z / 2.0, xy[:, 1] * z / 2.0, z])
    return PlainScene(mean=_f32(mean), scale=_f32(np.exp(logs).T), rot=_f32(q.T),
                      opacity=_f32(o), rgb=_f32(rgb.T),
                      feat=None if feat is None else _f32(feat.T))


def tiny_anchor_scene(seed: int, n_anchors: int = 24, k: int = 4, n_feat: int = 4,
                      l_s: float = 0.15, in_dim: int = 35) -> AnchorScene:
    """A few anchors in front of an identity camera for brute-force and
    finite-difference checks of the decoder.

    Draw order: anchor xy ~ U[-0.6,0.6]^2 scaled by depth/2, depth ~ U[2,4]
    (A,3 drawn as xy then z); features ~ N(0, 0.3) (A,32); offsets
    ~ N(0, 0.1) (A,k,3); then the head weights (anchor_weights).
    """
    rng = np.random.default_rng(seed)
    xy = rng.uniform(-0.6, 0.6, (n_anchors, 2))
    z = rng.uniform(2.0, 4.0, n_anchors)
    xyz = np.stack([xy[:, 0] * z / 2, xy[:, 1] * z / 2, z])
    feat = rng.normal(0.0, 0.3, (n_anchors, 32))
    off = rng.normal(0.0, 0.1, (n_anchors, k, 3))
    weights = anchor_weights(rng, k, in_dim=in_dim, n_feat=n_feat)
    return AnchorScene(xyz=_f32(xyz), feat=_f32(feat), off=_f32(off.reshape(n_anchors * k, 3).T),
                       k=k, weights=weights, l_s=l_s, in_dim=in_dim)


def room_cells(mode: str) -> np.ndarray:
    """Linear indices (i*150 + j)*150 + k of candidate anchor cells, ascending.

    mode 'shell': the 163 008 cells on the boundary of the 200x150x150 grid
    (the walls, floor and ceiling a depth camera sees); 'volume': all cells.
    """
    nx, ny, nz = GRID
    if mode == "volume":
        return np.arange(nx * ny * nz, dtype=np.int64)
    if mode != "shell":
        raise ValueError(mode)
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    shell = (i == 0) | (i == nx - 1) | (j == 0) | (j == ny - 1) | (k == 0) | (k == nz - 1)
    return np.flatnonzero(shell.ravel()).astype(np.int64)


def anchor_weights(rng: np.random.Generator, k: int, in_dim: int = 35, hidden: int = 32,
                   n_feat: int = 16) -> Dict[str, Dict[str, np.ndarray]]:
    """Per head, in HEADS order: W1 (hidden,in), b1 (hidden), W2 (k*m,hidden),
    b2 (k*m), each ~ U(+-1/sqrt(fan_in)). The feature head is skipped when
    n_feat == 0."""
    out = {}
    for name, m in HEADS:
        if name == "feat":
            if n_feat == 0:
                continue
            m = n_feat
        b1 = 1.0 / math.sqrt(in_dim)
        b2 = 1.0 / math.sqrt(hidden)
        W1 = rng.uniform(-b1, b1, (hidden, in_dim))
        c1 = rng.uniform(-b1, b1, hidden)
        W2 = rng.uniform(-b2, b2, (k * m, hidden))
        c2 = rng.uniform(-b2, b2, k * m)
        out[name] = dict(W1=_f32(W1), b1=_f32(c1), W2=_f32(W2), b2=_f32(c2))
    return out


def anchor_scene(seed: int, n_anchors: int, k: int = 10, mode: str = "shell",
                 n_feat: int = 16, in_dim: int = 35) -> AnchorScene:
    """Anchors on the 2 cm room grid.

    Draw order: cells = choice(candidates, A, replace=False) then sorted
    ascending; anchor features ~ N(0, 0.1) (A,32); offsets ~ N(0, 0.05) m
    (A,k,3); then the head weights (anchor_weights). Standard deviations are
    the second parameter of N(.,.).
    """
    rng = np.random.default_rng(seed)
    cand = room_cells(mode)
    cells = np.sort(rng.choice(cand, size=n_anchors, replace=False))
    nx, ny, nz = GRID
    i, rem = np.divmod(cells, ny * nz)
    j, kk = np.divmod(rem, nz)
    ijk = np.stack([i, j, kk]).astype(np.float64)
    xyz = ROOM_LO[:, None] + (ijk + 0.5) * VOXEL
    feat = rng.normal(0.0, 0.1, (n_anchors, 32))
    off = rng.normal(0.0, 0.05, (n_anchors, k, 3))
    weights = anchor_weights(rng, k, in_dim=in_dim, n_feat=n_feat)
    return AnchorScene(xyz=_f32(xyz), feat=_f32(feat),
                       off=_f32(off.reshape(n_anchors * k, 3).T), k=k,
                       weights=weights, in_dim=in_dim)


def targets(seed: int, height: int, width: int, channels: int) -> np.ndarray:
    """Per-pixel targets ~ U[0,1], shape (channels, H, W) float32."""
    rng = np.random.default_rng(seed)
    return _f32(rng.uniform(0.0, 1.0, (channels, height, width)))


def _hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def perturb_pose(T_wc: np.ndarray, rho, phi) -> np.ndarray:
    """Camera-to-world pose after the left perturbation T_cw <- Exp(xi) T_cw,
    xi = (rho, phi), with the closed-form SE(3) exponential (Rodrigues
    rotation and its left Jacobian for the translation)."""
    rho = np.asarray(rho, np.float64)
    phi = np.asarray(phi, np.float64)
    th = np.linalg.norm(phi)
    K = _hat(phi)
    if th < 1e-12:
        R = np.eye(3) + K
        V = np.eye(3) + 0.5 * K
    else:
        R = np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th**2 * K @ K
        V = np.eye(3) + (1 - math.cos(th)) / th**2 * K + (th - math.sin(th)) / th**3 * K @ K
    Twc = np.asarray(T_wc, np.float64)
    Rcw = Twc[:, :3].T
    tcw = -Rcw @ Twc[:, 3]
    R2 = R @ Rcw
    t2 = R @ tcw + V @ rho
    out = np.zeros((3, 4))
    out[:, :3] = R2.T
    out[:, 3] = -R2.T @ t2
    return _f32(out)


def _unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

def c1():
    """Plain 3DGS, 10k Gaussians at 160x120 (seed 0); targets rgb+depth (seed 1)."""
    scene = plain_scene(0, 10_000)
    cam = camera_c1()
    tgt = targets(1, cam.height, cam.width, 4)
    return scene, cam, tgt


def c2(mode: str = "shell", n_anchors: int = 20_000, seed: int = 2):
    """20k anchors x 10 on the 2 cm room grid at 640x480 with 16-d features;
    targets for all 21 channels (rgb, depth, 16 feat, alpha) from seed+100."""
    sc = anchor_scene(seed, n_anchors, 10, mode)
    cam = camera_c2()
    tgt = targets(seed + 100, cam.height, cam.width, 20)
    return sc, cam, tgt


def c3():
    """100k anchors -> 1M Gaussians on the shell (seed 3)."""
    return c2("shell", 100_000, seed=3)


def c4():
    """Tracking scene: the config-2 shell scene with the pose perturbed by
    2 cm and 1 degree about seeded unit axes (seed 4), per-pixel weights
    ~ U[0,1]."""
    sc, cam_gt, _ = c2("shell", 20_000, seed=2)
    rng = np.random.default_rng(4)
    u = _unit(rng)
    e = _unit(rng)
    rho0 = 0.02 * u
    phi0 = (math.pi / 180.0) * e
    T0 = perturb_pose(cam_gt.T_wc, rho0, phi0)
    weights = _f32(rng.uniform(0.0, 1.0, (cam_gt.height, cam_gt.width)))
    return sc, cam_gt, cam_gt.copy_with(T0), weights, (rho0, phi0)


def trajectory(seed: int, n_poses: int = 64):
    """Smooth camera path inside the room: the eye follows a seeded Lissajous
    curve around (0, 0, 1.5) and looks at a point that circles the far walls."""
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * math.pi, 4)
    amp = rng.uniform(0.3, 0.7, 3)
    poses = []
    for t in range(n_poses):
        s = 2 * math.pi * t / n_poses
        eye = (amp[0] * math.sin(s + ph[0]), 0.4 * amp[1] * math.sin(2 * s + ph[1]),
               1.5 + amp[2] * math.cos(s + ph[2]))
        tgt = (1.8 * math.cos(s + ph[3]), 0.3 * math.sin(s), 1.5 + 1.4 * math.sin(s + ph[3]))
        poses.append(look_at(eye, tgt, C2_UP))
    return poses


def c5():
    """Serving scene: 50k anchors x 10 on the shell (seed 5) and 64 poses."""
    sc = anchor_scene(5, 50_000, 10, "shell")
    return sc, trajectory(5)
