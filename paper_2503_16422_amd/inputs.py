"""Seeded synthetic inputs: 4D Gaussian scenes and a pinhole camera rig.

This module only draws random numbers and builds camera poses.  It holds none
of the rendering arithmetic, so both the CPU oracle tests and the HIP path can
take their inputs from it without sharing any of the method's code.

Scene parameterisation follows the 4D Gaussian primitive of Sec. 3 (4D mean,
4D scale, a left and a right quaternion for the 4D rotation, an opacity, and a
view-dependent colour stored as real spherical-harmonic coefficients of degree
three, 16 basis functions x RGB).  All arrays are float32 structure-of-arrays:

    mean          [4][n]   x, y, z, t
    log_scale     [4][n]   s = exp(log_scale), one standard deviation per axis
    q_left        [4][n]   (w, x, y, z), unit length as drawn
    q_right       [4][n]
    opacity_logit [n]      opacity = sigmoid(logit)
    sh            [16][3][n]   basis k (l*l + l + m), colour channel c

Draw order (one numpy PCG64 generator per scene): spatial means, temporal
means, log spatial scales, [lifespan labels], log temporal scales, q_left,
q_right, opacity logits, SH DC, SH rest.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SH_COEFFS = 16


@dataclasses.dataclass
class Scene:
    mean: np.ndarray
    log_scale: np.ndarray
    q_left: np.ndarray
    q_right: np.ndarray
    opacity_logit: np.ndarray
    sh: np.ndarray
    sh_degree: int = 3

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.mean[:, idx].copy(), self.log_scale[:, idx].copy(),
                     self.q_left[:, idx].copy(), self.q_right[:, idx].copy(),
                     self.opacity_logit[idx].copy(), self.sh[:, :, idx].copy(),
                     self.sh_degree)

    def arrays(self):
        return (self.mean, self.log_scale, self.q_left, self.q_right,
                self.opacity_logit, self.sh)


@dataclasses.dataclass
class Camera:
    """World-to-camera pinhole, OpenCV axes (x right, y down, z forward).

    x_cam = R @ x_world + tvec;  u = fx*x/z + cx,  v = fy*y/z + cy.
    Pixel (px, py) is sampled at (px + 0.5, py + 0.5).
    """
    R: np.ndarray          # (3, 3) float64, row-major
    tvec: np.ndarray       # (3,) float64
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.2

    @property
    def center(self) -> np.ndarray:
        return -self.R.T @ self.tvec


def _unit_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def make_scene(n: int, seed: int, log_t_scale, *, sh_degree: int = 3) -> Scene:
    """Draw n Gaussians.

    log_t_scale is (mu, sd) for a single normal, or a list of
    (weight, mu, sd) components for a mixture (the label is drawn first).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    xyz = rng.uniform(-1.0, 1.0, size=(3, n))
    t = rng.uniform(0.0, 1.0, size=(1, n))
    log_s_xyz = rng.normal(-4.0, 0.5, size=(3, n))
    if isinstance(log_t_scale, tuple):
        mu, sd = log_t_scale
        log_s_t = rng.normal(mu, sd, size=(1, n))
    else:
        weights = np.array([c[0] for c in log_t_scale], dtype=np.float64)
        labels = rng.choice(len(log_t_scale), size=n, p=weights / weights.sum())
        z = rng.standard_normal(n)
        mus = np.array([c[1] for c in log_t_scale])[labels]
        sds = np.array([c[2] for c in log_t_scale])[labels]
        log_s_t = (mus + sds * z)[None, :]
    q_l = _unit_quaternions(rng, n)
    q_r = _unit_quaternions(rng, n)
    logit = rng.standard_normal(n)
    sh = np.empty((SH_COEFFS, 3, n))
    sh[0] = rng.normal(0.0, 0.3, size=(3, n))
    sh[1:] = rng.normal(0.0, 0.05, size=(SH_COEFFS - 1, 3, n))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f32(np.concatenate([xyz, t])), f32(np.concatenate([log_s_xyz, log_s_t])),
                 f32(q_l), f32(q_r), f32(logit), f32(sh), sh_degree)


# Workload families --------------------------------------------------------
TINY_T_SCALE = (-2.5, 0.5)                      # 10k-Gaussian plain render
DENSE_T_SCALE = [(0.8, -4.5, 0.3), (0.2, -1.0, 0.3)]   # 80% short, 20% long lifespan
LONG_T_SCALE = (-1.0, 0.4)                      # pruned scene, long lifespans


def tiny_scene(n: int = 10_000, seed: int = 0) -> Scene:
    return make_scene(n, seed, TINY_T_SCALE)


def dense_scene(n: int = 3_000_000, seed: int = 0) -> Scene:
    return make_scene(n, seed, DENSE_T_SCALE)


def long_scene(n: int = 200_000, seed: int = 0) -> Scene:
    return make_scene(n, seed, LONG_T_SCALE)


def look_at_camera(phi_deg: float, radius: float, width: int, height: int,
                   fov_x_deg: float = 60.0, znear: float = 0.2) -> Camera:
    """Camera on the y=0 circle at angle phi (world y up), aimed at the origin."""
    phi = math.radians(phi_deg)
    C = radius * np.array([math.sin(phi), 0.0, math.cos(phi)])
    fwd = -C / np.linalg.norm(C)
    down = np.array([0.0, -1.0, 0.0])
    down = down - fwd * (down @ fwd)
    down /= np.linalg.norm(down)
    right = np.cross(down, fwd)
    R = np.stack([right, down, fwd])
    tvec = -R @ C
    f = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(R, tvec, f, f, width / 2.0, height / 2.0, width, height, znear)


def arc_cameras(n: int = 20, radius: float = 4.0, width: int = 1352, height: int = 1014,
                span_deg: float = 120.0):
    """n cameras evenly spaced on a span_deg arc centred on +z."""
    if n == 1:
        return [look_at_camera(0.0, radius, width, height)]
    return [look_at_camera(-span_deg / 2 + span_deg * k / (n - 1), radius, width, height)
            for k in range(n)]


def frame_times(n_frames: int = 300) -> np.ndarray:
    return np.arange(n_frames, dtype=np.float64) / (n_frames - 1)


def keyframe_windows(n_frames: int = 300, interval: int = 10):
    """Keyframes every `interval` frames plus the last frame.

    Returns (keyframe indices, list of (lo, hi) keyframe index pairs, window of
    each frame).  A frame that is itself a keyframe uses the window on its
    right; the last frame uses the last window.
    """
    keys = list(range(0, n_frames, interval))
    if keys[-1] != n_frames - 1:
        keys.append(n_frames - 1)
    windows = [(keys[i], keys[i + 1]) for i in range(len(keys) - 1)]
    frame_window = np.minimum(np.arange(n_frames) // interval, len(windows) - 1)
    return keys, windows, frame_window


def batched_scene_sizes():
    return [50_000, 80_000, 120_000, 160_000, 200_000, 260_000, 320_000, 400_000]


def batch_cameras(width: int = 800, height: int = 800):
    return [look_at_camera(phi, 4.0, width, height) for phi in (-60.0, -20.0, 20.0, 60.0)]
