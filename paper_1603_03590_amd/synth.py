"""Seeded synthetic frame pairs for optical-flow tests and benchmarks.

This module only makes inputs and ground truth.  It holds none of the flow
method's arithmetic, and both the GPU path's tests and the CPU oracle's tests
draw their inputs from here.

Two generators, standing in for the video workloads the paper measures on
(Sintel-shaped 1024x436 frames, VGA, wider KITTI-like frames):

* ``smooth_bump_pair``: a band-limited noise texture moved by a smooth flow
  made of four Gaussian bumps.
* ``layered_pair``: a textured background plus six textured rectangles, each
  layer under its own rigid motion (rotation about the layer centre plus a
  translation), drawn back to front, so layers occlude each other.

Conventions: frames are float32 ``[H][W]`` arrays in [0, 1]; flow is float64
``[2][H][W]`` (u along +x = columns, v along +y = rows) with
``I1(x + U(x)) ~= I0(x)``.  Every random number comes from
``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import ndimage

__all__ = [
    "texture",
    "smooth_bump_pair",
    "layered_pair",
    "FramePair",
    "batch_sizes",
]


@dataclass
class FramePair:
    I0: np.ndarray          # float32 [H][W] (colour: [C][H][W])
    I1: np.ndarray          # float32 [H][W] (colour: [C][H][W])
    flow: np.ndarray        # float64 [2][H][W], ground truth
    occluded: np.ndarray    # bool [H][W], True where x+flow is hidden or off-frame


def _upsample_linear(a: np.ndarray, factor: int, shape) -> np.ndarray:
    """Linear zoom by an integer factor, then crop to ``shape``."""
    if factor == 1:
        return a[: shape[0], : shape[1]]
    out = ndimage.zoom(a, factor, order=1, mode="nearest", grid_mode=False)
    return out[: shape[0], : shape[1]]


def texture(h: int, w: int, rng: np.random.Generator, octaves: int = 6) -> np.ndarray:
    """Band-limited ~1/f noise texture in [0, 1], float64 [h][w].

    Octave o is white noise on a grid 2^o times coarser, Gaussian-blurred
    (sigma 1 coarse pixel, so about 2^o full-resolution pixels), linearly
    zoomed to full size and scaled to unit standard deviation.  The octave sum
    is divided by sqrt(octaves) and mapped to clip(0.5 + z/6, 0, 1).
    """
    z = np.zeros((h, w), np.float64)
    for o in range(octaves):
        f = 1 << o
        hh, ww = h // f + 3, w // f + 3
        n = rng.standard_normal((hh, ww))
        n = ndimage.gaussian_filter(n, 1.0, mode="wrap") if o > 0 else n
        up = _upsample_linear(n, f, (h, w))
        up = up - up.mean()
        sd = up.std()
        z += up / (sd if sd > 0 else 1.0)
    z /= math.sqrt(octaves)
    return np.clip(0.5 + z / 6.0, 0.0, 1.0)


def _sample_bilinear(img: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Bilinear lookup with edge clamping, used only to render frames."""
    h, w = img.shape
    x0 = np.floor(x)
    y0 = np.floor(y)
    fx = x - x0
    fy = y - y0
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)
    xa = np.clip(x0, 0, w - 1)
    xb = np.clip(x0 + 1, 0, w - 1)
    ya = np.clip(y0, 0, h - 1)
    yb = np.clip(y0 + 1, 0, h - 1)
    top = img[ya, xa] * (1 - fx) + img[ya, xb] * fx
    bot = img[yb, xa] * (1 - fx) + img[yb, xb] * fx
    return top * (1 - fy) + bot * fy


def smooth_bump_pair(w: int, h: int, max_disp: float, seed: int,
                     noise_sigma: float = 0.01, n_bumps: int = 4, horizontal: bool = False,
                     channels: int = 1) -> FramePair:
    """I0 = texture; I1(y) = I0(y - v(y)) + noise, with v a sum of Gaussian bumps.

    The bump centres are uniform in the frame, widths uniform in
    [0.10, 0.25] * min(w, h), directions uniform; the field is rescaled so its
    largest displacement is ``max_disp`` px (``horizontal``: every bump
    points left or right, a rectified stereo pair).  Ground truth u solves
    u(x) = v(x + u(x)) (then I1(x + u) = I0(x)), by fixed-point iteration.

    ``channels`` > 1 gives colour frames ``[C][H][W]`` (planar): channel 0 is
    the grey pair above, drawn identically; channel c > 0 mixes that texture
    (weight 0.6) with a texture of its own (0.4), so the channels correlate
    as natural colour channels do, and carries noise of its own.  The extra
    draws come after every draw of the grey pair.
    """
    rng = np.random.default_rng(seed)
    pad = int(math.ceil(max_disp)) + 4
    canvas = texture(h + 2 * pad, w + 2 * pad, rng)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)

    cx = rng.uniform(0, w, n_bumps)
    cy = rng.uniform(0, h, n_bumps)
    sig = rng.uniform(0.10, 0.25, n_bumps) * min(w, h)
    ang = rng.uniform(0, 2 * math.pi, n_bumps)
    dir_x, dir_y = np.cos(ang), np.sin(ang)
    if horizontal:
        dir_x, dir_y = np.where(dir_x >= 0, 1.0, -1.0), np.zeros(n_bumps)

    def field(x, y):
        vx = np.zeros_like(x)
        vy = np.zeros_like(y)
        for k in range(n_bumps):
            g = np.exp(-((x - cx[k]) ** 2 + (y - cy[k]) ** 2) / (2 * sig[k] ** 2))
            vx += g * dir_x[k]
            vy += g * dir_y[k]
        return vx, vy

    vx, vy = field(xx, yy)
    scale = max_disp / max(np.sqrt(vx ** 2 + vy ** 2).max(), 1e-12)

    def v(x, y):
        a, b = field(x, y)
        return a * scale, b * scale

    I0 = canvas[pad:pad + h, pad:pad + w]
    vx, vy = v(xx, yy)
    I1 = _sample_bilinear(canvas, xx - vx + pad, yy - vy + pad)
    I1 = I1 + rng.normal(0.0, noise_sigma, I1.shape)

    # ground truth: u = v(x + u), a contraction because max|grad v| < 1 here
    ux = np.zeros_like(xx)
    uy = np.zeros_like(yy)
    for _ in range(200):
        nx, ny = v(xx + ux, yy + uy)
        delta = max(np.abs(nx - ux).max(), np.abs(ny - uy).max())
        ux, uy = nx, ny
        if delta < 1e-10:
            break
    occ = (xx + ux < 0) | (xx + ux > w - 1) | (yy + uy < 0) | (yy + uy > h - 1)
    if channels > 1:
        c0, c1 = [I0], [I1]
        for _ in range(1, channels):
            cv = 0.6 * canvas + 0.4 * texture(h + 2 * pad, w + 2 * pad, rng)
            c0.append(cv[pad:pad + h, pad:pad + w])
            J1 = _sample_bilinear(cv, xx - vx + pad, yy - vy + pad)
            c1.append(J1 + rng.normal(0.0, noise_sigma, J1.shape))
        I0, I1 = np.stack(c0), np.stack(c1)
    return FramePair(np.clip(I0, 0, 1).astype(np.float32),
                     np.clip(I1, 0, 1).astype(np.float32),
                     np.stack([ux, uy]), occ)


def _rot(theta):
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s], [s, c]])


def layered_pair(w: int, h: int, max_trans: float, seed: int,
                 n_rects: int = 6, max_rot_deg: float = 5.0,
                 noise_sigma: float = 0.01) -> FramePair:
    """Background plus ``n_rects`` rectangles, each under its own rigid motion.

    Layer k maps a frame-0 point x to R_k (x - c_k) + c_k + t_k, with R_k a
    rotation by U(-max_rot, max_rot) degrees about the layer centre c_k and t_k
    of length U(0, max_trans) at a uniform angle.  Rectangles have width
    U(0.1, 0.35)*w, height U(0.1, 0.35)*h and centres uniform in the frame;
    a later layer is drawn on top.  I1 is rendered by inverse mapping, with
    noise of standard deviation ``noise_sigma`` added to I1.  Ground truth at
    x is the motion of the top layer of frame 0 at x.
    """
    rng = np.random.default_rng(seed)
    diag = math.hypot(w, h)
    pad = int(math.ceil(max_trans + math.sin(math.radians(max_rot_deg)) * diag / 2)) + 8

    layers = []
    # background: whole (padded) frame, centred at the frame centre
    layers.append(dict(x0=-pad, y0=-pad, x1=w + pad, y1=h + pad,
                       c=np.array([(w - 1) / 2, (h - 1) / 2])))
    for _ in range(n_rects):
        rw = rng.uniform(0.1, 0.35) * w
        rh = rng.uniform(0.1, 0.35) * h
        cx = rng.uniform(0, w)
        cy = rng.uniform(0, h)
        layers.append(dict(x0=cx - rw / 2, y0=cy - rh / 2, x1=cx + rw / 2, y1=cy + rh / 2,
                           c=np.array([cx, cy])))
    for L in layers:
        th = math.radians(rng.uniform(-max_rot_deg, max_rot_deg))
        r = rng.uniform(0, max_trans)
        a = rng.uniform(0, 2 * math.pi)
        L["R"] = _rot(th)
        L["t"] = np.array([r * math.cos(a), r * math.sin(a)])
        # texture over the layer's bounding box (frame-0 coordinates) + 2 px margin
        tx0 = int(math.floor(L["x0"])) - 2
        ty0 = int(math.floor(L["y0"])) - 2
        tw = int(math.ceil(L["x1"])) + 2 - tx0 + 1
        th_ = int(math.ceil(L["y1"])) + 2 - ty0 + 1
        L["tex"] = texture(th_, tw, rng)
        L["tx0"], L["ty0"] = tx0, ty0

    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)

    def inside(L, x, y):
        return (x >= L["x0"]) & (x < L["x1"]) & (y >= L["y0"]) & (y < L["y1"])

    def sample(L, x, y):
        return _sample_bilinear(L["tex"], x - L["tx0"], y - L["ty0"])

    # frame 0: top layer at each pixel, texture at the pixel
    I0 = np.zeros((h, w))
    top0 = np.zeros((h, w), np.int64)
    for k, L in enumerate(layers):
        m = inside(L, xx, yy)
        I0[m] = sample(L, xx[m], yy[m])
        top0[m] = k

    # frame 1: inverse-map every pixel through each layer's motion
    I1 = np.zeros((h, w))
    top1 = np.full((h, w), -1, np.int64)
    pts = np.stack([xx.ravel(), yy.ravel()])
    for k, L in enumerate(layers):
        Rinv = L["R"].T
        q = Rinv @ (pts - (L["c"] + L["t"])[:, None]) + L["c"][:, None]
        qx = q[0].reshape(h, w)
        qy = q[1].reshape(h, w)
        m = inside(L, qx, qy)
        I1[m] = sample(L, qx[m], qy[m])
        top1[m] = k
    I1 = I1 + rng.normal(0.0, noise_sigma, I1.shape)

    # ground truth from the frame-0 top layer
    ux = np.zeros((h, w))
    uy = np.zeros((h, w))
    for k, L in enumerate(layers):
        m = top0 == k
        if not m.any():
            continue
        p = np.stack([xx[m], yy[m]])
        q = L["R"] @ (p - L["c"][:, None]) + (L["c"] + L["t"])[:, None]
        ux[m] = q[0] - p[0]
        uy[m] = q[1] - p[1]
    tx = xx + ux
    ty = yy + uy
    inframe = (tx >= 0) & (tx <= w - 1) & (ty >= 0) & (ty <= h - 1)
    txi = np.clip(np.rint(tx), 0, w - 1).astype(np.int64)
    tyi = np.clip(np.rint(ty), 0, h - 1).astype(np.int64)
    occ = ~inframe | (top1[tyi, txi] != top0)
    return FramePair(np.clip(I0, 0, 1).astype(np.float32),
                     np.clip(I1, 0, 1).astype(np.float32),
                     np.stack([ux, uy]), occ)


BATCH_SIZE_CHOICES = ((320, 240), (640, 480), (1024, 436), (1280, 720), (1920, 1080))


def batch_sizes(n: int, seed: int = 4000):
    """Sizes (w, h) of an uneven batch, drawn uniformly from BATCH_SIZE_CHOICES."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(BATCH_SIZE_CHOICES), n)
    return [BATCH_SIZE_CHOICES[i] for i in idx]
