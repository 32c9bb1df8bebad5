"""Seeded synthetic inputs for quarter-sampled video.

This module only *generates inputs*: high-resolution frames, quarter-sampling
masks and the measured (masked) frames a quarter-sampling sensor delivers.  It
holds none of the reconstruction arithmetic (motion estimation, checks,
projection, FSR).  Both the CPU oracle and the GPU path are fed from here.

Sampling model (Sec. 2.1 and the introduction): the sub-sampled image is the
high-resolution image times a binary mask, f_sub = f * b.  Quarter sampling
opens exactly one of the four high-resolution positions of every 2x2 cell.
With a dynamic mask (introduction, the read-out strategy of the dynamic-mask
work the paper builds on) every position of a 2x2 cell is read exactly once
within four frames and the pattern repeats every fourth frame.

Cell positions are numbered in raster order inside the cell:
0 = (0,0), 1 = (0,1), 2 = (1,0), 3 = (1,1).

The paper's test sequences (Spincalendar, JVET class C / class A) are not
available; the generators below stand in for them with the same frame sizes,
8-bit range and motion character (piecewise translation, occlusions).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "seed_for", "fixed_mask", "dynamic_masks", "mask_sequence",
    "bandlimited_noise", "video_translate_edges", "video_regions",
    "measured", "workload_c1", "workload_c2", "C4_SIZES", "workload_c4",
]

BASE_SEED = 220309200


def seed_for(config: int, stream: int = 0) -> int:
    """Seed of workload `config` (1-based), stream `stream`."""
    return BASE_SEED + 1000 * config + stream


def _cells_to_mask(pos: np.ndarray) -> np.ndarray:
    """(Hc, Wc) array of cell positions in 0..3 -> (2Hc, 2Wc) uint8 mask."""
    hc, wc = pos.shape
    m = np.zeros((2 * hc, 2 * wc), np.uint8)
    dy = (pos >> 1).astype(np.int64)
    dx = (pos & 1).astype(np.int64)
    yy = 2 * np.arange(hc)[:, None] + dy
    xx = 2 * np.arange(wc)[None, :] + dx
    m[yy, xx] = 1
    return m


def fixed_mask(h: int, w: int, rng: np.random.Generator) -> np.ndarray:
    """Fixed quarter mask: one uniformly random open position per 2x2 cell."""
    assert h % 2 == 0 and w % 2 == 0
    pos = rng.integers(0, 4, size=(h // 2, w // 2))
    return _cells_to_mask(pos)


def dynamic_masks(h: int, w: int, rng: np.random.Generator) -> np.ndarray:
    """Dynamic quarter mask period: (4, h, w) uint8.

    Each cell draws a random permutation pi of its four positions; frame t
    opens position pi[t mod 4].
    """
    assert h % 2 == 0 and w % 2 == 0
    hc, wc = h // 2, w // 2
    perm = np.argsort(rng.random((hc, wc, 4)), axis=-1)
    return np.stack([_cells_to_mask(perm[..., t]) for t in range(4)])


def mask_sequence(kind: str, n: int, h: int, w: int, rng: np.random.Generator) -> np.ndarray:
    """(n, h, w) masks, `kind` in {'fixed', 'dynamic'}."""
    if kind == "fixed":
        m = fixed_mask(h, w, rng)
        return np.broadcast_to(m, (n, h, w)).copy()
    if kind == "dynamic":
        p = dynamic_masks(h, w, rng)
        return np.stack([p[t % 4] for t in range(n)])
    raise ValueError(kind)


def bandlimited_noise(h: int, w: int, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """White N(0,1) noise low-pass filtered by a Gaussian transfer function
    of spatial std `sigma` pixels (periodic), scaled to unit expected
    variance (the filter's mean squared gain), so that fields much smoother
    than the canvas stay smooth instead of being blown up."""
    z = rng.standard_normal((h, w))
    fy = np.fft.fftfreq(h)[:, None]
    fx = np.fft.rfftfreq(w)[None, :]
    tf = np.exp(-2.0 * (np.pi * sigma) ** 2 * (fy ** 2 + fx ** 2))
    out = np.fft.irfft2(np.fft.rfft2(z) * tf, s=(h, w))
    full = np.exp(-2.0 * (np.pi * sigma) ** 2 * (fy ** 2 + np.fft.fftfreq(w)[None, :] ** 2))
    return out / np.sqrt(np.mean(full ** 2))


def _to_u8(x: np.ndarray) -> np.ndarray:
    return np.rint(np.clip(x, 0.0, 255.0)).astype(np.uint8)


def video_translate_edges(n: int, h: int, w: int, rng: np.random.Generator,
                          max_step: int = 3, n_edges: int = 8) -> tuple[np.ndarray, np.ndarray]:
    """Band-limited Gaussian noise plus straight edges, global integer
    translation of up to +-max_step px per frame.

    Returns (frames (n,h,w) uint8, offsets (n,2) int: crop origin of frame t
    in the canvas).  Frame t is the canvas crop at o_t = o_{t-1} + d_t.
    """
    margin = max_step * (n - 1) if n > 1 else 0
    ch, cw = h + 2 * margin, w + 2 * margin
    tex = 128.0 + 40.0 * bandlimited_noise(ch, cw, 1.5, rng)
    yy, xx = np.mgrid[0:ch, 0:cw].astype(np.float64)
    for _ in range(n_edges):
        py, px = rng.uniform(0, ch), rng.uniform(0, cw)
        ang = rng.uniform(0, 2 * np.pi)
        step = rng.uniform(20, 60) * rng.choice([-1.0, 1.0])
        side = (yy - py) * np.cos(ang) - (xx - px) * np.sin(ang) > 0
        tex = tex + step * side
    canvas = _to_u8(tex)
    offs = np.zeros((n, 2), np.int64)
    o = np.array([margin, margin])
    frames = np.empty((n, h, w), np.uint8)
    for t in range(n):
        if t > 0:
            o = o + rng.integers(-max_step, max_step + 1, size=2)
        offs[t] = o
        frames[t] = canvas[o[0]:o[0] + h, o[1]:o[1] + w]
    return frames, offs


def video_regions(n: int, h: int, w: int, rng: np.random.Generator, grid: int = 8,
                  vmax: int = 12, occl_frac: float = 0.05) -> np.ndarray:
    """Smooth texture with piecewise-translational local motion.

    The frame is split into a grid x grid array of rectangular regions; each
    region moves with its own constant integer velocity in U{-vmax..vmax}^2
    (frame t samples the texture at p - t*v).  Occluding squares with side
    U[27, 90] px, their own texture and velocity, are drawn on top until they
    cover at least `occl_frac` of the frame.
    """
    margin = vmax * max(n - 1, 0) + 1
    ch, cw = h + 2 * margin, w + 2 * margin

    def texture(th, tw):
        return (128.0 + 40.0 * bandlimited_noise(th, tw, 4.0, rng)
                + 30.0 * bandlimited_noise(th, tw, 32.0, rng))

    tex = texture(ch, cw)
    ry = (np.arange(h) * grid) // h
    rx = (np.arange(w) * grid) // w
    vel = rng.integers(-vmax, vmax + 1, size=(grid, grid, 2))
    vy = vel[ry[:, None], rx[None, :], 0]
    vx = vel[ry[:, None], rx[None, :], 1]
    squares = []
    area = 0
    while area < occl_frac * h * w:
        side = int(rng.integers(27, 91))
        y0 = int(rng.integers(0, max(h - side, 1)))
        x0 = int(rng.integers(0, max(w - side, 1)))
        sv = rng.integers(-vmax, vmax + 1, size=2)
        squares.append((side, y0, x0, sv, texture(side, side)))   # moves with the square
        area += side * side
    yy = np.arange(h)[:, None]
    xx = np.arange(w)[None, :]
    frames = np.empty((n, h, w), np.uint8)
    for t in range(n):
        f = tex[yy - t * vy + margin, xx - t * vx + margin]
        for side, y0, x0, sv, stex in squares:
            ty, tx = y0 + t * sv[0], x0 + t * sv[1]
            ys = np.arange(max(ty, 0), min(ty + side, h))
            xs = np.arange(max(tx, 0), min(tx + side, w))
            if ys.size == 0 or xs.size == 0:
                continue
            f[ys[:, None], xs[None, :]] = stex[ys[:, None] - ty, xs[None, :] - tx]
        frames[t] = _to_u8(f)
    return frames


def measured(frames: np.ndarray, masks: np.ndarray) -> np.ndarray:
    """Sensor output f * b (unmeasured positions hold 0)."""
    return (frames * masks).astype(np.uint8)


def workload_c1(seed: int | None = None):
    """CPU-sized recursive workload: 4 frames of 128x128, band-limited noise
    with 8 edges, global translation up to +-3 px per frame, fixed mask."""
    rng = np.random.default_rng(seed_for(1) if seed is None else seed)
    frames, _ = video_translate_edges(4, 128, 128, rng)
    masks = mask_sequence("fixed", 4, 128, 128, rng)
    return frames, masks


def workload_c2(n: int = 16, h: int = 1080, w: int = 1920, seed: int | None = None):
    """1080p workload: smooth texture, 8x8 grid of independently translating
    regions (+-12 px/frame), 5% occluding squares, dynamic mask."""
    rng = np.random.default_rng(seed_for(2) if seed is None else seed)
    frames = video_regions(n, h, w, rng)
    masks = mask_sequence("dynamic", n, h, w, rng)
    return frames, masks


# Batched multi-stream configuration: 16 CIF, 16 720p, 12 1080p and 4 2160p
# streams (H, W).
C4_SIZES = [(288, 352)] * 16 + [(720, 1280)] * 16 + [(1080, 1920)] * 12 + [(2160, 3840)] * 4


def workload_c4(n: int = 8, sizes=None):
    """Multi-stream workload: one (frames, masks) pair per stream, the 1080p
    generator at each stream's size, n frames each; even stream index ->
    fixed mask, odd -> dynamic.  Stream s uses seed_for(4, s)."""
    out = []
    for s, (h, w) in enumerate(C4_SIZES if sizes is None else sizes):
        rng = np.random.default_rng(seed_for(4, s))
        frames = video_regions(n, h, w, rng)
        masks = mask_sequence("fixed" if s % 2 == 0 else "dynamic", n, h, w, rng)
        out.append((frames, masks))
    return out
