"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds input generation only (images, masks, request mixes); it
contains none of the filtering method's arithmetic (no DCT, no filter, no
operator).  Everything is driven by numpy's PCG64 (``default_rng(seed)``), so
a seed fixes every value.

Image recipe (stands in for the natural images the paper filters; the paper
publishes no data set and its test block's values are not available):
    img[y][x] = clamp(floor(128 + 60 sin(x/7) cos(y/5) + n + 1/2), 0, 255),
    n ~ N(0, 10^2), x the column and y the row, both 0-based.

Quantised-coefficient recipe (stands in for the entropy-decoded blocks of a
JPEG-style codec; no standard table is reproduced): a table
    q[u][v] = round(q0 * (1 + slope * (u + v))),  q0 = 4, slope = 0.75,
growing with frequency like a codec's luminance table, and integer
coefficients round((X - dc_offset e_0) / q) of given coefficient blocks X.

Mask recipes:
  * box K x K (1/K^2 each);
  * sampled Gaussian, g(u, v) ~ exp(-(u^2+v^2) / (2 sigma^2)) on the K x K
    grid centred at 0, normalised to sum 1 (the 3x3, sigma = 1 mask of the
    paper's first experiment, Sec. III);
  * the magic square of order 3 (second experiment, Sec. III, Fig. 3), raw
    (sum 45) or divided by 45;
  * random masks with entries U(-1, 1), redrawn from the same stream until
    |sum| >= 1, then divided by their sum.  "Symmetric" averages the mask
    with its three mirror images (both axes) before normalising; "separable"
    is an outer product g h^T of two such 1-D masks.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

BORDER_ZERO = 0
BORDER_REPLICATE = 1


def image_u8(seed: int, h: int, w: int) -> np.ndarray:
    """One seeded ``h x w`` uint8 image from the recipe above."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((h, w)) * 10.0
    x = np.arange(w, dtype=np.float64)
    y = np.arange(h, dtype=np.float64)
    base = 128.0 + 60.0 * np.outer(np.cos(y / 5.0), np.sin(x / 7.0))
    return np.clip(np.floor(base + noise + 0.5), 0, 255).astype(np.uint8)


def box_mask(k: int) -> np.ndarray:
    return np.full((k, k), 1.0 / (k * k))


def gaussian_mask(k: int, sigma: float = 1.0) -> np.ndarray:
    r = np.arange(k, dtype=np.float64) - (k - 1) / 2.0
    g = np.exp(-(r[:, None] ** 2 + r[None, :] ** 2) / (2.0 * sigma * sigma))
    return g / g.sum()


def magic_square_3(normalised: bool = True) -> np.ndarray:
    m = np.array([[8.0, 1.0, 6.0], [3.0, 5.0, 7.0], [4.0, 9.0, 2.0]])
    return m / 45.0 if normalised else m


def delta_mask(kh: int, kw: int, dy: int = 0, dx: int = 0) -> np.ndarray:
    """K x K mask with a single 1 at offset (dy, dx) from the anchor
    floor((K-1)/2): it selects the pixel (i + dy, j + dx)."""
    W = np.zeros((kh, kw))
    W[(kh - 1) // 2 + dy, (kw - 1) // 2 + dx] = 1.0
    return W


def _unit_sum(rng, shape) -> np.ndarray:
    while True:
        m = rng.uniform(-1.0, 1.0, size=shape)
        s = m.sum()
        if abs(s) >= 1.0:
            return m / s


def random_mask(rng, kh: int, kw: int, symmetric: bool = False,
                separable: bool = False) -> np.ndarray:
    """Sum-1 random mask with entries drawn U(-1, 1) (redraw rule above)."""
    if separable:
        g = _unit_sum(rng, (kh,))
        h = _unit_sum(rng, (kw,))
        if symmetric:
            g = (g + g[::-1]) / 2.0
            h = (h + h[::-1]) / 2.0
            g = g / g.sum()
            h = h / h.sum()
        return np.outer(g, h)
    while True:
        m = _unit_sum(rng, (kh, kw))
        if symmetric:
            m = (m + m[::-1, :] + m[:, ::-1] + m[::-1, ::-1]) / 4.0
            if abs(m.sum()) < 1e-12:
                continue
            m = m / m.sum()
        return m


@dataclass
class MaskSpec:
    mask: np.ndarray
    border: int
    symmetric: bool
    separable: bool

    @property
    def shape(self):
        return self.mask.shape


def asym_mask_5x5(seed: int = 2) -> np.ndarray:
    """The 5 x 5 asymmetric, inseparable mask of the 512 x 512 workload."""
    return random_mask(np.random.default_rng(seed), 5, 5, symmetric=False, separable=False)


def mask_pool_16(seed: int = 3) -> list:
    """16 replicate-border masks, K uniform over {3, 5, 7}, symmetric or not
    with probability 1/2 (the batched 64-image workload)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(16):
        k = int(rng.choice([3, 5, 7]))
        sym = bool(rng.integers(0, 2))
        out.append(MaskSpec(random_mask(rng, k, k, symmetric=sym), BORDER_REPLICATE, sym, False))
    return out


def mask_set_32(seed: int = 5) -> list:
    """32 masks: 8 at each K in {3, 5, 7, 9}, spread evenly over
    symmetric/asymmetric x separable/inseparable x zero/replicate."""
    rng = np.random.default_rng(seed)
    out = []
    for k in (3, 5, 7, 9):
        for sym in (False, True):
            for sep in (False, True):
                for border in (BORDER_ZERO, BORDER_REPLICATE):
                    out.append(MaskSpec(random_mask(rng, k, k, symmetric=sym, separable=sep),
                                        border, sym, sep))
    return out


def coeff_like_fp32(seed: int, nblocks: int, N: int) -> np.ndarray:
    """FP32 values shaped like block-DCT coefficients of the image recipe
    without computing a DCT: a DC term in [N*40, N*220] and AC terms whose
    scale decays with frequency.  For shape and range tests only."""
    rng = np.random.default_rng(seed)
    u = np.arange(N)[:, None]
    v = np.arange(N)[None, :]
    scale = 60.0 / (1.0 + u + v)
    X = rng.standard_normal((nblocks, N, N)) * scale
    X[:, 0, 0] = rng.uniform(40.0 * N, 220.0 * N, size=nblocks)
    return X.astype(np.float32)


def quant_table(N: int, q0: float = 4.0, slope: float = 0.75) -> np.ndarray:
    """N x N quantisation table q[u][v] = round(q0 (1 + slope (u + v))), >= 1."""
    u = np.arange(N, dtype=np.float64)[:, None]
    v = np.arange(N, dtype=np.float64)[None, :]
    return np.maximum(np.round(q0 * (1.0 + slope * (u + v))), 1.0)


def quantize(X, qtable, dc_offset: float = 0.0) -> np.ndarray:
    """int16 coefficients round((X - dc_offset e_0) / q) of blocks ``[B, N, N]``
    (round half to even; the offset is taken off the DC term first)."""
    Xs = np.array(X, dtype=np.float64)
    Xs[..., 0, 0] -= dc_offset
    c = np.rint(Xs / np.asarray(qtable, dtype=np.float64))
    return np.clip(c, -32768, 32767).astype(np.int16)


@dataclass
class Request:
    rid: int
    arrival_s: float
    h: int
    w: int
    N: int
    mask_id: int
    payload: int


def request_mix(seed: int, rate_hz: float, count: int, n_payloads: int,
                side_min: int = 256, side_max: int = 4096, p_n16: float = 0.2,
                n_masks: int = 32) -> list:
    """Poisson arrivals at ``rate_hz``; sides uniform over the multiples of 8
    in [side_min, side_max]; block size 16 with probability ``p_n16``, else 8;
    one of ``n_masks`` masks; ``payload`` picks one of ``n_payloads``
    pre-generated device-resident images of that request's shape class."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    t = np.cumsum(gaps) - gaps[0]
    sides = np.arange(side_min, side_max + 1, 8)
    out = []
    for i in range(count):
        h = int(rng.choice(sides))
        w = int(rng.choice(sides))
        N = 16 if rng.random() < p_n16 else 8
        out.append(Request(i, float(t[i]), h, w, N, int(rng.integers(0, n_masks)),
                           int(rng.integers(0, n_payloads))))
    return out
