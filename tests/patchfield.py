"""A float64 field that exercises the two-record patch path.

Prequantization (Sec. IV: uniform bins of width 2eb, midpoint
reconstruction) keeps |x - x'| <= eb in exact arithmetic, but a value a few
ulps from a bin edge can land in the other bin once x * (1 / 2eb) and
q * 2eb are rounded to float64; such a point is stored exactly (a patch,
64 raw bits in two exception records).  The field below places many values
within three ulps of bin edges, so patches occur in a full tile, in ragged
edge tiles, in a tile with more exception records than fit a 64-record
staging slot, and in the same 32-point segment as outliers made by 2x2x2
checkerboard blocks of +-0.9 (Lorenzo residual of 8 * 0.9 / 2eb bins).

The range is fixed at vr = 2 by x = -1 and x = +1 at the first and last
points, so eb = 2 * sqrt(3) * 10^(-PSNR/20) (Eq. 7) is known in advance.
"""
import math

import numpy as np

from paper_1805_07384_amd import synth

SHAPE = (17, 33, 70)   # tile grid 2 x 3 x 3 of 16 x 16 x 32: full and ragged tiles
PSNR = 100.0
# 2x2x2 checkerboard blocks (z, y, x origin): tile (0,0,0), across the z
# tile edge, in the ragged x tile
BLOCKS = [(2, 4, 10), (9, 12, 3), (15, 20, 40), (8, 30, 66)]


def eb_of(psnr: float, vr: float = 2.0) -> float:
    return vr * (math.sqrt(3.0) * math.pow(10.0, -psnr / 20.0))


def f64_patch_field(shape=SHAPE, psnr=PSNR, seed=5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    g = synth.grf_numpy(shape, -3.0, seed).astype(np.float64)
    x = g / np.max(np.abs(g)) * 0.8
    e2 = 2.0 * eb_of(psnr)
    # density of bin-edge values: dense in tile (0, 0, 0), sparse elsewhere
    dens = np.full(shape, 0.03)
    dens[:16, :16, :32] = 0.4
    dens[16:, :, :] = 0.2
    m = rng.random(shape) < dens
    edge = (np.floor(x / e2) + 0.5) * e2
    steps = rng.integers(-3, 4, size=shape)
    for s in range(1, 4):
        edge = np.where(steps >= s, np.nextafter(edge, np.inf), edge)
        edge = np.where(steps <= -s, np.nextafter(edge, -np.inf), edge)
    x = np.where(m, edge, x)
    for (z, y, xx) in BLOCKS:
        for a in range(2):
            for b in range(2):
                for c in range(2):
                    x[z + a, y + b, xx + c] = 0.9 if (a + b + c) % 2 == 0 else -0.9
    x.flat[0] = -1.0
    x.flat[-1] = 1.0
    return np.ascontiguousarray(x)


def stream_positions(shape, tile=(16, 16, 32)) -> np.ndarray:
    """Stream position of every point: tiles row-major over the tile grid,
    points row-major inside the edge-clipped tile."""
    nz, ny, nx = shape
    tz, ty, tx = tile
    pos = np.empty(shape, dtype=np.int64)
    p = 0
    for z0 in range(0, nz, tz):
        for y0 in range(0, ny, ty):
            for x0 in range(0, nx, tx):
                blk = pos[z0:z0 + tz, y0:y0 + ty, x0:x0 + tx]
                blk[...] = p + np.arange(blk.size).reshape(blk.shape)
                p += blk.size
    return pos
