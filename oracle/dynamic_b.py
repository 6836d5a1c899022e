"""Per-tile b, a first step towards the dynamic b of the conclusion (test
infrastructure only, like the rest of this package).

The paper only suggests a b that varies over the image; the reading here:
for each 64x64 tile of an image whose sides are multiples of 64, the
location-map glide of Sec. III-A (initialisation, glide and update equations)
runs along each row of the tile from the tile's first column, which is kept
(label 1) like the first pixel of an image row.  For b = 2..7, Z_b(t) counts
the pixels whose b MSBs equal the tracker's.  b_t is the first b reaching the
largest b * Z_b(t) (the rule by which the method chooses its one b), and the
image's capacity is the sum over tiles of b_t * Z_{b_t}(t) bits.

Plain numpy: the glide steps column by column, all tile rows side by side.
"""
from __future__ import annotations

import numpy as np

TILE = 64
BMIN, BMAX = 2, 7


def tile_counts(I, tile: int = TILE) -> np.ndarray:
    """Z[ty, tx, b - BMIN] for b = BMIN..BMAX, each from its own glide."""
    I = np.asarray(I)
    assert I.dtype == np.uint8 and I.ndim == 2
    M, N = I.shape
    assert M % tile == 0 and N % tile == 0 and M > 0 and N > 0
    ty, tx = M // tile, N // tile
    seg = I.reshape(M, tx, tile).astype(np.int64)        # row i of every tile column tx
    Z = np.zeros((ty, tx, BMAX - BMIN + 1), dtype=np.int64)
    for b in range(BMIN, BMAX + 1):
        shift = 8 - b
        tracker = seg[:, :, 0] >> shift                    # the tile's first column starts the glide
        redundant = np.zeros((M, tx), dtype=np.int64)
        for c in range(1, tile):
            v = seg[:, :, c] >> shift
            same = v == tracker
            redundant += same
            tracker = np.where(same, tracker, v)           # the tracker moves to every non-redundant pixel
        Z[:, :, b - BMIN] = redundant.reshape(ty, tile, tx).sum(axis=1)
    return Z


def tile_b(I, tile: int = TILE):
    """(b_t as a (M/tile, N/tile) uint8 array, capacity in bits)."""
    Z = tile_counts(I, tile)
    bs = np.arange(BMIN, BMAX + 1, dtype=np.int64)
    score = Z * bs
    best = np.argmax(score, axis=2)                       # first maximum: the smaller b on ties
    cap = int(np.take_along_axis(score, best[..., None], axis=2).sum())
    return bs[best].astype(np.uint8), cap


__all__ = ["TILE", "BMIN", "BMAX", "tile_counts", "tile_b"]
