"""Per-tile b for the dynamic b of the conclusion (Sec. V, future work) --
test infrastructure only, like the rest of this package.

The paper only suggests a b that varies over the image.  The reading (the
same as the C oracle's demr_* functions, computed here a second, independent
way in plain numpy): one b per 64x64 tile of an image whose sides are
multiples of 64; a pixel (i, j), j >= 1, is redundant for b when its b MSBs
equal those of its left neighbour (i, j - 1) -- with one b for the whole image
exactly the pixels the Omega glide of Sec. III-A marks -- including the
first column of a tile, whose left neighbour lies in the tile before.  For
b = 2..7, Z_b(t) counts the tile's redundant pixels; b_t is the first b
reaching the largest b * Z_b(t) (the rule by which the method chooses its one
b), and the image's capacity is the sum over tiles of b_t * Z_{b_t}(t) bits.
"""
from __future__ import annotations

import numpy as np

TILE = 64
BMIN, BMAX = 2, 7


def tile_counts(I, tile: int = TILE) -> np.ndarray:
    """Z[ty, tx, b - BMIN] for b = BMIN..BMAX."""
    I = np.asarray(I)
    assert I.dtype == np.uint8 and I.ndim == 2
    M, N = I.shape
    assert M % tile == 0 and N % tile == 0 and M > 0 and N > 0
    x = np.zeros((M, N), dtype=np.int64)
    x[:, 1:] = I[:, 1:].astype(np.int64) ^ I[:, :-1].astype(np.int64)
    x[:, 0] = 0xFF                                      # column 0 has no left neighbour
    Z = np.zeros((M // tile, N // tile, BMAX - BMIN + 1), dtype=np.int64)
    for b in range(BMIN, BMAX + 1):
        same = (x >> (8 - b)) == 0
        Z[:, :, b - BMIN] = same.reshape(M // tile, tile, N // tile, tile).sum(axis=(1, 3))
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
