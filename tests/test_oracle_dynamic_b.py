"""Pins of the per-tile-b oracle (oracle/dynamic_b.py): the EMR oracle's own
b and capacity on one-tile images, a pure-Python glide, the left-neighbour
form of redundancy, closed forms and the tie rule."""
import numpy as np
import pytest

from oracle import dynamic_b as D
from oracle import oracle as O


def _smooth(seed, M, N, sigma=3.0):
    rng = np.random.default_rng(seed)
    y, x = np.indices((M, N))
    f = 128 + 60 * np.sin(x / 11.0 + seed) * np.cos(y / 13.0) + rng.normal(0, sigma, (M, N))
    return np.clip(np.rint(f), 0, 255).astype(np.uint8)


@pytest.mark.parametrize("seed,sigma", [(0, 1.0), (1, 3.0), (2, 8.0), (3, 30.0)])
def test_one_tile_image_equals_the_emr_choice(seed, sigma):
    """A 64x64 image is one tile whose first column is the image's: b_t and
    the capacity are the EMR oracle's b and capacity (its own glides and its
    own selection)."""
    I = _smooth(seed, 64, 64, sigma)
    b, cap = D.tile_b(I)
    _, meta = O.emr_encrypt(I, 5)
    assert (int(b[0, 0]), cap) == (meta.b, meta.capacity_bits)


def test_counts_match_a_pure_python_glide():
    """Every tile row glided pixel by pixel in plain Python (tile 8)."""
    rng = np.random.default_rng(4)
    I = (rng.integers(0, 4, (16, 24)) * 37 + rng.integers(0, 3, (16, 24))).astype(np.uint8)
    Z = D.tile_counts(I, tile=8)
    for ty in range(2):
        for tx in range(3):
            for b in range(D.BMIN, D.BMAX + 1):
                n = 0
                for r in range(8):
                    row = [int(v) for v in I[8 * ty + r, 8 * tx:8 * tx + 8]]
                    tracker = row[0]
                    for v in row[1:]:
                        if v >> (8 - b) == tracker >> (8 - b):
                            n += 1
                        else:
                            tracker = v
                assert Z[ty, tx, b - D.BMIN] == n


def test_counts_equal_the_left_neighbour_form():
    """A pixel is redundant exactly when its b MSBs equal its left
    neighbour's (the glide's tracker always shares them)."""
    I = _smooth(9, 128, 192, 4.0)
    Z = D.tile_counts(I)
    a = I.astype(np.int64)
    for b in range(D.BMIN, D.BMAX + 1):
        same = ((a[:, 1:] ^ a[:, :-1]) >> (8 - b)) == 0
        same[:, 63::64] = False                       # a tile's first column has no left pixel in the tile
        # columns 1..63 of tile tx are `same` columns 64 tx .. 64 tx + 62
        per = np.zeros((2, 3), np.int64)
        for ty in range(2):
            for tx in range(3):
                per[ty, tx] = same[64 * ty:64 * ty + 64, 64 * tx:64 * tx + 63].sum()
        assert np.array_equal(Z[:, :, b - D.BMIN], per)


def test_flat_and_noise_closed_forms():
    """A flat image: every pixel but the first column is redundant at any b,
    so b_t = 7 and 7 * 63 * 64 bits per tile.  Alternating 0 / 255 columns:
    nothing is redundant, b_t = 2 (the first b), capacity 0."""
    b, cap = D.tile_b(np.full((128, 256), 77, np.uint8))
    assert (b == 7).all() and cap == 8 * 7 * 63 * 64
    I = np.zeros((64, 128), np.uint8)
    I[:, 1::2] = 255
    b, cap = D.tile_b(I)
    assert (b == 2).all() and cap == 0


def _row_with_lambdas(lams, start=0):
    """A row whose pixel k + 1 shares exactly lams[k] leading bits with pixel k."""
    row = [start]
    for lam in lams:
        row.append(row[-1] ^ (0x80 >> lam))
    return row


@pytest.mark.parametrize("n2,n3,want", [(40, 80, 2), (40, 81, 3)])
def test_tie_goes_to_the_smaller_b(n2, n3, want):
    """Pixels sharing exactly 2 leading bits count for Z_2, exactly 3 for Z_2
    and Z_3, 0 for none: Z_2 = n2 + n3, Z_3 = n3, Z_b = 0 above.  With
    n3 = 2 n2, 2 Z_2 = 3 Z_3 and the smaller b wins; one more tips it."""
    lams = [2] * n2 + [3] * n3
    lams += [0] * (64 * 63 - len(lams))
    rows = [_row_with_lambdas(lams[63 * r:63 * r + 63], start=0) for r in range(64)]
    I = np.array(rows, dtype=np.uint8)
    Z = D.tile_counts(I)[0, 0]
    assert (Z[0], Z[1], Z[2:].sum()) == (n2 + n3, n3, 0)
    b, cap = D.tile_b(I)
    assert int(b[0, 0]) == want and cap == max(2 * (n2 + n3), 3 * n3)
