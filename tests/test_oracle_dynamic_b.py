"""Pins of the dynamic-b oracle (one b per 64x64 tile, the conclusion's future
work under this library's reading; C functions demr_* and the numpy tile
counts of oracle/dynamic_b.py): the EMR oracle's results on images where
every tile takes the same b (one-tile images, flat images), an independent
numpy count, a pure-Python glide along whole rows, hand-worked two-tile and
tie cases, a brute-force search over every b assignment, and the round-trip
invariants."""
import itertools

import numpy as np
import pytest

from oracle import dynamic_b as D
from oracle import oracle as O
from paper_2302_07992_amd import inputs


def _smooth(seed, M, N, sigma=3.0):
    rng = np.random.default_rng(seed)
    y, x = np.indices((M, N))
    f = 128 + 60 * np.sin(x / 11.0 + seed) * np.cos(y / 13.0) + rng.normal(0, sigma, (M, N))
    return np.clip(np.rint(f), 0, 255).astype(np.uint8)


def _full_trip(I, k1, k2, nonce, emr):
    """Every role of one variant at full capacity; returns all outputs."""
    if emr:
        Ie, m = O.emr_encrypt(I, k1, nonce=nonce)
    else:
        Ie, m, bt = O.demr_encrypt(I, k1, nonce=nonce)
    nb = int(m.capacity_bits)
    msg = np.random.default_rng(k2).integers(0, 256, (nb + 7) // 8 + 1).astype(np.uint8)
    if emr:
        W = O.emr_embed(Ie, m.b, msg, nb, k2, nonce=nonce)
        g = O.emr_extract(W, m.b, nb, k2, nonce=nonce)
        r = O.emr_recover(W, m.b, k1, nonce=nonce)
    else:
        W = O.demr_embed(Ie, bt, msg, nb, k2, nonce=nonce)
        g = O.demr_extract(W, bt, nb, k2, nonce=nonce)
        r = O.demr_recover(W, bt, k1, nonce=nonce)
    return Ie, m, W, g, r, msg, nb


@pytest.mark.parametrize("seed,sigma", [(0, 1.0), (1, 3.0), (2, 8.0), (3, 30.0)])
def test_one_tile_image_equals_emr(seed, sigma):
    """A 64x64 image is one tile: its b, the capacity, and every role's output
    are the EMR oracle's (its own Omega glide, selection, hiding and omega
    recovery); the b table holds that b."""
    I = _smooth(seed, 64, 64, sigma)
    a = _full_trip(I, 5, 6, 9, emr=True)
    d = _full_trip(I, 5, 6, 9, emr=False)
    _, _, bt = O.demr_encrypt(I, 5, nonce=9)
    assert bt.shape == (1, 1) and int(bt[0, 0]) == a[1].b
    assert (d[1].redundant, d[1].capacity_bits) == (a[1].redundant, a[1].capacity_bits)
    for x, y in zip(a[:1] + a[2:5], d[:1] + d[2:5]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("value", [0, 77, 255])
def test_flat_image_equals_emr_with_b7(value):
    """Flat 192x256: every tile takes b = 7 (7 * 64 * 63 bits per tile, 7 * 64 *
    64 for tiles not on column 0), the image the EMR oracle encrypts with b = 7,
    and every role agrees with EMR."""
    I = np.full((192, 256), value, np.uint8)
    tb, Z = O.demr_tile_b(I)
    assert (tb == 7).all()
    cap = sum(7 * 64 * (63 if tx == 0 else 64) for tx in range(4)) * 3
    a = _full_trip(I, 11, 12, 13, emr=True)
    d = _full_trip(I, 11, 12, 13, emr=False)
    assert a[1].b == 7 and d[1].capacity_bits == a[1].capacity_bits == cap
    for x, y in zip(a[:1] + a[2:5], d[:1] + d[2:5]):
        assert np.array_equal(x, y)


def test_same_b_everywhere_equals_emr():
    """Whenever every tile takes the same b, dynamic b is EMR with that b (the
    global b is then the same: each tile's b maximises its own b Z_b(t), so it
    maximises the sum); checked on smooth images until 5 such cases."""
    found = 0
    for seed in range(60):
        I = inputs.make_image_np(seed, 128, 192, 3, 2.0)
        tb, _ = O.demr_tile_b(I)
        if len(set(tb.ravel().tolist())) != 1:
            continue
        a = _full_trip(I, seed + 1, seed + 2, seed, emr=True)
        d = _full_trip(I, seed + 1, seed + 2, seed, emr=False)
        assert a[1].b == int(tb[0, 0]) and a[1].capacity_bits == d[1].capacity_bits
        for x, y in zip(a[:1] + a[2:5], d[:1] + d[2:5]):
            assert np.array_equal(x, y)
        found += 1
        if found == 5:
            break
    assert found == 5


@pytest.mark.parametrize("seed", range(4))
def test_tile_counts_match_numpy_and_a_python_row_glide(seed):
    """Z_b(t) of the C oracle equals the numpy left-neighbour count, and a
    pure-Python Omega glide along whole image rows with a fixed b marks, inside
    each tile, the same pixels (one b: the glide is the left-neighbour rule)."""
    I = inputs.make_image_np(seed, 128, 192, 2 + seed, (1.0, 3.0, 8.0, 20.0)[seed])
    tb, Z = O.demr_tile_b(I)
    assert np.array_equal(Z, D.tile_counts(I))
    b_np, _ = D.tile_b(I)
    assert np.array_equal(tb, b_np)
    for b in (2, 5, 7):
        n = np.zeros((2, 3), np.int64)
        for i in range(128):
            row = [int(v) for v in I[i]]
            omega = row[0]
            for j in range(1, 192):
                if row[j] >> (8 - b) == omega >> (8 - b):
                    n[i // 64, j // 64] += 1
                else:
                    omega = row[j]
        assert np.array_equal(Z[:, :, b - 2], n)


def test_hand_worked_two_tiles():
    """64x128: tile 0 holds values below 32 whose bit 4 flips at every step
    (the top 3 bits always equal, the top 4 never): Z_3 = 64 * 63, Z_b = 0 for
    b >= 4, so b = 3 and 12,096 bits.  Tile 1 is flat at 200; its first column
    differs from the values below 32 at the left, so Z_b = 64 * 63 for every
    b: b = 7 and 28,224 bits.  Dynamic b: 40,320 bits.  One b for the image
    (Z_3 = 8,064, Z_b = 4,032 for b >= 4): b = 7 and 28,224 bits."""
    rng = np.random.default_rng(5)
    I = np.empty((64, 128), np.uint8)
    I[:, :64] = (16 * (np.arange(64) % 2))[None, :] + rng.integers(0, 16, (64, 64))
    I[:, 64:] = 200
    tb, Z = O.demr_tile_b(I)
    assert tb.tolist() == [[3, 7]]
    assert Z[0, 0].tolist() == [64 * 63, 64 * 63, 0, 0, 0, 0] and Z[0, 1].tolist() == [64 * 63] * 6
    _, m, _ = O.demr_encrypt(I, 1)
    _, me = O.emr_encrypt(I, 1)
    assert (m.b, m.redundant, m.capacity_bits) == (0, 2 * 64 * 63, 40320)
    assert (me.b, me.capacity_bits) == (7, 28224)


@pytest.mark.parametrize("seed", range(3))
def test_capacity_is_the_best_assignment(seed):
    """Brute force over all 6^4 choices of b for the four tiles of a 128x128
    image: the oracle's capacity is the largest total, reached by its own
    choice; and it is never below the EMR capacity."""
    I = inputs.make_image_np(100 + seed, 128, 128, 4, (2.0, 6.0, 12.0)[seed])
    tb, Z = O.demr_tile_b(I)
    best = 0
    for bs in itertools.product(range(2, 8), repeat=4):
        tot = sum(b * Z[t // 2, t % 2, b - 2] for t, b in enumerate(bs))
        best = max(best, tot)
    _, m, _ = O.demr_encrypt(I, 3)
    mine = sum(int(tb[t // 2, t % 2]) * Z[t // 2, t % 2, int(tb[t // 2, t % 2]) - 2] for t in range(4))
    assert m.capacity_bits == best == mine
    _, me = O.emr_encrypt(I, 3)
    assert m.capacity_bits >= me.capacity_bits


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
    tb, Z = O.demr_tile_b(I)
    assert (Z[0, 0, 0], Z[0, 0, 1], Z[0, 0, 2:].sum()) == (n2 + n3, n3, 0)
    assert int(tb[0, 0]) == want
    b_np, cap = D.tile_b(I)
    assert int(b_np[0, 0]) == want and cap == max(2 * (n2 + n3), 3 * n3)


@pytest.mark.parametrize("shape", [(64, 64), (128, 192), (256, 256), (192, 320)])
@pytest.mark.parametrize("kind", ["smooth", "noise", "checker", "mixed"])
def test_round_trip_invariants(shape, kind):
    """Every b table entry is a tile's b (the encrypted-order table is a
    permutation of the tile table); the payload comes back at full and partial
    length; the recovered image equals the original above the LSB plane."""
    M, N = shape
    if kind == "smooth":
        I = inputs.make_image_np(M + N, M, N, 6, 3.0)
    elif kind == "noise":
        I = np.random.default_rng(M).integers(0, 256, (M, N)).astype(np.uint8)
    elif kind == "checker":
        r, c = np.indices((M, N))
        I = (((r // 3 + c // 5) % 2) * 255).astype(np.uint8)
    else:
        I = inputs.make_image_np(M * N, M, N, 8, 3.0)
        I[:, : N // 2] = np.random.default_rng(2).integers(0, 256, (M, N // 2))
    tb, _ = O.demr_tile_b(I)
    Ie, m, bt = O.demr_encrypt(I, 21, nonce=M)
    assert sorted(bt.ravel().tolist()) == sorted(tb.ravel().tolist())
    for frac in (1.0, 0.37):
        nb = int(m.capacity_bits * frac)
        msg = np.random.default_rng(nb).integers(0, 256, (nb + 7) // 8 + 1).astype(np.uint8)
        W = O.demr_embed(Ie, bt, msg, nb, 22, nonce=M)
        assert np.array_equal(W & 1, Ie & 1)
        g = O.demr_extract(W, bt, nb, 22, nonce=M)
        full = nb // 8
        assert np.array_equal(g[:full], msg[:full])
        if nb % 8:
            assert g[full] >> (8 - nb % 8) == msg[full] >> (8 - nb % 8)
        r = O.demr_recover(W, bt, 21, nonce=M)
        assert np.array_equal(r >> 1, I >> 1)
    with pytest.raises(ValueError):
        O.demr_embed(Ie, bt, np.zeros(int(m.capacity_bits) // 8 + 2, np.uint8), int(m.capacity_bits) + 1, 22)
