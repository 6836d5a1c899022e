"""Host logic of the serving loop: the pool allocator, arrivals and the
admission footprint (no GPU)."""
import numpy as np
import pytest

from paper_2302_07992_amd import serve


def test_arena_ring_reuse_and_wrap():
    a = serve.Arena(4096, device="cpu")
    assert a.base % 256 == 0 and a.available() == 4096
    b1 = a.alloc(1000)          # rounds to 1024
    b2 = a.alloc(2048)
    assert (b1[0], b1[1], b2[0], b2[1]) == (0, 1024, 1024, 3072)
    assert a.available() == 1024
    assert a.alloc(1025) is None
    a.release(b2)               # out of order: nothing reclaimed yet
    assert a.available() == 1024
    a.release(b1)               # oldest released: everything free
    assert a.available() == 4096 and not a.blocks
    b3 = a.alloc(3072)
    b4 = a.alloc(512)
    a.release(b3)
    # free: [3584, 4096) and [0, 3072); a 2048 block wraps to the start
    b5 = a.alloc(2048)
    assert b5[0] == 0
    assert a.available() == 1024
    a.release(b4)
    a.release(b5)
    assert a.available() == 4096


def test_arena_blocks_never_overlap_random():
    rng = np.random.default_rng(3)
    a = serve.Arena(1 << 16, device="cpu")
    live = []
    for _ in range(3000):
        if live and (rng.random() < 0.45 or a.available() < 4096):
            blk = live.pop(int(rng.integers(len(live))))
            a.release(blk)
        else:
            blk = a.alloc(int(rng.integers(1, 8192)))
            if blk is None:
                continue
            assert 0 <= blk[0] < blk[1] <= a.size
            for o in live:
                assert blk[1] <= o[0] or o[1] <= blk[0], (blk, o)
            live.append(blk)
    for blk in live:
        a.release(blk)
    assert a.available() == a.size


def test_poisson_arrivals_rate():
    t = serve.poisson_arrivals(20000, 1000.0, seed=1)
    assert np.all(np.diff(t) >= 0)
    gaps = np.diff(np.concatenate(([0.0], t)))
    assert abs(gaps.mean() - 1e-3) < 3e-5          # mean 1/rate
    assert abs(gaps.std() - 1e-3) < 5e-5           # exponential: std = mean


def test_footprint_covers_outputs():
    wl = serve.Workload(kind=np.array([0, 1, 0, 1], np.int8), side=np.array([256, 512, 100, 4096], np.int32),
                        seed=np.arange(4), nbits=np.array([0, 700000, 0, 45_000_000]),
                        k1=np.zeros(4, np.uint64), k2=np.zeros(4, np.uint64), in_ptr=np.zeros(4, np.uint64),
                        msg_ptr=np.zeros(4, np.uint64), meta_ptr=np.zeros(4, np.uint64))
    ob = wl.out_bytes()
    assert ob[0] == 65536 + 256
    assert ob[1] == (700000 + 127) // 128 * 16 // 256 * 256 + 256 * ((((700000 + 127) // 128 * 16) % 256) > 0) + 262144
    fp = wl.footprint()
    assert np.all(fp > ob)
    assert fp[2] - ob[2] >= 100 * 100 // 2      # untiled shape: larger workspace bound
