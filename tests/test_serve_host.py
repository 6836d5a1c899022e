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


def test_batch_tables_fields_and_layout():
    """A batch's job tables: every field of every op comes from its request
    (inputs, keys, nonce, sizes, payload bits), and the outputs are laid out
    back to back from the base, 256-byte aligned, without overlap: EMBED
    requests' marked image then meta, then RECOVER requests' payload then
    restored image."""
    from paper_2302_07992_amd import rdhei as R
    rng = np.random.default_rng(7)
    n = 400
    wl = serve.Workload(kind=np.where(rng.random(n) < 0.6, serve.EMBED_REQ, serve.RECOVER_REQ).astype(np.int8),
                        side=rng.choice([64, 256, 512, 1024], n).astype(np.int32), seed=np.arange(n) * 3 + 1,
                        nbits=rng.integers(0, 200000, n), k1=np.arange(n, dtype=np.uint64) * 5 + 1,
                        k2=np.arange(n, dtype=np.uint64) * 7 + 2, in_ptr=np.arange(n, dtype=np.uint64) * 4096 + 256,
                        msg_ptr=np.arange(n, dtype=np.uint64) * 512 + 1024, meta_ptr=np.arange(n, dtype=np.uint64) * 256 + 512)

    class Host:                 # the table builder needs no device state
        _tmpl = {}
        _templates = staticmethod(serve.Server._templates)

    base = 1 << 40
    for trial in range(50):
        a = int(rng.integers(0, n - 40))
        idx = np.arange(a, a + int(rng.integers(1, 40)))
        tabs, out, total = serve.Server._tables(Host(), wl, idx, base)
        ops = {op: t for op, t, _ in tabs}
        e, r = out["e"], out["r"]
        assert sorted(np.concatenate([e, r]).tolist()) == idx.tolist()
        assert np.all(wl.kind[e] == serve.EMBED_REQ) and np.all(wl.kind[r] == serve.RECOVER_REQ)
        spans = []
        if len(e):
            enc, emb = ops[R.OP_ENCRYPT], ops[R.OP_EMBED]
            px = wl.pixels[e]
            assert np.array_equal(enc["inp"], wl.in_ptr[e]) and np.array_equal(enc["key"], wl.k1[e])
            assert np.array_equal(enc["nonce"], wl.seed[e].astype(np.uint64))
            assert np.array_equal(emb["msg"], wl.msg_ptr[e]) and np.array_equal(emb["key"], wl.k2[e])
            assert np.array_equal(emb["nbits"], wl.nbits[e]) and not emb["inp"].any() and not emb["nonce"].any()
            assert np.array_equal(enc["out"], emb["out"]) and np.array_equal(enc["meta"], emb["meta"])
            assert np.array_equal(enc["height"], wl.side[e]) and np.array_equal(emb["width"], wl.side[e])
            spans += [(int(o), int(o) + int(p)) for o, p in zip(enc["out"], px)]
            spans += [(int(m), int(m) + R.META_BYTES) for m in enc["meta"]]
        if len(r):
            ext, rec = ops[R.OP_EXTRACT], ops[R.OP_RECOVER]
            assert np.array_equal(ext["inp"], wl.in_ptr[r]) and np.array_equal(rec["inp"], wl.in_ptr[r])
            assert np.array_equal(ext["meta"], wl.meta_ptr[r]) and np.array_equal(rec["meta"], wl.meta_ptr[r])
            assert np.array_equal(ext["key"], wl.k2[r]) and np.array_equal(rec["key"], wl.k1[r])
            assert np.array_equal(ext["nbits"], wl.nbits[r]) and not rec["nbits"].any() and not rec["msg"].any()
            spans += [(int(m), int(m) + int(b)) for m, b in zip(ext["msg"], serve.msg_bytes(wl.nbits[r]))]
            spans += [(int(o), int(o) + int(p)) for o, p in zip(rec["out"], wl.pixels[r])]
        spans.sort()
        assert all(s0 % 256 == 0 and base <= s0 and s1 <= base + total for s0, s1 in spans)
        assert all(a1 <= b0 for (_, a1), (b0, _) in zip(spans, spans[1:]))
