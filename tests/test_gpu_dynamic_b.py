"""Parity of the per-tile-b kernel (rdhei_tile_b) with oracle/dynamic_b.py (the
dynamic-b reading: the location-map rule carried over tile borders),
bit-exact (integer counts and choices), through the C ABI."""
import numpy as np
import pytest
import torch

from oracle import dynamic_b as D
from paper_2302_07992_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2302_07992_amd import rdhei
    return rdhei


@pytest.fixture(scope="module")
def ctx(R):
    return R.Context(0)


def _check(ctx, imgs):
    d = [torch.from_numpy(np.ascontiguousarray(I)).cuda() for I in imgs]
    tb, cap = ctx.tile_b(d)
    torch.cuda.synchronize()
    tb, cap = tb.cpu().numpy(), cap.cpu().numpy()
    off = 0
    for i, I in enumerate(imgs):
        b, c = D.tile_b(I)
        n = b.size
        assert np.array_equal(tb[off:off + n].reshape(b.shape), b), f"image {i} {I.shape}"
        assert int(cap[i]) == c, f"image {i} {I.shape}: gpu {int(cap[i])} oracle {c}"
        off += n


def test_tile_b_batch_matches_oracle(R, ctx):
    """Images of several tiled shapes and textures in one call."""
    print("[tile_b] batch", flush=True)
    shapes = [(64, 64), (128, 192), (512, 512), (64, 1024), (320, 256), (1024, 1024)]
    imgs = [inputs.make_image_np(40 + i, M, N, 2 + 3 * i, (1.0, 3.0, 8.0, 20.0)[i % 4])
            for i, (M, N) in enumerate(shapes)]
    imgs.append(np.full((128, 128), 200, np.uint8))
    imgs.append(np.random.default_rng(1).integers(0, 256, (192, 64)).astype(np.uint8))
    _check(ctx, imgs)


def test_tile_b_large_image(R, ctx):
    """A 4096 x 4096 image: 4,096 tiles, more than the grid."""
    print("[tile_b] 4096^2", flush=True)
    _check(ctx, [inputs.make_image_np(77, 4096, 4096, 8, 3.0)])


def test_one_tile_image_equals_the_gpu_emr_choice(R, ctx):
    """On a 64x64 image the tile's b and capacity are the b and capacity that
    encryption records in the meta."""
    I = inputs.make_image_np(5, 64, 64, 8, 3.0)
    d = torch.from_numpy(I).cuda()
    meta = R.new_meta()
    ctx.encrypt(d, torch.empty_like(d), 9, meta)
    m = R.read_meta(meta)
    tb, cap = ctx.tile_b([d])
    assert (int(tb.cpu()[0]), int(cap.cpu()[0])) == (m.b, m.capacity_bits)


def test_tile_b_invalid_arguments(R, ctx):
    for shape in [(64, 100), (100, 64), (32, 64)]:
        with pytest.raises(R.RdheiError):
            ctx.tile_b([torch.zeros(shape, dtype=torch.uint8, device="cuda")])
    buf = torch.zeros(64 * 64 + 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(R.RdheiError):
        ctx.tile_b([buf[1:].view(64, 64)])                 # not 16-byte aligned


# ---- dynamic b end to end (RDHEI_DEMR): every role against the oracle ----------
from oracle import oracle as O


def _demr_round_trip(R, ctx, imgs, k1s, k2s, nonces, frac=1.0, plans=False):
    """encrypt -> embed -> extract -> recover over a batch, each op one direct
    batched launch (or one graph plan); every output against the oracle."""
    n = len(imgs)
    shapes = [I.shape for I in imgs]
    d_in = [torch.from_numpy(np.ascontiguousarray(I)).cuda() for I in imgs]
    enc = [torch.empty_like(x) for x in d_in]
    rec = [torch.empty_like(x) for x in d_in]
    bts = [torch.full(((M // 64) * (N // 64),), 0xEE, dtype=torch.uint8, device="cuda") for M, N in shapes]
    metas = R.new_meta(n)
    mp = [metas[i] for i in range(n)]

    def run(op, jobs):
        if plans:
            p = R.Plan(ctx, op, jobs)
            p.run()
            p.run()          # a graph replay gives the same bytes (every stage is idempotent but embedding,
            # which rewrites the same MSBs from the same labels)
            torch.cuda.synchronize()
            p.close()
        else:
            ctx.run_batch(op, jobs)
    run(R.OP_ENCRYPT, R.make_jobs(d_in, enc, None, mp, k1s, None, shapes, method=R.DEMR, nonces=nonces, btabs=bts))
    torch.cuda.synchronize()
    ms = R.read_meta(metas)
    oracle = [O.demr_encrypt(I, k, nonce=z) for I, k, z in zip(imgs, k1s, nonces)]
    for i, (Ie_o, mo, bt_o) in enumerate(oracle):
        assert (ms[i].status, ms[i].method, ms[i].b) == (0, R.DEMR, 0), i
        assert (ms[i].redundant, ms[i].capacity_bits) == (mo.redundant, mo.capacity_bits), i
        assert np.array_equal(bts[i].cpu().numpy(), bt_o.ravel()), f"b table {i} {shapes[i]}"
        assert np.array_equal(enc[i].cpu().numpy(), Ie_o), f"encrypt {i} {shapes[i]}"
    caps = [int(m.capacity_bits * frac) for m in ms]
    msgs = [inputs.make_payload(k, c).numpy() for k, c in zip(k2s, caps)]
    d_msg = []
    for m, c in zip(msgs, caps):
        buf = torch.zeros(R.msg_bytes(c), dtype=torch.uint8, device="cuda")
        if m.size:
            buf[: m.size] = torch.from_numpy(m).cuda()
        d_msg.append(buf)
    got = [torch.full((R.msg_bytes(c),), 0xAB, dtype=torch.uint8, device="cuda") for c in caps]
    run(R.OP_EMBED, R.make_jobs(None, enc, d_msg, mp, k2s, caps, shapes, method=R.DEMR, btabs=bts))
    run(R.OP_EXTRACT, R.make_jobs(enc, None, got, mp, k2s, caps, shapes, method=R.DEMR, btabs=bts))
    run(R.OP_RECOVER, R.make_jobs(enc, rec, None, mp, k1s, None, shapes, method=R.DEMR, btabs=bts))
    torch.cuda.synchronize()
    assert all(m.status == 0 for m in R.read_meta(metas))
    for i in range(n):
        Ie_o, mo, bt_o = oracle[i]
        W = O.demr_embed(Ie_o, bt_o, msgs[i], caps[i], k2s[i], nonce=nonces[i])
        e = enc[i].cpu().numpy()
        mism = np.argwhere(e != W)
        assert mism.size == 0, f"embed {i} {shapes[i]} at {mism[:5].tolist()} of {len(mism)}"
        nb = (caps[i] + 7) // 8
        g = got[i].cpu().numpy()
        assert np.array_equal(g[:nb], O.demr_extract(W, bt_o, caps[i], k2s[i], nonce=nonces[i])), f"extract {i}"
        assert np.array_equal(g[:nb], msgs[i][:nb])
        r = rec[i].cpu().numpy()
        r_o = O.demr_recover(W, bt_o, k1s[i], nonce=nonces[i])
        mism = np.argwhere(r != r_o)
        assert mism.size == 0, f"recover {i} {shapes[i]} at {mism[:5].tolist()} of {len(mism)}"
        assert np.array_equal(r >> 1, imgs[i] >> 1)
    return ms


DEMR_SHAPES = [(64, 64), (128, 192), (256, 256), (512, 512), (64, 1024), (192, 320)]


@pytest.mark.parametrize("hide_mode", [0, 1, 2, 3], ids=["auto", "whole", "counted", "one_pass"])
@pytest.mark.parametrize("frac", [1.0, 0.37])
def test_demr_batch_matches_oracle(R, hide_mode, frac):
    """Dynamic b (one b per 64x64 tile, the conclusion's future work): a batch
    of tiled shapes and textures, hiding by whole images, counted steps or
    steps in one pass, full and partial payloads, every role equal to the
    oracle."""
    print(f"[demr] batch hide_mode={hide_mode} frac={frac}", flush=True)
    c = R.Context(0)
    c.set_option(R.OPT_HIDE_MODE, hide_mode)
    imgs = [inputs.make_image_np(70 + i, M, N, 2 + 5 * i, (1.0, 3.0, 8.0, 20.0)[i % 4]) for i, (M, N) in
            enumerate(DEMR_SHAPES)]
    imgs.append(np.full((128, 128), 91, np.uint8))
    imgs.append(np.random.default_rng(3).integers(0, 256, (64, 192)).astype(np.uint8))
    n = len(imgs)
    _demr_round_trip(R, c, imgs, [300 + i for i in range(n)], [400 + i for i in range(n)],
                     [(7 * i) << 33 | i for i in range(n)], frac=frac)


def test_demr_per_image_matches_oracle(R):
    """RDHEI_OPT_WG_PER_IMAGE 2 (encryption and recovery of each image in
    one workgroup): per-tile b, the image totals, the b table and I_e, then
    every role, equal to the oracle, direct and as graph plans."""
    print("[demr] encrypt per image", flush=True)
    c = R.Context(0)
    c.set_option(R.OPT_WG_PER_IMAGE, 2)
    imgs = [inputs.make_image_np(170 + i, M, N, 2 + 5 * i, (1.0, 3.0, 8.0, 20.0)[i % 4]) for i, (M, N) in
            enumerate(DEMR_SHAPES)]
    imgs += [_mixed_rows(23, 256, 1024), np.full((128, 128), 91, np.uint8),
             np.random.default_rng(4).integers(0, 256, (64, 192)).astype(np.uint8)]
    n = len(imgs)
    for plans in (False, True):
        _demr_round_trip(R, c, imgs, [500 + i for i in range(n)], [600 + i for i in range(n)],
                         [(11 * i) << 31 | i for i in range(n)], plans=plans)


def _mixed_rows(seed, M, N):
    """Tiles whose b differ (noise under a fixed top, flat, smooth) and rows
    with no label across whole tiles and segments."""
    rng = np.random.default_rng(seed)
    I = inputs.make_image_np(seed, M, N, 6, 3.0)
    for tx in range(N // 64):
        cols = slice(64 * tx, 64 * tx + 64)
        kind = (tx + seed) % 4
        if kind == 0:
            I[:, cols] = 0x40 | rng.integers(0, 64, (M, 64))       # top 2 bits fixed: b = 2
        elif kind == 1:
            I[:, cols] = 0x5A                                       # flat: b = 7
        elif kind == 2:
            I[:, cols] = 0x60 | rng.integers(0, 16, (M, 64))        # top 4 bits fixed
    for r in range(0, M, 5):
        I[r] = (37 * r) % 256                                       # a whole row without a label
    return I.astype(np.uint8)


@pytest.mark.parametrize("qseg", [1, 2])
@pytest.mark.parametrize("shape", [(256, 1024), (128, 1536)], ids=lambda s: f"{s[0]}x{s[1]}")
def test_demr_rows_across_segments(R, qseg, shape):
    """Band pairs cut into short work units (RDHEI_OPT_QUAD_SEG): rows whose
    first label lies tiles or whole segments to the right, through tiles of
    different b, are completed by the fix-up from the restored last pixel of
    the nearest segment that has one; against the oracle."""
    print(f"[demr] segments qseg={qseg} {shape}", flush=True)
    c = R.Context(0)
    c.set_option(R.OPT_QUAD_SEG, qseg)
    imgs = [_mixed_rows(5 + qseg, *shape), inputs.make_image_np(9, *shape, 4, 2.0)]
    ms = _demr_round_trip(R, c, imgs, [11, 12], [21, 22], [31, 32])
    tb, _ = O.demr_tile_b(imgs[0])
    assert len(set(tb.ravel().tolist())) >= 3


def test_demr_plans_chacha_and_large(R):
    """Graph-captured plans under ChaCha20 with nonces, and one 2048 x 2048
    image (hidden by counted steps; finalisation across workgroups is only
    for larger images)."""
    print("[demr] plans chacha20", flush=True)
    c = R.Context(0)
    c.set_option(R.OPT_KEYSTREAM, R.KEYSTREAM_CHACHA20)
    imgs = [inputs.make_image_np(90 + i, 256, 384, 8, 3.0) for i in range(3)]
    with O.keystream_family(O.KEYSTREAM_CHACHA20):
        _demr_round_trip(R, c, imgs, [1, 2, 3], [4, 5, 6], [7, 8, 9], plans=True)
    print("[demr] 2048^2", flush=True)
    _demr_round_trip(R, R.Context(0), [inputs.make_image_np(91, 2048, 2048, 8, 3.0)], [13], [14], [15], frac=0.8)


def test_demr_capacity_equals_tile_b_and_beats_one_b(R, ctx):
    """The capacity encryption records equals what rdhei_tile_b computes, and
    is never below the EMR capacity of the same image."""
    imgs = [inputs.make_image_np(200 + i, 256, 256, 2 + 7 * i, (1.0, 3.0, 8.0, 20.0)[i % 4]) for i in range(8)]
    d = [torch.from_numpy(I).cuda() for I in imgs]
    _, cap = ctx.tile_b(d)
    cap = cap.cpu().numpy()
    for i, I in enumerate(imgs):
        _, mo, _ = O.demr_encrypt(I, 1)
        _, me = O.emr_encrypt(I, 1)
        assert int(cap[i]) == mo.capacity_bits >= me.capacity_bits


def test_demr_invalid_arguments(R, ctx):
    """Sides not multiples of 64, a missing b table, and the single-image
    entry points (batch only for dynamic b) are rejected on the host."""
    meta = R.new_meta()
    x = torch.zeros(64, 100, dtype=torch.uint8, device="cuda")
    bt = torch.zeros(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(R.RdheiError):
        ctx.run_batch(R.OP_ENCRYPT, R.make_jobs([x], [torch.empty_like(x)], None, [meta], [1], None, [(64, 100)],
                                                method=R.DEMR, btabs=[bt]))
    y = torch.zeros(128, 128, dtype=torch.uint8, device="cuda")
    with pytest.raises(R.RdheiError):
        ctx.run_batch(R.OP_ENCRYPT, R.make_jobs([y], [torch.empty_like(y)], None, [meta], [1], None, [(128, 128)],
                                                method=R.DEMR))
    with pytest.raises(R.RdheiError):
        ctx.encrypt(y, torch.empty_like(y), 1, meta, method=R.DEMR)


def test_demr_4096_big_image_matches_oracle(R):
    """A 4096 x 4096 image (4,096 tiles: the statistics and pyramid are
    finalised across workgroups, the b totals in the top pass; 4,096 hiding
    steps with bit-weighted ranks) through every role against the oracle,
    with a payload ending inside a pixel."""
    print("[demr] 4096^2", flush=True)
    I = inputs.make_band_image(17, 4096, 4096, 8, 3.0, "cpu").numpy()
    _demr_round_trip(R, R.Context(0), [I], [27], [28], [29], frac=0.91)
