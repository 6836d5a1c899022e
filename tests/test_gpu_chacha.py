"""Parity of the ChaCha20 keystream family (RDHEI_OPT_KEYSTREAM) with the
oracle under the same family, element by element through the C ABI: the
tiled and per-pixel EMR paths, both hiding schemes, batched plans and LMR.
The oracle's ChaCha20 is pinned against OpenSSL in the CPU tests."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2302_07992_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2302_07992_amd import rdhei
    return rdhei


@pytest.fixture(scope="module")
def cctx(R):
    c = R.Context(0)
    c.set_option(R.OPT_KEYSTREAM, R.KEYSTREAM_CHACHA20)
    return c


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _msg_dev(R, msg, nbits):
    buf = torch.zeros(R.msg_bytes(nbits), dtype=torch.uint8, device="cuda")
    if msg.size:
        buf[: msg.size] = torch.from_numpy(msg).cuda()
    return buf


@pytest.mark.parametrize("shape,frac", [((64, 64), 1.0), ((256, 256), 1.0), ((512, 512), 0.37), ((1024, 1024), 1.0),
                                        ((2048, 1024), 1.0), ((4096, 4096), 1.0), ((100, 63), 1.0), ((33, 47), 0.5),
                                        ((1, 9), 1.0)],
                         ids=lambda v: f"{v[0]}x{v[1]}" if isinstance(v, tuple) else f"f{v}")
def test_emr_chacha_roundtrip_matches_oracle(R, cctx, shape, frac):
    M, N = shape
    k1, k2 = 0x0123456789ABCDEF + M, 0x0FEDCBA987654321 + N
    print(f"[chacha emr] shape={M}x{N} frac={frac}", flush=True)
    I = inputs.make_image_np(M * 3 + N, M, N, 8, 3.0)
    with O.keystream_family(O.KEYSTREAM_CHACHA20):
        Ie_o, mo = O.emr_encrypt(I, k1)
        nbits = int(mo.capacity_bits * frac)
        msg = inputs.make_payload(k2 & 0xFFFF, nbits).numpy()
        Iem_o = O.emr_embed(Ie_o, mo.b, msg, nbits, k2)
        got_o = O.emr_extract(Iem_o, mo.b, nbits, k2)
        rec_o = O.emr_recover(Iem_o, mo.b, k1)
    d_img = _dev(I)
    d_enc = torch.empty_like(d_img)
    meta = R.new_meta()
    cctx.encrypt(d_img, d_enc, k1, meta)
    m = R.read_meta(meta)
    assert (m.status, m.b, m.capacity_bits) == (0, mo.b, mo.capacity_bits)
    assert np.array_equal(d_enc.cpu().numpy(), Ie_o)
    cctx.embed(d_enc, meta, _msg_dev(R, msg, nbits), nbits, k2)
    assert np.array_equal(d_enc.cpu().numpy(), Iem_o)
    d_out = torch.zeros(R.msg_bytes(nbits), dtype=torch.uint8, device="cuda")
    cctx.extract(d_enc, meta, d_out, nbits, k2)
    nb = (nbits + 7) // 8
    assert np.array_equal(d_out.cpu().numpy()[:nb], got_o)
    assert np.array_equal(d_out.cpu().numpy()[:nb], msg[:nb])
    d_rec = torch.empty_like(d_img)
    cctx.recover(d_enc, meta, d_rec, k1)
    assert np.array_equal(d_rec.cpu().numpy(), rec_o)
    assert np.array_equal(d_rec.cpu().numpy() >> 1, I >> 1)


@pytest.mark.parametrize("hide_mode", [1, 2, 3], ids=["whole", "counted", "one_pass"])
def test_batched_chacha_plan_matches_oracle(R, hide_mode):
    """A graph-captured batch of tiled and per-pixel images under ChaCha20;
    hiding walks images whole (one wave each) or in counted steps."""
    print(f"[chacha batched] hide_mode={hide_mode}", flush=True)
    ctx = R.Context(0)
    ctx.set_option(R.OPT_KEYSTREAM, R.KEYSTREAM_CHACHA20)
    ctx.set_option(R.OPT_HIDE_MODE, hide_mode)
    shapes = [(64, 64), (256, 256), (33, 47), (512, 512), (100, 63), (320, 256)]
    imgs = [inputs.make_image_np(300 + i, *s, 2 + i, (1, 3, 8)[i % 3]) for i, s in enumerate(shapes)]
    n = len(imgs)
    d_in = [_dev(I) for I in imgs]
    d_enc = [torch.empty_like(x) for x in d_in]
    d_rec = [torch.empty_like(x) for x in d_in]
    metas = R.new_meta(n)
    k1s = [(7 << 40) + i for i in range(n)]
    k2s = [(9 << 50) + i for i in range(n)]
    R.Plan(ctx, R.OP_ENCRYPT, R.make_jobs(d_in, d_enc, None, [metas[i] for i in range(n)], k1s, None, shapes)).run()
    torch.cuda.synchronize()
    ms = R.read_meta(metas)
    caps = [m.capacity_bits for m in ms]
    msgs = [inputs.make_payload(50 + i, c).numpy() for i, c in enumerate(caps)]
    d_msg = [_msg_dev(R, m, c) for m, c in zip(msgs, caps)]
    R.Plan(ctx, R.OP_EMBED, R.make_jobs(None, d_enc, d_msg, [metas[i] for i in range(n)], k2s, caps, shapes)).run()
    d_got = [torch.zeros(R.msg_bytes(c), dtype=torch.uint8, device="cuda") for c in caps]
    R.Plan(ctx, R.OP_EXTRACT, R.make_jobs(d_enc, None, d_got, [metas[i] for i in range(n)], k2s, caps, shapes)).run()
    R.Plan(ctx, R.OP_RECOVER, R.make_jobs(d_enc, d_rec, None, [metas[i] for i in range(n)], k1s, None, shapes)).run()
    torch.cuda.synchronize()
    with O.keystream_family(O.KEYSTREAM_CHACHA20):
        for i in range(n):
            Ie_o, mo = O.emr_encrypt(imgs[i], k1s[i])
            assert (ms[i].b, caps[i]) == (mo.b, mo.capacity_bits)
            Iem_o = O.emr_embed(Ie_o, mo.b, msgs[i], caps[i], k2s[i])
            assert np.array_equal(d_enc[i].cpu().numpy(), Iem_o), f"image {i} {shapes[i]}"
            nb = (caps[i] + 7) // 8
            assert np.array_equal(d_got[i].cpu().numpy()[:nb], msgs[i])
            assert np.array_equal(d_rec[i].cpu().numpy(), O.emr_recover(Iem_o, mo.b, k1s[i]))


def test_chacha_per_image_matches_oracle(R):
    """Encryption and recovery one workgroup per image
    (RDHEI_OPT_WG_PER_IMAGE 2) under ChaCha20 with per-image nonces: meta,
    I_e and I' equal the oracle's."""
    print("[chacha encrypt per image]", flush=True)
    ctx = R.Context(0)
    ctx.set_option(R.OPT_KEYSTREAM, R.KEYSTREAM_CHACHA20)
    ctx.set_option(R.OPT_WG_PER_IMAGE, 2)
    shapes = [(64, 64), (256, 256), (512, 512), (320, 256), (128, 1024), (576, 192)]
    imgs = [inputs.make_image_np(340 + i, *s, 2 + i, (1, 3, 8)[i % 3]) for i, s in enumerate(shapes)]
    n = len(imgs)
    d_in = [_dev(I) for I in imgs]
    d_enc = [torch.empty_like(x) for x in d_in]
    metas = R.new_meta(n)
    k1s = [(5 << 44) + i for i in range(n)]
    nonces = [(3 << 61) | i for i in range(n)]
    plan = R.Plan(ctx, R.OP_ENCRYPT, R.make_jobs(d_in, d_enc, None, [metas[i] for i in range(n)], k1s, None, shapes,
                                                  nonces=nonces))
    assert plan.stages() == ["encrypt_images"]
    plan.run()
    torch.cuda.synchronize()
    ms = R.read_meta(metas)
    d_rec = [torch.empty_like(x) for x in d_in]
    rp = R.Plan(ctx, R.OP_RECOVER, R.make_jobs(d_enc, d_rec, None, [metas[i] for i in range(n)], k1s, None, shapes))
    assert rp.stages() == ["recover_images"]
    rp.run()
    torch.cuda.synchronize()
    with O.keystream_family(O.KEYSTREAM_CHACHA20):
        for i in range(n):
            Ie_o, mo = O.emr_encrypt(imgs[i], k1s[i], nonce=nonces[i])
            assert (ms[i].b, ms[i].capacity_bits, ms[i].nonce) == (mo.b, mo.capacity_bits, nonces[i])
            assert np.array_equal(d_enc[i].cpu().numpy(), Ie_o), f"image {i} {shapes[i]}"
            assert np.array_equal(d_rec[i].cpu().numpy(), O.emr_recover(Ie_o, mo.b, k1s[i], nonce=nonces[i]))


@pytest.mark.parametrize("shape", [(256, 256), (100, 90)], ids=lambda s: f"{s[0]}x{s[1]}")
def test_lmr_chacha_matches_oracle(R, cctx, shape):
    """LMR under ChaCha20 (tiled and per-pixel): encrypted image, marked
    image, payload and the exact recovery."""
    M, N = shape
    print(f"[chacha lmr] shape={M}x{N}", flush=True)
    I = inputs.make_image_np(M + 11 * N, M, N, 8, 1.0)
    k1, k2 = 0xABCDEF0123 + M, 0x5555AAAA + N
    with O.keystream_family(O.KEYSTREAM_CHACHA20):
        Ie_o, mo, stream = O.lmr_encode(I, k1, 4)
        assert Ie_o is not None
        eta_rot, l_rot = O.lmr_decompress(stream, M, N)
        nbits = int(mo.capacity_bits)
        msg = inputs.make_payload(5, nbits).numpy()
        Iem_o = O.lmr_embed(Ie_o, mo.b, l_rot, msg, nbits, k2)
        rec_o = O.lmr_recover(Iem_o, mo.b, 4, k1, l_rot, eta_rot)
    d_img = _dev(I)
    d_enc = torch.empty_like(d_img)
    meta = R.new_meta()
    cctx.encrypt(d_img, d_enc, k1, meta, method=R.LMR)
    assert np.array_equal(d_enc.cpu().numpy(), Ie_o)
    cctx.embed(d_enc, meta, _msg_dev(R, msg, nbits), nbits, k2, method=R.LMR)
    assert np.array_equal(d_enc.cpu().numpy(), Iem_o)
    d_got = torch.zeros(R.msg_bytes(nbits), dtype=torch.uint8, device="cuda")
    cctx.extract(d_enc, meta, d_got, nbits, k2, method=R.LMR)
    assert np.array_equal(d_got.cpu().numpy()[:(nbits + 7) // 8], msg)
    d_rec = torch.empty_like(d_img)
    cctx.recover(d_enc, meta, d_rec, k1, method=R.LMR)
    assert np.array_equal(d_rec.cpu().numpy(), rec_o)
    assert np.array_equal(d_rec.cpu().numpy(), I)


def test_keystream_families_differ_and_must_match(R, cctx):
    """The two families encrypt differently; a recipient on the other family
    does not get the image back; bad option values are refused."""
    I = inputs.make_image_np(4, 256, 256, 8, 3.0)
    pctx = R.Context(0)
    d_img = _dev(I)
    e_c, e_p = torch.empty_like(d_img), torch.empty_like(d_img)
    m_c, m_p = R.new_meta(), R.new_meta()
    cctx.encrypt(d_img, e_c, 77, m_c)
    pctx.encrypt(d_img, e_p, 77, m_p)
    assert R.read_meta(m_c).b == R.read_meta(m_p).b
    assert not torch.equal(e_c, e_p)
    rec = torch.empty_like(d_img)
    pctx.recover(e_c, m_c, rec, 77)
    assert not np.array_equal(rec.cpu().numpy() >> 1, I >> 1)
    for bad in (-1, 2):
        with pytest.raises(R.RdheiError):
            pctx.set_option(R.OPT_KEYSTREAM, bad)


def test_lmr_batch_chacha_matches_oracle(R):
    """The batched LMR roles under ChaCha20 (device stages batched, host map
    coder): encrypted images and marked images equal the oracle's, payloads
    and exact recovery."""
    print("[chacha lmr batch]", flush=True)
    ctx = R.Context(0)
    ctx.set_option(R.OPT_KEYSTREAM, R.KEYSTREAM_CHACHA20)
    shapes = [(256, 256), (128, 320), (100, 90), (64, 64)]
    imgs = [inputs.make_image_np(900 + i, *s, 8, (1.0, 3.0)[i % 2]) for i, s in enumerate(shapes)]
    n = len(imgs)
    d_in = [_dev(I) for I in imgs]
    k1s, k2s = [(3 << 33) + i for i in range(n)], [(5 << 35) + i for i in range(n)]
    enc = [torch.zeros_like(x) for x in d_in]
    metas = R.new_meta(n)
    mp = [metas[i] for i in range(n)]
    ctx.lmr_batch(R.OP_ENCRYPT, R.make_jobs(d_in, enc, None, mp, k1s, None, shapes, method=R.LMR), threads=2)
    ms = R.read_meta(metas)
    assert all(m.status == 0 for m in ms)
    caps = [m.capacity_bits for m in ms]
    msgs = [inputs.make_payload(20 + i, c).numpy() for i, c in enumerate(caps)]
    d_msg = [_msg_dev(R, m, c) for m, c in zip(msgs, caps)]
    with O.keystream_family(O.KEYSTREAM_CHACHA20):
        want = [O.lmr_encode(I, k, 4) for I, k in zip(imgs, k1s)]
        for i in range(n):
            assert (ms[i].b, ms[i].capacity_bits) == (want[i][1].b, want[i][1].capacity_bits), i
            assert np.array_equal(enc[i].cpu().numpy(), want[i][0]), i
    ctx.lmr_batch(R.OP_EMBED, R.make_jobs(None, enc, d_msg, mp, k2s, caps, shapes, method=R.LMR))
    got = [torch.zeros(R.msg_bytes(c), dtype=torch.uint8, device="cuda") for c in caps]
    ctx.lmr_batch(R.OP_EXTRACT, R.make_jobs(enc, None, got, mp, k2s, caps, shapes, method=R.LMR))
    rec = [torch.zeros_like(x) for x in d_in]
    ctx.lmr_batch(R.OP_RECOVER, R.make_jobs(enc, rec, None, mp, k1s, None, shapes, method=R.LMR))
    torch.cuda.synchronize()
    with O.keystream_family(O.KEYSTREAM_CHACHA20):
        for i in range(n):
            Ie_o, mo, stream = want[i]
            eta_rot, l_rot = O.lmr_decompress(stream, *shapes[i])
            assert np.array_equal(enc[i].cpu().numpy(), O.lmr_embed(Ie_o, mo.b, l_rot, msgs[i], caps[i], k2s[i])), i
            assert np.array_equal(got[i].cpu().numpy()[:(caps[i] + 7) // 8], msgs[i]), i
            assert torch.equal(rec[i], d_in[i]), i
