"""Serving loop on the GPU: every request's outputs are byte-identical when
served alone (single-image entry points) and inside mixed continuous
batches, and match the oracle."""
import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2302_07992_amd import serve
    return serve


@pytest.fixture(scope="module")
def R():
    from paper_2302_07992_amd import rdhei
    return rdhei


@pytest.fixture(scope="module")
def workload(S, R):
    # tiled and untiled sides; 48 requests of the 60/40 mix
    print("[serve] building workload", flush=True)
    return S.make_workload(48, seed=5, sides=[64, 128, 256, 96, 100, 320], weights=[3, 3, 2, 1, 1, 1],
                           keep_originals=True)


def _alone(R, wl, i):
    """Request i through the single-image entry points, on its own."""
    ctx = R.Context()
    M = int(wl.side[i])
    nbits = int(wl.nbits[i])
    if wl.kind[i] == 0:
        enc = torch.empty(M, M, dtype=torch.uint8, device="cuda")
        meta = R.new_meta()
        msg = torch.zeros(R.msg_bytes(nbits), dtype=torch.uint8, device="cuda")
        msg[: wl.payloads[i].numel()] = wl.payloads[i]
        ctx.encrypt(wl.images[i], enc, int(wl.k1[i]), meta, nonce=int(wl.seed[i]))
        ctx.embed(enc, meta, msg, nbits, int(wl.k2[i]))
        torch.cuda.synchronize()
        return {"marked": enc.cpu().numpy(), "meta": meta.cpu().numpy()}
    meta_in = _meta_of(R, wl, i)
    msg = torch.zeros(R.msg_bytes(nbits), dtype=torch.uint8, device="cuda")
    rec = torch.empty(M, M, dtype=torch.uint8, device="cuda")
    ctx.extract(wl.images[i], meta_in, msg, nbits, int(wl.k2[i]))
    ctx.recover(wl.images[i], meta_in, rec, int(wl.k1[i]))
    torch.cuda.synchronize()
    return {"recovered": rec.cpu().numpy(), "payload": msg.cpu().numpy()}


def _meta_of(R, wl, i):
    """The resident metadata tensor of RECOVER request i."""
    for t in wl.keep:
        if t.data_ptr() == int(wl.meta_ptr[i]):
            return t
    raise KeyError(i)


def _serve(S, wl, arrivals, **kw):
    got = {}

    def keep(i, views):
        got[i] = {k: v.cpu().numpy().copy() for k, v in views.items()}

    srv = S.Server(on_complete=keep, **kw)
    res = srv.run(wl, arrivals)
    return res, got


def _bits(a, nbits):
    return np.unpackbits(np.asarray(a, np.uint8))[:nbits]


@pytest.mark.parametrize("mode", ["burst", "poisson", "per_request"])
def test_served_equals_alone(S, R, workload, mode):
    wl = workload
    n = len(wl)
    print(f"[serve] isolation mode={mode} n={n}", flush=True)
    if mode == "burst":
        arrivals = np.zeros(n)                        # all queued at once: large batches
        kw = dict(pool_bytes=1 << 20, streams=2)      # pool binds: several batches
    elif mode == "poisson":
        arrivals = S.poisson_arrivals(n, 20000.0, seed=2)
        kw = dict(pool_bytes=4 << 20, streams=3)
    else:
        arrivals = S.poisson_arrivals(n, 20000.0, seed=2)
        kw = dict(pool_bytes=4 << 20, per_request=True)
    res, got = _serve(S, wl, arrivals, **kw)
    assert res.rejected == 0
    assert sorted(got) == list(range(n))
    assert np.all(np.isfinite(res.latency_s)) and np.all(res.latency_s > 0)
    if mode == "burst":
        assert 1 < res.batches < n                    # admission split the burst
    if mode == "per_request":
        assert res.batches == n
    for i in range(n):
        ref = _alone(R, wl, i)
        if wl.kind[i] == 0:
            assert np.array_equal(got[i]["marked"], ref["marked"]), i
            assert np.array_equal(got[i]["meta"], ref["meta"]), i
        else:
            nb = int(wl.nbits[i])
            assert np.array_equal(got[i]["recovered"], ref["recovered"]), i
            assert np.array_equal(_bits(got[i]["payload"], nb), _bits(ref["payload"], nb)), i


def test_served_matches_oracle(S, R, workload):
    """Served outputs against the oracle: the marked image of EMBED requests,
    and the payload and restored image of RECOVER requests."""
    wl = workload
    n = len(wl)
    res, got = _serve(S, wl, np.zeros(n), pool_bytes=2 << 20, streams=2)
    assert res.rejected == 0
    checked = 0
    for i in range(n):
        I = wl.images[i].cpu().numpy()
        k1, k2, nb, nz = int(wl.k1[i]), int(wl.k2[i]), int(wl.nbits[i]), int(wl.seed[i])
        pay = wl.payloads[i].cpu().numpy()
        if wl.kind[i] == 0:
            Ie, mo = O.emr_encrypt(I, k1, nonce=nz)
            assert mo.capacity_bits == nb
            marked = O.emr_embed(Ie, mo.b, pay, nb, k2, nonce=nz)
            assert np.array_equal(got[i]["marked"], marked), i
        else:
            orig = wl.originals[i].cpu().numpy()
            _, mo = O.emr_encrypt(orig, k1, nonce=nz)
            assert np.array_equal(_bits(got[i]["payload"], nb), _bits(pay, nb)), i
            assert np.array_equal(got[i]["recovered"], O.emr_recover(I, mo.b, k1, nonce=nz)), i
            assert np.all((got[i]["recovered"] ^ orig) <= 1)
        checked += 1
    assert checked == n


def test_served_chacha_matches_oracle(S, R):
    """A server on the ChaCha20 keystream family (RECOVER inputs prepared
    under ChaCha20 too) against the oracle under the same family."""
    print("[serve] chacha20", flush=True)
    cctx = R.Context()
    cctx.set_option(R.OPT_KEYSTREAM, R.KEYSTREAM_CHACHA20)
    wl = S.make_workload(24, seed=11, sides=[64, 128, 100, 256], weights=[2, 2, 1, 1], ctx=cctx, keep_originals=True)
    n = len(wl)
    res, got = _serve(S, wl, np.zeros(n), pool_bytes=2 << 20, streams=2, keystream=R.KEYSTREAM_CHACHA20)
    assert res.rejected == 0 and sorted(got) == list(range(n))
    with O.keystream_family(O.KEYSTREAM_CHACHA20):
        for i in range(n):
            I = wl.images[i].cpu().numpy()
            k1, k2, nb, nz = int(wl.k1[i]), int(wl.k2[i]), int(wl.nbits[i]), int(wl.seed[i])
            pay = wl.payloads[i].cpu().numpy()
            if wl.kind[i] == 0:
                Ie, mo = O.emr_encrypt(I, k1, nonce=nz)
                assert mo.capacity_bits == nb
                assert np.array_equal(got[i]["marked"], O.emr_embed(Ie, mo.b, pay, nb, k2, nonce=nz)), i
            else:
                orig = wl.originals[i].cpu().numpy()
                _, mo = O.emr_encrypt(orig, k1, nonce=nz)
                assert np.array_equal(_bits(got[i]["payload"], nb), _bits(pay, nb)), i
                assert np.array_equal(got[i]["recovered"], O.emr_recover(I, mo.b, k1, nonce=nz)), i


def test_request_larger_than_pool_is_rejected(S, workload):
    wl = workload
    big = int(np.argmax(wl.footprint()))
    pool = int(wl.footprint()[big]) - 1024
    res, got = _serve(S, wl, np.zeros(len(wl)), pool_bytes=pool, streams=1)
    assert res.rejected >= 1
    assert not np.isfinite(res.latency_s[big])
    assert big not in got


def test_run_roles_equals_run_batch_per_op(R):
    """rdhei_run_roles (every op of a batch in one call, one table upload,
    one shared workspace) gives the bytes of one rdhei_run_batch per op: a
    mixed batch of new requests (encrypt then embed) and returning ones
    (extract and recover), tiled and per-pixel shapes."""
    from paper_2302_07992_amd import inputs
    print("[serve] run_roles against run_batch", flush=True)
    ctx = R.Context(0)
    shapes = [(256, 256), (128, 320), (100, 63), (512, 512)]
    n = len(shapes)
    imgs = [inputs.make_image(900 + i, M, N, 8, 3.0, "cuda") for i, (M, N) in enumerate(shapes)]
    k1 = [11 + i for i in range(n)]
    k2 = [21 + i for i in range(n)]
    # capacities and a marked image for every shape (the returning requests' inputs)
    metas0 = R.new_meta(n)
    marked = [torch.empty_like(x) for x in imgs]
    ctx.run_batch(R.OP_ENCRYPT, R.make_jobs(imgs, marked, None, [metas0[i] for i in range(n)], k1, None, shapes,
                                             nonces=list(range(n))))
    torch.cuda.synchronize()
    caps = [int(m.capacity_bits) for m in R.read_meta(metas0)]
    msgs = [inputs.make_payload(k, c, "cuda") for k, c in zip(k2, caps)]
    bufs = []
    for m, c in zip(msgs, caps):
        b = torch.zeros(R.msg_bytes(c), dtype=torch.uint8, device="cuda")
        b[: m.numel()] = m
        bufs.append(b)
    ctx.run_batch(R.OP_EMBED, R.make_jobs(None, marked, bufs, [metas0[i] for i in range(n)], k2, caps, shapes))
    torch.cuda.synchronize()

    def once(use_roles):
        metas = R.new_meta(n)
        mp = [metas[i] for i in range(n)]
        enc = [torch.empty_like(x) for x in imgs]
        got = [torch.zeros(R.msg_bytes(c), dtype=torch.uint8, device="cuda") for c in caps]
        rec = [torch.empty_like(x) for x in imgs]
        roles = [(R.OP_ENCRYPT, R.make_jobs(imgs, enc, None, mp, k1, None, shapes, nonces=list(range(n)))),
                 (R.OP_EMBED, R.make_jobs(None, enc, bufs, mp, k2, caps, shapes)),
                 (R.OP_EXTRACT, R.make_jobs(marked, None, got, [metas0[i] for i in range(n)], k2, caps, shapes)),
                 (R.OP_RECOVER, R.make_jobs(marked, rec, None, [metas0[i] for i in range(n)], k1, None, shapes))]
        if use_roles:
            wsb = ctx.roles_workspace_size(roles)
            assert wsb >= max(ctx.workspace_size(op, t) for op, t in roles)
            ws = torch.empty(wsb + 256, dtype=torch.uint8, device="cuda")
            base = (ws.data_ptr() + 255) // 256 * 256
            ctx.run_roles(roles, base, wsb)
        else:
            for op, t in roles:
                ctx.run_batch(op, t)
        torch.cuda.synchronize()
        return ([e.cpu() for e in enc], [g.cpu() for g in got], [r.cpu() for r in rec], metas.cpu())

    a, b = once(False), once(True)
    for xa, xb in zip(a[:3], b[:3]):
        for u, v in zip(xa, xb):
            assert torch.equal(u, v)
    assert torch.equal(a[3], b[3])
    for g, m, c in zip(a[1], msgs, caps):
        assert torch.equal(g[: c // 8], m[: c // 8].cpu())
