"""Parity of the batched image-metric kernels (rdhei_metrics, Sec. IV
metrics) with the metric oracle, through the C ABI.

Everything but the final divisions and logarithms is integer on both sides
(level counts, differing pixels, sums of |a - b| and (a - b)^2, 7x7 window
sums), so entropy, chi-square, NPCR, UACI and PSNR agree to the last few
ulps (relative 1e-12); SSIM is the mean of up to millions of per-window
doubles computed in the same order on both sides, added in a different
order: relative 1e-10."""
import math

import numpy as np
import pytest
import torch

from oracle import metrics as OM

pytestmark = pytest.mark.gpu

REL = [1e-12, 1e-12, 1e-12, 1e-12, 1e-12, 1e-12, 1e-12, 1e-10]


@pytest.fixture(scope="module")
def R():
    from paper_2302_07992_amd import rdhei
    return rdhei


@pytest.fixture(scope="module")
def ctx(R):
    return R.Context(0)


def _close(got, want, k):
    if math.isnan(want):
        return math.isnan(got)
    if math.isinf(want):
        return got == want
    return abs(got - want) <= REL[k] * max(1.0, abs(want))


def _check(R, ctx, pairs_np, ssim=True, align=True):
    """pairs_np: list of (a, b or None) numpy uint8 images."""
    pairs = []
    keep = []
    for a, b in pairs_np:
        if align:
            da = torch.from_numpy(np.ascontiguousarray(a)).cuda()
            db = torch.from_numpy(np.ascontiguousarray(b)).cuda() if b is not None else None
        else:   # one byte past a 16-byte boundary: the byte-by-byte path
            ba = torch.zeros(a.size + 1, dtype=torch.uint8, device="cuda")
            ba[1:] = torch.from_numpy(a.ravel()).cuda()
            da = ba[1:].view(a.shape)
            keep.append(ba)
            db = None
            if b is not None:
                bb = torch.zeros(b.size + 1, dtype=torch.uint8, device="cuda")
                bb[1:] = torch.from_numpy(b.ravel()).cuda()
                db = bb[1:].view(b.shape)
                keep.append(bb)
        pairs.append((da, db))
    out = ctx.metrics(pairs, ssim=ssim)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for i, (a, b) in enumerate(pairs_np):
        want = OM.image_metrics(a, b, with_ssim=ssim)
        for k in range(8):
            assert _close(float(got[i, k]), float(want[k]), k), \
                f"pair {i} {a.shape} {R.METRIC_NAMES[k]}: gpu {got[i, k]!r} oracle {want[k]!r}"


def _pair(seed, M, N, kind="noisy"):
    rng = np.random.default_rng(seed)
    y, x = np.indices((M, N))
    a = np.clip(128 + 60 * np.sin(x / 17.0 + seed) * np.cos(y / 23.0) + rng.normal(0, 4, (M, N)), 0, 255)
    a = np.rint(a).astype(np.uint8)
    if kind == "same":
        return a, a.copy()
    if kind == "random":
        return a, rng.integers(0, 256, (M, N)).astype(np.uint8)
    return a, np.clip(a.astype(np.int64) + rng.integers(-9, 10, (M, N)), 0, 255).astype(np.uint8)


SHAPES = [(1, 1), (5, 9), (6, 40), (7, 7), (8, 13), (64, 64), (100, 63), (130, 257), (512, 512), (300, 1000),
          (1100, 70)]


@pytest.mark.parametrize("align", [True, False], ids=["aligned", "unaligned"])
def test_metrics_match_oracle(R, ctx, align):
    """A batch of pairs of every shape (below the window, one window, several
    SSIM tiles in both directions, ragged sizes), noisy, random and identical
    pairs, and single images."""
    print(f"[metrics] align={align}", flush=True)
    pairs = []
    for i, (M, N) in enumerate(SHAPES):
        pairs.append(_pair(10 + i, M, N, ["noisy", "random", "same"][i % 3]))
    pairs.append((_pair(99, 90, 110)[0], None))
    _check(R, ctx, pairs, ssim=True, align=align)


def test_metrics_without_ssim_and_multi_run_images(R, ctx):
    """Images of several 256K-pixel runs (histograms and sums added across
    workgroups); SSIM not asked for comes back NaN."""
    print("[metrics] multi-run", flush=True)
    pairs = [_pair(5, 1024, 1024, "random"), _pair(6, 700, 1300), _pair(7, 513, 511, "same")]
    _check(R, ctx, pairs, ssim=False)
    _check(R, ctx, pairs[:2], ssim=True)


def test_metrics_full_size_image(R, ctx):
    """A 4096 x 4096 pair (64 runs, 1,024 SSIM tiles) and an image against its
    complement (NPCR 100 unless a pixel is 127.5, which none is)."""
    print("[metrics] 4096^2", flush=True)
    a, b = _pair(8, 4096, 4096)
    _check(R, ctx, [(a, b), (a, (255 - a).astype(np.uint8))], ssim=True)


def test_metrics_invalid_arguments(R, ctx):
    z = torch.zeros(8, 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(R.RdheiError):
        ctx.metrics([(z, torch.zeros(8, 9, dtype=torch.uint8, device="cuda"))])
    lib = R.load_library()
    arr = (R.MetricJobStruct * 1)()
    arr[0].a, arr[0].b, arr[0].height, arr[0].width = z.data_ptr(), None, 0, 8
    out = torch.empty(8, dtype=torch.float64, device="cuda")
    import ctypes
    assert lib.rdhei_metrics(ctx.h, arr, 1, 0, ctypes.c_void_p(out.data_ptr()), None) == R.EINVAL
    arr[0].height = 8
    assert lib.rdhei_metrics(ctx.h, arr, 1, 4, ctypes.c_void_p(out.data_ptr()), None) == R.EINVAL
    assert lib.rdhei_metrics(ctx.h, arr, 1, 0, None, None) == R.EINVAL
