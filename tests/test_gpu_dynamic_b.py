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
