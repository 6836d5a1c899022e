"""Host-side checks of the C-ABI library (no GPU needed): it loads, it exports
every entry point the header declares, and the host-only LMR map coder
round-trips bit planes."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rdhei.h")


@pytest.fixture(scope="module")
def R():
    from paper_2302_07992_amd import rdhei
    if not os.path.exists(rdhei.LIB_PATH):
        from paper_2302_07992_amd import build
        build.build()
    rdhei.load_library()
    return rdhei


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rdhei_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_function_is_exported(R):
    lib = ctypes.CDLL(R.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(names) == sorted(R.EXPORTS)


def test_strerror_and_version(R):
    lib = R.load_library()
    assert lib.rdhei_strerror(R.ECAPACITY).decode().startswith("message")
    assert b"gfx950" in lib.rdhei_version()


def test_host_argument_errors_need_no_gpu(R):
    lib = R.load_library()
    assert lib.rdhei_ctx_create(None, 0) == R.EINVAL
    assert lib.rdhei_encrypt(None, None, None, 4, 4, 1, 0, None, None) == R.EINVAL
    assert lib.rdhei_plan_run(None, None) == R.EINVAL


def _plane(rng, M, N, kind):
    if kind == "blocks":
        y, x = np.mgrid[0:M, 0:N]
        a = (((y // 7) + (x // 5)) % 3 == 0).astype(np.uint8)
    elif kind == "noise":
        a = (rng.random((M, N)) < 0.3).astype(np.uint8)
    else:
        a = np.zeros((M, N), np.uint8)
    return np.packbits(a.ravel())


@pytest.mark.parametrize("shape", [(1, 1), (3, 5), (16, 16), (37, 101), (256, 256)])
def test_lmr_coder_roundtrip(R, shape):
    M, N = shape
    rng = np.random.default_rng(M * N)
    for ke in ("blocks", "zeros", "noise"):
        for kl in ("noise", "blocks"):
            eta, lb = _plane(rng, M, N, ke), _plane(rng, M, N, kl)
            stream, bits = R.lmr_compress(eta, lb, M, N, 64 + 2 * M * N)
            assert bits == 8 * stream.size
            e2, l2 = R.lmr_decompress(stream, M, N)
            assert np.array_equal(e2, eta) and np.array_equal(l2, lb)


def test_lmr_coder_reports_no_fit(R):
    rng = np.random.default_rng(1)
    M, N = 64, 64
    eta = np.packbits((rng.random(M * N) < 0.5).astype(np.uint8))
    lb = np.packbits((rng.random(M * N) < 0.5).astype(np.uint8))
    with pytest.raises(R.RdheiError) as ei:
        R.lmr_compress(eta, lb, M, N, M * N // 8)
    assert ei.value.code == R.ENOFIT
