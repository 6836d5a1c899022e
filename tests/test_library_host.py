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


def test_header_constants_match_the_binding(R):
    """Every integer #define RDHEI_<NAME> of the header that the binding also
    names (as <NAME>) has the same value there: options, keystream families,
    methods, ops, status codes, metric layout."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    defs = dict(re.findall(r"#define\s+RDHEI_([A-Z0-9_]+)\s+\(?(-?\d+)\)?\s*$", text, flags=re.M))
    checked = 0
    for name, value in defs.items():
        if hasattr(R, name):
            assert getattr(R, name) == int(value), name
            checked += 1
    for name in ("OPT_KEYSTREAM", "KEYSTREAM_PHILOX", "KEYSTREAM_CHACHA20", "OPT_LMR_MIN_LEVEL", "METRIC_COUNT"):
        assert name in defs and hasattr(R, name), name
    assert checked >= 10


def test_strerror_and_version(R):
    lib = R.load_library()
    assert lib.rdhei_strerror(R.ECAPACITY).decode().startswith("message")
    assert b"gfx950" in lib.rdhei_version()


def test_host_argument_errors_need_no_gpu(R):
    lib = R.load_library()
    assert lib.rdhei_ctx_create(None, 0) == R.EINVAL
    assert lib.rdhei_encrypt(None, None, None, 4, 4, 1, 0, 0, None, None) == R.EINVAL
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


def test_library_coder_matches_oracle_coder(R):
    """The library's host map coder and the oracle's independent coder emit
    identical streams for the same bit planes (both follow one coder
    definition), and each decodes the other's stream."""
    import oracle as O
    from paper_2302_07992_amd import inputs
    rng = np.random.default_rng(4)
    cases = []
    for (M, N) in [(16, 16), (37, 101), (128, 128)]:
        y, x = np.mgrid[0:M, 0:N]
        cases.append((M, N, (((y // 7) + (x // 5)) % 3 == 0).astype(np.uint8),
                      (rng.random((M, N)) < 0.25).astype(np.uint8)))
    I = inputs.make_image_np(2, 256, 256, 8, 1.0)
    l_rot, eta_rot = O.lmr_rotated_maps(I, 5, 4, 11)
    cases.append((256, 256, eta_rot, l_rot))
    for M, N, eta, l in cases:
        want = O.lmr_compress(eta, l, 64 + M * N)
        got, bits = R.lmr_compress(np.packbits(eta.ravel()), np.packbits(l.ravel()), M, N, 64 + M * N)
        assert bits == 8 * got.size
        assert np.array_equal(got, want)
        e2, l2 = R.lmr_decompress(want, M, N)
        assert np.array_equal(np.unpackbits(e2)[:M * N], eta.ravel())
        assert np.array_equal(np.unpackbits(l2)[:M * N], l.ravel())
