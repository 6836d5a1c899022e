"""Pins of the metric oracle (Sec. IV metrics) against closed forms, library
routines and brute force, independent of the oracle's own vectorised code."""
import math

import numpy as np
import pytest

from oracle import metrics as OM


def _rng(seed):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- entropy, chi-square
def test_entropy_and_chi2_closed_forms():
    """Entropy equation: every level equally often -> 8 bits; one level -> 0;
    two levels half and half -> 1.  Chi-square equation: 256 MN sum (P -
    1/256)^2 is 0 for the flat histogram, 255 MN for one level and 127 MN for
    two equal halves (2 (127/256)^2 + 254/256^2 = 127/256)."""
    flat = np.arange(256 * 64, dtype=np.int64).reshape(64, 256).astype(np.uint8)
    assert OM.entropy(flat) == 8.0
    assert OM.chi2(flat) == 0.0
    const = np.full((37, 53), 200, np.uint8)
    assert OM.entropy(const) == 0.0
    assert OM.chi2(const) == pytest.approx(255 * 37 * 53, rel=1e-12)
    half = np.zeros((40, 50), np.uint8)
    half[:, 25:] = 9
    assert OM.entropy(half) == pytest.approx(1.0, abs=1e-15)
    assert OM.chi2(half) == pytest.approx(127 * 40 * 50, rel=1e-12)


def test_entropy_matches_library_routine():
    """Entropy equation against scipy.stats.entropy of the level counts."""
    from scipy.stats import entropy as sp_entropy
    I = _rng(1).integers(0, 256, (97, 61)).astype(np.uint8)
    I[:30] //= 7                                     # a skewed histogram
    counts = np.bincount(I.ravel(), minlength=256)
    assert OM.entropy(I) == pytest.approx(sp_entropy(counts, base=2), rel=1e-13)


def test_chi2_equals_pearson_statistic():
    """The printed chi-square equals Pearson's statistic against the uniform
    expectation MN/256 (scipy.stats.chisquare)."""
    from scipy.stats import chisquare
    I = _rng(2).integers(0, 256, (128, 96)).astype(np.uint8)
    I[:, :20] = 17
    counts = np.bincount(I.ravel(), minlength=256)
    assert OM.chi2(I) == pytest.approx(chisquare(counts).statistic, rel=1e-12)


# ---------------------------------------------------------------- NPCR, UACI, PSNR
def test_npcr_uaci_closed_forms():
    """NPCR/UACI equations: an image against itself 0 / 0; all-0 against
    all-255 100 / 100; one changed pixel of 10,000 -> 0.01 %; against its
    complement UACI = mean |2 I - 255| / 255."""
    I = _rng(3).integers(0, 256, (100, 100)).astype(np.uint8)
    assert OM.npcr(I, I) == 0.0 and OM.uaci(I, I) == 0.0
    z, f = np.zeros((20, 30), np.uint8), np.full((20, 30), 255, np.uint8)
    assert OM.npcr(z, f) == 100.0 and OM.uaci(z, f) == 100.0
    J = I.copy()
    J[50, 50] ^= 1
    assert OM.npcr(I, J) == pytest.approx(0.01, abs=1e-15)
    C = (255 - I).astype(np.uint8)
    expect = 100.0 * sum(abs(2 * int(v) - 255) for v in I.ravel()) / (255.0 * I.size)
    assert OM.uaci(I, C) == pytest.approx(expect, rel=1e-14)


def test_psnr_closed_forms():
    """PSNR: identical -> infinite; off by one everywhere -> 20 log10 255;
    0 against 255 -> 0 dB; one pixel off by 16 in 64x64 -> 10 log10(255^2
    4096 / 256)."""
    I = _rng(4).integers(0, 255, (64, 64)).astype(np.uint8)
    assert math.isinf(OM.psnr(I, I))
    assert OM.psnr(I, I + 1) == pytest.approx(20 * math.log10(255), rel=1e-14)
    assert OM.psnr(np.zeros((8, 8), np.uint8), np.full((8, 8), 255, np.uint8)) == 0.0
    J = I.copy()
    J[3, 3] = (int(J[3, 3]) + 16) % 256 if J[3, 3] < 240 else J[3, 3] - 16
    assert OM.psnr(I, J) == pytest.approx(10 * math.log10(255.0 ** 2 * 4096 / 256), rel=1e-14)


# ---------------------------------------------------------------- SSIM
def test_ssim_identity_and_symmetry():
    """SSIM of an image with itself is exactly 1; SSIM is symmetric."""
    I = _rng(5).integers(0, 256, (33, 41)).astype(np.uint8)
    J = _rng(6).integers(0, 256, (33, 41)).astype(np.uint8)
    assert OM.ssim(I, I) == 1.0
    assert OM.ssim(I, J) == pytest.approx(OM.ssim(J, I), rel=1e-15)


def test_ssim_constant_images_closed_form():
    """Two flat images have no variance, so only the luminance term is left:
    (2 c1 c2 + C1) / (c1^2 + c2^2 + C1), C1 = (0.01 * 255)^2."""
    C1 = (0.01 * 255) ** 2
    for c1, c2 in [(0, 0), (10, 200), (128, 127), (255, 0)]:
        a, b = np.full((9, 12), c1, np.uint8), np.full((9, 12), c2, np.uint8)
        expect = (2 * c1 * c2 + C1) / (c1 * c1 + c2 * c2 + C1)
        assert OM.ssim(a, b) == pytest.approx(expect, rel=1e-14)


def test_ssim_single_window_sample_statistics():
    """A 7x7 image is one window: the (co)variances are the sample ones
    (numpy's ddof=1), the means numpy's."""
    a = _rng(7).integers(0, 256, (7, 7)).astype(np.uint8)
    b = _rng(8).integers(0, 256, (7, 7)).astype(np.uint8)
    x, y = a.astype(np.float64).ravel(), b.astype(np.float64).ravel()
    C1, C2 = (0.01 * 255) ** 2, (0.03 * 255) ** 2
    cxy = np.cov(x, y, ddof=1)
    expect = ((2 * x.mean() * y.mean() + C1) * (2 * cxy[0, 1] + C2)) / (
        (x.mean() ** 2 + y.mean() ** 2 + C1) * (cxy[0, 0] + cxy[1, 1] + C2))
    assert OM.ssim(a, b) == pytest.approx(expect, rel=1e-12)


def test_ssim_windows_brute_force():
    """Every 7x7 window inside the image, enumerated one by one and scored
    with numpy's mean and ddof=1 covariance, then averaged."""
    a = _rng(9).integers(0, 256, (11, 14)).astype(np.uint8)
    b = np.clip(a.astype(np.int64) + _rng(10).integers(-20, 21, a.shape), 0, 255).astype(np.uint8)
    C1, C2 = (0.01 * 255) ** 2, (0.03 * 255) ** 2
    vals = []
    for r in range(a.shape[0] - 6):
        for c in range(a.shape[1] - 6):
            x = a[r:r + 7, c:c + 7].astype(np.float64).ravel()
            y = b[r:r + 7, c:c + 7].astype(np.float64).ravel()
            k = np.cov(x, y, ddof=1)
            vals.append(((2 * x.mean() * y.mean() + C1) * (2 * k[0, 1] + C2))
                        / ((x.mean() ** 2 + y.mean() ** 2 + C1) * (k[0, 0] + k[1, 1] + C2)))
    assert len(vals) == 5 * 8
    assert OM.ssim(a, b) == pytest.approx(float(np.mean(vals)), rel=1e-12)


def test_ssim_undefined_below_window():
    assert math.isnan(OM.ssim(np.zeros((6, 50), np.uint8), np.zeros((6, 50), np.uint8)))
    assert math.isnan(OM.ssim(np.zeros((50, 6), np.uint8), np.zeros((50, 6), np.uint8)))
