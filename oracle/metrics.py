"""Image quality and security metrics of arXiv 2302.07992, Sec. IV
(test infrastructure only, like the rest of this package).

Plain numpy in float64, one function per metric, each written from its
definition:

* Shannon entropy and chi-square test of one image: Sec. IV-B, entropy and
  chi-square equations (256 grey levels, P = level count / pixel count).
* NPCR and UACI between an original image and another one: Sec. IV-B, NPCR
  and UACI equations.  The printed indicator of the NPCR sum is 1 where the
  two pixels are equal; the metric's name ("changing pixel rate"), the cited
  source and the table's values near 99.6 % for an image against its
  encryption all say it counts pixels that differ, which is what this does.
* PSNR between two 8-bit images (Sec. IV, the similarity measure of Table
  EMR_results and Table analysis): 10 log10(255^2 / MSE), infinite when equal.
* SSIM (Sec. IV; the paper does not say which variant): mean structural
  similarity with a 7x7 uniform window, sample (co)variances (49/48),
  K1 = 0.01, K2 = 0.03, L = 255, over every window that lies inside the image;
  NaN for images smaller than the window.
"""
from __future__ import annotations

import numpy as np

SSIM_WIN = 7
SSIM_K1, SSIM_K2, SSIM_L = 0.01, 0.03, 255.0


def _u8(a) -> np.ndarray:
    a = np.asarray(a)
    assert a.dtype == np.uint8 and a.ndim == 2
    return a


def histogram(I) -> np.ndarray:
    """Count of each grey level 0..255."""
    return np.bincount(_u8(I).ravel(), minlength=256).astype(np.int64)


def entropy(I) -> float:
    """Shannon entropy in bits: -sum P log2 P over the levels that occur."""
    I = _u8(I)
    P = histogram(I) / float(I.size)
    nz = P[P > 0]
    return float(-np.sum(nz * np.log2(nz)))


def chi2(I) -> float:
    """Chi-square test as printed: 256 (h w) sum_i (P_i - 1/256)^2."""
    I = _u8(I)
    P = histogram(I) / float(I.size)
    return float(256.0 * I.size * np.sum((P - 1.0 / 256.0) ** 2))


def npcr(I, J) -> float:
    """Percentage of pixel positions where the two images differ."""
    I, J = _u8(I), _u8(J)
    assert I.shape == J.shape
    return float(100.0 * np.count_nonzero(I != J) / I.size)


def uaci(I, J) -> float:
    """Mean absolute difference as a percentage of 255."""
    I, J = _u8(I), _u8(J)
    assert I.shape == J.shape
    d = np.abs(I.astype(np.int64) - J.astype(np.int64))
    return float(100.0 * d.sum() / (255.0 * I.size))


def psnr(I, J) -> float:
    """10 log10(255^2 / MSE); infinite for identical images."""
    I, J = _u8(I), _u8(J)
    assert I.shape == J.shape
    d = I.astype(np.int64) - J.astype(np.int64)
    sq = int((d * d).sum())
    if sq == 0:
        return float("inf")
    return float(10.0 * np.log10(255.0 * 255.0 / (sq / float(I.size))))


def _window_sums(X: np.ndarray, w: int) -> np.ndarray:
    """Sum of X over every w x w window inside the image (top-left anchored)."""
    c = np.cumsum(np.cumsum(np.pad(X, ((1, 0), (1, 0))), axis=0), axis=1)
    return c[w:, w:] - c[:-w, w:] - c[w:, :-w] + c[:-w, :-w]


def ssim(I, J) -> float:
    """Mean SSIM over the windows inside the image (see the module note)."""
    I, J = _u8(I), _u8(J)
    assert I.shape == J.shape
    M, N = I.shape
    w = SSIM_WIN
    if M < w or N < w:
        return float("nan")
    a, b = I.astype(np.int64), J.astype(np.int64)
    n = float(w * w)
    sa, sb = _window_sums(a, w), _window_sums(b, w)
    saa, sbb, sab = _window_sums(a * a, w), _window_sums(b * b, w), _window_sums(a * b, w)
    ua, ub = sa / n, sb / n
    cov = n / (n - 1.0)
    va = cov * (saa / n - ua * ua)
    vb = cov * (sbb / n - ub * ub)
    vab = cov * (sab / n - ua * ub)
    C1, C2 = (SSIM_K1 * SSIM_L) ** 2, (SSIM_K2 * SSIM_L) ** 2
    S = ((2.0 * ua * ub + C1) * (2.0 * vab + C2)) / ((ua * ua + ub * ub + C1) * (va + vb + C2))
    return float(S.mean())


def image_metrics(I, J=None, with_ssim: bool = True) -> np.ndarray:
    """The eight per-pair values in the library's order: entropy and
    chi-square of I, of J, NPCR, UACI, PSNR and SSIM of (I, J); NaN where J is
    absent (or SSIM not asked for)."""
    nan = float("nan")
    out = [entropy(I), chi2(I), nan, nan, nan, nan, nan, nan]
    if J is not None:
        out[2:7] = [entropy(J), chi2(J), npcr(I, J), uaci(I, J), psnr(I, J)]
        if with_ssim:
            out[7] = ssim(I, J)
    return np.array(out, dtype=np.float64)


__all__ = ["histogram", "entropy", "chi2", "npcr", "uaci", "psnr", "ssim", "image_metrics",
           "SSIM_WIN", "SSIM_K1", "SSIM_K2", "SSIM_L"]
