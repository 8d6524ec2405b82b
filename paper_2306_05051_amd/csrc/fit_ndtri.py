"""Fits the FP32 inverse normal CDF used by the HIP kernels.

Structure after M. Giles, "Approximating the erfinv function" (GPU Computing
Gems, 2011): with x = 2q - 1 and w = -log((1-x)(1+x)),
    erfinv(x) = x * P1(w - 2.5)          for w < 5
    erfinv(x) = x * P2(sqrt(w) - 3)      otherwise,
and Phi^-1(q) = sqrt(2) erfinv(2q - 1).  The coefficients are fitted here
(weighted least squares on the relative error, FP64, against
scipy.special.erfinv) rather than taken from the paper, and the printed
table is pasted into glint_device.hpp.  The script also reports the FP32
error over every uniform the method can draw, q = (2k+1) 2^-24.

Run:  python paper_2306_05051_amd/csrc/fit_ndtri.py
"""
import numpy as np
from scipy.special import erfinv

DEG = 8


def fit(lo, hi, transform, n=20000):
    # Chebyshev nodes in the fitted variable
    t = np.cos(np.pi * (np.arange(n) + 0.5) / n)
    v = 0.5 * (lo + hi) + 0.5 * (hi - lo) * t
    x = transform(v)
    y = erfinv(x) / x
    V = np.vander(v, DEG + 1)
    c, *_ = np.linalg.lstsq(V / y[:, None], np.ones_like(y), rcond=None)
    return c


def w_of_x(x):
    return -np.log((1 - x) * (1 + x))


def x_of_w(w):
    return np.sqrt(-np.expm1(-w))


def main():
    c1 = fit(-2.5, 2.5, lambda s: x_of_w(s + 2.5))
    wmax = w_of_x(1 - 2.0**-23)
    c2 = fit(np.sqrt(5.0) - 3.0, np.sqrt(wmax + 0.5) - 3.0, lambda s: x_of_w((s + 3.0) ** 2))
    f1 = c1.astype(np.float32)
    f2 = c2.astype(np.float32)
    # FP32 evaluation over every q = (2k+1) 2^-24 (fma-free Horner: an upper bound)
    k = np.arange(2**23, dtype=np.int64)
    q = ((2 * k + 1).astype(np.float64) * 2.0**-24)
    x = (2.0 * q - 1.0).astype(np.float32)
    w = -np.log(((np.float32(1) - x) * (np.float32(1) + x)).astype(np.float32)).astype(np.float32)
    central = w < np.float32(5.0)
    s1 = (w - np.float32(2.5)).astype(np.float32)
    s2 = (np.sqrt(w).astype(np.float32) - np.float32(3.0)).astype(np.float32)
    p = np.where(central, f1[0], f2[0]).astype(np.float32)
    for i in range(1, DEG + 1):
        p = (np.where(central, s1, s2) * p + np.where(central, f1[i], f2[i])).astype(np.float32)
    z = (np.float32(np.sqrt(2.0)) * p * x).astype(np.float32).astype(np.float64)
    from scipy.special import ndtri
    ref = ndtri(q)
    rel = np.abs(z - ref) / np.maximum(np.abs(ref), 1e-30)
    absd = np.abs(z - ref)
    print("max rel err", rel.max(), "at q", q[rel.argmax()], " max abs err", absd.max())
    print("central:")
    print(",\n".join(f"    {v:.9e}f" for v in f1))
    print("tail:")
    print(",\n".join(f"    {v:.9e}f" for v in f2))


if __name__ == "__main__":
    main()
