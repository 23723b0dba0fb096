"""Radial basis and polynomial envelope (oracle).

Bessel basis (n = 1..n_b):
    B_n(d) = sqrt(2/r_c) * sin(n*pi*d/r_c) / d
Polynomial envelope of order p (x = d/r_c):
    f(x) = 1 - (p+1)(p+2)/2 x^p + p(p+2) x^(p+1) - p(p+1)/2 x^(p+2)
         (p = 6: 1 - 28 x^6 + 48 x^7 - 21 x^8), so f(1) = f'(1) = f''(1) = 0.
Edge features: e_n(d) = f(d) * B_n(d).
"""
from __future__ import annotations

import numpy as np


def bessel_basis(d: np.ndarray, r_cut: float, n_basis: int):
    """B [E, n_b] and dB/dd [E, n_b]."""
    d = np.asarray(d, dtype=np.float64)[:, None]
    k = np.arange(1, n_basis + 1, dtype=np.float64)[None, :] * np.pi / r_cut
    pref = np.sqrt(2.0 / r_cut)
    s, c = np.sin(k * d), np.cos(k * d)
    B = pref * s / d
    dB = pref * (k * d * c - s) / (d * d)
    return B, dB


def envelope(d: np.ndarray, r_cut: float, p: int):
    """f and df/dd; f = 0 for d >= r_cut."""
    x = np.asarray(d, dtype=np.float64) / r_cut
    a = (p + 1) * (p + 2) / 2.0
    b = p * (p + 2.0)
    c = p * (p + 1) / 2.0
    f = 1.0 - a * x ** p + b * x ** (p + 1) - c * x ** (p + 2)
    df = (-a * p * x ** (p - 1) + b * (p + 1) * x ** p - c * (p + 2) * x ** (p + 1)) / r_cut
    inside = x < 1.0
    return np.where(inside, f, 0.0), np.where(inside, df, 0.0)


def radial_features(d: np.ndarray, r_cut: float, n_basis: int, p: int):
    """e = f*B [E, n_b] and de/dd [E, n_b]."""
    B, dB = bessel_basis(d, r_cut, n_basis)
    f, df = envelope(d, r_cut, p)
    return f[:, None] * B, df[:, None] * B + f[:, None] * dB
