"""Brute-force evaluations of the paper's defining sums, for pinning the oracle on tiny inputs.

TEST INFRASTRUCTURE ONLY (same import rule as ``scd_oracle``). Everything here is pure-Python loops over
Python complex numbers, with no numpy FFT, so that a mistake in the vectorised oracle (a sign, a shifted
frame, a transposed index) shows up as a disagreement with these direct sums.
"""
from __future__ import annotations

import cmath
import math


def demodulate_eq1(x, n, f, win):
    """Complex demodulate of Eq. (1) at time n and (continuous) frequency f.

    X_T(n, f) = sum_r a(r) x(n - r) exp(-i 2 pi f (n - r)), with the length-Np window a(r) supported on
    r in [-Np/2, Np/2 - 1] and a(d - j) = win[j], d = Np/2 - 1. Samples outside [0, len(x)) are zero.
    """
    Np = len(win)
    d = Np // 2 - 1
    acc = 0j
    for j in range(Np):
        r = d - j
        m = n - r
        if 0 <= m < len(x):
            acc += win[j] * x[m] * cmath.exp(-2j * math.pi * f * m)
    return acc


def scd_eq2(demod_x, demod_y, times):
    """Eq. (2) with g = 1 over the given times: sum_r X(r) conj(Y(r))."""
    return sum(demod_x(r) * demod_y(r).conjugate() for r in times)


def ssca_cell_eq2(x, win, k, q):
    """SSCA cell [k][q] from Eq. (1)-(2) directly.

    The SSCA correlates the demodulate at f1 = f_k (window win) with a one-sample-window demodulate of x at
    f2 = -q/N, i.e. x(r) exp(-i 2 pi f2 r). With f1 = f + alpha/2 and f2 = f - alpha/2 this is the cell
    alpha = f_k + q/N, f = (f_k - q/N)/2. Eq. (3)'s down-conversion drops a constant exp(+i 2 pi k d / Np)
    that Eq. (1) carries, so the Eq. (3) estimate equals exp(-i 2 pi k d / Np) times the Eq. (2) sum.
    """
    N = len(x)
    Np = len(win)
    d = Np // 2 - 1
    fk = k / Np
    f2 = -q / N
    acc = 0j
    for n in range(N):
        a = demodulate_eq1(x, n, fk, win)
        b = x[n] * cmath.exp(-2j * math.pi * f2 * n)
        acc += a * b.conjugate()
    return cmath.exp(-2j * math.pi * k * d / Np) * acc


def ssca_cross_cell_eq2(x, y, win, k, q, conjugate=False):
    """Cross SSCA cell [k][q] from Eq. (1)-(2) with two inputs: the demodulate of x at f_k (window win)
    times the conjugate of y's one-sample demodulate y(r) exp(+i 2 pi q r / N) (Eq. (2)'s Y*). The
    conjugate form multiplies by that demodulate itself, taken at the mirrored frequency: y(r) exp(-i 2 pi q r / N).
    The constant exp(-i 2 pi k d / Np) relates Eq. (1) to Eq. (3) as in ``ssca_cell_eq2``."""
    N = len(x)
    Np = len(win)
    d = Np // 2 - 1
    acc = 0j
    for n in range(N):
        a = demodulate_eq1(x, n, k / Np, win)
        if conjugate:
            acc += a * y[n] * cmath.exp(-2j * math.pi * q * n / N)
        else:
            acc += a * (y[n] * cmath.exp(2j * math.pi * q * n / N)).conjugate()
    return cmath.exp(-2j * math.pi * k * d / Np) * acc


def fam_cell_eq15(x, win, L, P, k, l, q):
    """FAM cell [k][l][q] from Eq. (1) demodulates sampled at times pL and the P-point sum of Eq. (5).

    S = sum_p X_T(pL, f_k) conj(X_T(pL, f_l)) exp(-i 2 pi p q / P), with Eq. (1) demodulates; the Eq. (3)
    form differs by the constant exp(-i 2 pi (k - l) d / Np) (see ``ssca_cell_eq2``). The input is cut to
    N = P*L samples.
    """
    xs = list(x[: P * L])
    Np = len(win)
    d = Np // 2 - 1
    acc = 0j
    for p in range(P):
        a = demodulate_eq1(xs, p * L, k / Np, win)
        b = demodulate_eq1(xs, p * L, l / Np, win)
        acc += a * b.conjugate() * cmath.exp(-2j * math.pi * p * q / P)
    return cmath.exp(-2j * math.pi * (k - l) * d / Np) * acc


def fam_cross_cell_eq15(x, y, win, L, P, k, l, q, conjugate=False):
    """Cross FAM cell [k][l][q]: Eq. (1) demodulates of x at f_k and of y at f_l, sampled at pL, their
    Eq. (2) product (y's conjugated, or not in the conjugate form) and the P-point sum of Eq. (5). The Eq. (3)
    form differs by exp(-i 2 pi (k - l) d / Np), or exp(-i 2 pi (k + l) d / Np) in the conjugate form."""
    xs, ys = list(x[: P * L]), list(y[: P * L])
    Np = len(win)
    d = Np // 2 - 1
    acc = 0j
    for p in range(P):
        a = demodulate_eq1(xs, p * L, k / Np, win)
        b = demodulate_eq1(ys, p * L, l / Np, win)
        acc += a * (b if conjugate else b.conjugate()) * cmath.exp(-2j * math.pi * p * q / P)
    return cmath.exp(-2j * math.pi * (k + l if conjugate else k - l) * d / Np) * acc


def channelize_direct(x, Np, L, P, win):
    """Eq. (3) written as a double loop (no FFT): X_T[p][k]."""
    d = Np // 2 - 1
    out = [[0j] * Np for _ in range(P)]
    for p in range(P):
        for k in range(Np):
            acc = 0j
            for j in range(Np):
                m = p * L - d + j
                if 0 <= m < len(x):
                    acc += win[j] * x[m] * cmath.exp(-2j * math.pi * k * j / Np)
            out[p][k] = acc * cmath.exp(-2j * math.pi * ((k * p * L) % Np) / Np)
    return out


def correlogram_psd(x, win, k):
    """Blackman-Tukey estimate at f_k with lag window win[tau + d]:

    sum_tau win[tau + d] R(tau) exp(-i 2 pi f_k tau), R(tau) = sum_n x[n + tau] conj(x[n]) (zero-padded),
    tau in [-d, Np - 1 - d]. The SSCA alpha = 0 cell of strip k equals exp(-i 2 pi k d / Np) times this.
    """
    Np = len(win)
    d = Np // 2 - 1
    N = len(x)
    acc = 0j
    for tau in range(-d, Np - d):
        r = 0j
        for n in range(N):
            if 0 <= n + tau < N:
                r += x[n + tau] * x[n].conjugate()
        acc += win[tau + d] * r * cmath.exp(-2j * math.pi * k * tau / Np)
    return cmath.exp(-2j * math.pi * k * d / Np) * acc


def dft_direct(v):
    """Plain O(n^2) DFT sum_n v[n] exp(-i 2 pi n q / len(v))."""
    n = len(v)
    return [sum(v[m] * cmath.exp(-2j * math.pi * m * q / n) for m in range(n)) for q in range(n)]
