"""FP64 CPU oracle of the FAM and SSCA spectral correlation density estimators.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this module. The GPU library never calls it, and the two share no code: this file computes every
quantity from the paper's definitions with numpy complex128 arithmetic. Its only library primitive is the
DFT (``numpy.fft.fft``, an exact factorisation of the DFT sum).

Notation (paper, Sec. II):
  x        complex input, zero outside [0, len(x))
  Np       channel count of the channelizer (N_P)
  d        = Np/2 - 1, the frame centre offset of Eq. (3)
  w[j]     window value multiplying frame sample j (j = 0..Np-1), i.e. a(d - j) of Eq. (3)
  omega_M  = exp(-2*pi*i/M)

Readings of points where the paper is silent or inconsistent (they are listed with reasons in the design
notes): frames are centred as in Eq. (3); the down-conversion factor is exactly Eq. (3)'s
exp(-i 2 pi k p L / Np) with the integer exponent reduced mod Np; g = g_d = 1 with no normalisation; outputs
use natural DFT order in both k and q; FAM returns all P complex bins.
"""
from __future__ import annotations

import numpy as np


def _omega_pow(e, m):
    """omega_m ** e for integer e, with the exponent reduced mod m before the float conversion."""
    e = np.mod(np.asarray(e, dtype=np.int64), m)
    return np.exp(-2j * np.pi * e.astype(np.float64) / m)


# --------------------------------------------------------------------------------------------------------------
# Channelizer: Eq. (3), Sec. II-B "Complex Demodulate".
# --------------------------------------------------------------------------------------------------------------
def channelize(x, Np, L, P, win):
    """X_T[p][k] for p in [0,P), k in [0,Np) following Eq. (3).

    X_T[p][k] = omega_Np^{(k p L) mod Np} * sum_j w[j] x[pL - d + j] omega_Np^{k j}

    The bracket of Eq. (3) is an Np-point DFT of the windowed frame; the trailing factor is the down-conversion.
    """
    x = np.asarray(x, dtype=np.complex128)
    w = np.asarray(win, dtype=np.float64)
    n = len(x)
    d = Np // 2 - 1
    p = np.arange(P, dtype=np.int64)[:, None]
    j = np.arange(Np, dtype=np.int64)[None, :]
    idx = p * L - d + j
    inside = (idx >= 0) & (idx < n)
    frames = np.where(inside, x[np.clip(idx, 0, n - 1)], 0.0)
    Y = np.fft.fft(frames * w[None, :], axis=1)
    k = np.arange(Np, dtype=np.int64)[None, :]
    return Y * _omega_pow(k * p * L, Np)


# --------------------------------------------------------------------------------------------------------------
# SSCA: Eq. (6)-(7), Sec. II-C.
# --------------------------------------------------------------------------------------------------------------
def ssca_demodulate_strip(x, Np, win, k):
    """X_T[n][k] for all n of the SSCA channelizer (L = 1), channel k only.

    Written as an FIR filter with taps w[j] omega_Np^{k j} over the centred frame, followed by the
    down-conversion omega_Np^{(k n) mod Np}. This is Eq. (3) with L = 1, evaluated per channel.
    """
    x = np.asarray(x, dtype=np.complex128)
    w = np.asarray(win, dtype=np.float64)
    n = len(x)
    d = Np // 2 - 1
    j = np.arange(Np)
    h = w * _omega_pow(k * j, Np)
    xp = np.concatenate([np.zeros(d, np.complex128), x, np.zeros(Np - 1 - d, np.complex128)])
    y = np.zeros(n, np.complex128)
    for jj in range(Np):            # y[n] = sum_j h[j] x[n - d + j]
        y += h[jj] * xp[jj:jj + n]
    return y * _omega_pow(k * np.arange(n, dtype=np.int64), Np)


def ssca_strip(x, Np, win, k):
    """Row k of the SSCA estimate: S[k][q] = sum_n X_T[n][k] conj(x[n]) omega_N^{n q}, q in [0, N).

    Eq. (6) gives the channel-data product X_g = X_T * conj(x) (g = 1); Eq. (7) is its N-point DFT. The sum
    runs over n = 0..N-1 (natural DFT order), the indexing the paper's 2-D decomposition uses.
    """
    x = np.asarray(x, dtype=np.complex128)
    xg = ssca_demodulate_strip(x, Np, win, k) * np.conj(x)
    return np.fft.fft(xg)


def ssca(x, Np, win):
    """Full SSCA estimate S[k][q], shape [Np][N], complex128."""
    x = np.asarray(x, dtype=np.complex128)
    return np.stack([ssca_strip(x, Np, win, k) for k in range(Np)])


def ssca_block(x, offset, N, Np, win):
    """SSCA of the block n in [offset, offset + N) of a longer signal x (a stream of blocks): the channelizer
    of Eq. (3) runs on the whole signal, so frames at the block edges see the true neighbouring samples (zero
    only outside x), and the sum of Eq. (7) runs over the block:
    S[k][q] = sum_{n<N} X_T[offset + n][k] conj(x[offset + n]) omega_N^{n q}. Blocks start at multiples of Np,
    where Eq. (3)'s down-conversion factor omega_Np^{(k n) mod Np} is the same counted from the block's start."""
    x = np.asarray(x, dtype=np.complex128)
    out = np.empty((Np, N), np.complex128)
    xb = x[offset:offset + N]
    for k in range(Np):
        xt = ssca_demodulate_strip(x, Np, win, k)[offset:offset + N]
        out[k] = np.fft.fft(xt * np.conj(xb))
    return out


def ssca_cross_strip(x, y, Np, win, k, conjugate=False):
    """Row k of the cross SCD of x and y (Eq. (2) with a second input y, Sec. II-A) by SSCA: the demodulate of
    y has a one-sample window, so the channel-data product of Eq. (6) takes conj(y[n]) in place of conj(x[n]):
    S_xy[k][q] = sum_n X_T[n][k] conj(y[n]) omega_N^{n q}. With conjugate=True the product takes y[n] itself
    (the conjugate SCD, a library form: the paper treats the conjugated product only)."""
    x = np.asarray(x, dtype=np.complex128)
    y = np.asarray(y, dtype=np.complex128)
    xg = ssca_demodulate_strip(x, Np, win, k) * (y if conjugate else np.conj(y))
    return np.fft.fft(xg)


def ssca_cross(x, y, Np, win, conjugate=False):
    """Full cross (or conjugate) SSCA estimate, shape [Np][N], complex128; see ``ssca_cross_strip``."""
    return np.stack([ssca_cross_strip(x, y, Np, win, k, conjugate) for k in range(Np)])


def ssca_2dfft(x, Np, win, M1):
    """The paper's SSCA_2DFFT (Sec. III-B, Eq. (10)-(16)): same result as ``ssca`` via a decomposed DFT.

    X_g is reshaped to X_g^{2D}(m1, m2, k) = X_g(m1*M2 + m2, k); Stage 1 takes M1-point DFTs over m1 and
    multiplies by the rotation factor exp(-j 2 pi m2 m1' / N); Stage 2 takes M2-point DFTs over m2. The
    result S^{2D}(m1', m2', k) sits at output bin q = m1' + M1*m2'.
    """
    x = np.asarray(x, dtype=np.complex128)
    N = len(x)
    M2 = N // M1
    assert M1 * M2 == N
    xt = channelize(x, Np, 1, N, win)                       # [n][k]
    xg = xt * np.conj(x)[:, None]
    xg2 = xg.reshape(M1, M2, Np)                           # (m1, m2, k)
    s1 = np.fft.fft(xg2, axis=0)                           # (m1', m2, k)
    m1p = np.arange(M1, dtype=np.int64)[:, None, None]
    m2 = np.arange(M2, dtype=np.int64)[None, :, None]
    s1 = s1 * _omega_pow(m1p * m2, N)
    s2 = np.fft.fft(s1, axis=1)                            # (m1', m2', k)
    out = np.empty((Np, N), np.complex128)
    q = (np.arange(M1)[:, None] + M1 * np.arange(M2)[None, :]).reshape(-1)
    out[:, q] = s2.reshape(M1 * M2, Np).T
    return out


def ssca_coords(Np, N):
    """(f, alpha) of each SSCA cell [k][q] with f_s = 1: alpha = f_k + q_c/N, f = (f_k - q_c/N)/2.

    f_k = k_c/Np uses the signed (wrapped) channel index, q_c the signed bin index (Sec. II-C and the
    coordinate map at the end of Sec. III-B, read with signed k and q).
    """
    k = np.arange(Np)
    kc = ((k + Np // 2) % Np) - Np // 2
    q = np.arange(N)
    qc = ((q + N // 2) % N) - N // 2
    fk = (kc / Np)[:, None]
    a = fk + (qc / N)[None, :]
    f = (fk - (qc / N)[None, :]) / 2.0
    return f, a


# --------------------------------------------------------------------------------------------------------------
# FAM: Eq. (4)-(5), Sec. II-B.
# --------------------------------------------------------------------------------------------------------------
def fam(x, Np, L, P, win):
    """FAM estimate S[k][l][q] = sum_p X_T[p][k] conj(X_T[p][l]) omega_P^{p q}, shape [Np][Np][P].

    The input length is N = P*L (samples beyond it are ignored; frames reaching past it see zeros). The
    conjugate products of Eq. (5) are formed for all Np^2 channel pairs and each is followed by a P-point DFT
    (g_d = 1).
    """
    x = np.asarray(x, dtype=np.complex128)[: P * L]
    xt = channelize(x, Np, L, P, win)                       # [p][k]
    z = xt[:, :, None] * np.conj(xt)[:, None, :]           # [p][k][l]
    s = np.fft.fft(z, axis=0)                              # [q][k][l]
    return np.ascontiguousarray(s.transpose(1, 2, 0))


def fam_cross(x, y, Np, L, P, win, conjugate=False):
    """Cross FAM of x and y (Eq. (2) and (5) with a second input): S_xy[k][l][q] =
    sum_p X_T[p][k] conj(Y_T[p][l]) omega_P^{p q}, Y_T the Eq. (3) channelizer output of y. With
    conjugate=True the product takes Y_T[p][l] itself (the conjugate SCD, a library form)."""
    x = np.asarray(x, dtype=np.complex128)[: P * L]
    y = np.asarray(y, dtype=np.complex128)[: P * L]
    xt = channelize(x, Np, L, P, win)
    yt = channelize(y, Np, L, P, win)
    z = xt[:, :, None] * (yt if conjugate else np.conj(yt))[:, None, :]
    s = np.fft.fft(z, axis=0)
    return np.ascontiguousarray(s.transpose(1, 2, 0))


def fam_coords(Np, L, P):
    """(f, alpha) of each FAM cell [k][l][q]: f = (f_k + f_l)/2, alpha = f_k - f_l + q_c/(P L)."""
    k = np.arange(Np)
    kc = ((k + Np // 2) % Np) - Np // 2
    fk = kc / Np
    q = np.arange(P)
    qc = ((q + P // 2) % P) - P // 2
    f = (fk[:, None, None] + fk[None, :, None]) / 2.0 + 0.0 * qc[None, None, :]
    a = fk[:, None, None] - fk[None, :, None] + (qc / (P * L))[None, None, :]
    return f, a


def fam_paper_view(S):
    """|S|^2 over the central half of the q axis (-P/4 <= q_c < P/4), in natural order [0..P/4-1, -P/4..-1]."""
    P = S.shape[-1]
    keep = np.concatenate([np.arange(0, P // 4), np.arange(P - P // 4, P)])
    return np.abs(S[..., keep]) ** 2
