"""Seeded synthetic signal generators.

This module only draws test signals. It holds none of the estimator's arithmetic, so both the FP64 oracle
tests and the GPU path may consume its outputs without sharing any code with each other.

All generators return complex128 numpy arrays; callers cast to complex64 for the GPU path. Randomness comes
from ``numpy.random.Generator(PCG64(seed))``.

Recipes (the paper fixes only the DSSS BPSK test signal of its accuracy experiment; the rest are this
library's choices):

* rectangular pulses with an integer number of samples per symbol, random symbol timing and carrier phase;
* BPSK and AM use a real carrier ``cos(2*pi*fc*n + theta)``; QPSK, 16-QAM and MSK use a complex carrier;
* QPSK symbols are (+-1 +- 1j)/sqrt(2); 16-QAM symbols are {+-1, +-3}^2 / sqrt(10);
* MSK is continuous-phase FSK with modulation index 1/2;
* AM is (1 + 0.5 m[n]) cos(2*pi*fc*n + theta) with m a smoothed, unit-RMS Gaussian message;
* SNR is E|s|^2 / E|w|^2 over the full band, with circular complex white Gaussian noise w.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 250618003

MODULATIONS = ("bpsk", "qpsk", "qam16", "msk", "am", "noise")


def rng_for(config: int, index: int) -> np.random.Generator:
    """Generator for signal ``index`` of workload ``config`` (seed = 250618003 + 1000*config + index)."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + 1000 * config + index))


def rng_keyed(*keys: int) -> np.random.Generator:
    """Generator for an arbitrary tuple of integer keys (no overlap between different tuples)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, *keys])))


def _symbols_to_samples(sym: np.ndarray, sps: int, n: int, rng: np.random.Generator) -> np.ndarray:
    """Rectangular pulse shaping with a random timing offset in [0, sps)."""
    off = int(rng.integers(0, sps))
    idx = (np.arange(n) + off) // sps
    return sym[idx]


def _n_symbols(n: int, sps: int) -> int:
    return n // sps + 2


def add_noise(s: np.ndarray, snr_db: float, rng: np.random.Generator) -> np.ndarray:
    """Add circular complex white Gaussian noise at the given SNR (E|s|^2 / E|w|^2, full band)."""
    ps = float(np.mean(np.abs(s) ** 2))
    if ps == 0.0:
        ps = 1.0
    var = ps * 10.0 ** (-snr_db / 10.0)
    w = rng.standard_normal(len(s)) + 1j * rng.standard_normal(len(s))
    return s + w * np.sqrt(var / 2.0)


def bpsk(n, fc, sps, snr_db, rng, real_carrier=True):
    b = rng.choice(np.array([-1.0, 1.0]), size=_n_symbols(n, sps))
    base = _symbols_to_samples(b, sps, n, rng)
    theta = rng.uniform(0.0, 2.0 * np.pi)
    t = np.arange(n)
    if real_carrier:
        s = base * np.cos(2.0 * np.pi * fc * t + theta)
    else:
        s = base * np.exp(1j * (2.0 * np.pi * fc * t + theta))
    return add_noise(s.astype(np.complex128), snr_db, rng)


def qpsk(n, fc, sps, snr_db, rng):
    re = rng.choice(np.array([-1.0, 1.0]), size=_n_symbols(n, sps))
    im = rng.choice(np.array([-1.0, 1.0]), size=_n_symbols(n, sps))
    sym = (re + 1j * im) / np.sqrt(2.0)
    base = _symbols_to_samples(sym, sps, n, rng)
    theta = rng.uniform(0.0, 2.0 * np.pi)
    s = base * np.exp(1j * (2.0 * np.pi * fc * np.arange(n) + theta))
    return add_noise(s, snr_db, rng)


def qam16(n, fc, sps, snr_db, rng):
    lv = np.array([-3.0, -1.0, 1.0, 3.0])
    m = _n_symbols(n, sps)
    sym = (rng.choice(lv, size=m) + 1j * rng.choice(lv, size=m)) / np.sqrt(10.0)
    base = _symbols_to_samples(sym, sps, n, rng)
    theta = rng.uniform(0.0, 2.0 * np.pi)
    s = base * np.exp(1j * (2.0 * np.pi * fc * np.arange(n) + theta))
    return add_noise(s, snr_db, rng)


def msk(n, fc, sps, snr_db, rng):
    """Continuous-phase binary FSK with h = 1/2: the phase moves by +-pi/2 over each symbol."""
    b = rng.choice(np.array([-1.0, 1.0]), size=_n_symbols(n, sps))
    per_sample = _symbols_to_samples(b, sps, n, rng) * (np.pi / 2.0) / sps
    phase = np.cumsum(per_sample)
    theta = rng.uniform(0.0, 2.0 * np.pi)
    s = np.exp(1j * (phase + 2.0 * np.pi * fc * np.arange(n) + theta))
    return add_noise(s, snr_db, rng)


def am(n, fc, sps, snr_db, rng):
    """Real-carrier AM; the message is white Gaussian smoothed by a length-sps moving average."""
    g = rng.standard_normal(n + sps)
    msg = np.convolve(g, np.ones(sps) / sps, mode="valid")[:n]
    msg = msg / (np.sqrt(np.mean(msg ** 2)) + 1e-30)
    theta = rng.uniform(0.0, 2.0 * np.pi)
    s = (1.0 + 0.5 * msg) * np.cos(2.0 * np.pi * fc * np.arange(n) + theta)
    return add_noise(s.astype(np.complex128), snr_db, rng)


def noise(n, rng):
    """Unit-variance circular complex white Gaussian noise."""
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2.0)


def m_sequence(length_pow: int = 5, taps=(5, 3)) -> np.ndarray:
    """A +-1 maximal-length sequence of period 2^length_pow - 1 from a Fibonacci LFSR (x^5 + x^3 + 1)."""
    nbit = length_pow
    state = [1] * nbit
    out = []
    for _ in range(2 ** nbit - 1):
        out.append(state[-1])
        fb = 0
        for t in taps:
            fb ^= state[t - 1]
        state = [fb] + state[:-1]
    return np.where(np.array(out) > 0, 1.0, -1.0)


def dsss_bpsk(n, snr_db, rng, chip_rate=0.25, gain=31):
    """Direct-sequence spread BPSK: one data bit spans `gain` chips of a length-31 m-sequence, each chip
    lasting 1/chip_rate samples (chip rate 0.25 with f_s = 1), real baseband, plus complex AWGN."""
    code = m_sequence(5)
    assert len(code) == gain
    spc = int(round(1.0 / chip_rate))
    nchips = n // spc + 2 * gain
    nbits = nchips // gain + 1
    bits = rng.choice(np.array([-1.0, 1.0]), size=nbits)
    chips = np.repeat(bits, gain)[:nchips] * np.tile(code, nbits)[:nchips]
    off = int(rng.integers(0, spc))
    s = chips[(np.arange(n) + off) // spc].astype(np.complex128)
    return add_noise(s, snr_db, rng)


def generate(kind: str, n: int, rng: np.random.Generator, fc: float, sps: int, snr_db: float) -> np.ndarray:
    if kind == "bpsk":
        return bpsk(n, fc, sps, snr_db, rng)
    if kind == "qpsk":
        return qpsk(n, fc, sps, snr_db, rng)
    if kind == "qam16":
        return qam16(n, fc, sps, snr_db, rng)
    if kind == "msk":
        return msk(n, fc, sps, snr_db, rng)
    if kind == "am":
        return am(n, fc, sps, snr_db, rng)
    if kind == "noise":
        return noise(n, rng)
    raise ValueError(kind)


def hamming(n: int) -> np.ndarray:
    """Symmetric Hamming window 0.54 - 0.46 cos(2 pi j / (n-1))."""
    j = np.arange(n)
    return 0.54 - 0.46 * np.cos(2.0 * np.pi * j / (n - 1))
