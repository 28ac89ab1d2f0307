"""The five seeded workloads the library is tested and measured on.

Each function returns plain numpy arrays (complex128 signals, float64 windows) plus the estimator parameters.
Nothing here computes any part of the estimator.

1. one real-carrier BPSK signal of 1024 samples (fc 0.05, 8 samples/symbol, 0 dB); SSCA Np=32, N=1024; FAM
   Np=32, L=8, P=32 on its first 256 samples; Hamming windows.
2. 16 signals drawn from {BPSK, QPSK, MSK, noise}, fc ~ U[0.02, 0.2], sps ~ U{4..16}, SNR ~ U[-10, 10] dB;
   SSCA Np=64 on 2^16 samples; FAM Np=256, L=64, P=256 on the first 16384 samples.
3. one QPSK signal of 2^20 samples, complex carrier 0.1, 8 samples/symbol, 5 dB; SSCA Np=64 (headline).
4. learned-selector training/evaluation signals over {BPSK, QPSK, 16-QAM, MSK, AM, noise}, fc ~ U[0.02, 0.3],
   sps ~ U{4..16}, SNR ~ U[-10, 10] dB; SSCA Np=256, N=2^18.
5. 64 signals of lengths 2^e, e ~ U{14..20}, mixed modulations, SNR ~ U[-10, 15] dB; Np=64 for even
   indices and 128 for odd ones.
"""
from __future__ import annotations

import numpy as np

from . import signals as sg


def cfg1():
    rng = sg.rng_for(1, 0)
    x = sg.bpsk(1024, 0.05, 8, 0.0, rng, real_carrier=True)
    return dict(x=x, ssca=dict(N=1024, Np=32, win=sg.hamming(32)),
                fam=dict(Np=32, L=8, P=32, win=sg.hamming(32)))


def cfg2_signal(i: int, n: int = 1 << 16):
    rng = sg.rng_for(2, i)
    kind = ("bpsk", "qpsk", "msk", "noise")[int(rng.integers(0, 4))]
    fc = float(rng.uniform(0.02, 0.2))
    sps = int(rng.integers(4, 17))
    snr = float(rng.uniform(-10.0, 10.0))
    return kind, sg.generate(kind, n, rng, fc, sps, snr)


def cfg2(batch: int = 16):
    xs = [cfg2_signal(i)[1] for i in range(batch)]
    return dict(x=np.stack(xs), ssca=dict(N=1 << 16, Np=64, win=sg.hamming(64)),
                fam=dict(Np=256, L=64, P=256, win=sg.hamming(256)))


def cfg3(n: int = 1 << 20):
    rng = sg.rng_for(3, 0)
    x = sg.qpsk(n, 0.1, 8, 5.0, rng)
    return dict(x=x, ssca=dict(N=n, Np=64, win=sg.hamming(64)))


SPLITS = {"train": 0, "val": 1, "test": 2}


def cfg4_signal(i: int, n: int = 1 << 18, split: str = "train"):
    """Signal i of a selector data set split ("train", "val", "test"); the splits' seeds never overlap."""
    rng = sg.rng_keyed(4, SPLITS[split], i)
    kind = sg.MODULATIONS[int(rng.integers(0, len(sg.MODULATIONS)))]
    fc = float(rng.uniform(0.02, 0.3))
    sps = int(rng.integers(4, 17))
    snr = float(rng.uniform(-10.0, 10.0))
    return kind, sg.generate(kind, n, rng, fc, sps, snr)


def selector_signal(i: int, split: str = "train", emin: int = 14, emax: int = 20):
    """Training signal for the Np = 64 / 128 selectors: length 2^e, e ~ U{emin..emax}, and the modulation,
    carrier, rate and SNR ranges of the combined workload (SNR ~ U[-10, 15] dB)."""
    rng = sg.rng_keyed(6, SPLITS[split], i)
    e = int(rng.integers(emin, emax + 1))
    kind = sg.MODULATIONS[int(rng.integers(0, len(sg.MODULATIONS)))]
    fc = float(rng.uniform(0.02, 0.3))
    sps = int(rng.integers(4, 17))
    snr = float(rng.uniform(-10.0, 15.0))
    return kind, sg.generate(kind, 1 << e, rng, fc, sps, snr)


def cfg5_signal(i: int):
    rng = sg.rng_for(5, i)
    e = int(rng.integers(14, 21))
    kind = sg.MODULATIONS[int(rng.integers(0, len(sg.MODULATIONS)))]
    fc = float(rng.uniform(0.02, 0.3))
    sps = int(rng.integers(4, 17))
    snr = float(rng.uniform(-10.0, 15.0))
    np_ = 64 if i % 2 == 0 else 128
    return dict(kind=kind, x=sg.generate(kind, 1 << e, rng, fc, sps, snr), N=1 << e, Np=np_,
                win=sg.hamming(np_))
