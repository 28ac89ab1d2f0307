"""The paper's accuracy workload (Sec. IV-A): DSSS BPSK at 10 dB SNR, processing gain 31 (a length-31
m-sequence), chip rate 0.25, f_s = 1, with a Chebyshev window of 100 dB sidelobe attenuation (the window Alg. 1
and Alg. 2 name). FAM runs at N = 2048, Np = 256, P = 32 (L = 64) and SSCA at N = 2^20, Np = 64, as in the
paper's experiments.

The paper reports an average relative error (9.94e-5 for FAM against MATLAB in double precision, 1.08e-6 for
SSCA against a C++ SSCA with the same FFT coefficients) without defining the average. Here it is read as
sum |S - S_ref| / sum |S_ref| over every cell, against the FP64 oracle, and each form is held to a bound well
above what it reaches (parity unpinned against the paper's figures, whose references differ from ours)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from scipy.signal.windows import chebwin  # noqa: E402

import paper_2506_18003_amd as scd  # noqa: E402
from oracle import scd_oracle as O  # noqa: E402
from synth import signals as sg  # noqa: E402

pytestmark = pytest.mark.gpu

BOUND = {"fp32": 1e-5, "split_fp16": 1e-5, "split_bf16": 1e-4, "bf16": 1e-2}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _err(S, ref):
    return float(np.abs(S - ref).sum() / np.abs(ref).sum())


def _win(Np):
    return chebwin(Np, at=100).astype(np.float32)


@pytest.fixture(scope="module")
def ssca_case():
    x = sg.dsss_bpsk(1 << 20, 10.0, sg.rng_for(95, 1)).astype(np.complex64)
    w = _win(64)
    return x, w, O.ssca(x.astype(np.complex128), 64, w.astype(np.float64))


@pytest.mark.parametrize("prec", ["fp32", "split_fp16", "split_bf16", "bf16"])
def test_paper_accuracy_workload_ssca(dev, ssca_case, prec):
    x, w, ref = ssca_case
    S = scd.ssca(torch.from_numpy(x).to(dev), 64, win=torch.from_numpy(w).to(dev), precision=prec)
    e = _err(S.cpu().numpy(), ref)
    print(f"SSCA N=2^20 Np=64 DSSS BPSK {prec}: average relative error {e:.3e} (paper: 1.08e-6)")
    assert e <= BOUND[prec], e


def test_paper_accuracy_workload_fam(dev):
    x = sg.dsss_bpsk(2048, 10.0, sg.rng_for(95, 0)).astype(np.complex64)
    w = _win(256)
    ref = O.fam(x.astype(np.complex128), 256, 64, 32, w.astype(np.float64))
    S = scd.fam(torch.from_numpy(x).to(dev), 256, 64, 32, win=torch.from_numpy(w).to(dev))
    e = _err(S.cpu().numpy(), ref)
    print(f"FAM N=2048 Np=256 P=32 DSSS BPSK fp32: average relative error {e:.3e} (paper: 9.94e-5)")
    assert e <= BOUND["fp32"], e
