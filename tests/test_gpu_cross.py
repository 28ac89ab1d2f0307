"""Cross and conjugate SSCA (scd_ssca_cross_ex) on the GPU against the FP64 oracle's ssca_cross, over sizes
that take the paired and single-subset Stage 1, both down-conversion forms, a batch and y = x."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2506_18003_amd as scd  # noqa: E402
from oracle import scd_oracle as O  # noqa: E402
from synth import signals as sg  # noqa: E402

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-4  # max |S - S_ref| / max |S_ref|, the bar of the auto SSCA parity tests


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _g(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x).astype(np.complex64)).to(dev)


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("conjugate", [False, True])
@pytest.mark.parametrize("N,Np", [(1024, 16), (4096, 64), (1 << 14, 32), (1 << 16, 256)])
def test_cross_matches_oracle(dev, N, Np, conjugate):
    x = sg.bpsk(N, 0.09, 5, 2.0, sg.rng_for(99, N + Np)).astype(np.complex64)
    y = sg.qpsk(N, 0.13, 7, 1.0, sg.rng_for(99, N + Np + 1)).astype(np.complex64)
    w = sg.hamming(Np).astype(np.float32)
    S = scd.ssca_cross(_g(x, dev), _g(y, dev), Np, win=torch.from_numpy(w).to(dev), conjugate=conjugate)
    ref = O.ssca_cross(x.astype(np.complex128), y.astype(np.complex128), Np, w.astype(np.float64), conjugate)
    assert _rel(S.cpu().numpy(), ref) <= TOL_FP32


def test_cross_batch_paired_stage1(dev):
    """A batch of two at N = 2^16, Np = 64 runs the paired Stage 1; each signal matches the oracle."""
    N, Np = 1 << 16, 64
    xs = np.stack([sg.msk(N, 0.1, 8, 3.0, sg.rng_for(100, b)) for b in range(2)]).astype(np.complex64)
    ys = np.stack([sg.noise(N, sg.rng_for(101, b)) for b in range(2)]).astype(np.complex64)
    S = scd.ssca_cross(_g(xs, dev), _g(ys, dev), Np).cpu().numpy()
    w = sg.hamming(Np).astype(np.float32).astype(np.float64)
    for b in range(2):
        ref = O.ssca_cross(xs[b].astype(np.complex128), ys[b].astype(np.complex128), Np, w)
        assert _rel(S[b], ref) <= TOL_FP32, b


def test_cross_with_itself_is_the_auto_scd(dev):
    x = _g(sg.qpsk(1 << 15, 0.1, 8, 5.0, sg.rng_for(102, 0)), dev)
    assert torch.equal(scd.ssca_cross(x, x, 64), scd.ssca(x, 64))


@pytest.mark.parametrize("conjugate", [False, True])
@pytest.mark.parametrize("Np,L,P", [(16, 4, 64), (64, 16, 128), (256, 64, 32), (32, 1, 1024), (16, 16, 4), (32, 8, 64),
                                    (64, 4, 256)])
def test_fam_cross_matches_oracle(dev, Np, L, P, conjugate):
    x = sg.bpsk(P * L, 0.06, 6, 2.0, sg.rng_for(103, Np + P)).astype(np.complex64)
    y = sg.msk(P * L, 0.11, 8, 4.0, sg.rng_for(104, Np + P)).astype(np.complex64)
    w = sg.hamming(Np).astype(np.float32)
    S = scd.fam_cross(_g(x, dev), _g(y, dev), Np, L, P, win=torch.from_numpy(w).to(dev), conjugate=conjugate)
    ref = O.fam_cross(x.astype(np.complex128), y.astype(np.complex128), Np, L, P, w.astype(np.float64), conjugate)
    assert _rel(S.cpu().numpy(), ref) <= TOL_FP32


def test_fam_cross_batch_and_small_workspace(dev):
    """A batch of three through a caller workspace that holds one signal's X_T and Y_T (so three chunks)."""
    Np, L, P = 64, 16, 64
    xs = np.stack([sg.qpsk(P * L, 0.1, 8, 0.0, sg.rng_for(105, b)) for b in range(3)]).astype(np.complex64)
    ys = np.stack([sg.noise(P * L, sg.rng_for(106, b)) for b in range(3)]).astype(np.complex64)
    ws = torch.empty(2 * scd.fam_workspace_size(Np, L, P) // 8, dtype=torch.complex64, device=dev)
    S = scd.fam_cross(_g(xs, dev), _g(ys, dev), Np, L, P, workspace=ws).cpu().numpy()
    w = sg.hamming(Np).astype(np.float32).astype(np.float64)
    for b in range(3):
        ref = O.fam_cross(xs[b].astype(np.complex128), ys[b].astype(np.complex128), Np, L, P, w)
        assert _rel(S[b], ref) <= TOL_FP32, b


def test_fam_cross_with_itself_is_the_auto_fam(dev):
    x = _g(sg.bpsk(4096, 0.08, 5, 1.0, sg.rng_for(107, 0)), dev)
    assert torch.equal(scd.fam_cross(x, x, 64, 16, 256), scd.fam(x, 64, 16, 256))
