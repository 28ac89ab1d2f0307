"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on the same seeded inputs.

Bar (FP32 path): max |S_gpu - S_oracle| / max |S_oracle| <= 1e-4. The oracle sees exactly the complex64
samples and float32 window the GPU sees, promoted to float64.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2506_18003_amd as scd  # noqa: E402
from oracle import scd_oracle as O  # noqa: E402
from synth import signals as sg  # noqa: E402
from synth import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
TOL_FP32 = 1e-4


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def to_gpu(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x).astype(np.complex64)).to(dev)


def f64(x):
    return np.asarray(x).astype(np.complex64).astype(np.complex128)


def w32(n):
    return sg.hamming(n).astype(np.float32)


def test_ssca_cfg1(dev):
    c = W.cfg1()
    x, p = c["x"], c["ssca"]
    S = scd.ssca(to_gpu(x, dev), p["Np"], win=torch.from_numpy(w32(p["Np"])).to(dev)).cpu().numpy()
    ref = O.ssca(f64(x), p["Np"], w32(p["Np"]).astype(np.float64))
    assert rel(S, ref) <= TOL_FP32


def test_fam_cfg1(dev):
    c = W.cfg1()
    p = c["fam"]
    x = c["x"][: p["P"] * p["L"]]
    S = scd.fam(to_gpu(x, dev), p["Np"], p["L"], p["P"], win=torch.from_numpy(w32(p["Np"])).to(dev)).cpu().numpy()
    ref = O.fam(f64(x), p["Np"], p["L"], p["P"], w32(p["Np"]).astype(np.float64))
    assert rel(S, ref) <= TOL_FP32


@pytest.mark.parametrize("N,Np", [(1024, 16), (2048, 16), (4096, 64), (8192, 256), (1 << 14, 128), (1 << 15, 32)])
def test_ssca_sizes(dev, N, Np):
    x = sg.bpsk(N, 0.11, 5, 2.0, sg.rng_for(50, N + Np))
    w = w32(Np)
    S = scd.ssca(to_gpu(x, dev), Np, win=torch.from_numpy(w).to(dev)).cpu().numpy()
    ref = O.ssca(f64(x), Np, w.astype(np.float64))
    assert rel(S, ref) <= TOL_FP32


# Pair tiles of 16, 32 and 64 channels (P <= 64 takes min(Np, 64)); single-stage, uniform-radix (wave-local)
# and mixed-radix transforms.
@pytest.mark.parametrize("Np,L,P", [(16, 4, 64), (16, 16, 4), (64, 16, 128), (256, 64, 32), (128, 1, 1024),
                                    (32, 8, 64), (64, 4, 16), (128, 8, 8), (32, 16, 256), (64, 2, 512)])
def test_fam_sizes(dev, Np, L, P):
    x = sg.qpsk(P * L, 0.07, 6, 3.0, sg.rng_for(51, Np + L + P))
    w = w32(Np)
    S = scd.fam(to_gpu(x, dev), Np, L, P, win=torch.from_numpy(w).to(dev)).cpu().numpy()
    ref = O.fam(f64(x), Np, L, P, w.astype(np.float64))
    assert rel(S, ref) <= TOL_FP32


def test_ssca_cfg2_batch(dev):
    c = W.cfg2()
    p = c["ssca"]
    xs = c["x"]
    S = scd.ssca(to_gpu(xs, dev), p["Np"], win=torch.from_numpy(w32(p["Np"])).to(dev)).cpu().numpy()
    w = w32(p["Np"]).astype(np.float64)
    for b in range(xs.shape[0]):
        assert rel(S[b], O.ssca(f64(xs[b]), p["Np"], w)) <= TOL_FP32, b


def test_fam_cfg2_batch(dev):
    c = W.cfg2()
    p = c["fam"]
    n = p["P"] * p["L"]
    xs = np.ascontiguousarray(c["x"][:, :n])
    S = scd.fam(to_gpu(xs, dev), p["Np"], p["L"], p["P"], win=torch.from_numpy(w32(p["Np"])).to(dev))
    w = w32(p["Np"]).astype(np.float64)
    Sc = S.cpu().numpy()
    for b in (0, 7, 15):
        assert rel(Sc[b], O.fam(f64(xs[b]), p["Np"], p["L"], p["P"], w)) <= TOL_FP32, b
    # exact conjugate symmetry of the estimator, within FP32 rounding, on every signal
    P = p["P"]
    T = torch.conj(S.transpose(1, 2)[..., (-torch.arange(P, device=dev)) % P])
    d = (S - T).abs().amax(dim=(1, 2, 3)) / S.abs().amax(dim=(1, 2, 3))
    assert float(d.max()) <= TOL_FP32


def test_ssca_cfg3_full_size_sampled_strips(dev):
    """N = 2^20, Np = 64 in the launch configuration the benchmark times; strips compared in full."""
    c = W.cfg3()
    x, p = c["x"], c["ssca"]
    w = w32(p["Np"])
    S = scd.ssca(to_gpu(x, dev), p["Np"], win=torch.from_numpy(w).to(dev))
    xf = f64(x)
    strips = (0, 1, 6, 13, 31, 32, 51, 63)
    refs = {k: O.ssca_strip(xf, p["Np"], w.astype(np.float64), k) for k in strips}
    peak = max(np.abs(r).max() for r in refs.values())
    for k in strips:
        g = S[k].cpu().numpy()
        assert np.abs(g - refs[k]).max() / peak <= TOL_FP32, k


@pytest.mark.parametrize("N,Np,strips", [
    (1 << 20, 128, (0, 3, 8, 67, 100, 127)),       # paired Stage 1 at Np = 128 (both subsets of a pair)
    (1 << 18, 256, (0, 5, 21, 130, 200, 255)),     # paired Stage 1 at Np = 256, 16 taps per lane
])
def test_ssca_large_np_sampled_strips(dev, N, Np, strips):
    """The paired Stage 1 at Np = 128 and 256 on grids that fill the GPU; strips compared in full."""
    x = sg.qpsk(N, 0.1, 8, 5.0, sg.rng_for(53, Np))
    w = w32(Np)
    S = scd.ssca(to_gpu(x, dev), Np, win=torch.from_numpy(w).to(dev))
    xf = f64(x)
    refs = {k: O.ssca_strip(xf, Np, w.astype(np.float64), k) for k in strips}
    peak = max(np.abs(r).max() for r in refs.values())
    for k in strips:
        assert np.abs(S[k].cpu().numpy() - refs[k]).max() / peak <= TOL_FP32, k


def test_stages_equal_whole(dev):
    N, Np = 1 << 16, 64
    x = to_gpu(sg.qpsk(N, 0.1, 8, 5.0, sg.rng_for(52, 0)), dev)
    S = scd.ssca(x, Np)
    inter = torch.empty(Np * N, dtype=torch.complex64, device=dev)
    out = torch.empty(Np, N, dtype=torch.complex64, device=dev)
    scd.ssca_stage1(x, Np, inter)
    scd.ssca_stage2(inter, N, Np, out)
    assert torch.equal(out, S)


def test_edge_zero_and_impulse(dev):
    N, Np = 4096, 32
    z = scd.ssca(torch.zeros(N, dtype=torch.complex64, device=dev), Np)
    assert float(z.abs().max()) == 0.0
    for n0 in (0, 5, N // 2, N - 1):
        x = np.zeros(N, np.complex128)
        x[n0] = 1.0 - 0.5j
        S = scd.ssca(to_gpu(x, dev), Np).cpu().numpy()
        ref = O.ssca(x, Np, w32(Np).astype(np.float64))
        assert rel(S, ref) <= TOL_FP32, n0


def test_edge_energy_at_signal_ends(dev):
    """Frames that hang over either end of the signal see zeros (the ragged edges of the framing)."""
    N, Np = 2048, 64
    x = np.zeros(N, np.complex128)
    x[:40] = sg.noise(40, sg.rng_for(53, 0))
    x[-40:] = sg.noise(40, sg.rng_for(53, 1))
    S = scd.ssca(to_gpu(x, dev), Np).cpu().numpy()
    assert rel(S, O.ssca(x, Np, w32(Np).astype(np.float64))) <= TOL_FP32


def test_edge_energy_at_signal_ends_full_size(dev):
    """The headline configuration (N = 2^20, Np = 64, Np dividing M2): frames that start before sample 0 or end
    after sample N-1 read zeros there and the true samples elsewhere, on sampled strips."""
    N, Np = 1 << 20, 64
    x = np.zeros(N, np.complex128)
    x[:100] = sg.noise(100, sg.rng_for(53, 2))
    x[-100:] = sg.noise(100, sg.rng_for(53, 3))
    S = scd.ssca(to_gpu(x, dev), Np).cpu().numpy()
    w = w32(Np).astype(np.float64)
    for k in (0, 17, 33, 63):
        ref = O.ssca_strip(x, Np, w, k)
        assert np.abs(S[k] - ref).max() <= TOL_FP32 * np.abs(ref).max(), k


def test_determinism(dev):
    x = to_gpu(sg.qpsk(1 << 16, 0.1, 8, 5.0, sg.rng_for(54, 0)), dev)
    a = scd.ssca(x, 64)
    b = scd.ssca(x, 64)
    assert torch.equal(a, b)
    y = to_gpu(sg.qpsk(1 << 14, 0.1, 8, 5.0, sg.rng_for(54, 1)), dev)
    assert torch.equal(scd.fam(y, 256, 64, 256), scd.fam(y, 256, 64, 256))


def test_batch_strides_and_small_workspace(dev):
    """A strided batch (x rows padded), a caller workspace holding 2 of 5 intermediates (forces chunking)."""
    N, Np, B = 4096, 32, 5
    xs = np.stack([sg.msk(N, 0.05 * (b + 1), 6, 4.0, sg.rng_for(55, b)) for b in range(B)])
    pad = torch.zeros(B, N + 64, dtype=torch.complex64, device=dev)
    pad[:, :N] = to_gpu(xs, dev)
    xv = pad[:, :N]
    ws = torch.empty(2 * Np * N, dtype=torch.complex64, device=dev)
    S = scd.ssca(xv, Np, workspace=ws).cpu().numpy()
    for b in range(B):
        assert rel(S[b], O.ssca(f64(xs[b]), Np, w32(Np).astype(np.float64))) <= TOL_FP32, b


def test_workspace_too_small_is_an_error(dev):
    x = to_gpu(sg.noise(4096, sg.rng_for(56, 0)), dev)
    ws = torch.empty(16, dtype=torch.complex64, device=dev)
    with pytest.raises(scd.ScdError) as e:
        scd.ssca(x, 32, workspace=ws)
    assert e.value.code == -4


def test_nonsymmetric_window(dev):
    N, Np = 2048, 32
    x = sg.qam16(N, 0.2, 4, 6.0, sg.rng_for(57, 0))
    w = np.linspace(0.05, 1.0, Np).astype(np.float32)
    S = scd.ssca(to_gpu(x, dev), Np, win=torch.from_numpy(w).to(dev)).cpu().numpy()
    assert rel(S, O.ssca(f64(x), Np, w.astype(np.float64))) <= TOL_FP32
    F = scd.fam(to_gpu(x[:1024], dev), Np, 8, 128, win=torch.from_numpy(w).to(dev)).cpu().numpy()
    assert rel(F, O.fam(f64(x[:1024]), Np, 8, 128, w.astype(np.float64))) <= TOL_FP32


TOL_SPLIT = 1e-3


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
@pytest.mark.parametrize("N,Np", [(1024, 32), (2048, 16), (1 << 14, 64), (1 << 16, 64), (8192, 128)])
def test_ssca_split_precision(dev, prec, N, Np):
    x = sg.qpsk(N, 0.13, 6, 4.0, sg.rng_for(60, N + Np))
    w = w32(Np)
    S = scd.ssca(to_gpu(x, dev), Np, win=torch.from_numpy(w).to(dev), precision=prec).cpu().numpy()
    assert rel(S, O.ssca(f64(x), Np, w.astype(np.float64))) <= TOL_SPLIT


def test_ssca_split_bf16_cfg3_full_size(dev):
    """The headline workload in split-BF16: sampled strips against the FP64 oracle, error <= 1e-3 of peak,
    and the unsplit BF16 ablation measurably worse."""
    c = W.cfg3()
    x, p = c["x"], c["ssca"]
    w = w32(p["Np"])
    xg, wg = to_gpu(x, dev), torch.from_numpy(w).to(dev)
    S = scd.ssca(xg, p["Np"], win=wg, precision="split_bf16")
    S1 = scd.ssca(xg, p["Np"], win=wg, precision="bf16")
    xf = f64(x)
    strips = (0, 6, 13, 51)
    refs = {k: O.ssca_strip(xf, p["Np"], w.astype(np.float64), k) for k in strips}
    peak = max(np.abs(r).max() for r in refs.values())
    e_split = max(np.abs(S[k].cpu().numpy() - refs[k]).max() for k in strips) / peak
    e_plain = max(np.abs(S1[k].cpu().numpy() - refs[k]).max() for k in strips) / peak
    assert e_split <= TOL_SPLIT
    assert e_plain > 10 * e_split


def test_ssca_split_fp16_cfg3_full_size(dev):
    """The headline workload with the split-FP16 channelizer (x is well inside the FP16 range): sampled strips,
    spread over all four channel subsets, against the FP64 oracle within 1e-3 of peak, and the unsplit FP16
    ablation measurably worse."""
    c = W.cfg3()
    x, p = c["x"], c["ssca"]
    w = w32(p["Np"])
    xg, wg = to_gpu(x, dev), torch.from_numpy(w).to(dev)
    S = scd.ssca(xg, p["Np"], win=wg, precision="split_fp16")
    S1 = scd.ssca(xg, p["Np"], win=wg, precision="fp16")
    xf = f64(x)
    strips = (1, 6, 32, 63)
    refs = {k: O.ssca_strip(xf, p["Np"], w.astype(np.float64), k) for k in strips}
    peak = max(np.abs(r).max() for r in refs.values())
    e_split = max(np.abs(S[k].cpu().numpy() - refs[k]).max() for k in strips) / peak
    e_plain = max(np.abs(S1[k].cpu().numpy() - refs[k]).max() for k in strips) / peak
    assert e_split <= TOL_SPLIT
    assert e_plain > 10 * e_split


def test_ssca_split_batch(dev):
    N, Np, B = 1 << 14, 128, 3
    xs = np.stack([sg.bpsk(N, 0.04 * (b + 1), 5, 0.0, sg.rng_for(61, b)) for b in range(B)])
    S = scd.ssca(to_gpu(xs, dev), Np, precision="split_bf16").cpu().numpy()
    for b in range(B):
        assert rel(S[b], O.ssca(f64(xs[b]), Np, w32(Np).astype(np.float64))) <= TOL_SPLIT, b
