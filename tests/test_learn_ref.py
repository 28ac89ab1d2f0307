"""Pins of the FP64 learned-selector reference (CPU only)."""
import numpy as np
import pytest

from oracle import learn_ref as LR
from oracle import scd_oracle as O
from synth import signals as sg


def _small_params(Np=4, hidden=8, seed=0):
    rng = np.random.default_rng(seed)
    p = LR.init_params(Np, rng, hidden=hidden)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.standard_normal(p[k].shape) * 0.1
    return p


def test_mlp_gradients_match_central_differences():
    Np, B = 4, 5
    rng = np.random.default_rng(1)
    p = _small_params(Np)
    F = rng.standard_normal((B, 2 * Np))
    y = (rng.random((B, Np)) > 0.5).astype(float)
    cache = LR.mlp_forward(p, F)
    g = LR.mlp_backward(p, F, y, cache)

    def loss(pp, FF=F):
        return LR.bce(LR.mlp_forward(pp, FF)["s"], y)

    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        for idx in [tuple(rng.integers(0, s) for s in p[name].shape) for _ in range(6)]:
            pp = {k: v.copy() for k, v in p.items()}
            pp[name][idx] += h
            lp = loss(pp)
            pp[name][idx] -= 2 * h
            lm = loss(pp)
            num = (lp - lm) / (2 * h)
            assert abs(num - g[name][idx]) <= 1e-6 + 1e-5 * abs(num), (name, idx, num, g[name][idx])
    for _ in range(6):
        i, j = rng.integers(0, B), rng.integers(0, 2 * Np)
        Fp, Fm = F.copy(), F.copy()
        Fp[i, j] += h
        Fm[i, j] -= h
        num = (loss(p, Fp) - loss(p, Fm)) / (2 * h)
        assert abs(num - g["F"][i, j]) <= 1e-6 + 1e-5 * abs(num)


def test_adam_first_step_closed_form():
    """With zero moments the first bias-corrected step is lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p = np.ones(4)
    newp, m, v = LR.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(newp, p - 0.01 * g / (np.abs(g) + 1e-8), atol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_round_against_torch_and_ties():
    torch = pytest.importorskip("torch")
    a = np.random.default_rng(2).standard_normal(1000) * 10.0 ** np.random.default_rng(3).uniform(-5, 5, 1000)
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(LR.bf16_round(a), ref)
    assert LR.bf16_round(1.0 + 2.0 ** -8) == 1.0                       # tie -> even (1.0)
    assert LR.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6       # tie -> even (1 + 2^-6)
    assert LR.bf16_round(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7           # representable


def test_labels_pure_noise_all_zero_and_bpsk_has_active_strips():
    N, Np = 8192, 16
    w = sg.hamming(Np)
    lab, ratio = LR.labels_from_scd(O.ssca(sg.noise(N, sg.rng_for(70, 0)), Np, w))
    assert lab.sum() == 0 and ratio.max() < LR.T_LABEL
    lab, ratio = LR.labels_from_scd(O.ssca(sg.bpsk(N, 0.1, 4, 20.0, sg.rng_for(70, 1)), Np, w))
    assert lab.sum() >= 2


def test_label_threshold_matches_false_alarm_design():
    """|S|^2 of complex Gaussian noise is exponential: P(max of 2^18 bins > T mean) is about 1e-3."""
    p_bin = np.exp(-LR.T_LABEL)
    assert 5e-4 < (1 - (1 - p_bin) ** (1 << 18)) < 2e-3


def test_features_noise_vs_bpsk():
    N, Np = 1 << 14, 16
    w = sg.hamming(Np)
    fn = LR.features(sg.noise(N, sg.rng_for(71, 0)), Np, w)
    fb = LR.features(sg.bpsk(N, 0.1, 4, 15.0, sg.rng_for(71, 1)), Np, w)
    assert abs(fn[:Np].mean()) < 1e-12 and abs(fb[:Np].mean()) < 1e-12   # PSD part is centred
    # noise: peak-to-mean of ~1000 averaged exponential bins stays small; BPSK: strong cyclic peaks
    assert fn[Np:].max() < 1.5
    assert fb[Np:].max() > 3.0


def test_acp_equals_sum_of_segment_periodograms():
    N, Np = 1 << 14, 16
    x = sg.qpsk(N, 0.1, 8, 5.0, sg.rng_for(72, 0))
    A = LR.acp(x, Np, sg.hamming(Np))
    hop = N // LR.B_F
    direct = np.zeros_like(A)
    for b in range(LR.B_F):
        direct += np.abs(O.ssca(x[b * hop: b * hop + LR.N_C], Np, sg.hamming(Np))) ** 2
    assert np.allclose(A, direct, rtol=1e-12)
