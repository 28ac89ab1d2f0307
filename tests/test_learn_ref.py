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


@pytest.mark.parametrize("N", [4096, 8192])
def test_labels_pure_noise_all_zero_and_bpsk_has_active_strips(N):
    Np = 16
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


@pytest.mark.parametrize("Np,nc", [(16, 1024), (64, 1024), (8, 256)])
def test_alpha0_bin_is_where_the_coordinate_map_puts_alpha_zero(Np, nc):
    """q0(k) (the PSD bin of the features) is the unique bin of strip k whose cycle frequency, by the
    coordinate map pinned against the Eq. (2) sums, is zero modulo 1 (alpha = -1 in the Nyquist strip)."""
    _, a = O.ssca_coords(Np, nc)
    q0 = LR.alpha0_bin(Np, nc)
    for k in range(Np):
        zeros = np.flatnonzero(np.abs(((a[k] + 0.5) % 1.0) - 0.5) < 1e-12)
        assert zeros.tolist() == [q0[k]], (k, zeros, q0[k])


@pytest.mark.parametrize("Np,N", [(16, 4096), (8, 2048)])
def test_label_guard_is_alpha_distance_from_zero_mod_1(Np, N):
    """The label's off-guard bins of strip k are exactly the cells whose coordinate-map alpha lies at least
    1/256 away from 0 modulo 1."""
    _, a = O.ssca_coords(Np, N)
    for k in range(Np):
        aw = ((a[k] + 0.5) % 1.0) - 0.5
        assert np.array_equal(LR.label_off_mask(k, Np, N), np.abs(aw) >= 1.0 / 256 - 1e-12), k


def test_psd_feature_peaks_at_a_tone_channel():
    """A complex tone at f = 3/16 puts its power in the alpha = 0 cell of strip 3: the PSD feature peaks
    there, above its neighbours that see it through the window's main lobe (a q0 read at alpha = 2 f_k
    instead would not see it)."""
    N, Np = 1 << 14, 16
    n = np.arange(N)
    x = np.exp(2j * np.pi * 3 / Np * n) + 0.01 * sg.noise(N, sg.rng_for(73, 0))
    f = LR.features(x, Np, sg.hamming(Np))
    assert int(np.argmax(f[:Np])) == 3 and f[3] - np.sort(f[:Np])[-2] > 0.5


def _bf16_exact_params(Np, hidden, rng):
    """Weights and features in {-1, 0, 1}, zero biases: every GEMM input of the forward pass is an integer
    of magnitude <= 256, so bf16 rounding leaves the forward pass exact."""
    p = {"W1": rng.integers(-1, 2, (hidden, 2 * Np)).astype(float), "b1": np.zeros(hidden),
         "W2": rng.integers(-1, 2, (hidden, hidden)).astype(float), "b2": np.zeros(hidden),
         "W3": rng.integers(-1, 2, (Np, hidden)).astype(float), "b3": np.zeros(Np)}
    return p


def test_bf16_forward_rounds_only_gemm_inputs():
    """With bf16-exact inputs and activations the bf16 forward equals the FP64 forward bit for bit; with
    general inputs it differs, by no more than the bf16 unit roundoff 2^-8 per rounded GEMM operand."""
    rng = np.random.default_rng(5)
    Np, hidden, B = 4, 8, 6
    p = _bf16_exact_params(Np, hidden, rng)
    F = rng.integers(-1, 2, (B, 2 * Np)).astype(float)
    c64, c16 = LR.mlp_forward(p, F), LR.mlp_forward(p, F, bf16=True)
    for k in ("a1", "a2", "z", "s"):
        assert np.array_equal(c64[k], c16[k]), k
    p = _small_params(Np, hidden)
    F = rng.standard_normal((B, 2 * Np))
    c64, c16 = LR.mlp_forward(p, F), LR.mlp_forward(p, F, bf16=True)
    scale = np.abs(F) @ np.abs(p["W1"]).T
    d = np.abs(c16["a1"] - c64["a1"])
    assert 0 < d.max() and np.all(d <= 2.01 * 2.0 ** -8 * scale)


def _backward_scale(p, F, cache):
    """Element-wise size of every gradient's terms: the backward pass run on absolute values."""
    B, Np = cache["s"].shape
    adz = np.abs(cache["s"]) / (B * Np) + 1.0 / (B * Np)
    m2, m1 = (cache["a2"] > 0), (cache["a1"] > 0)
    g = {"W3": adz.T @ np.abs(cache["h2"])}
    dh2 = adz @ np.abs(p["W3"])
    g["W2"] = (dh2 * m2).T @ np.abs(cache["h1"])
    dh1 = (dh2 * m2) @ np.abs(p["W2"])
    g["W1"] = (dh1 * m1).T @ np.abs(F)
    g["F"] = (dh1 * m1) @ np.abs(p["W1"])
    return g


def test_bf16_backward_within_rounding_bound_of_exact_backward():
    """The bf16 backward (the GPU kernels' comparator) rounds the operands of every backward GEMM. On the same
    forward cache it must equal the exact backward (itself pinned by central differences) within the error
    those roundings allow: each term carries at most two rounded factors per GEMM, and the error compounds
    over at most three layers, so |g16 - g64| <= 8 * 2^-8 * (the same backward on absolute values). A
    transposed weight or a mask taken from the wrong layer breaks that bound."""
    rng = np.random.default_rng(6)
    Np, hidden, B = 4, 8, 5
    p = _small_params(Np, hidden, seed=3)
    F = rng.standard_normal((B, 2 * Np))
    y = (rng.random((B, Np)) > 0.5).astype(float)
    cache = LR.mlp_forward(p, F, bf16=True)
    g16 = LR.mlp_backward(p, F, y, cache, bf16=True)
    g64 = LR.mlp_backward(p, F, y, cache, bf16=False)
    sc = _backward_scale(p, F, cache)
    bound = 8 * 2.0 ** -8
    for k in ("W3", "W2", "W1", "F"):
        d = np.abs(g16[k] - g64[k])
        assert d.max() > 0, k
        assert np.all(d <= bound * sc[k] + 1e-300), (k, (d / sc[k]).max())
    # Planted mistakes in an exact backward, each of which the bound catches.
    dz = (cache["s"] - y) / (B * Np)
    da2 = (dz @ p["W3"]) * (cache["a2"] > 0)
    wrong_t = ((da2 @ p["W2"].T) * (cache["a1"] > 0)).T @ F
    wrong_mask = ((da2 @ p["W2"]) * (cache["a2"] > 0)).T @ F
    for wrong in (wrong_t, wrong_mask):
        assert np.any(np.abs(wrong - g16["W1"]) > bound * sc["W1"])
