"""GPU parity of the learned strip selector against its FP64 reference (oracle/learn_ref.py)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2506_18003_amd as scd  # noqa: E402
from paper_2506_18003_amd import selector as SEL  # noqa: E402
from oracle import learn_ref as LR  # noqa: E402
from oracle import scd_oracle as O  # noqa: E402
from synth import signals as sg  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def f64(x):
    return np.asarray(x).astype(np.complex64).astype(np.complex128)


def gpu(x, dev, dtype=torch.complex64):
    return torch.as_tensor(np.ascontiguousarray(x), device=dev).to(dtype)


# The segments start every N/16 samples, so N = 2^20 places them 64 Ki apart; the oracle only reads the 16
# segments, which keeps the large case cheap.
@pytest.mark.parametrize("N,Np", [(1 << 14, 16), (1 << 15, 64), (1 << 14, 256), (1 << 20, 64), (1 << 17, 128)])
def test_features_match_reference(dev, N, Np):
    xs = [sg.bpsk(N, 0.08, 6, 8.0, sg.rng_for(80, N + Np)), sg.noise(N, sg.rng_for(80, 1 + Np))]
    w = sg.hamming(Np).astype(np.float32)
    F = SEL.features(gpu(np.stack(xs), dev), Np, win=torch.from_numpy(w).to(dev)).cpu().numpy()
    for b, x in enumerate(xs):
        ref = LR.features(f64(x), Np, w.astype(np.float64))
        assert np.abs(F[b] - ref).max() <= 2e-3, b


def test_features_batch_spans_launch_chunks(dev):
    """Ten signals in one call (the features run at most 8 signals per launch): each row equals the feature of its
    signal computed alone."""
    N, Np = 1 << 14, 32
    xs = np.stack([sg.qpsk(N, 0.05 + 0.02 * i, 4 + i, 3.0, sg.rng_for(83, i)) for i in range(10)])
    w = torch.from_numpy(sg.hamming(Np).astype(np.float32)).to(dev)
    F = SEL.features(gpu(xs, dev), Np, win=w).cpu().numpy()
    for i in range(10):
        assert np.array_equal(F[i], SEL.features(gpu(xs[i], dev), Np, win=w).cpu().numpy()[0]), i


def test_labels_match_reference(dev):
    N, Np = 8192, 32
    xs = [sg.bpsk(N, 0.1, 4, 15.0, sg.rng_for(81, 0)), sg.noise(N, sg.rng_for(81, 1)),
          sg.qpsk(N, 0.2, 8, 3.0, sg.rng_for(81, 2))]
    S = scd.ssca(gpu(np.stack(xs), dev), Np)
    lab, ratio = SEL.strip_labels(S)
    lab, ratio = lab.cpu().numpy(), ratio.cpu().numpy()
    for b, x in enumerate(xs):
        rl, rr = LR.labels_from_scd(O.ssca(f64(x), Np, sg.hamming(Np).astype(np.float32).astype(np.float64)))
        assert np.allclose(ratio[b], rr, rtol=1e-3), b
        clear = np.abs(rr - LR.T_LABEL) > 1e-2 * LR.T_LABEL   # decisions away from the threshold must agree
        assert np.array_equal(lab[b][clear], rl[clear]), b


def _params_dict(p, Np):
    out = {}
    for name, (off, size) in SEL.layout(Np).items():
        a = p[off:off + size].astype(np.float64)
        if name == "W1":
            a = a.reshape(SEL.HIDDEN, 2 * Np)
        elif name == "W2":
            a = a.reshape(SEL.HIDDEN, SEL.HIDDEN)
        elif name == "W3":
            a = a.reshape(Np, SEL.HIDDEN)
        out[name] = a
    return out


TOL_GEMM = 1e-4  # |GPU - FP64| per element, relative to the sum of |terms| (the dot product's error scale)


def _bf(a):
    return LR.bf16_round(np.asarray(a, np.float64))


def _check_gemm(got, A, B, bias=None, name=""):
    """got == bf16(A) @ bf16(B) (+ bias) element by element, within TOL_GEMM of the absolute-sum scale: both sides
    take the same bf16-rounded operands, so only the FP32 accumulation order differs."""
    a, b = _bf(A), _bf(B)
    ref = a @ b + (0.0 if bias is None else bias)
    scale = np.abs(a) @ np.abs(b) + (0.0 if bias is None else np.abs(bias)) + 1e-30
    err = np.abs(np.asarray(got, np.float64) - ref) / scale
    assert err.max() <= TOL_GEMM, (name, float(err.max()))


@pytest.mark.parametrize("Np,B", [(16, 37), (64, 70), (128, 33), (256, 20)])
def test_mlp_forward_backward_match_bf16_reference_elementwise(dev, Np, B):
    """Every layer of the forward and backward pass, element by element: each GPU GEMM against the FP64 product
    of the same bf16-rounded operands (taken from the GPU's own previous layer), within 1e-4 of the dot
    product's absolute-sum scale; ReLU, the sigmoid and the BCE gradient to FP32 rounding."""
    rng = np.random.default_rng(Np + B)
    p = SEL.init_params(Np, seed=3)
    for name in ("b1", "b2", "b3"):
        off, size = SEL.layout(Np)[name]
        p[off:off + size] = rng.standard_normal(size) * 0.1
    X = rng.standard_normal((B, 2 * Np)).astype(np.float32)
    Y = (rng.random((B, Np)) > 0.6).astype(np.float32)
    pg, Xg, Yg = gpu(p, dev, torch.float32), gpu(X, dev, torch.float32), gpu(Y, dev, torch.float32)
    act, z, s = SEL.mlp_forward(pg, Xg, Np)
    grads = torch.empty_like(pg)
    scratch = torch.empty(B * (Np + 2 * SEL.HIDDEN), dtype=torch.float32, device=dev)
    dx = torch.empty_like(Xg)
    from paper_2506_18003_amd import _lib
    _lib.check(_lib.lib().scd_mlp_backward(Np, B, pg.data_ptr(), Xg.data_ptr(), act.data_ptr(), s.data_ptr(),
                                           Yg.data_ptr(), grads.data_ptr(), scratch.data_ptr(), dx.data_ptr(),
                                           torch.cuda.current_stream(dev).cuda_stream))
    P = _params_dict(p, Np)
    a1, h1, a2, h2 = (t.cpu().numpy().astype(np.float64) for t in act)
    z, s = z.cpu().numpy().astype(np.float64), s.cpu().numpy().astype(np.float64)
    # forward
    _check_gemm(a1, X, P["W1"].T, P["b1"], "a1")
    assert np.array_equal(h1, np.maximum(a1, 0.0))
    _check_gemm(a2, h1, P["W2"].T, P["b2"], "a2")
    assert np.array_equal(h2, np.maximum(a2, 0.0))
    _check_gemm(z, h2, P["W3"].T, P["b3"], "z")
    assert np.abs(s - 1.0 / (1.0 + np.exp(-z))).max() <= 4e-7
    # backward
    sc = scratch.cpu().numpy().astype(np.float64)
    dz = sc[:B * Np].reshape(B, Np)
    d2 = sc[B * Np:B * Np + B * SEL.HIDDEN].reshape(B, SEL.HIDDEN)
    d1 = sc[B * Np + B * SEL.HIDDEN:].reshape(B, SEL.HIDDEN)
    assert np.abs(dz - (s - Y) / (B * Np)).max() <= 1e-6 / (B * Np)
    g = _params_dict(grads.cpu().numpy(), Np)
    _check_gemm(g["W3"], dz.T, h2, name="dW3")
    assert np.abs(g["b3"] - dz.sum(axis=0)).max() <= TOL_GEMM * np.abs(dz).sum(axis=0).max()
    assert np.array_equal(d2, d2 * (a2 > 0))  # the ReLU mask of layer 2
    pre2 = _bf(dz) @ _bf(P["W3"])
    scale2 = np.abs(_bf(dz)) @ np.abs(_bf(P["W3"])) + 1e-30
    assert (np.abs(d2 - pre2 * (a2 > 0)) / scale2).max() <= TOL_GEMM
    _check_gemm(g["W2"], d2.T, h1, name="dW2")
    assert np.abs(g["b2"] - d2.sum(axis=0)).max() <= TOL_GEMM * np.abs(d2).sum(axis=0).max() + 1e-30
    pre1 = _bf(d2) @ _bf(P["W2"])
    scale1 = np.abs(_bf(d2)) @ np.abs(_bf(P["W2"])) + 1e-30
    assert (np.abs(d1 - pre1 * (a1 > 0)) / scale1).max() <= TOL_GEMM
    _check_gemm(g["W1"], d1.T, X, name="dW1")
    assert np.abs(g["b1"] - d1.sum(axis=0)).max() <= TOL_GEMM * np.abs(d1).sum(axis=0).max() + 1e-30
    _check_gemm(dx.cpu().numpy(), d1, P["W1"], name="dx")
    # End to end against the FP64 reference's own chain: operands that land on either side of a bf16 rounding
    # boundary add up to 8 * 2^-8 of the absolute-sum scale (the bound the CPU pin of the reference uses).
    cache = LR.mlp_forward(P, X.astype(np.float64), bf16=True)
    gr = LR.mlp_backward(P, X.astype(np.float64), Y.astype(np.float64), cache, bf16=True)
    bound = 8 * 2.0 ** -8
    scale_w3 = np.abs(_bf(cache["s"] - Y)).T @ np.abs(_bf(cache["h2"])) / (B * Np) + 1e-30
    assert (np.abs(g["W3"] - gr["W3"]) / scale_w3).max() <= bound


def test_adam_matches_reference(dev):
    rng = np.random.default_rng(5)
    n = 1000
    p, m, v = rng.standard_normal(n), np.zeros(n), np.zeros(n)
    pg, mg, vg = (gpu(a, dev, torch.float32) for a in (p, m, v))
    for t in range(1, 4):
        gr = rng.standard_normal(n)
        SEL.adam_step(pg, gpu(gr, dev, torch.float32), mg, vg, t, lr=1e-2)
        p, m, v = LR.adam_step(p, gr, m, v, t, lr=1e-2)
    assert np.allclose(pg.cpu().numpy(), p, rtol=1e-5, atol=1e-6)


def test_select_mask_and_confidence(dev):
    s = np.array([[0.95, 0.02, 0.5, 0.99], [0.97, 0.01, 0.03, 0.92]] * 1, np.float32)
    s = np.tile(s, (1, 4))
    mask, conf = SEL.select(gpu(s, dev, torch.float32), 0.4)
    assert np.array_equal(mask.cpu().numpy(), (s >= 0.4).astype(np.uint8))
    assert np.allclose(conf.cpu().numpy(), np.minimum.reduce(np.maximum(s, 1 - s), axis=1))


def test_training_lowers_loss(dev):
    """A learnable rule (strip active when its ACP-like feature is positive) is fitted by the GPU loop."""
    Np, B = 16, 256
    rng = np.random.default_rng(6)
    X = rng.standard_normal((B, 2 * Np)).astype(np.float32)
    Y = (X[:, Np:] > 0.3).astype(np.float32)
    tr = SEL.Trainer(Np, dev, seed=1, lr=3e-3)
    Xg, Yg = gpu(X, dev, torch.float32), gpu(Y, dev, torch.float32)
    first = None
    for it in range(150):
        s = tr.step(Xg, Yg)
        if it == 0:
            first = LR.bce(s.cpu().numpy().astype(np.float64), Y)
    last = LR.bce(SEL.mlp_forward(tr.params, Xg, Np)[2].cpu().numpy().astype(np.float64), Y)
    assert last < 0.3 * first


def _fixed_selector(Np, keep, dev):
    """A selector whose output ignores the features: strip k scores sigmoid(+-12) by keep[k]."""
    p = np.zeros(SEL.param_count(Np), np.float32)
    off, size = SEL.layout(Np)["b3"]
    p[off:off + size] = np.where(keep, 12.0, -12.0)
    return SEL.Selector(Np, p, np.zeros(2 * Np, np.float32), np.ones(2 * Np, np.float32), 0.5, 0.9).to(dev)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_learned_ssca_selected_strips_equal_full(dev, prec):
    N, Np = 1 << 16, 64
    x = gpu(sg.qpsk(N, 0.1, 8, 5.0, sg.rng_for(82, 0)), dev)
    keep = np.zeros(Np, bool)
    keep[[0, 3, 17, 18, 40, 63]] = True
    sel = _fixed_selector(Np, keep, dev)
    sentinel = torch.full((Np, N), complex(7.0, -7.0), dtype=torch.complex64, device=dev)
    out, mask, fb = SEL.ssca_learned(x, sel, precision=prec, out=sentinel.clone())
    assert not fb
    assert np.array_equal(mask.cpu().numpy().astype(bool), keep)
    full = scd.ssca(x, Np, precision=prec)
    k = torch.from_numpy(np.nonzero(keep)[0]).to(dev)
    nk = torch.from_numpy(np.nonzero(~keep)[0]).to(dev)
    assert torch.equal(out[k], full[k])
    assert torch.equal(out[nk], sentinel[nk])


def test_learned_ssca_no_strip_selected(dev):
    """All scores below theta and a confident selector: nothing is computed and out is left untouched (the
    Stage 1 and Stage 2 grids exit on the device-side selection)."""
    N, Np = 1 << 15, 64
    x = gpu(sg.qpsk(N, 0.1, 8, 5.0, sg.rng_for(84, 0)), dev)
    sel = _fixed_selector(Np, np.zeros(Np, bool), dev)
    sentinel = torch.full((Np, N), complex(3.0, 1.0), dtype=torch.complex64, device=dev)
    out, mask, fb = SEL.ssca_learned(x, sel, out=sentinel.clone())
    assert not fb and int(mask.sum()) == 0
    assert torch.equal(out, sentinel)


@pytest.mark.parametrize("Np,strips", [(64, [2]), (64, [5, 9]), (16, [0, 7, 15]), (128, [1, 127])])
def test_learned_ssca_partial_selections(dev, Np, strips):
    """Selections that leave one subset of a pair (or, at Np = 16, of the single-subset kernel) unused: the
    chosen strips equal the full SSCA and every other row keeps its previous content."""
    N = 1 << 16
    x = gpu(sg.bpsk(N, 0.07, 6, 4.0, sg.rng_for(85, Np)), dev)
    keep = np.zeros(Np, bool)
    keep[strips] = True
    sel = _fixed_selector(Np, keep, dev)
    sentinel = torch.full((Np, N), complex(-2.0, 5.0), dtype=torch.complex64, device=dev)
    out, mask, fb = SEL.ssca_learned(x, sel, out=sentinel.clone())
    assert not fb and np.array_equal(mask.cpu().numpy().astype(bool), keep)
    full = scd.ssca(x, Np)
    k = torch.from_numpy(np.nonzero(keep)[0]).to(dev)
    nk = torch.from_numpy(np.nonzero(~keep)[0]).to(dev)
    assert torch.equal(out[k], full[k])
    assert torch.equal(out[nk], sentinel[nk])


def test_learned_ssca_fallback_forced(dev):
    N, Np = 1 << 14, 32
    x = gpu(sg.bpsk(N, 0.1, 8, 5.0, sg.rng_for(83, 0)), dev)
    keep = np.zeros(Np, bool)
    keep[:3] = True
    sel = _fixed_selector(Np, keep, dev)
    sel.conf_min = 1.0  # no selector output can be that confident: forces the full SSCA
    out, mask, fb = SEL.ssca_learned(x, sel)
    assert fb and int(mask.sum()) == Np
    assert torch.equal(out, scd.ssca(x, Np))


MODELS = os.path.join(os.path.dirname(SEL.__file__), "models")


def _model(Np, dev):
    path = f"{MODELS}/selector_np{Np}.npz"
    if not os.path.exists(path):
        pytest.skip(f"no trained model for Np={Np}")
    return SEL.Selector.load(path, dev)


def test_trained_selector_recall_on_held_out_cfg4(dev):
    """Held-out signals of the Np = 256, N = 2^18 selector workload (test-split seeds): strip recall >= 0.99
    with the committed model and its calibrated threshold (fallback counted as full recall), and fewer strips
    computed than the full SSCA, which is what the network gains over the method without it."""
    from synth import workloads as W
    sel = _model(256, dev)
    Np, N, count = 256, 1 << 18, 96
    tp = pos = work = 0
    for i in range(0, count, 8):
        xs = np.stack([W.cfg4_signal(j, N, "test")[1] for j in range(i, i + 8)]).astype(np.complex64)
        x = torch.from_numpy(xs).to(dev)
        lab, _ = SEL.strip_labels(scd.ssca(x, Np))
        feat = SEL.features(x, Np)
        s = sel.scores(feat).cpu().numpy()
        lab = lab.cpu().numpy() > 0.5
        conf = np.min(np.maximum(s, 1 - s), axis=1)
        chosen = s >= sel.theta
        chosen[conf < sel.conf_min] = True
        tp += (chosen & lab).sum()
        pos += lab.sum()
        work += chosen.sum()
    recall = tp / max(1, pos)
    assert recall >= 0.99, recall
    assert work < count * Np


def test_combined_workload_split_bf16_learned(dev):
    """The combined form on signals of the cfg-5 recipe (uneven lengths 2^14..2^20; Np = 64 for even indices,
    128 for odd): split-BF16 + learned selection + fallback. Every selected strip equals the full split-BF16
    SSCA's, the recall over the labels of the full FP32 SSCA is >= 0.99 for each Np, and the split-BF16 strips
    stay within 1e-3 of the FP64 oracle."""
    from synth import workloads as W
    sels = {64: _model(64, dev), 128: _model(128, dev)}
    tp = {64: 0, 128: 0}
    pos = {64: 0, 128: 0}
    for i in range(16):
        c = W.cfg5_signal(i)
        Np = c["Np"]
        assert Np == (64 if i % 2 == 0 else 128)
        x = torch.from_numpy(c["x"].astype(np.complex64)).to(dev)
        out, mask, fb = SEL.ssca_learned(x, sels[Np], precision="split_bf16")
        full32 = scd.ssca(x, Np)
        full16 = scd.ssca(x, Np, precision="split_bf16")
        m = mask.cpu().numpy().astype(bool)
        lab = SEL.strip_labels(full32)[0].cpu().numpy()[0] > 0.5
        tp[Np] += (m & lab).sum()
        pos[Np] += lab.sum()
        k = torch.from_numpy(np.nonzero(m)[0]).to(dev)
        assert torch.equal(out[k], full16[k]), i
        if m.any():
            kk = int(np.nonzero(m)[0][0])
            ref = O.ssca_strip(f64(c["x"]), Np, sg.hamming(Np).astype(np.float32).astype(np.float64), kk)
            g = out[kk].cpu().numpy()
            assert np.abs(g - ref).max() <= 1e-3 * np.abs(ref).max(), i
    for Np in (64, 128):
        assert tp[Np] / max(1, pos[Np]) >= 0.99, Np


def _random_selector(Np, dev, seed):
    """A selector with non-zero random weights, biases and feature statistics (not trained)."""
    rng = np.random.default_rng(seed)
    p = SEL.init_params(Np, seed=seed)
    for name in ("b1", "b2", "b3"):
        off, size = SEL.layout(Np)[name]
        p[off:off + size] = rng.standard_normal(size) * 0.3
    mu = rng.standard_normal(2 * Np).astype(np.float32)
    sigma = rng.uniform(0.5, 2.0, 2 * Np).astype(np.float32)
    return SEL.Selector(Np, p, mu, sigma, theta=0.5, conf_min=0.6).to(dev)


@pytest.mark.parametrize("Np,which", [(64, "trained"), (128, "trained"), (256, "trained"), (64, "random"),
                                      (128, "random")])
def test_fused_selector_chain_matches_reference(dev, Np, which):
    """The fused inference chain of the learned form (raw features -> PSD centring and standardisation inside the
    first layer -> bf16 GEMVs -> sigmoid -> threshold -> fallback), run alone by scd_selector_run, against the
    FP64 reference of the same chain on the GPU's own features: scores element by element within the bf16
    bound; mask and fallback equal to thresholding those scores; and scd_ssca_learned's mask equal to it."""
    from synth import workloads as W
    sel = _model(Np, dev) if which == "trained" else _random_selector(Np, dev, 7 + Np)
    P = _params_dict(sel.params.cpu().numpy(), Np)
    mu, sigma = sel.mu.cpu().numpy().astype(np.float64), sel.sigma.cpu().numpy().astype(np.float64)
    for i in range(4):
        xs = W.selector_signal(i, "test", emin=15, emax=16)[1] if Np < 256 else W.cfg4_signal(i, 1 << 16, "test")[1]
        x = gpu(xs, dev)
        scores, mask, conf, fell = SEL.run_selector(x, sel)
        feat = SEL.features(x, Np).cpu().numpy()[0].astype(np.float64)  # PSD part centred, as the chain centres it
        f = (feat - mu) / sigma
        cache = LR.mlp_forward(P, f[None, :], bf16=True)
        # |dz| <= 8 * 2^-8 * (abs-sum scale of the last layer); the sigmoid's slope is at most 1/4
        zscale = np.abs(_bf(cache["h2"])) @ np.abs(_bf(P["W3"])).T + np.abs(P["b3"])
        got = scores.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - cache["s"][0]) <= 0.25 * 8 * 2.0 ** -8 * zscale[0] + 1e-6), (i, Np, which)
        m = mask.cpu().numpy().astype(bool)
        c = float(np.min(np.maximum(got, 1 - got)))
        assert abs(float(conf.item()) - c) <= 1e-7
        fb = bool(fell.item())
        assert fb == (c < sel.conf_min)
        assert np.array_equal(m, np.ones(Np, bool) if fb else got >= sel.theta)
        _, m2, fb2 = SEL.ssca_learned(x, sel)
        assert np.array_equal(m2.cpu().numpy().astype(bool), m) and fb2 == fb
