"""scd_ssca_batch on the GPU: a ragged list of signals (different N and Np, with and without a learned
selection) gives, item by item, exactly what the single-signal entry points give on the same stream."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2506_18003_amd as scd  # noqa: E402
from paper_2506_18003_amd import selector as SEL  # noqa: E402
from synth import signals as sg  # noqa: E402

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _x(x, dev):
    return torch.as_tensor(np.ascontiguousarray(x).astype(np.complex64), device=dev)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_ragged_batch_equals_single_calls(dev, prec):
    sel = SEL.Selector.load(os.path.join(ROOT, "paper_2506_18003_amd", "models", "selector_np64.npz"), dev)
    specs = [  # (N, Np, signal, learned selection)
        (1 << 14, 32, sg.bpsk(1 << 14, 0.07, 6, 5.0, sg.rng_for(90, 0)), False),
        (1 << 16, 64, sg.qpsk(1 << 16, 0.12, 8, 3.0, sg.rng_for(90, 1)), True),
        (1024, 16, sg.msk(1024, 0.05, 8, 0.0, sg.rng_for(90, 2)), False),
        (1 << 15, 128, sg.noise(1 << 15, sg.rng_for(90, 3)), False),
        (1 << 14, 64, sg.bpsk(1 << 14, 0.2, 4, -5.0, sg.rng_for(90, 4)), True),
    ]
    items = [dict(x=_x(x, dev), Np=Np, selector=sel if learned else None) for N, Np, x, learned in specs]
    got = scd.ssca_batch(items, precision=prec)
    for i, (it, (out, mask)) in enumerate(zip(items, got)):
        if it["selector"] is None:
            assert mask is None
            assert torch.equal(out, scd.ssca(it["x"], it["Np"], precision=prec)), i
        else:
            ref, rmask, _ = SEL.ssca_learned(it["x"], sel, precision=prec)
            assert torch.equal(mask, rmask), i
            assert torch.equal(out, ref), i


def test_ragged_batch_bad_item_is_named(dev):
    x = _x(sg.noise(4096, sg.rng_for(91, 0)), dev)
    with pytest.raises(scd.ScdError, match="item 1"):
        scd.ssca_batch([dict(x=x, Np=32), dict(x=x, Np=8192)])
