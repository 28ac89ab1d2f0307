"""GPU round trips of the selector model lifecycle (scd_model_create / save / load / read / selector /
destroy) through the C ABI, and the learned SSCA run from a loaded model file."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2506_18003_amd import selector as SEL  # noqa: E402
from synth import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
MODELS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2506_18003_amd", "models")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _arrays(Np):
    s = SEL.Selector.load(os.path.join(MODELS, f"selector_np{Np}.npz"))
    return s, np.asarray(s.params, np.float32), np.asarray(s.mu, np.float32), np.asarray(s.sigma, np.float32)


@pytest.mark.parametrize("Np", [64, 128, 256])
def test_create_read_save_load_round_trip(dev, tmp_path, Np):
    s, p, mu, sg = _arrays(Np)
    with torch.cuda.device(dev):
        m = SEL.Model.create(Np, p, mu, sg, s.theta, s.conf_min)
        rp, rmu, rsg = m.read()
        assert np.array_equal(rp, p) and np.array_equal(rmu, mu) and np.array_equal(rsg, sg)
        c = m.c_struct()
        assert (c.Np, c.theta, c.conf_min) == (Np, np.float32(s.theta), np.float32(s.conf_min))
        assert c.params % 16 == 0 and c.mu == c.params + 4 * p.size and c.sigma == c.mu + 8 * Np
        path = tmp_path / "m.scdm"
        m.save(str(path))
        # The saved file is byte-identical to the committed one written from the same arrays.
        assert path.read_bytes() == open(os.path.join(MODELS, f"selector_np{Np}.scdm"), "rb").read()
        m2 = SEL.Model.load(str(path))
        for a, b in zip(m2.read(), (p, mu, sg)):
            assert np.array_equal(a, b)
        assert (m2.Np, m2.theta, m2.conf_min) == (Np, float(np.float32(s.theta)), float(np.float32(s.conf_min)))
        m.close()
        m2.close()
        m2.close()  # closing twice is harmless


def test_learned_ssca_from_loaded_model_matches_selector_arrays(dev):
    """scd_ssca_learned with the scd_selector view of a model loaded from its committed file gives the same
    output rows, mask and fallback flag, bit for bit, as with the same arrays held in torch tensors."""
    Np = 64
    s, _, _, _ = _arrays(Np)
    sel_t = s.to(dev)
    with torch.cuda.device(dev):
        m = SEL.Model.load(os.path.join(MODELS, f"selector_np{Np}.scdm"))
        for i in range(3):
            x = torch.from_numpy(W.selector_signal(i, "test", emin=16, emax=16)[1].astype(np.complex64)).to(dev)
            N = x.shape[0]
            o1 = torch.zeros(Np, N, dtype=torch.complex64, device=dev)
            o2 = torch.zeros(Np, N, dtype=torch.complex64, device=dev)
            _, k1, f1 = SEL.ssca_learned(x, sel_t, out=o1)
            _, k2, f2 = SEL.ssca_learned(x, m, out=o2)
            assert torch.equal(k1, k2) and f1 == f2, i
            assert torch.equal(o1, o2), i
        m.close()
