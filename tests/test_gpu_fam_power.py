"""The FAM power form (scd_fam_power_ex): the kernel's |S|^2 over -P/4 <= q_c < P/4 equals, bit for bit, the paper's
view taken from the complex grid the same kernels compute, and matches the oracle's view of its FP64 FAM."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2506_18003_amd as scd  # noqa: E402
from oracle import scd_oracle as O  # noqa: E402
from synth import signals as sg  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("Np,L,P", [(16, 4, 4), (32, 8, 32), (64, 16, 128), (256, 64, 32), (16, 1, 1024), (64, 8, 256)])
def test_fam_power_equals_view_of_complex_grid(dev, Np, L, P):
    x = sg.bpsk(P * L, 0.07, 6, 3.0, sg.rng_for(97, Np + P)).astype(np.complex64)
    xt = torch.from_numpy(x).to(dev)
    pw = scd.fam_power(xt, Np, L, P)
    assert pw.shape == (Np, Np, P // 2)
    assert torch.equal(pw, scd.fam_paper_view(scd.fam(xt, Np, L, P)))
    w = sg.hamming(Np).astype(np.float32).astype(np.float64)
    ref = O.fam_paper_view(O.fam(x.astype(np.complex128), Np, L, P, w))
    assert np.abs(pw.cpu().numpy() - ref).max() <= 1e-5 * ref.max()


def test_fam_power_batch_strides(dev):
    Np, L, P = 64, 16, 64
    xs = np.stack([sg.qpsk(P * L + 100, 0.1, 8, 0.0, sg.rng_for(98, b)) for b in range(3)]).astype(np.complex64)
    xt = torch.from_numpy(xs).to(dev)[:, : P * L]  # rows at a stride longer than one signal
    pw = scd.fam_power(xt, Np, L, P)
    for b in range(3):
        assert torch.equal(pw[b], scd.fam_power(xt[b].contiguous(), Np, L, P)), b
