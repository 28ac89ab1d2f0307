"""scd_ssca_noalloc, the entry point that allocates nothing (its scratch is a file-scope device array), called
through the C ABI: equal bit for bit to scd_ssca_ex on the same inputs, on calls in a row with shrinking
sizes (the second call finds the first one's tables and intermediate in the shared scratch), and rejecting a
grid beyond its scratch before any device work."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2506_18003_amd as scd  # noqa: E402
from paper_2506_18003_amd import _lib  # noqa: E402
from synth import signals as sg  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _noalloc(x, Np, win, out):
    o = _lib.ScdOpts()
    o.stream = torch.cuda.current_stream(x.device).cuda_stream
    return _lib.lib().scd_ssca_noalloc(x.data_ptr(), x.shape[0], Np, win.data_ptr(), out.data_ptr(), ctypes.byref(o))


def test_noalloc_matches_ssca_ex_on_calls_in_a_row(dev):
    assert _lib.lib().scd_ssca_noalloc_limit() == 64 << 20
    cases = [(1 << 17, 64), (1 << 14, 32), (1024, 16), (1 << 15, 256)]  # 8 Np N: 64 MiB (the limit), then smaller
    for i, (N, Np) in enumerate(cases):
        x = torch.from_numpy(sg.qpsk(N, 0.11, 8, 5.0, sg.rng_for(120, i)).astype(np.complex64)).to(dev)
        w = torch.from_numpy(sg.hamming(Np).astype(np.float32)).to(dev)
        out = torch.full((Np, N), float("nan"), dtype=torch.complex64, device=dev)
        with torch.cuda.device(dev):
            _lib.check(_noalloc(x, Np, w, out))
        ref = scd.ssca(x, Np, win=w)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (N, Np)


def test_noalloc_rejects_a_grid_beyond_its_scratch(dev):
    N, Np = 1 << 18, 64  # 8 Np N = 128 MiB
    x = torch.zeros(N, dtype=torch.complex64, device=dev)
    w = torch.ones(Np, dtype=torch.float32, device=dev)
    out = torch.zeros(8, dtype=torch.complex64, device=dev)
    with torch.cuda.device(dev):
        assert _noalloc(x, Np, w, out) == _lib.SCD_ERR_SIZE
    assert b"scratch" in _lib.lib().scd_last_error()
