"""SSCA of blocks of a longer signal (scd_ssca_block_ex): each block matches the oracle's ssca_block, whose
frames at the block edges read the neighbouring samples, over the single-subset and paired Stage 1 and at
the signal's left edge, middle and right edge; a whole-signal block is scd_ssca bit for bit."""
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


@pytest.mark.parametrize("length,N,Np,offset", [(4096, 1024, 64, 0), (4096, 1024, 64, 1024), (4096, 1024, 16, 3072),
                                                (1 << 16, 1 << 14, 32, 1 << 15), (1 << 18, 1 << 17, 64, 1 << 17)])
def test_block_matches_oracle(dev, length, N, Np, offset):
    x = sg.qpsk(length, 0.1, 6, 3.0, sg.rng_for(110, length + offset + Np)).astype(np.complex64)
    w = sg.hamming(Np).astype(np.float32)
    S = scd.ssca_block(torch.from_numpy(x).to(dev), offset, N, Np, win=torch.from_numpy(w).to(dev)).cpu().numpy()
    ref = O.ssca_block(x.astype(np.complex128), offset, N, Np, w.astype(np.float64))
    assert np.abs(S - ref).max() <= TOL_FP32 * np.abs(ref).max()


def test_whole_signal_block_is_ssca(dev):
    x = torch.from_numpy(sg.bpsk(1 << 15, 0.07, 5, 2.0, sg.rng_for(111, 0)).astype(np.complex64)).to(dev)
    assert torch.equal(scd.ssca_block(x, 0, 1 << 15, 64), scd.ssca(x, 64))


def test_stream_of_blocks(dev):
    x = sg.msk(4 * 4096, 0.12, 8, 5.0, sg.rng_for(112, 0)).astype(np.complex64)
    xt = torch.from_numpy(x).to(dev)
    w = sg.hamming(32).astype(np.float64)
    offs = []
    for off, S in scd.ssca_stream(xt, 4096, 32):
        ref = O.ssca_block(x.astype(np.complex128), off, 4096, 32, w)
        assert np.abs(S.cpu().numpy() - ref).max() <= TOL_FP32 * np.abs(ref).max(), off
        offs.append(off)
    assert offs == [0, 4096, 8192, 12288]


@pytest.mark.parametrize("nb,slots,outputs", [(9, 4, 2), (5, 3, 1), (2, 4, 3), (1, 4, 2)])
def test_receiver_streams_host_blocks(dev, nb, slots, outputs):
    """Blocks pushed from pinned host memory through the receiver's fixed ring of device slots (more blocks
    than slots, so slots and output buffers are reused) come back in order, equal bit for bit to ssca_block of
    the whole signal resident on the device (copy and estimate overlap on two streams)."""
    N, Np = 4096, 64
    x = sg.qpsk(nb * N, 0.1, 8, 4.0, sg.rng_for(113, nb + slots), ).astype(np.complex64)
    full = torch.from_numpy(x).to(dev)
    rx = scd.SscaReceiver(N, Np, dev, slots=slots, outputs=outputs)
    got = []
    for b in range(nb):
        blk = torch.empty(N, dtype=torch.complex64, pin_memory=True)
        blk.copy_(torch.from_numpy(x[b * N:(b + 1) * N]))
        r = rx.push(blk)
        if r is not None:
            got.append((r[0], r[1].clone()))  # the output buffer is reused `outputs` estimates later
    off, S = rx.finish()
    got.append((off, S.clone()))
    torch.cuda.synchronize()
    assert [o for o, _ in got] == [b * N for b in range(nb)]
    for off, S in got:
        assert torch.equal(S, scd.ssca_block(full, off, N, Np)), off
    assert rx.ring_bytes == 8 * (slots * N + 2 * Np)  # fixed device memory, whatever the stream length
