"""scd_ssca_strips: the SSCA restricted to a list of strips (one GPU's share of an SSCA split by strips).

Listed rows equal the full call's to FP32 rounding and the FP64 oracle's strip (Eq. (6)-(7)) within 1e-4 of the
peak; unlisted rows keep the caller's values exactly. (A shorter list gives a smaller Stage-1 grid, for which the
launch may take the paired instead of the single-subset kernel or the reverse; their folds round differently.) Cases cover the single-subset and
paired Stage 1, both down-conversion forms, the split-BF16 MFMA Stage 1 with a pair count that is not a power of
two, N = 1024 (where Stage 1 alone is the transform), batches, and the empty and full lists."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2506_18003_amd as scd  # noqa: E402
from oracle import scd_oracle as O  # noqa: E402
from synth import signals as sg  # noqa: E402

pytestmark = pytest.mark.gpu
TOL_FP32 = 1e-4


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _x(N, seed, dev, batch=None):
    if batch is None:
        x = sg.qpsk(N, 0.1, 8, 5.0, sg.rng_for(96, seed))
    else:
        x = np.stack([sg.bpsk(N, 0.05 + 0.01 * b, 6, 3.0, sg.rng_for(96, seed + b)) for b in range(batch)])
    return torch.from_numpy(x.astype(np.complex64)).to(dev)


def _shard(Np, G, r):
    """Strips of GPU r of G: whole channel subsets (k = c mod Np/16) while G <= Np/16, else half subsets."""
    S = Np // 16
    if G <= S:
        return [k for k in range(Np) if (k % S) % G == r]
    per = Np // G
    c, h = r % S, r // S
    ks = [k for k in range(Np) if k % S == c]
    return ks[h * per:(h + 1) * per]


TOL_SAME = 1e-5  # two FP32 folds of the same sums: a few roundings apart


def _check_rows(out, full, sentinel, ks):
    Np = out.shape[-2]
    nk = [k for k in range(Np) if k not in set(ks)]
    if ks:
        a, b = out[..., ks, :], full[..., ks, :]
        assert float((a - b).abs().max() / b.abs().max()) <= TOL_SAME
    if nk:
        assert torch.equal(out[..., nk, :], sentinel[..., nk, :])


@pytest.mark.parametrize("N,Np,prec,ks", [
    (1 << 20, 64, "fp32", _shard(64, 8, 5)),           # single-subset Stage 1, half a subset
    (1 << 20, 64, "fp32", _shard(64, 4, 2)),           # one whole subset
    (1 << 18, 64, "fp32", [0, 7, 9, 62]),              # paired Stage 1, three subsets
    (1 << 16, 32, "fp32", [31]),
    (1 << 12, 128, "fp32", [5, 77, 100]),             # M2 = 4 < Np: per-frame down-conversion
    (1 << 16, 128, "split_bf16", [0, 9, 18, 26]),      # three of four subset pairs (grid rounded up)
    (1 << 16, 64, "split_bf16", [3, 4]),
    (1024, 32, "fp32", [5, 17, 30]),                   # N = 1024: listed rows copied out of Stage 1
])
def test_strips_equal_full_call(dev, N, Np, prec, ks):
    x = _x(N, len(ks) + Np, dev)
    full = scd.ssca(x, Np, precision=prec)
    sentinel = torch.full((Np, N), complex(7.0, -3.0), dtype=torch.complex64, device=dev)
    out = scd.ssca_strips(x, Np, ks, precision=prec, out=sentinel.clone())
    torch.cuda.synchronize()
    _check_rows(out, full, sentinel, ks)


def test_strips_against_oracle_at_full_size(dev):
    N, Np = 1 << 20, 64
    ks = _shard(64, 8, 3)
    x = _x(N, 1, dev)
    out = scd.ssca_strips(x, Np, ks).cpu().numpy()
    xh = x.cpu().numpy().astype(np.complex128)
    w = sg.hamming(Np).astype(np.float32).astype(np.float64)
    for k in (ks[0], ks[-1]):
        ref = O.ssca_strip(xh, Np, w, k)
        assert float(np.abs(out[k] - ref).max() / np.abs(ref).max()) <= TOL_FP32


def test_strips_batch_and_unsorted_list(dev):
    N, Np = 1 << 15, 64
    ks = [50, 3, 17, 40, 8]
    x = _x(N, 2, dev, batch=3)
    full = scd.ssca(x, Np)
    sentinel = torch.full((3, Np, N), complex(-1.0, 2.0), dtype=torch.complex64, device=dev)
    out = scd.ssca_strips(x, Np, ks, out=sentinel.clone())
    torch.cuda.synchronize()
    _check_rows(out, full, sentinel, ks)


def test_shards_cover_the_full_call(dev):
    N, Np, G = 1 << 17, 64, 8
    x = _x(N, 3, dev)
    full = scd.ssca(x, Np)
    out = torch.zeros(Np, N, dtype=torch.complex64, device=dev)
    seen = []
    for r in range(G):
        ks = _shard(Np, G, r)
        seen += ks
        scd.ssca_strips(x, Np, ks, out=out)
    torch.cuda.synchronize()
    assert sorted(seen) == list(range(Np))
    assert float((out - full).abs().max() / full.abs().max()) <= TOL_SAME


def test_empty_and_full_lists(dev):
    N, Np = 1 << 14, 32
    x = _x(N, 4, dev)
    sentinel = torch.full((Np, N), complex(1.0, 1.0), dtype=torch.complex64, device=dev)
    out = scd.ssca_strips(x, Np, [], out=sentinel.clone())
    torch.cuda.synchronize()
    assert torch.equal(out, sentinel)
    out = scd.ssca_strips(x, Np, range(Np), out=sentinel.clone())
    assert torch.equal(out, scd.ssca(x, Np))  # the full list launches the same kernels as scd_ssca


def test_strips_reject_other_precisions(dev):
    x = _x(1 << 14, 5, dev)
    for prec in ("split_fp16", "bf16"):
        with pytest.raises(scd.ScdError):
            scd.ssca_strips(x, 64, [1, 2], precision=prec)


def test_strips_batch_through_a_small_workspace(dev):
    """Three signals through a caller workspace that holds one intermediate (three chunks), with a selection."""
    N, Np = 1 << 15, 64
    ks = [2, 6, 33, 63]
    x = _x(N, 6, dev, batch=3)
    ws = torch.empty(Np * N, dtype=torch.complex64, device=dev)
    full = scd.ssca(x, Np)
    sentinel = torch.full((3, Np, N), complex(0.5, -0.5), dtype=torch.complex64, device=dev)
    out = scd.ssca_strips(x, Np, ks, out=sentinel.clone(), workspace=ws)
    torch.cuda.synchronize()
    _check_rows(out, full, sentinel, ks)


def test_strips_batch_at_n1024(dev):
    """N = 1024 (Stage 1 alone is the transform): each signal's listed rows come from the library's scratch."""
    N, Np = 1024, 64
    ks = [0, 17, 40, 63]
    x = _x(N, 7, dev, batch=3)
    full = scd.ssca(x, Np)
    sentinel = torch.full((3, Np, N), complex(4.0, 4.0), dtype=torch.complex64, device=dev)
    out = scd.ssca_strips(x, Np, ks, out=sentinel.clone())
    torch.cuda.synchronize()
    _check_rows(out, full, sentinel, ks)
