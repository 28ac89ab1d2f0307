"""Spectral correlation density (FAM and SSCA) on AMD MI355X.

Thin Python layer over the C ABI in include/scd.h. torch supplies device memory and the current stream;
every numerical step runs in the library's HIP kernels (``libscd.so``), and the calls fail loudly if that
library is missing.

    S = ssca(x, Np)                 # x: complex64 CUDA tensor [N] or [B, N]  ->  [Np, N] or [B, Np, N]
    S = fam(x, Np, L, P)            # x: [P*L] or [B, P*L]                      ->  [Np, Np, P] or [B, Np, Np, P]
    f, alpha = ssca_coords(Np, N)   # the (f, alpha) of each SSCA cell
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import PRECISIONS, ScdError  # noqa: F401

__all__ = ["ssca", "ssca_block", "ssca_stream", "SscaReceiver", "ssca_cross", "ssca_batch", "ssca_stage1", "ssca_stage2", "fam", "fam_cross", "fam_power", "ssca_coords", "fam_coords", "fam_paper_view", "hamming", "ScdError",
           "ssca_workspace_size", "fam_workspace_size", "shutdown", "version"]

_win_cache: dict = {}


def hamming(n: int) -> np.ndarray:
    """Symmetric Hamming window 0.54 - 0.46 cos(2 pi j / (n - 1)), float64."""
    j = np.arange(n)
    return 0.54 - 0.46 * np.cos(2.0 * np.pi * j / (n - 1))


def _torch():
    import torch
    return torch


def _window(win, Np, device):
    torch = _torch()
    if win is None:
        key = (Np, str(device))
        w = _win_cache.get(key)
        if w is None:
            w = torch.tensor(hamming(Np), dtype=torch.float32, device=device)
            _win_cache[key] = w
        return w
    if not isinstance(win, torch.Tensor):
        win = torch.tensor(np.asarray(win), dtype=torch.float32, device=device)
    if win.dtype != torch.float32 or win.device != device or not win.is_contiguous() or win.numel() != Np:
        raise ValueError(f"win must be a contiguous float32 tensor of {Np} values on {device}")
    return win


def _check_x(x):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or x.dtype != torch.complex64 or not x.is_cuda:
        raise TypeError("x must be a complex64 CUDA tensor")
    if x.dim() not in (1, 2):
        raise ValueError("x must be [N] or [B, N]")
    if x.stride(-1) != 1:
        raise ValueError("x must be contiguous along its last axis")


def _opts(x, precision, batch, x_stride, out_stride, workspace):
    torch = _torch()
    o = _lib.ScdOpts()
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.batch = batch
    o.x_stride = x_stride
    o.out_stride = out_stride
    o.stream = torch.cuda.current_stream(x.device).cuda_stream
    if workspace is not None:
        if not workspace.is_cuda or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous CUDA tensor")
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return o


def ssca(x, Np: int, win=None, precision="fp32", out=None, workspace=None):
    """SSCA estimate S[k][q] (k < Np, q < N) of each signal in x; see scd_ssca in include/scd.h."""
    torch = _torch()
    _check_x(x)
    N = x.shape[-1]
    B = 1 if x.dim() == 1 else x.shape[0]
    w = _window(win, Np, x.device)
    shape = (Np, N) if x.dim() == 1 else (B, Np, N)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=x.device)
    elif tuple(out.shape) != shape or out.dtype != torch.complex64 or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous complex64 tensor of shape {shape}")
    xs = x.stride(0) if x.dim() == 2 else 0
    o = _opts(x, precision, B, xs, Np * N, workspace)
    with torch.cuda.device(x.device):
        _lib.check(_lib.lib().scd_ssca_ex(x.data_ptr(), N, Np, w.data_ptr(), out.data_ptr(), ctypes.byref(o)))
    return out


def ssca_strips(x, Np: int, strips, win=None, precision="fp32", out=None, workspace=None):
    """SSCA of each signal in x restricted to the listed strips (distinct k in [0, Np)); only those rows of out
    are written. One GPU's share of an SSCA split by strips; see scd_ssca_strips in include/scd.h."""
    torch = _torch()
    _check_x(x)
    N = x.shape[-1]
    B = 1 if x.dim() == 1 else x.shape[0]
    w = _window(win, Np, x.device)
    shape = (Np, N) if x.dim() == 1 else (B, Np, N)
    if out is None:
        out = torch.zeros(shape, dtype=torch.complex64, device=x.device)
    elif tuple(out.shape) != shape or out.dtype != torch.complex64 or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous complex64 tensor of shape {shape}")
    ks = np.ascontiguousarray(np.asarray(list(strips), dtype=np.int32).reshape(-1))
    xs = x.stride(0) if x.dim() == 2 else 0
    o = _opts(x, precision, B, xs, Np * N, workspace)
    with torch.cuda.device(x.device):
        _lib.check(_lib.lib().scd_ssca_strips(x.data_ptr(), N, Np, w.data_ptr(), ks.ctypes.data, int(ks.size),
                                              out.data_ptr(), ctypes.byref(o)))
    return out


def ssca_block(x, offset: int, N: int, Np: int, win=None, out=None, workspace=None):
    """SSCA of the block [offset, offset + N) of the signal x ([len] complex64), with frames at the block's
    edges reading the neighbouring samples; see scd_ssca_block_ex."""
    torch = _torch()
    _check_x(x)
    if x.dim() != 1:
        raise ValueError("x must be one signal [len]")
    w = _window(win, Np, x.device)
    if out is None:
        out = torch.empty(Np, N, dtype=torch.complex64, device=x.device)
    elif tuple(out.shape) != (Np, N) or out.dtype != torch.complex64 or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous complex64 tensor of shape {(Np, N)}")
    o = _opts(x, "fp32", 1, 0, Np * N, workspace)
    with torch.cuda.device(x.device):
        _lib.check(_lib.lib().scd_ssca_block_ex(x.data_ptr(), x.shape[0], offset, N, Np, w.data_ptr(), out.data_ptr(),
                                                ctypes.byref(o)))
    return out


def ssca_stream(x, N: int, Np: int, win=None):
    """Consecutive blocks of N samples of a resident signal x, each estimated with its true neighbours
    (ssca_block at offsets 0, N, 2N, ...); yields (offset, S) in order, enqueued on the current stream."""
    for off in range(0, x.shape[-1] - N + 1, N):
        yield off, ssca_block(x, off, N, Np, win=win)


class SscaReceiver:
    """Continuous streaming SSCA of blocks of N samples arriving from the host (scd_receiver_* in
    include/scd.h): fixed device memory, a ring of `slots` device blocks owned by the library and `outputs`
    output tensors owned here and reused in rotation. push(block) waits until the ring slot it reuses is free (the
    estimate `slots` - 1 blocks back has finished: the ring bounds how far the host runs ahead), copies one
    pinned complex64 CPU tensor [N] on the receiver's copy stream and enqueues the estimate of the block before it
    on the current stream; it returns (offset, S [Np, N]) for that block (None for the first). finish() returns
    the last block's estimate.
    A returned S is overwritten `outputs` estimates later, in stream order: read or copy it before then. A pushed
    host block must not be modified until wait_copy() (or finish()) has returned; this object keeps a reference
    to the last `slots` blocks meanwhile. The estimates equal ssca_block of the whole signal resident on the
    device, bit for bit."""

    def __init__(self, N: int, Np: int, device, win=None, slots: int = 4, outputs: int = 2):
        torch = _torch()
        self.N, self.Np, self.device = N, Np, torch.device(device)
        self.win = _window(win, Np, self.device)
        with torch.cuda.device(self.device):
            self.out = [torch.empty(Np, N, dtype=torch.complex64, device=self.device) for _ in range(outputs)]
            ptrs = (ctypes.c_void_p * outputs)(*[o.data_ptr() for o in self.out])
            self._h = ctypes.c_void_p()
            stream = torch.cuda.current_stream(self.device).cuda_stream
            _lib.check(_lib.lib().scd_receiver_create(N, Np, self.win.data_ptr(), slots, ptrs, outputs, stream,
                                                      ctypes.byref(self._h)))
        self.slots = slots
        self.ring_bytes = 8 * (slots * N + 2 * Np)
        self._hold = []

    def _result(self, idx, off):
        return None if idx.value < 0 else (off.value, self.out[idx.value])

    def push(self, block):
        """Enqueue one host block; returns the estimate of the block before it, or None for the first."""
        torch = _torch()
        if block.shape != (self.N,) or block.dtype != torch.complex64 or block.device.type != "cpu":
            raise ValueError(f"a block is a complex64 CPU tensor of {self.N} samples")
        if not block.is_contiguous():
            raise ValueError("a block must be contiguous")
        idx, off = ctypes.c_int(-1), ctypes.c_int64(0)
        _lib.check(_lib.lib().scd_receiver_push(self._h, block.data_ptr(), ctypes.byref(idx), ctypes.byref(off)))
        self._hold.append(block)
        if len(self._hold) > self.slots:
            self._hold.pop(0)
        return self._result(idx, off)

    def wait_copy(self):
        _lib.check(_lib.lib().scd_receiver_wait_copy(self._h))

    def finish(self):
        """Estimate the last block (zeros after it) and wait for every copy."""
        idx, off = ctypes.c_int(-1), ctypes.c_int64(0)
        _lib.check(_lib.lib().scd_receiver_finish(self._h, ctypes.byref(idx), ctypes.byref(off)))
        self._hold.clear()
        return self._result(idx, off)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(_lib.lib().scd_receiver_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ssca_cross(x, y, Np: int, win=None, conjugate=False, out=None, workspace=None):
    """Cross SCD of x and y by SSCA (conj(y[n]) in the channel-data product; y[n] with conjugate=True);
    x and y alike ([N] or [B, N]); see scd_ssca_cross_ex."""
    torch = _torch()
    _check_x(x)
    _check_x(y)
    if y.shape != x.shape or y.device != x.device or (x.dim() == 2 and y.stride(0) != x.stride(0)):
        raise ValueError("y must have x's shape, device and row stride")
    N = x.shape[-1]
    B = 1 if x.dim() == 1 else x.shape[0]
    w = _window(win, Np, x.device)
    shape = (Np, N) if x.dim() == 1 else (B, Np, N)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=x.device)
    elif tuple(out.shape) != shape or out.dtype != torch.complex64 or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous complex64 tensor of shape {shape}")
    xs = x.stride(0) if x.dim() == 2 else 0
    o = _opts(x, "fp32", B, xs, Np * N, workspace)
    with torch.cuda.device(x.device):
        _lib.check(_lib.lib().scd_ssca_cross_ex(x.data_ptr(), y.data_ptr(), N, Np, w.data_ptr(), int(bool(conjugate)),
                                                out.data_ptr(), ctypes.byref(o)))
    return out


def ssca_batch(items, precision="fp32", workspace=None):
    """SSCA of several signals of any lengths and channel counts in one call; see scd_ssca_batch.

    `items` is a list of dicts with keys x (complex64 CUDA tensor [N]) and Np, and optionally win, out and
    selector (a selector.Selector: only the strips it picks are computed, the other rows of out stay zero).
    Returns one (out, mask) pair per item; mask is the uint8 [Np] selection, None for items without a selector.
    """
    torch = _torch()
    if not items:
        return []
    dev = items[0]["x"].device
    arr = (_lib.ScdSscaItem * len(items))()
    keep, res = [], []
    for i, it in enumerate(items):
        x, Np = it["x"], int(it["Np"])
        _check_x(x)
        if x.dim() != 1 or x.device != dev:
            raise ValueError("every item's x must be one signal [N] on the same device")
        N = x.shape[-1]
        w = _window(it.get("win"), Np, dev)
        sel = it.get("selector")
        out = it.get("out")
        if out is None:
            out = (torch.zeros if sel is not None else torch.empty)(Np, N, dtype=torch.complex64, device=dev)
        elif tuple(out.shape) != (Np, N) or out.dtype != torch.complex64 or not out.is_contiguous():
            raise ValueError(f"item {i}: out must be a contiguous complex64 tensor of shape {(Np, N)}")
        mask = torch.empty(Np, dtype=torch.uint8, device=dev) if sel is not None else None
        arr[i].x, arr[i].N, arr[i].Np, arr[i].win, arr[i].out = x.data_ptr(), N, Np, w.data_ptr(), out.data_ptr()
        if sel is not None:
            cs = sel.c_struct()
            keep.append(cs)
            arr[i].selector = ctypes.pointer(cs)
            arr[i].mask = mask.data_ptr()
        keep.append(w)
        res.append((out, mask))
    o = _opts(items[0]["x"], precision, 1, 0, 0, workspace)
    with torch.cuda.device(dev):
        _lib.check(_lib.lib().scd_ssca_batch(arr, len(items), ctypes.byref(o)))
    return res


def ssca_stage1(x, Np: int, inter, win=None, precision="fp32"):
    """Stage 1 of SSCA_2DFFT into `inter` (complex64, Np*N elements per signal); see scd_ssca_stage1_ex."""
    torch = _torch()
    _check_x(x)
    N = x.shape[-1]
    B = 1 if x.dim() == 1 else x.shape[0]
    w = _window(win, Np, x.device)
    if inter.dtype != torch.complex64 or not inter.is_contiguous() or inter.numel() != B * Np * N:
        raise ValueError("inter must be a contiguous complex64 tensor of batch*Np*N elements")
    o = _opts(x, precision, B, x.stride(0) if x.dim() == 2 else 0, Np * N, None)
    with torch.cuda.device(x.device):
        _lib.check(_lib.lib().scd_ssca_stage1_ex(x.data_ptr(), N, Np, w.data_ptr(), inter.data_ptr(),
                                                 ctypes.byref(o)))
    return inter


def ssca_stage2(inter, N: int, Np: int, out):
    """Stage 2 of SSCA_2DFFT from `inter` into out ([.., Np, N] complex64); see scd_ssca_stage2_ex."""
    torch = _torch()
    B = inter.numel() // (Np * N)
    if out.dtype != torch.complex64 or not out.is_contiguous() or out.numel() != B * Np * N:
        raise ValueError("out must be a contiguous complex64 tensor of batch*Np*N elements")
    o = _opts(inter, "fp32", B, Np * N, Np * N, None)
    with torch.cuda.device(inter.device):
        _lib.check(_lib.lib().scd_ssca_stage2_ex(inter.data_ptr(), N, Np, out.data_ptr(), ctypes.byref(o)))
    return out


def fam(x, Np: int, L: int | None = None, P: int | None = None, win=None, out=None, workspace=None):
    """FAM estimate S[k][l][q] of each signal in x (default L = Np/4, P = len/L); see scd_fam."""
    torch = _torch()
    _check_x(x)
    if L is None:
        L = Np // 4
    if P is None:
        P = x.shape[-1] // L
    if x.shape[-1] < P * L:
        raise ValueError(f"x has {x.shape[-1]} samples, FAM needs P*L = {P * L}")
    B = 1 if x.dim() == 1 else x.shape[0]
    w = _window(win, Np, x.device)
    shape = (Np, Np, P) if x.dim() == 1 else (B, Np, Np, P)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=x.device)
    elif tuple(out.shape) != shape or out.dtype != torch.complex64 or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous complex64 tensor of shape {shape}")
    xs = x.stride(0) if x.dim() == 2 else 0
    o = _opts(x, "fp32", B, xs, Np * Np * P, workspace)
    with torch.cuda.device(x.device):
        _lib.check(_lib.lib().scd_fam_ex(x.data_ptr(), Np, L, P, w.data_ptr(), out.data_ptr(), ctypes.byref(o)))
    return out


def fam_cross(x, y, Np: int, L: int | None = None, P: int | None = None, win=None, conjugate=False, out=None,
              workspace=None):
    """Cross FAM of x and y (conj(Y_T) in the product; Y_T itself with conjugate=True), x and y alike;
    see scd_fam_cross_ex."""
    torch = _torch()
    _check_x(x)
    _check_x(y)
    if y.shape != x.shape or y.device != x.device or (x.dim() == 2 and y.stride(0) != x.stride(0)):
        raise ValueError("y must have x's shape, device and row stride")
    if L is None:
        L = Np // 4
    if P is None:
        P = x.shape[-1] // L
    if x.shape[-1] < P * L:
        raise ValueError(f"x has {x.shape[-1]} samples, FAM needs P*L = {P * L}")
    B = 1 if x.dim() == 1 else x.shape[0]
    w = _window(win, Np, x.device)
    shape = (Np, Np, P) if x.dim() == 1 else (B, Np, Np, P)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=x.device)
    elif tuple(out.shape) != shape or out.dtype != torch.complex64 or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous complex64 tensor of shape {shape}")
    xs = x.stride(0) if x.dim() == 2 else 0
    o = _opts(x, "fp32", B, xs, Np * Np * P, workspace)
    with torch.cuda.device(x.device):
        _lib.check(_lib.lib().scd_fam_cross_ex(x.data_ptr(), y.data_ptr(), Np, L, P, w.data_ptr(),
                                               int(bool(conjugate)), out.data_ptr(), ctypes.byref(o)))
    return out


def fam_power(x, Np: int, L: int | None = None, P: int | None = None, win=None, out=None, workspace=None):
    """The paper's FAM output, |S[k][l][q]|^2 over -P/4 <= q_c < P/4 ([.., Np, Np, P/2] float32, bins in the order of
    fam_paper_view), written by the FAM kernel itself; see scd_fam_power_ex."""
    torch = _torch()
    _check_x(x)
    if L is None:
        L = Np // 4
    if P is None:
        P = x.shape[-1] // L
    if x.shape[-1] < P * L:
        raise ValueError(f"x has {x.shape[-1]} samples, FAM needs P*L = {P * L}")
    B = 1 if x.dim() == 1 else x.shape[0]
    w = _window(win, Np, x.device)
    shape = (Np, Np, P // 2) if x.dim() == 1 else (B, Np, Np, P // 2)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=x.device)
    elif tuple(out.shape) != shape or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous float32 tensor of shape {shape}")
    xs = x.stride(0) if x.dim() == 2 else 0
    o = _opts(x, "fp32", B, xs, Np * Np * (P // 2), workspace)
    with torch.cuda.device(x.device):
        _lib.check(_lib.lib().scd_fam_power_ex(x.data_ptr(), Np, L, P, w.data_ptr(), out.data_ptr(),
                                               ctypes.byref(o)))
    return out


def ssca_workspace_size(N: int, Np: int, batch: int = 1) -> int:
    v = ctypes.c_size_t()
    _lib.check(_lib.lib().scd_ssca_workspace_size(N, Np, batch, ctypes.byref(v)))
    return v.value


def fam_workspace_size(Np: int, L: int, P: int, batch: int = 1) -> int:
    v = ctypes.c_size_t()
    _lib.check(_lib.lib().scd_fam_workspace_size(Np, L, P, batch, ctypes.byref(v)))
    return v.value


def shutdown() -> None:
    _lib.lib().scd_shutdown()


def version() -> int:
    return _lib.lib().scd_version()


def _signed(n: int) -> np.ndarray:
    i = np.arange(n)
    return ((i + n // 2) % n) - n // 2


def ssca_coords(Np: int, N: int):
    """(f, alpha) arrays [Np, N] of the SSCA cells (f_s = 1): alpha = f_k + q_c/N, f = (f_k - q_c/N)/2."""
    fk = (_signed(Np) / Np)[:, None]
    qn = (_signed(N) / N)[None, :]
    return (fk - qn) / 2.0, fk + qn


def fam_coords(Np: int, L: int, P: int):
    """(f, alpha) arrays [Np, Np, P] of the FAM cells: f = (f_k + f_l)/2, alpha = f_k - f_l + q_c/(P L)."""
    fk = _signed(Np) / Np
    qa = _signed(P) / (P * L)
    f = np.broadcast_to(((fk[:, None] + fk[None, :]) / 2.0)[:, :, None], (Np, Np, P))
    a = (fk[:, None] - fk[None, :])[:, :, None] + qa[None, None, :]
    return f, a


def fam_paper_view(S):
    """|S|^2 over the central half of the alpha-offset axis (-P/4 <= q_c < P/4), natural order
    [0..P/4-1, -P/4..-1]; the bins the paper's FFT2 stage keeps. A view of a complex grid already computed
    (re^2 + im^2, each operation rounded to FP32, as fam_power's kernel computes it)."""
    torch = _torch()
    P = S.shape[-1]
    idx = torch.cat([torch.arange(0, P // 4), torch.arange(P - P // 4, P)]).to(S.device)
    T = S.index_select(-1, idx)
    return T.real.square() + T.imag.square()
