"""CPU-only checks of the C ABI: the library loads, exports every function include/scd.h declares, and
rejects bad arguments with the documented codes before touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_2506_18003_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(scd_[a-z_0-9]+)\s*\(", text, re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libscd.so not built")
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert "scd_ssca" in names and "scd_fam" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version(L):
    assert L.scd_version() >> 16 == 1


def _fake(addr):
    return ctypes.c_void_p(addr)


X, W, O = 0x10000000, 0x20000000, 0x30000000


@pytest.mark.parametrize("N,Np,code", [
    (1000, 32, _lib.SCD_ERR_SIZE), (512, 32, _lib.SCD_ERR_SIZE), (1 << 21, 32, _lib.SCD_ERR_SIZE),
    (1024, 8, _lib.SCD_ERR_SIZE), (1024, 512, _lib.SCD_ERR_SIZE), (1024, 48, _lib.SCD_ERR_SIZE),
])
def test_ssca_size_errors(L, N, Np, code):
    assert L.scd_ssca(_fake(X), N, Np, _fake(W), _fake(O)) == code
    assert L.scd_last_error()


def test_ssca_null_and_alias(L):
    assert L.scd_ssca(None, 1024, 32, _fake(W), _fake(O)) == _lib.SCD_ERR_NULL
    assert L.scd_ssca(_fake(X), 1024, 32, None, _fake(O)) == _lib.SCD_ERR_NULL
    assert L.scd_ssca(_fake(X), 1024, 32, _fake(W), None) == _lib.SCD_ERR_NULL
    # out overlapping x
    assert L.scd_ssca(_fake(X), 1024, 32, _fake(W), _fake(X + 64)) == _lib.SCD_ERR_ALIAS
    # out overlapping win
    assert L.scd_ssca(_fake(X), 1024, 32, _fake(O + 8 * 1024), _fake(O)) == _lib.SCD_ERR_ALIAS


def test_ssca_ex_option_errors(L):
    o = _lib.ScdOpts()
    o.precision = 9
    assert L.scd_ssca_ex(_fake(X), 1024, 32, _fake(W), _fake(O), ctypes.byref(o)) == _lib.SCD_ERR_SIZE
    o = _lib.ScdOpts()
    o.batch = 2
    o.x_stride = 100  # < N
    assert L.scd_ssca_ex(_fake(X), 1024, 32, _fake(W), _fake(O), ctypes.byref(o)) == _lib.SCD_ERR_SIZE
    o = _lib.ScdOpts()
    o.workspace_bytes = 10
    assert L.scd_ssca_ex(_fake(X), 1024, 32, _fake(W), _fake(O), ctypes.byref(o)) == _lib.SCD_ERR_NULL
    o = _lib.ScdOpts()
    o.workspace = X + 8
    o.workspace_bytes = 1 << 20
    assert L.scd_ssca_ex(_fake(X), 2048, 32, _fake(W), _fake(O), ctypes.byref(o)) == _lib.SCD_ERR_ALIAS
    o = _lib.ScdOpts()
    o.workspace = 0x50000000
    o.workspace_bytes = 1024
    assert L.scd_ssca_ex(_fake(X), 2048, 32, _fake(W), _fake(O), ctypes.byref(o)) == _lib.SCD_ERR_NOMEM


@pytest.mark.parametrize("Np,Lh,P,code", [
    (32, 8, 3, _lib.SCD_ERR_SIZE), (32, 64, 32, _lib.SCD_ERR_SIZE), (32, 3, 32, _lib.SCD_ERR_SIZE),
    (8, 2, 32, _lib.SCD_ERR_SIZE), (32, 8, 2048, _lib.SCD_ERR_SIZE), (256, 256, 512, _lib.SCD_ERR_SIZE),
])
def test_fam_size_errors(L, Np, Lh, P, code):
    assert L.scd_fam(_fake(X), Np, Lh, P, _fake(W), _fake(O)) == code


def test_fam_alias_and_null(L):
    assert L.scd_fam(None, 32, 8, 32, _fake(W), _fake(O)) == _lib.SCD_ERR_NULL
    assert L.scd_fam(_fake(X), 32, 8, 32, _fake(W), _fake(X)) == _lib.SCD_ERR_ALIAS


def test_workspace_size(L):
    v = ctypes.c_size_t()
    assert L.scd_ssca_workspace_size(1 << 20, 64, 1, ctypes.byref(v)) == 0
    assert v.value == 8 * 64 * (1 << 20)
    assert L.scd_ssca_workspace_size(1024, 64, 3, ctypes.byref(v)) == 0 and v.value == 0
    assert L.scd_ssca_workspace_size(1000, 64, 1, ctypes.byref(v)) == _lib.SCD_ERR_SIZE
    assert L.scd_fam_workspace_size(256, 64, 256, 16, ctypes.byref(v)) == 0
    assert v.value == 8 * 256 * 256 * 16
    assert L.scd_ssca_workspace_size(1024, 64, 1, None) == _lib.SCD_ERR_NULL


def test_split_precision_np256_unsupported(L):
    o = _lib.ScdOpts()
    o.precision = _lib.PRECISIONS["split_bf16"]
    assert L.scd_ssca_ex(_fake(X), 4096, 256, _fake(W), _fake(O), ctypes.byref(o)) == _lib.SCD_ERR_UNSUPPORTED


def test_learned_entry_errors(L):
    assert L.scd_mlp_param_count(256) == 262912
    assert L.scd_mlp_param_count(100) == _lib.SCD_ERR_SIZE
    v = ctypes.c_size_t()
    assert L.scd_features(None, 1 << 14, 64, _fake(W), _fake(O), None) == _lib.SCD_ERR_NULL
    assert L.scd_features(_fake(X), 1 << 12, 64, _fake(W), _fake(O), None) == _lib.SCD_ERR_SIZE
    sel = _lib.ScdSelector()
    sel.Np = 64
    fb = ctypes.c_int()
    assert L.scd_ssca_learned(_fake(X), 1 << 16, 64, _fake(W), ctypes.byref(sel), _fake(O), _fake(O + 8),
                              ctypes.byref(fb), None) == _lib.SCD_ERR_MODEL
    sel.params, sel.mu, sel.sigma = 0x1000, 0x2000, 0x3000
    assert L.scd_ssca_learned(_fake(X), 1 << 16, 32, _fake(W), ctypes.byref(sel), _fake(O), _fake(O + 8),
                              ctypes.byref(fb), None) == _lib.SCD_ERR_MODEL
    sel.params = 0x1004  # parameters must be 16-byte aligned
    assert L.scd_ssca_learned(_fake(X), 1 << 16, 64, _fake(W), ctypes.byref(sel), _fake(O), _fake(O + 8),
                              None, None) == _lib.SCD_ERR_MODEL
    assert L.scd_adam_step(0, _fake(X), _fake(W), _fake(O), _fake(O), 1, 1e-3, 0.9, 0.999, 1e-8, None) == _lib.SCD_ERR_SIZE


def test_ssca_batch_errors(L):
    o = _lib.ScdOpts()
    assert L.scd_ssca_batch(None, -1, None) == _lib.SCD_ERR_SIZE
    assert L.scd_ssca_batch(None, 1, None) == _lib.SCD_ERR_NULL
    assert L.scd_ssca_batch(None, 0, None) == _lib.SCD_OK
    items = (_lib.ScdSscaItem * 2)()
    o.batch = 2
    assert L.scd_ssca_batch(items, 2, ctypes.byref(o)) == _lib.SCD_ERR_SIZE
    o.batch, o.x_stride = 1, 5
    assert L.scd_ssca_batch(items, 2, ctypes.byref(o)) == _lib.SCD_ERR_UNSUPPORTED
    # The first failing item stops the call and is named in the message.
    items[0].x, items[0].N, items[0].Np, items[0].win, items[0].out = _fake(X), 3000, 64, _fake(W), _fake(O)
    assert L.scd_ssca_batch(items, 2, None) == _lib.SCD_ERR_SIZE
    assert L.scd_last_error().startswith(b"item 0:")
    sel = _lib.ScdSelector()
    sel.Np = 64
    items[0].N, items[0].selector, items[0].mask = 1 << 16, ctypes.pointer(sel), _fake(O + 8)
    assert L.scd_ssca_batch(items, 1, None) == _lib.SCD_ERR_MODEL
    assert L.scd_last_error().startswith(b"item 0:")


def test_fam_power_errors(L):
    assert L.scd_fam_power_ex(None, 64, 16, 64, _fake(W), _fake(O), None) == _lib.SCD_ERR_NULL
    assert L.scd_fam_power_ex(_fake(X), 64, 16, 2, _fake(W), _fake(O), None) == _lib.SCD_ERR_SIZE
    assert L.scd_fam_power_ex(_fake(X), 64, 128, 64, _fake(W), _fake(O), None) == _lib.SCD_ERR_SIZE
    o = _lib.ScdOpts()
    o.precision = _lib.PRECISIONS["split_bf16"]
    assert L.scd_fam_power_ex(_fake(X), 64, 16, 64, _fake(W), _fake(O), ctypes.byref(o)) == _lib.SCD_ERR_UNSUPPORTED


def test_ssca_cross_errors(L):
    assert L.scd_ssca_cross_ex(_fake(X), None, 4096, 64, _fake(W), 0, _fake(O), None) == _lib.SCD_ERR_NULL
    assert L.scd_ssca_cross_ex(_fake(X), _fake(X + 0x100000), 3000, 64, _fake(W), 0, _fake(O), None) == _lib.SCD_ERR_SIZE
    assert L.scd_ssca_cross_ex(_fake(X), _fake(O), 4096, 64, _fake(W), 1, _fake(O), None) == _lib.SCD_ERR_ALIAS
    o = _lib.ScdOpts()
    o.precision = _lib.PRECISIONS["split_bf16"]
    assert L.scd_ssca_cross_ex(_fake(X), _fake(X + 0x100000), 4096, 64, _fake(W), 0, _fake(O),
                               ctypes.byref(o)) == _lib.SCD_ERR_UNSUPPORTED


def test_fam_cross_errors(L):
    assert L.scd_fam_cross_ex(_fake(X), None, 64, 16, 64, _fake(W), 0, _fake(O), None) == _lib.SCD_ERR_NULL
    assert L.scd_fam_cross_ex(_fake(X), _fake(X + 0x100000), 64, 16, 2, _fake(W), 0, _fake(O), None) == _lib.SCD_ERR_SIZE
    assert L.scd_fam_cross_ex(_fake(X), _fake(O), 64, 16, 64, _fake(W), 1, _fake(O), None) == _lib.SCD_ERR_ALIAS


def test_ssca_block_errors(L):
    assert L.scd_ssca_block_ex(_fake(X), 8192, 100, 4096, 64, _fake(W), _fake(O), None) == _lib.SCD_ERR_SIZE
    assert L.scd_ssca_block_ex(_fake(X), 8192, 6144, 4096, 64, _fake(W), _fake(O), None) == _lib.SCD_ERR_SIZE
    assert L.scd_ssca_block_ex(_fake(X), (1 << 27) + 64, 0, 4096, 64, _fake(W), _fake(O), None) == _lib.SCD_ERR_SIZE
    assert L.scd_ssca_block_ex(_fake(X), 0, 0, 4096, 64, _fake(W), _fake(O), None) == _lib.SCD_ERR_SIZE
    o = _lib.ScdOpts()
    o.precision = _lib.PRECISIONS["split_bf16"]
    assert L.scd_ssca_block_ex(_fake(X), 8192, 4096, 4096, 64, _fake(W), _fake(O), ctypes.byref(o)) == _lib.SCD_ERR_UNSUPPORTED


# ---- selector model files and lifecycle (host-side checks; no device call is reached) ---------------------
MODELS = os.path.join(ROOT, "paper_2506_18003_amd", "models")


def _fnv1a(b: bytes) -> int:
    h = 2166136261
    for c in b:
        h = ((h ^ c) * 16777619) & 0xFFFFFFFF
    return h


def _npz_model(Np):
    import json
    import numpy as np

    d = np.load(os.path.join(MODELS, f"selector_np{Np}.npz"))
    m = json.load(open(os.path.join(MODELS, f"selector_np{Np}.json")))
    return (np.ascontiguousarray(d["params"], np.float32), np.ascontiguousarray(d["mu"], np.float32),
            np.ascontiguousarray(d["sigma"], np.float32), m["theta"], m["conf_min"])


def _write(L, path, Np, p, mu, sg, theta, conf):
    return L.scd_model_write(os.fsencode(str(path)), Np, p.ctypes.data, mu.ctypes.data, sg.ctypes.data, theta, conf)


@pytest.mark.parametrize("Np", [64, 128, 256])
def test_model_file_layout_and_committed_files(L, tmp_path, Np):
    """scd_model_write lays the file out as the header documents (parsed here with struct, hash recomputed), and
    the committed .scdm files are exactly what it writes from the trained selectors' arrays."""
    import struct

    import numpy as np

    p, mu, sg, theta, conf = _npz_model(Np)
    path = tmp_path / "m.scdm"
    assert _write(L, path, Np, p, mu, sg, theta, conf) == 0
    b = path.read_bytes()
    assert b[:4] == b"SCDM"
    version, np_, n, th, cf = struct.unpack("<IiiFf".replace("F", "f"), b[4:24])
    assert (version, np_, n) == (1, Np, L.scd_mlp_param_count(Np))
    assert th == np.float32(theta) and cf == np.float32(conf)
    arr = np.frombuffer(b[24:-4], np.float32)
    assert np.array_equal(arr, np.concatenate([p, mu, sg]))
    assert struct.unpack("<I", b[-4:])[0] == _fnv1a(b[:-4])
    assert (open(os.path.join(MODELS, f"selector_np{Np}.scdm"), "rb").read()) == b


def test_model_load_rejects_bad_files(L, tmp_path):
    p, mu, sg, theta, conf = _npz_model(64)
    good = tmp_path / "good.scdm"
    assert _write(L, good, 64, p, mu, sg, theta, conf) == 0
    b = good.read_bytes()
    h = ctypes.c_void_p(123)
    cases = {
        "missing": None,
        "magic": b"SCDX" + b[4:],
        "version": b[:4] + (2).to_bytes(4, "little") + b[8:],
        "np": b[:8] + (48).to_bytes(4, "little") + b[12:],
        "truncated": b[:-100],
        "extra": b + b"\0",
        "corrupt": b[:1000] + bytes([b[1000] ^ 1]) + b[1001:],
        "short": b[:10],
    }
    for name, content in cases.items():
        path = tmp_path / f"{name}.scdm"
        if content is not None:
            path.write_bytes(content)
        assert L.scd_model_load(os.fsencode(str(path)), ctypes.byref(h)) == _lib.SCD_ERR_MODEL, name
        assert not h.value, name
        assert L.scd_last_error()
    assert L.scd_model_load(None, ctypes.byref(h)) == _lib.SCD_ERR_NULL
    assert L.scd_model_load(os.fsencode(str(good)), None) == _lib.SCD_ERR_NULL


def test_model_create_and_write_reject_bad_values(L, tmp_path):
    import numpy as np

    p, mu, sg, theta, conf = _npz_model(64)
    h = ctypes.c_void_p()
    create = lambda Np, pp, mm, ss, t, c, out=ctypes.byref(h): L.scd_model_create(
        Np, pp.ctypes.data if pp is not None else None, mm.ctypes.data, ss.ctypes.data, t, c, out)
    assert create(64, p, mu, sg, theta, conf, None) == _lib.SCD_ERR_NULL
    assert create(64, None, mu, sg, theta, conf) == _lib.SCD_ERR_NULL
    assert create(48, p, mu, sg, theta, conf) == _lib.SCD_ERR_SIZE
    assert create(64, p, mu, sg, 1.5, conf) == _lib.SCD_ERR_MODEL
    assert create(64, p, mu, sg, theta, -0.1) == _lib.SCD_ERR_MODEL
    bad_sigma = sg.copy()
    bad_sigma[3] = 0.0
    assert create(64, p, mu, bad_sigma, theta, conf) == _lib.SCD_ERR_MODEL
    bad_p = p.copy()
    bad_p[1000] = np.nan
    assert create(64, bad_p, mu, sg, theta, conf) == _lib.SCD_ERR_MODEL
    assert _write(L, tmp_path / "x.scdm", 64, bad_p, mu, sg, theta, conf) == _lib.SCD_ERR_MODEL
    assert _write(L, tmp_path / "no_such_dir" / "x.scdm", 64, p, mu, sg, theta, conf) == _lib.SCD_ERR_MODEL
    assert L.scd_model_write(None, 64, p.ctypes.data, mu.ctypes.data, sg.ctypes.data, theta, conf) == _lib.SCD_ERR_NULL
    assert L.scd_model_destroy(None) == 0
    assert L.scd_model_save(None, b"x") == _lib.SCD_ERR_NULL
    assert L.scd_model_selector(None, None) == _lib.SCD_ERR_NULL


def test_receiver_rejects_bad_arguments(L):
    h = ctypes.c_void_p(1)
    outs = (ctypes.c_void_p * 2)(_fake(O), _fake(O + 0x10000000))
    create = lambda N, Np, win, slots, o, n, out=ctypes.byref(h): L.scd_receiver_create(N, Np, win, slots, o, n, None, out)
    assert create(1 << 16, 64, _fake(W), 4, outs, 2, None) == _lib.SCD_ERR_NULL
    assert create(1 << 16, 64, None, 4, outs, 2) == _lib.SCD_ERR_NULL and not h.value
    assert create(1 << 16, 64, _fake(W), 4, None, 2) == _lib.SCD_ERR_NULL
    assert create(1000, 64, _fake(W), 4, outs, 2) == _lib.SCD_ERR_SIZE
    assert create(1 << 21, 64, _fake(W), 4, outs, 2) == _lib.SCD_ERR_SIZE
    assert create(1 << 16, 48, _fake(W), 4, outs, 2) == _lib.SCD_ERR_SIZE
    assert create(1 << 16, 64, _fake(W), 2, outs, 2) == _lib.SCD_ERR_SIZE
    assert create(1 << 16, 64, _fake(W), 4, outs, 0) == _lib.SCD_ERR_SIZE
    nul = (ctypes.c_void_p * 2)(_fake(O), None)
    assert create(1 << 16, 64, _fake(W), 4, nul, 2) == _lib.SCD_ERR_NULL
    assert L.scd_receiver_push(None, _fake(X), None, None) == _lib.SCD_ERR_NULL
    assert L.scd_receiver_finish(None, None, None) == _lib.SCD_ERR_NULL
    assert L.scd_receiver_wait_copy(None) == _lib.SCD_ERR_NULL
    assert L.scd_receiver_destroy(None) == 0


def test_ssca_strips_rejects_bad_strip_lists(L):
    def call(ks, n=None, N=1024, Np=32, o=_fake(O)):
        arr = (ctypes.c_int * max(1, len(ks)))(*ks)
        return L.scd_ssca_strips(_fake(X), N, Np, _fake(W), arr, len(ks) if n is None else n, o, None)
    assert call([0, 32]) == _lib.SCD_ERR_SIZE  # outside [0, Np)
    assert call([-1]) == _lib.SCD_ERR_SIZE
    assert call([3, 5, 3]) == _lib.SCD_ERR_SIZE  # listed twice
    assert call([0], n=33) == _lib.SCD_ERR_SIZE  # more strips than Np
    assert call([0], n=-1) == _lib.SCD_ERR_SIZE
    assert L.scd_ssca_strips(_fake(X), 1024, 32, _fake(W), None, 2, _fake(O), None) == _lib.SCD_ERR_NULL
    assert call([], n=0) == 0  # nothing to compute
    assert call([], n=0, o=None) == _lib.SCD_ERR_NULL
    # the checks of scd_ssca_ex still apply, before any GPU work
    assert call([1], N=1000) == _lib.SCD_ERR_SIZE
    assert call([1], Np=48) == _lib.SCD_ERR_SIZE
    assert call([1], o=_fake(X + 64)) == _lib.SCD_ERR_ALIAS
    assert call([1], o=None) == _lib.SCD_ERR_NULL
    o = _lib.ScdOpts()
    o.precision = _lib.PRECISIONS["split_fp16"]
    arr = (ctypes.c_int * 1)(1)
    assert L.scd_ssca_strips(_fake(X), 1024, 32, _fake(W), arr, 1, _fake(O), ctypes.byref(o)) == \
        _lib.SCD_ERR_UNSUPPORTED
