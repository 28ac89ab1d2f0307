"""CPU checks of the gfx950 code the SSCA kernels compile to (no GPU needed).

* Every out-of-range-safe sample load is one 64-bit buffer load addressed through the range-checked VGPR
  offset (plus, at most, an immediate offset, which the buffer range check includes: the checked offset is the
  32-bit sum of both); a split or narrowed load would read past the signal instead of the zero padding, and a
  scalar offset would escape the check.
* No Stage-1 form (the headline kernel, its selection form, subset pairs, the per-frame down-conversion of
  short signals, the cross forms, every Np) and no Stage-2 kernel spills registers.
* No LDS table fill in the Stage-1, FAM and selector kernels is a loop that waits for each load before the next
  (a strided copy loop whose trip count the compiler cannot see compiles to load, wait, LDS write per entry, so
  a workgroup pays one memory round trip per entry before it starts). Stage 2 keeps such loops on purpose.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_18003_amd", "csrc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


pytestmark = pytest.mark.skipif(not os.path.exists(_hipcc()), reason="hipcc not available")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    out = tmp_path_factory.mktemp("asm") / "ssca.s"
    subprocess.run([_hipcc(), *FLAGS, "-S", "--cuda-device-only", os.path.join(CSRC, "ssca_fp32.hip"), "-o",
                    str(out)], check=True, capture_output=True)
    return out.read_text()


def test_sample_loads_are_single_64bit_range_checked(asm):
    loads = [ln.split() for ln in asm.splitlines() if "buffer_load" in ln]
    assert loads
    for ins in loads:
        assert ins[0] == "buffer_load_dwordx2", ins
        # operands: vdst, voffset, srsrc, soffset (0), offen [, offset:imm]
        ops = [o.rstrip(",") for o in ins[1:]]
        assert ops[3] == "0" and ops[4] == "offen", ins
        assert len(ops) == 5 or (len(ops) == 6 and re.fullmatch(r"offset:\d+", ops[5])), ins


def _spills(asm):
    out = {}
    for m in re.finditer(r"\.name:\s+(\S+)(.*?)\.vgpr_spill_count:\s+(\d+)", asm, re.S):
        out[m.group(1)] = int(m.group(3))
    return out


def test_hot_kernels_do_not_spill(asm):
    sp = _spills(asm)
    # every Stage-1 form (each Np, both down-conversion forms, selection, subset pairs, cross forms) and Stage 2
    hot = [n for n in sp if "ssca_pass1_fp32" in n or "ssca_pass2_fp32" in n]
    assert any("pass1_fp32ILi64ELb1ELb0ELb0E" in n for n in hot)  # the headline kernel
    assert any("pass1_fp32ILi64ELb1ELb1ELb0E" in n for n in hot)  # the same with a device-side selection
    assert any("pass1_fp32ILi64ELb0E" in n for n in hot)          # per-frame down-conversion (Np does not divide M2)
    assert any("pass2" in n for n in hot)
    for n in hot:
        assert sp[n] == 0, n


def _device_asm(tmp_path_factory, name):
    out = tmp_path_factory.mktemp("asm") / (name + ".s")
    subprocess.run([_hipcc(), *FLAGS, "-S", "--cuda-device-only", os.path.join(CSRC, name + ".hip"), "-o", str(out)],
                   check=True, capture_output=True)
    return out.read_text()


def _serial_fill_loops(asm):
    """Kernel name -> short loops (at most 40 lines from header to back branch) whose body issues a global or
    buffer load, then waits for every outstanding load, then writes LDS."""
    found = {}
    for m in re.finditer(r"^(_Z\S+):\s*(?:;.*)?$", asm, re.M):
        end = asm.find(".Lfunc_end", m.start())
        lines = asm[m.start():end].splitlines()
        labels = {}
        for k, ln in enumerate(lines):
            lm = re.match(r"^(\.LBB\d+_\d+):", ln)
            if lm:
                labels[lm.group(1)] = k
        for k, ln in enumerate(lines):
            bm = re.search(r"s_(?:cbranch_\w+|branch)\s+(\.LBB\d+_\d+)", ln)
            if not bm or bm.group(1) not in labels or labels[bm.group(1)] >= k or k - labels[bm.group(1)] > 40:
                continue
            body = "\n".join(lines[labels[bm.group(1)]:k])
            ld = re.search(r"(?:global|buffer)_load", body)
            wt = re.search(r"s_waitcnt vmcnt\(0\)", body[ld.end():]) if ld else None
            if wt and "ds_write" in body[ld.end() + wt.end():]:
                found.setdefault(m.group(1), []).append(labels[bm.group(1)])
    return found


def test_detector_sees_a_serial_fill_loop():
    fake = "\n".join(["_Zfake:", ".LBB0_1:", "\tglobal_load_dwordx2 v[4:5], v[2:3], off", "\ts_waitcnt vmcnt(0)",
                      "\tds_write_b64 v3, v[4:5]", "\ts_cbranch_execnz .LBB0_1", ".Lfunc_end0:"])
    assert _serial_fill_loops(fake) == {"_Zfake": [1]}


@pytest.mark.parametrize("name, kernels", [
    ("ssca_fp32", ("ssca_pass1_fp32",)),
    ("ssca_mfma", ("ssca_pass1_mfma",)),
    ("fam_fp32", ("fam_chan_fp32", "fam_pair_fp32ILi16", "fam_pair_fp32ILi32", "fam_pair_fp32ILi64",
                  "fam_pair_fp32ILi128", "fam_pair_fp32ILi256", "fam_pair_fp32ILi512", "fam_pair_fp32ILi1024")),
    ("learn", ("seg_periodogram_kernel", "infer_l12_kernel", "infer_l3_select_kernel")),
])
def test_table_fills_issue_their_loads_together(request, tmp_path_factory, name, kernels):
    # ssca_fp32 reuses the module's compile (about a minute); the others take seconds
    asm = request.getfixturevalue("asm") if name == "ssca_fp32" else _device_asm(tmp_path_factory, name)
    names = re.findall(r"^(_Z\S+):\s*(?:;.*)?$", asm, re.M)
    assert all(any(k in n for n in names) for k in kernels), "a checked kernel was not compiled"
    bad = {n: v for n, v in _serial_fill_loops(asm).items() if any(k in n for k in kernels)}
    assert not bad, bad
