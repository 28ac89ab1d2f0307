"""CPU checks of the gfx950 code the SSCA kernels compile to (no GPU needed).

* Every out-of-range-safe sample load is one 64-bit buffer load addressed through the range-checked VGPR
  offset (plus, at most, an immediate offset, which the buffer range check includes: the checked offset is the
  32-bit sum of both); a split or narrowed load would read past the signal instead of the zero padding, and a
  scalar offset would escape the check.
* No Stage-1 form (the headline kernel, its selection form, subset pairs, the per-frame down-conversion of
  short signals, the cross forms, every Np) and no Stage-2 kernel spills registers.
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
