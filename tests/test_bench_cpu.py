"""Host-side pieces of bench.py: the rocprofv3 counter summaries, the source-digest gate on measured traffic and
the oracle's all-core leg (no GPU)."""
import csv
import importlib.util
import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    # Registered under its own name with the repository root on sys.path, so the oracle leg's spawned workers
    # can import the pool function.
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    sys.modules["bench"] = mod
    spec.loader.exec_module(mod)
    return mod


def _pmc_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


PASS1 = "void scd::(anonymous namespace)::ssca_pass1_fp32<64, true, false, false, 0>(HIP_vector_type<float, 2u> const*)"
PASS2 = "scd::(anonymous namespace)::ssca_pass2_fp32_32x32(HIP_vector_type<float, 2u> const*)"
CALIB = "void at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<float, float, float, MulFunctor<float> > >"


def test_counter_table_averages_per_kernel_and_counter(bench, tmp_path):
    a = tmp_path / "a.csv"
    _pmc_csv(a, [(PASS1, "SQ_WAVES", 16384), (PASS1, "SQ_WAVES", 16384), (PASS1, "SQ_INSTS_VALU", 70e6),
                 (PASS1, "SQ_INSTS_VALU", 74e6), (PASS2, "SQ_WAVES", 100)])
    t = bench.counter_table([str(a)]).splitlines()
    assert t[0].startswith("| kernel | counter |")
    rows = {tuple(c.strip() for c in line.strip("|").split("|")[:2]): line for line in t[2:]}
    assert "| 2 | 7.2e+07 |" in rows[("ssca_pass1_fp32<64, true, false, false, 0>", "SQ_INSTS_VALU")]
    assert "| 2 | 16384 |" in rows[("ssca_pass1_fp32<64, true, false, false, 0>", "SQ_WAVES")]
    assert "| 1 | 100 |" in rows[("ssca_pass2_fp32_32x32", "SQ_WAVES")]


def test_write_traffic_scales_each_counter_by_its_calibration(bench, tmp_path):
    f, w, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    # FETCH_SIZE reads the 256 MiB calibration read as 128 MiB (factor 2), WRITE_SIZE reads it exactly (factor 1).
    _pmc_csv(f, [(CALIB, "FETCH_SIZE", 131072), (PASS1, "FETCH_SIZE", 1000), (PASS1, "FETCH_SIZE", 3000),
                 (PASS2, "FETCH_SIZE", 262144)])
    _pmc_csv(w, [(CALIB, "WRITE_SIZE", 262144), (PASS1, "WRITE_SIZE", 524288), (PASS2, "WRITE_SIZE", 524288)])
    d = bench.write_traffic(str(f), str(w), path=str(out))
    assert json.load(open(out)) == d
    assert d["calibration"]["FETCH_SIZE"]["factor"] == pytest.approx(2.0)
    assert d["calibration"]["WRITE_SIZE"]["factor"] == pytest.approx(1.0)
    p1, p2 = d["kernels"]["ssca_pass1"], d["kernels"]["ssca_pass2"]
    assert p1["fetch_bytes"] == 2 * 2000 * 1024 and p1["write_bytes"] == 512 << 20
    assert p2["fetch_bytes"] == 512 << 20 and p2["bytes_per_launch"] == 1 << 30
    assert d["source_digest"] == bench.source_digest()


def test_write_traffic_needs_exactly_one_calibration_reading(bench, tmp_path):
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _pmc_csv(f, [(PASS1, "FETCH_SIZE", 1000), (PASS2, "FETCH_SIZE", 1000)])
    _pmc_csv(w, [(CALIB, "WRITE_SIZE", 262144), (PASS1, "WRITE_SIZE", 1), (PASS2, "WRITE_SIZE", 1)])
    with pytest.raises(SystemExit):
        bench.write_traffic(str(f), str(w), path=str(tmp_path / "t.json"))


def test_measured_traffic_only_for_the_digest_it_was_taken_on(bench, tmp_path):
    p = tmp_path / "t.json"
    json.dump({"source_digest": "abc", "kernels": {"ssca_pass1": {"bytes_per_launch": 123}}}, open(p, "w"))
    assert bench.measured_traffic("ssca_pass1", "abc", path=str(p)) == 123
    assert bench.measured_traffic("ssca_pass1", "abd", path=str(p)) is None
    assert bench.measured_traffic("ssca_pass2", "abc", path=str(p)) is None
    assert bench.measured_traffic("ssca_pass1", "abc", path=str(tmp_path / "missing.json")) is None


def test_committed_traffic_summary_matches_the_current_sources(bench):
    """The committed counter summary was taken on the FP32 SSCA sources as they are now (else the bench reports
    no measured traffic and the summary must be re-taken)."""
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic_ssca_n2p20_np64.json")))
    assert d["source_digest"] == bench.source_digest()


def test_oracle_pool_leg_equals_single_process(bench):
    from oracle import scd_oracle as O
    from synth import signals as sg

    x = sg.qpsk(2048, 0.1, 8, 5.0, sg.rng_for(90, 0)).astype(np.complex128)
    w = sg.hamming(16)
    S1, _ = bench.cpu_oracle_ssca(x, 16, w, 1)
    S2, _ = bench.cpu_oracle_ssca(x, 16, w, 2)
    assert np.array_equal(S1, S2)
    assert np.abs(S1 - O.ssca(x, 16, w)).max() <= 1e-9 * np.abs(S1).max()


@pytest.mark.parametrize("Np,G", [(64, 1), (64, 2), (64, 4), (64, 8), (128, 8), (256, 16), (32, 4)])
def test_shard_strips_partition_the_strips(bench, Np, G):
    shards = [bench.shard_strips(Np, G, r) for r in range(G)]
    assert sorted(k for sh in shards for k in sh) == list(range(Np))
    assert all(len(sh) == Np // G for sh in shards)
    S = Np // 16
    if G <= S:  # whole subsets: no subset is split over two GPUs
        for sh in shards:
            subsets = {k % S for k in sh}
            assert all(k in sh for c in subsets for k in range(c, Np, S))
