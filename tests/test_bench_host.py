"""Host-side arithmetic of bench.py's measurement objects (no GPU): the
issue roofline, the recorded instruction mixes and the CPU description."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_issue_roofline_prices_each_class_at_its_rate():
    """A launch of 1e9 FMA and 1e9 transcendental wave instructions, probed
    at 32 and 8 lane-ops per SIMD per rated clock: it needs
    1e9 * 64 / (32 c) + 1e9 * 64 / (8 c) seconds with c = 1024 SIMDs x 2.4 GHz;
    timed at exactly that, the fraction is 1 and the ceiling rate is the
    harmonic combination 2 / (64/32 + 64/8) = 0.2 wave instructions per
    SIMD-clock."""
    c = 1024 * 2.4e9
    rates = {k: 16.0 * c for k in bench.PROBE_KINDS}
    rates["fma_f32"] = 32.0 * c
    rates["exp_f32"] = 8.0 * c
    mix = {"per_launch": {"FMA_F32": 1e9, "TRANS_F32": 1e9}, "lanes_active_per_instr": 0.9}
    need = 1e9 * 64 / (32 * c) + 1e9 * 64 / (8 * c)
    r = bench.issue_roofline(mix, rates, need * 1e3)
    assert r["frac"] == pytest.approx(1.0, rel=1e-12)
    assert r["ceiling_wave_instr_per_simd_clock"] == pytest.approx(0.2, rel=1e-12)
    assert r["achieved_wave_instr_per_simd_clock"] == pytest.approx(0.2, rel=1e-12)
    assert r["class_mix"] == pytest.approx({"FMA_F32": 0.5, "TRANS_F32": 0.5})
    # twice as long: half the ceiling
    assert bench.issue_roofline(mix, rates, 2 * need * 1e3)["frac"] == pytest.approx(0.5)
    assert bench.issue_roofline(None, rates, 1.0) is None


def test_every_counted_class_has_a_probe_kind():
    assert set(bench.VALU_CLASS_PROBE.values()) <= set(bench.PROBE_KINDS)


def test_recorded_mixes_are_consistent():
    """Each record of profiles/valu_mix.json: classes sum to SQ_INSTS_VALU,
    every class is priced, the sources it names exist."""
    path = os.path.join(ROOT, "profiles", "valu_mix.json")
    rec = json.load(open(path))
    keys = [k for k in rec if not k.startswith("_")]
    assert keys
    for k in keys:
        r = rec[k]
        tot = sum(r["per_launch"].values())
        raw = r["sq_insts_valu_raw"]
        assert tot == pytest.approx(sum(raw) / len(raw), rel=1e-9), k
        assert set(r["per_launch"]) <= set(bench.VALU_CLASS_PROBE), k
        assert all(v >= 0 for v in r["per_launch"].values()), k
        assert 0 < r["lanes_active_per_instr"] <= 1.0, k
        for f in r["sources"]:
            assert os.path.exists(os.path.join(ROOT, "paper_2304_06835_amd", "csrc", f)), (k, f)


def test_recorded_mix_is_ignored_once_sources_change(tmp_path):
    good = bench.kernel_source_hash(["tsit5.hip"])
    rec = {"w/a/f": {"sources": ["tsit5.hip"], "source_hash": "0000000000000000",
                     "per_launch": {"FMA_F32": 1.0}},
           "w/a/g": {"sources": ["tsit5.hip"], "source_hash": good,
                     "per_launch": {"FMA_F32": 1.0}}}
    path = tmp_path / "valu_mix.json"
    path.write_text(json.dumps(rec))
    assert bench.recorded_valu_mix("w/a/f", str(path)) is None
    assert bench.recorded_valu_mix("w/a/g", str(path))["per_launch"] == {"FMA_F32": 1.0}
    assert bench.recorded_valu_mix("missing", str(path)) is None


def test_cpu_model_reports_the_host():
    m = bench.cpu_model()
    assert m["logical_cpus"] and m["logical_cpus"] >= 1
    assert 1 <= m["affinity"] <= m["logical_cpus"]
    assert m["model"] is None or isinstance(m["model"], str)


def test_training_flops_per_sample():
    """Forward 2 (4*256 + 2*256^2 + 256*48), the weight gradients the same,
    the input gradients of layers 2..4 2 (2*256^2 + 256*48)."""
    fwd = 2 * (4 * 256 + 2 * 256 * 256 + 256 * 48)
    assert bench.MLP_FLOPS_PER_QUERY == fwd == 288768
    assert bench.MLP_TRAIN_FLOPS_PER_SAMPLE == 2 * fwd + 2 * (2 * 256 * 256 + 256 * 48) == 864256


def test_coissue_ceiling_counts_the_inference_kernels_work():
    """The probe units of one 16-query subtile add up to the fused kernel's
    296 products (16 + 128 + 128 + 24 row-block x k-block tiles) and 192 SiLU
    rows (768 activations x 16 queries / 64 lanes), and the ceiling is the
    probe time of those units over the kernel time."""
    prod = (bench.INFER_SUBTILE["mfma_then_silu"] + bench.INFER_SUBTILE["mfma"]) * bench.MIX_PRODUCTS
    rows = (bench.INFER_SUBTILE["mfma_then_silu"] + bench.INFER_SUBTILE["silu"]) * bench.MIX_ROWS
    assert abs(prod - 296) < 1e-9 and abs(rows - 192) < 1e-9
    rates = {"mfma": 2e9, "silu": 1e9, "mfma_then_silu": 5e8}
    q = 1 << 20
    r = bench.coissue_ceiling(q, 10.0, rates)
    want_s = q / 16 * (256 / 24 / 5e8 + 40 / 24 / 2e9 + 64 / 12 / 1e9)
    assert abs(r["ceiling_ms"] - want_s * 1e3) < 1e-9
    assert abs(r["frac"] - want_s * 1e3 / 10.0) < 1e-12
    # 24 products of 16 x 16 x 32 per wave-iteration against the bf16 peak
    assert abs(r["probe_products_frac_of_peak"] - 2e9 * 24 * 16384 / 2.5e15) < 1e-12


def _write_pmc(d, rows):
    """A rocprofv3 counter CSV with the columns record_counters reads."""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w") as fh:
        fh.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for disp, kern, name, val in rows:
            fh.write(f'{disp},"{kern}",{name},{val}\n')


def test_record_counters_from_pmc_csvs(tmp_path):
    """bench.py --record-counters: per-dispatch sums of each counter over the
    CSV's rows (one row per XCD here), means over the kernel's dispatches,
    OTHER as the uncounted remainder, lane activity from the F64 pass, and
    HBM bytes scaled by the 1 GiB copy's counter reading (first write
    dispatch dropped as cold); other kernels' rows are ignored."""
    root = tmp_path / "pmc"
    cls = {"FMA_F32": 40, "MUL_F32": 20, "ADD_F32": 5, "TRANS_F32": 3, "INT32": 2, "INT64": 1,
           "CVT": 1}
    for key, (tag, match, _src, _k) in bench.MIX_RUNS.items():
        kern = f"void ens::{match}(ens::LaunchArgs)"
        a, c = [], []
        for disp, scale in ((1, 1.0), (2, 3.0)):
            for xcd in range(2):  # each counter read on two XCDs, half each
                a.append((disp, kern, "SQ_INSTS_VALU", 50 * scale))
                for k, v in cls.items():
                    a.append((disp, kern, f"SQ_INSTS_VALU_{k}", v / 2 * scale))
                for k in ("FMA", "ADD", "MUL", "TRANS"):
                    c.append((disp, kern, f"SQ_INSTS_VALU_{k}_F64", 1 / 2 * scale))
                c += [(disp, kern, "SQ_ACTIVE_INST_VALU", 100 / 2), (disp, kern, "SQ_THREAD_CYCLES_VALU",
                      0.75 * 64 * 100 / 2), (disp, kern, "SQ_WAVES", 8 / 2),
                      (disp, kern, "SQ_BUSY_CYCLES", 1000 / 2)]
            a.append((disp + 10, "other_kernel", "SQ_INSTS_VALU", 1e9))
        _write_pmc(str(root / f"mixA_{tag}"), a)
        _write_pmc(str(root / f"mixC_{tag}"), c)
    copy = "__amd_rocclr_copyBuffer"
    _write_pmc(str(root / "pmc_copy_FETCH"), [(1, copy, "FETCH_SIZE", 524288), (2, copy, "FETCH_SIZE", 12)])
    _write_pmc(str(root / "pmc_copy_WRITE"), [(1, copy, "WRITE_SIZE", 1048576)])
    for tag in ("h", "st"):
        k = "void ens::tsit5_sorted<float, ens::Lorenz, 256, 1, false>(ens::LaunchArgs)"
        _write_pmc(str(root / f"pmc_{tag}_FETCH"), [(1, k, "FETCH_SIZE", 1000), (2, k, "FETCH_SIZE", 3000)])
        _write_pmc(str(root / f"pmc_{tag}_WRITE"), [(1, k, "WRITE_SIZE", 9e9), (2, k, "WRITE_SIZE", 4000)])
    out = tmp_path / "out"
    out.mkdir()
    mix, tr = bench.record_counters(str(root), str(out))
    r = mix["lorenz_fp32/tsit5/sorted/dense"]
    assert r["dispatches"] == [2, 2]
    # means over dispatches of scale 1 and 3: twice the base counts
    assert r["per_launch"]["FMA_F32"] == 80 and r["per_launch"]["F64"] == 8
    # SQ_INSTS_VALU averages 200; the counted classes 144, F64 8
    assert r["per_launch"]["OTHER"] == 200 - 2 * sum(cls.values()) - 8
    assert abs(r["lanes_active_per_instr"] - 0.75) < 1e-12
    assert r["source_hash"] == bench.kernel_source_hash(bench.TSIT5_SOURCES)
    t = tr["lorenz_fp32/sorted/dense"]
    assert t["hbm_read_bytes_per_launch"] == 2000 * 1024 * 2.0   # fetch scale 1 GiB / 512 MiB read
    assert t["hbm_write_bytes_per_launch"] == 4000 * 1024 * 1.0  # first dispatch dropped
    assert json.load(open(out / "valu_mix.json"))["gbm/em/plain"]["per_launch"]["MUL_F32"] == 40
    assert json.load(open(out / "traffic.json"))["lorenz_fp32/sorted_staged/dense"]["fetch_kib_raw"] == [1000, 3000]
