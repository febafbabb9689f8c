"""Host checks of how bench.py reads the committed profile summaries: the
counter block of a kernel (not of another kernel whose name it prefixes),
only when the block's source digest matches, and the HBM traffic line."""
import bench


def _write(root, name, text):
    d = root / "profiles"
    d.mkdir(exist_ok=True)
    (d / name).write_text(text)


COUNTERS = """# header
commands ...

k_project_rows<10>  (45 launches per step, 66.0 ms per step)
  sources: aaaa
  SQ_INSTS_VALU                    1e+10
  VALU issue rate             1.2500 of the 16-lane rate
  ACTIVE_INST_VALU2 / VALU    0.3500
  wait share of wave cycles   0.4000
  L2 hit rate                 0.7000
  LDS bank-conflict share     0.0200
  MFMA busy                   0.0000
  VALU lane-slots per segment 15.0000 (2.2e+11)

k_project_rows_split<10, 1>  (45 launches per step, 64.0 ms per step)
  sources: bbbb
  VALU issue rate             0.9000 of the 16-lane rate
  MFMA busy                   0.0100
"""


def test_counter_block_of_the_named_kernel(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _write(tmp_path, "counters_head.txt", COUNTERS)
    plain = bench.profiled_counters("k_project_rows", "aaaa", "head")
    assert plain["valu_issue_vs_16_lane_rate"] == 1.25 and plain["valu_lane_slots_per_segment"] == 15.0
    assert plain["l2_hit"] == 0.7 and plain["wait_share"] == 0.4 and plain["valu2_share"] == 0.35
    split = bench.profiled_counters("k_project_rows_split", "bbbb", "head")
    assert split == {"valu_issue_vs_16_lane_rate": 0.9, "mfma_busy": 0.01}


def test_counters_taken_on_other_sources_are_not_used(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _write(tmp_path, "counters_head.txt", COUNTERS)
    assert bench.profiled_counters("k_project_rows", "bbbb", "head") == {}
    assert bench.profiled_counters("k_psf4", "aaaa", "head") == {}
    assert bench.profiled_counters("k_project_rows", "aaaa", "contrast") == {}


def test_traffic_line(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _write(tmp_path, "hbm_traffic_k_psf_head.txt", "# x\nsources: cccc\ntraffic_bytes_per_step: 3.25e+10\n")
    assert bench.profiled_traffic("k_psf", "cccc", "head") == 3.25e10
    assert bench.profiled_traffic("k_psf", "dddd", "head") is None
    assert bench.profiled_traffic("k_project_rows", "cccc", "head") is None


def test_measured_ceilings_price_walks_by_the_steps_taken():
    """A walk priced by the model count (every Siddon segment) gets no rate
    against the measured ceilings, since it crosses uniform bricks in one step
    and can outrun them; its executed-steps entry, and every other entry, does."""
    walk = bench.alu_roof("k_project_rows<8>", 60e12, 1000.0,
                          executed=bench.alu_roof("same launches", 20e12, 1000.0))
    psf = {"kernel": "k_psf4", "bound": "alu", "achieved": 100.0, "unit": "TFLOP/s", "peak": 157.3, "frac": 0.64}
    result = {"roofline": {"kernel": "k_project_rows<8>", "bound": "alu", "achieved": 60.0, "unit": "Top/s",
                           "peak": 78.65, "frac": 0.76, "frac_executed": 0.25},
              "kernels": {"k_project_rows": walk, "k_psf": psf}}
    bench.apply_measured_ceilings(result, {"fma_f32_TFLOPs": 120.0, "copy_GBps": 5000.0, "mfma_bf16_TFLOPs": 2000.0})
    assert "frac_measured" not in result["roofline"] and "frac_measured" not in walk
    assert walk["executed"]["measured_peak"] == 60.0 and walk["executed"]["frac_measured"] == round(20.0 / 60.0, 4)
    assert psf["measured_peak"] == 120.0 and psf["frac_measured"] == round(100.0 / 120.0, 4)


def test_atomic_rows_take_the_measured_ceiling_as_peak():
    e = {"kernel": "k_image_rays<true>", "bound": "atomic", "achieved": 30.0, "peak": None, "unit": "Gatomic/s",
         "frac": None}
    result = {"next": {"image_projector": {"backproject": {"roofline": e}}}}
    bench.apply_measured_ceilings(result, {"fma_f32_TFLOPs": 120.0, "copy_GBps": 5000.0, "mfma_bf16_TFLOPs": 2000.0,
                                           "atomic_add_f32_Gps": 120.0})
    assert e["measured_peak"] == 120.0 and e["peak"] == 120.0 and e["frac"] == 0.25


def test_scattered_atomic_view_takes_its_own_ceiling():
    v = {"kernel": "k_image_rays<true>", "bound": "atomic_scattered", "achieved": 30.0, "peak": None,
         "unit": "Gatomic/s", "frac": None}
    e = {"kernel": "k_image_rays<true>", "bound": "atomic", "achieved": 30.0, "peak": None, "unit": "Gatomic/s",
         "frac": None, "scattered_view": v}
    result = {"next": {"image_projector": {"backproject": {"roofline": e}}}}
    bench.apply_measured_ceilings(result, {"fma_f32_TFLOPs": 120.0, "copy_GBps": 5000.0, "mfma_bf16_TFLOPs": 2000.0,
                                           "atomic_add_f32_Gps": 300.0, "atomic_add_f32_scattered_Gps": 40.0})
    assert e["peak"] == 300.0 and e["frac"] == 0.1
    assert v["peak"] == 40.0 and v["frac"] == 0.75
