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
