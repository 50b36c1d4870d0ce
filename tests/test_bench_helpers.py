"""Host-side checks of the measurement helpers in bench.py: the source hash
that ties a counter table to the code it was taken on, the reading of those
tables, and the per-kernel byte models.  No GPU needed."""
import os
import shutil

import bench


def _fake_tree(tmp_path, text):
    csrc = tmp_path / "paper_1603_02655_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "a.hip").write_text(text)
    (csrc / "notes.txt").write_text("not code")
    return tmp_path


def test_source_hash_ignores_comments_and_whitespace(tmp_path, monkeypatch):
    a = _fake_tree(tmp_path / "a", "int f() { return 1; } // one\n/* block */\n")
    b = _fake_tree(tmp_path / "b", "int f()   {\n  return 1;\n}\n// another comment\n")
    c = _fake_tree(tmp_path / "c", "int f() { return 2; }\n")
    monkeypatch.setattr(bench, "ROOT", str(a))
    ha = bench.census_source_hash()
    monkeypatch.setattr(bench, "ROOT", str(b))
    hb = bench.census_source_hash()
    monkeypatch.setattr(bench, "ROOT", str(c))
    hc = bench.census_source_hash()
    assert ha == hb and ha != hc and len(ha) == 16


def test_source_hash_skips_serving_and_tuner_sources(tmp_path, monkeypatch):
    root = _fake_tree(tmp_path, "int f() { return 1; }\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    h0 = bench.census_source_hash()
    csrc = root / "paper_1603_02655_amd" / "csrc"
    for name in bench.NOT_CENSUS_SOURCES:
        (csrc / name).write_text("int serve_something() { return 3; }\n")
    assert bench.census_source_hash() == h0
    (csrc / "tc_census.hip").write_text("int k() { return 4; }\n")
    assert bench.census_source_hash() != h0


def test_measured_traffic_only_for_the_current_sources(tmp_path, monkeypatch):
    root = _fake_tree(tmp_path, "int g() { return 0; }\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    h = bench.census_source_hash()
    (root / "profiles").mkdir()
    table = ("| kernel | source hash | FETCH_SIZE KiB/launch | WRITE_SIZE KiB/launch | fetch scale | write scale | traffic bytes/launch |\n"
             "|---|---|---|---|---|---|---|\n"
             f"| k_census_hub<true> | `{h}` | 1.0 | 1.0 | 2.0 | 1.0 | 3072 |\n"
             "| k_census_lane<true> | `0123456789abcdef` | 1.0 | 1.0 | 2.0 | 1.0 | 999 |\n")
    (root / "profiles" / "hbm_traffic_rmat.md").write_text(table)
    assert bench.measured_traffic("rmat", "k_census_hub<true>") == 3072.0
    assert bench.measured_traffic("rmat", "k_census_lane<true>") is None      # other sources
    assert bench.measured_traffic("citation", "k_census_hub<true>") is None   # no table


def test_committed_traffic_tables_parse():
    # every row of the committed traffic tables has a 16-digit hash and a byte count
    for name in ("hbm_traffic_rmat.md", "hbm_traffic_citation.md", "hbm_traffic_batch.md"):
        path = os.path.join(bench.ROOT, "profiles", name)
        rows = [ln for ln in open(path) if ln.startswith("| k_census") and ln.count("|") == 8]
        assert rows, name
        for ln in rows:
            cells = [c.strip().strip("`") for c in ln.strip().strip("|").split("|")]
            assert len(cells) == 7 and len(cells[1]) == 16 and float(cells[6]) > 0


def test_measured_valu_busy_only_for_the_current_sources(tmp_path, monkeypatch):
    root = _fake_tree(tmp_path, "int g() { return 0; }\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    h = bench.census_source_hash()
    (root / "profiles").mkdir()
    row = "| k_census_hub<true, 1024u> | 2.0 | 4.5e+06 | 0.97 | 0.47 | 0.36 | 0.21 |\n"
    (root / "profiles" / "sq_counters_rmat.md").write_text(f"Source hash `{h}`.\n\n" + row)
    (root / "profiles" / "sq_counters_citation.md").write_text("Source hash `0123456789abcdef`.\n\n" + row)
    assert bench.measured_valu_busy("rmat", "k_census_hub<true, 1024u>") == 0.97
    assert bench.measured_valu_busy("rmat", "k_census_lane<true>") is None
    assert bench.measured_valu_busy("citation", "k_census_hub<true, 1024u>") is None   # other sources
    assert bench.measured_valu_busy("batch", "k_census_hub<true, 1024u>") is None      # no table


def test_kernel_key_names_the_template_instance():
    t = {"hub_tile": 2048, "wave_tile": 512, "group_size": 512, "group_tile": 8192}
    assert bench.kernel_key("k_census_hub", True, t) == "k_census_hub<true, 2048u, 512u>"
    assert bench.kernel_key("k_census_hub", True, t, 256) == "k_census_hub<true, 2048u, 256u>"
    assert bench.kernel_key("k_census_wave", False, t) == "k_census_wave<false, 512>"
    assert bench.kernel_key("k_census_group", True, t) == "k_census_group<true, 512, 8192>"
    assert bench.kernel_key("k_census_lane", True, t) == "k_census_lane<true>"
    assert bench.kernel_key("k_census_totals", True, t) == "k_census_totals"


def test_census_bytes_model():
    info = {"bucket_cost": [10, 20, 30, 40], "bucket_dyads": [1, 2, 3, 4], "hub_stream": 100, "hub_staged": 50,
            "tri_bucket_cost": [5, 0, 0, 7], "tri_bucket_edges": [2, 0, 0, 3], "tri_stream": 11, "tri_staged": 13,
            "asym_dyads": 6, "mutual_dyads": 4}
    # dyad path: 4 B per merged entry + 8 B per record, hub 4 B per streamed and staged entry + 8 B per record
    assert bench.census_bytes(info, 9, False) == 4 * 60 + 8 * 6 + 4 * 150 + 8 * 4
    # forward-list path adds the totals pass: 16 B per neighbour entry (2 per dyad) + 16 B per row
    assert bench.census_bytes(info, 9, True) == 16 * 2 * 10 + 16 * 9 + 4 * 5 + 8 * 2 + 4 * 24 + 8 * 3
