"""Host-side logic of bench.py that its JSON line depends on (CPU only): the per-row byte and
flop figures of the roofline, the source hash that decides whether the committed byte-counter
records still apply, and the refusal of more than one GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_bytes_per_row():
    # scalar: d 8 + m 8 (+ 1 flag); 2x2: D 32 + M 32 + 1; CohJones Nd = 10: d 8 + M 80
    assert bench.bytes_per_row(1, 1, False) == 16
    assert bench.bytes_per_row(1, 1, True) == 17
    assert bench.bytes_per_row(4, 1, True) == 65
    assert bench.bytes_per_row(1, 10, False) == 88


def test_gram_flop_figures():
    # per-unit figure: both antennas' Hermitian Nd x Nd blocks, unique entries, 8 flops per
    # complex product (880 at Nd = 10); the pass's own count 4 Nd^2 + 8 Nd; issued: three
    # 16x16x4 MFMAs (2048 flops each) per four samples
    assert bench.unit_gram_flop_per_row(1, 10) == 880
    assert bench.unit_gram_flop_per_row(1, 1) == 16
    assert bench.gram_flop_per_row(1, 10) == 480
    assert bench.gram_issued_flop_per_row(1, 10) == 3 * 2048 / 4
    # 2x2, Nd = 10: 40 model columns + 4 data columns in three 16-column tiles
    assert bench.gram_flop_per_row(4, 10) == 4 * 40 * 40 + 8 * 40 * 4
    assert bench.unit_gram_flop_per_row(4, 10) == bench.gram_flop_per_row(4, 10)
    assert bench.gram_issued_flop_per_row(4, 10) == (3 * 3 + 3 * 3) * 2048 / 4


def test_code_only_drops_comments_and_keeps_strings():
    src = 'int a; // note\n/* block\n comment */ const char* s = "//kept /* too */";\nchar q = \'x\'; f("a\\"b");\n'
    out = bench._code_only(src)
    assert "note" not in out and "block" not in out
    assert '"//kept /* too */"' in out
    assert '"a\\"b"' in out
    assert bench._code_only(src + "// trailing\n") == bench._code_only(src) + "\n"


def test_source_hash_and_traffic_records():
    for fam in bench.KERNEL_SOURCES:
        h = bench.source_hash(fam)
        assert len(h) == 16 and h == bench.source_hash(fam)
    assert bench.measured_traffic("no_such_kernel/no_such_workload") is None


def test_traffic_record_without_sources_is_not_reported(tmp_path, monkeypatch):
    # a tree that ships the records but not the kernel sources cannot match a record to its
    # build: no traffic figure, and no crash
    import json
    (tmp_path / "profiles").mkdir()
    rec = {"dd_gram_dmaf_kernel/cohjones_na64": {"traffic_bytes_per_launch": 1.0, "src_sha": "0" * 16}}
    (tmp_path / "profiles" / "pmc_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("dd_gram_dmaf_kernel/cohjones_na64") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_committed_traffic_records_match_the_sources():
    # a committed byte-counter record taken on the sources in the tree is reported for the
    # default solve of its workload and for no other run; records taken on other sources
    # are reported for none (the counter runs have to be taken again)
    import json
    import pytest
    recs = json.load(open(os.path.join(ROOT, "profiles", "pmc_traffic.json")))
    assert recs
    stale = [k for k, r in recs.items() if r["src_sha"] != bench.source_hash(k.split("_", 1)[0])]
    for key, rec in recs.items():
        want = None if key in stale else rec["traffic_bytes_per_launch"]
        assert bench.measured_traffic(key) == want
        assert bench.measured_traffic(key, default_solve=False) is None
    if stale:
        pytest.skip(f"records taken on other sources (take the counter runs again): {stale}")
