"""CPU checks of bench.py's host logic: the HBM traffic it reports comes only
from a counter record taken from the current library sources in the atom order
being timed, and `--gpus N` with N > 1 is refused (one GPU)."""
import json
import os
import subprocess
import sys

import pytest

import bench


def _record(tmp_path, **over):
    rec = {"source_sha256": bench.kernel_source_hash(), "atom_order": bench.DEFAULT_ORDER,
           "fetch_factor": 2.0, "write_factor": 1.0,
           "kernels": {"chain_pairs": {"fetch_bytes": 3.0e8, "write_bytes": 1.5e9,
                                       "fetch_kib": 1.0, "write_kib": 1.0}}}
    rec.update(over)
    p = tmp_path / "summary.md"
    p.write_text("# summary\n\nsome text\n\ntraffic-record: " + json.dumps(rec) + "\n")
    return str(p)


def test_traffic_is_read_from_a_matching_record(tmp_path):
    t, detail = bench.traffic_from_counters("chain_pairs", _record(tmp_path))
    assert t == pytest.approx(1.8e9)
    assert detail["fetch_bytes"] == 3.0e8 and detail["write_bytes"] == 1.5e9


@pytest.mark.parametrize("over,why", [
    ({"source_sha256": "0" * 64}, "kernel sources changed"),
    ({"atom_order": "identity"}, "another atom order"),
    ({"kernels": {}}, "no counters for chain_pairs"),
])
def test_stale_or_foreign_records_give_no_traffic(tmp_path, over, why):
    t, detail = bench.traffic_from_counters("chain_pairs", _record(tmp_path, **over))
    assert t is None and why in detail


def test_timed_order_must_match(tmp_path):
    p = _record(tmp_path)
    other = "spatial" if bench.DEFAULT_ORDER != "spatial" else "blocks"
    t, detail = bench.traffic_from_counters("chain_pairs", p, other)
    assert t is None and "another atom order" in detail


def test_missing_summary(tmp_path):
    t, detail = bench.traffic_from_counters("chain_pairs", str(tmp_path / "absent.md"))
    assert t is None and detail == "no counter summary"


def test_committed_summaries_carry_a_record():
    # the committed summaries name the order they were taken in and the two
    # copy-calibration factors
    for path in (bench.COUNTER_SUMMARY, bench.EREMD_COUNTER_SUMMARY):
        with open(path) as f:
            lines = [l for l in f if l.startswith("traffic-record: ")]
        rec = json.loads(lines[-1][len("traffic-record: "):])
        assert {"source_sha256", "atom_order", "fetch_factor", "write_factor",
                "kernels"} <= set(rec)
        assert set(rec["kernels"]) == {"radii_pairs", "energy_pairs", "chain_pairs"}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, WORLD_SIZE="1"))
    assert r.returncode == 2 and "one GPU only" in r.stderr
