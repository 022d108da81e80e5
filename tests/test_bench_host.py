"""Host logic of bench.py (no GPU): which committed counter record the bench reports."""
import json
import os

import bench


def _write(tmp_path, name, d):
    prof = tmp_path / "profiles"
    prof.mkdir(exist_ok=True)
    (prof / name).write_text(json.dumps(d))


def test_pmc_traffic_picks_the_record_of_the_launch(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    la = {"waves_per_block": 2, "blocks_per_cu": 0, "chunk_trees": 1024, "stack_depth": 6}
    lb = dict(la, waves_per_block=4, stack_depth=8)
    _write(tmp_path, "walk_fisher_pmc.json",
           {"kernel_source_sha256": "abc", "hbm_bytes_per_launch": 2.0, "launch": lb,
            "by_launch": [{"launch": la, "hbm_bytes_per_launch": 1.0}, {"launch": lb, "hbm_bytes_per_launch": 2.0}]})
    assert bench.pmc_traffic("abc", la) == (1.0, la)
    assert bench.pmc_traffic("abc", lb) == (2.0, lb)
    # no record for this launch: the latest one, with its launch
    assert bench.pmc_traffic("abc", dict(la, waves_per_block=1)) == (2.0, lb)
    # counters taken on another source are not reported
    assert bench.pmc_traffic("other", la) == (None, None)


def test_committed_counter_records_name_their_launch():
    with open(os.path.join(bench.ROOT, "profiles", "walk_fisher_pmc.json")) as f:
        d = json.load(f)
    launches = [r["launch"] for r in d["by_launch"]]
    assert d["launch"] in launches and len({json.dumps(x, sort_keys=True) for x in launches}) == len(launches)
    for r in d["by_launch"]:
        assert r["hbm_bytes_per_launch"] >= d["algorithmic_bytes_per_launch"]
