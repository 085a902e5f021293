"""Autotuner bookkeeping on the CPU: workload keys and the JSON cache."""
import json

from paper_2003_05293_amd import autotune
from workload import Grid


def test_single_key_distinguishes_shapes():
    a = autotune.single_key(Grid(1152, 1152), 100, 30, 1 / 16, "fp32")
    assert a != autotune.single_key(Grid(1152, 1152), 101, 30, 1 / 16, "fp32")
    assert a != autotune.single_key(Grid(1152, 1152), 100, 30, 1 / 16, "mixed")
    assert a != autotune.single_key(Grid(1920, 1152), 100, 30, 1 / 16, "fp32")
    assert a == autotune.single_key(Grid(1152, 1152), 100, 30, 0.0625, "fp32")


def test_table_round_trip(tmp_path):
    path = tmp_path / "t.json"
    t = autotune.Table(str(path))
    key = autotune.single_key(Grid(64, 64), 5, 3, 0.5, "fp32")
    t.entries[key] = {"full_block_cap": 0, "subset_block_cap": 256, "pass_form": 1, "ms": 1.0,
                      "sweep_ms": {"full=0,subset=256,form=1": 1.0}}
    t.save()
    again = autotune.Table(str(path))
    assert again.entries == json.loads(path.read_text())
    assert autotune.Table.as_tune(again.entries[key]) == {"full_block_cap": 0,
                                                          "subset_block_cap": 256,
                                                          "pass_form": 1,
                                                          "chain_passes": 0}
