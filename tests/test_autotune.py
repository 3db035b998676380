"""CPU checks of the autotuner's bins and table lookup, and of the committed
table's contents."""
import json

from paper_1705_05443_amd import autotune as A


def test_size_bins():
    assert A.size_bin(65536, 2, "strong", "f64", 16) == "d2-strong-f64-r16-n16"
    assert A.size_bin(1 << 20, 3, "h2", "bf16", 64) == "d3-strong-bf16-r64-n20"
    assert A.size_bin(2048, 1, "weak", "f64", 1) == "d1-weak-f64-r1-n11"
    # right-hand-side classes and nearest power of two
    assert A.size_bin(3000, 1, "weak", "f32", 17).endswith("-r64-n12")
    assert A.size_bin(100000, 2, "strong", "f32", 2).endswith("-r16-n17")


def test_lookup_exact_then_nearest_bin():
    table = {
        "d2-strong-f64-r16-n16": {"shape": {"mv_split_nodes": 256, "mv_xcd_run": 4}},
        "d2-strong-f64-r16-n20": {"shape": {"mv_split_nodes": 4096, "mv_xcd_run": 64}},
        "d3-strong-f32-r64-n20": {"shape": {"mv_split_nodes": 64, "mv_xcd_run": 1}},
    }
    assert A.lookup(65536, 2, "strong", "f64", 16, table)["mv_xcd_run"] == 4
    assert A.lookup(1 << 19, 2, "strong", "f64", 16, table)["mv_xcd_run"] == 64
    assert A.lookup(1 << 17, 2, "strong", "f64", 16, table)["mv_xcd_run"] == 4
    assert A.lookup(65536, 2, "strong", "f32", 16, table) is None
    assert A.lookup(65536, 3, "strong", "f32", 64, table)["mv_split_nodes"] == 64


def test_committed_table_holds_valid_shapes():
    table = A.load_table()
    for key, entry in table.items():
        assert key.startswith("d") and "-r" in key and "-n" in key
        shp = entry["shape"]
        assert shp["mv_split_nodes"] in A.KNOBS["mv_split_nodes"]
        assert shp["mv_xcd_run"] in A.KNOBS["mv_xcd_run"]
        assert entry["ms"] > 0
    json.dumps(table)
