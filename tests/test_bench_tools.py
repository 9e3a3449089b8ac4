"""Host-side helpers of bench.py: the kernel-code hash that guards the
committed traffic measurement, and the kernel-duration summary."""
import csv

import bench


def test_code_hash_ignores_comments_only():
    code = "int f(int x) {\n    return x + 1;  // one more\n}\n"
    same = "/* header */\nint f(int x) {\n\n    return x + 1;\n}\n// trailing note\n"
    other = "int f(int x) {\n    return x + 2;\n}\n"
    assert bench._code_only(code) == bench._code_only(same)
    assert bench._code_only(code) != bench._code_only(other)


def test_kernel_stats_table_is_capped(tmp_path):
    path = tmp_path / "stats.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage",
                                          "MinNs", "MaxNs"])
        w.writeheader()
        for i in range(40):
            w.writerow({"Name": f"k{i}", "Calls": 1, "TotalDurationNs": 1000 * (i + 1),
                        "AverageNs": 1000 * (i + 1), "Percentage": 1.0, "MinNs": 1, "MaxNs": 2})
    out = tmp_path / "stats.md"
    bench.write_kernel_stats(str(path), "cmd", str(out), max_rows=5)
    text = out.read_text()
    assert "of 40" in text
    assert "`k39`" in text and "`k0`" not in text
    assert len([ln for ln in text.splitlines() if ln.startswith("| `")]) == 5
