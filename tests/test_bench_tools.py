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


def test_kernel_classes_of_the_counter_summaries():
    """Demangled kernel names map to the classes whose bytes the counter
    summaries compare with the algorithmic bytes."""
    cases = {
        "__amd_rocclr_copyBuffer": "copy",
        "void haar::fwd2d_kernel<haar::StF32, haar::StF32, haar::StF32, 4, 4, 8, 64, 2, true>(haar::Pass2D, long, long)":
            "fwd2d f32",
        "void haar::inv2d_kernel<haar::StBF16, haar::StBF16, haar::StBF16, 8, 8, 4, 64, true>(haar::Pass2D, long, long)":
            "inv2d bf16",
        "void haar::plan2d_kernel<haar::StBF16, 8, 32, true, false, false, false>(haar::PlanItem2D const*)":
            "plan2d inv bf16",
        "void haar::plan1d_kernel<haar::StF32, false, false, false, true>(haar::PlanItem1D const*)": "plan1d fwd f32",
        "void haar::shrink2d_full_kernel<haar::StF32, 8, 64, 1, false, true>(void const*, void*)": "l1grad2d f32",
        "void haar::shrink2d_full_kernel<haar::StF32, 8, 64, 0, true, true>(void const*, void*)": "shrink2d f32",
        "void haar::shrink1d_full_kernel<haar::StF32, 16, 256, true>(void const*, void*)": "shrink1d f32",
        "haar::l1_loss_reduce_kernel(double const*, double*, long, long)": "l1 loss reduce",
        "void haar::(anonymous namespace)::fwd3d_full_kernel<haar::StBF16, false, 3, false, true>(Pass3D)":
            "fwd3d bf16",
        "void haar::(anonymous namespace)::inv3d_tail_kernel<haar::StF32>(haar::(anonymous namespace)::Tail3D)":
            "inv3d f32",
        "void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<float>>(int)": None,
    }
    for name, cls in cases.items():
        assert bench._kernel_class(name) == cls, name


def test_traffic_summary_scales_by_the_reference_copy(tmp_path, monkeypatch):
    """Counter rows of two passes -> HBM bytes per dispatch, scaled by what
    the same counter reads for the 64 MiB reference copy (the probe's first
    four dispatches), against the algorithmic bytes of the kernel class."""
    import json
    monkeypatch.setattr(bench, "RAW_DIR", str(tmp_path))
    kind = "fused"
    with open(bench._alg_file(kind), "w") as f:
        json.dump({"shrink2d f32": 128 << 20}, f)
    copy = "__amd_rocclr_copyBuffer"
    k = "void haar::shrink2d_full_kernel<haar::StF32, 8, 64, 0, true, true>(void const*, void*)"
    ref_kib = bench.H * bench.W * 4 / 1024.0          # 64 MiB

    def write(path, counter, copy_val, k_val):
        with open(path, "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for i in range(4):
                w.writerow({"Dispatch_Id": i, "Kernel_Name": copy, "Counter_Name": counter,
                            "Counter_Value": copy_val})
            for i in range(4, 8):
                w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": counter, "Counter_Value": k_val})
    # the copy reads half of what it moves on this counter and writes all of it
    write(tmp_path / "f.csv", "FETCH_SIZE", ref_kib / 2, ref_kib / 2)
    write(tmp_path / "w.csv", "WRITE_SIZE", ref_kib, ref_kib)
    out = tmp_path / "t.md"
    bench.write_traffic_kind(kind, str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "cmd", str(out))
    row = [ln for ln in out.read_text().splitlines() if ln.startswith("| shrink2d f32")][0]
    assert row.rstrip(" |").endswith("1.0000"), row
