"""Host logic of bench.py that turns rocprofv3 counter tables into HBM bytes
per launch: the copy calibration, the choice of launches priced, and the
per-kernel records the roofline line reads."""

import csv

import bench

FIELDS = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
COPY = "__amd_rocclr_copyBuffer"


def _write(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def _lat(flags, prec="float", shape="64, 4, 1"):
    return f"void rlb::(anonymous namespace)::k_step_lattice<{prec}, {shape}, {flags}>(...)"


def test_write_traffic_scales_by_the_copy_and_prices_plain_steps(tmp_path):
    cells = 1000
    kib = 1024.0
    # the 1 GiB copy: FETCH_SIZE reads half the bytes, WRITE_SIZE all of them
    fetch = [(COPY, "131072", "FETCH_SIZE", (1 << 29) / kib)]
    write = [(COPY, "131072", "WRITE_SIZE", (1 << 30) / kib)]
    alg = 2 * 38 * 4 * cells
    # priced: no diagnostics, no extended model; either store kind
    fetch.append((_lat("false, false, true"), "1", "FETCH_SIZE", alg / 2 / 2 / kib))
    write.append((_lat("false, false, true"), "1", "WRITE_SIZE", alg / 2 / kib))
    fetch.append((_lat("false, false, false", shape="256, 1, 1"), "1", "FETCH_SIZE",
                  alg / 2 / kib))  # 2x the algorithmic read bytes once scaled
    write.append((_lat("false, false, false", shape="256, 1, 1"), "1", "WRITE_SIZE",
                  alg / 2 / kib))
    # not priced: fused diagnostics, extended model
    for flags in ("true, false, true", "false, true, true"):
        fetch.append((_lat(flags, shape="128, 2, 1"), "1", "FETCH_SIZE", 1.0))
        write.append((_lat(flags, shape="128, 2, 1"), "1", "WRITE_SIZE", 1.0))
    _write(tmp_path / "f.csv", fetch)
    _write(tmp_path / "w.csv", write)
    out = bench.write_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), cells=cells)
    assert abs(out["_calibration"]["scale"]["FETCH_SIZE"] - 2.0) < 1e-12
    assert abs(out["_calibration"]["scale"]["WRITE_SIZE"] - 1.0) < 1e-12
    names = sorted(k for k in out if not k.startswith("_"))
    assert names == ["k_step_lattice<float,256,1,1>", "k_step_lattice<float,64,4,1>"]
    rec = out["k_step_lattice<float,64,4,1>"]
    assert rec["algorithmic_bytes"] == alg
    assert abs(rec["ratio"] - 1.0) < 1e-12
    assert abs(out["k_step_lattice<float,256,1,1>"]["ratio"] - 1.5) < 1e-12
    assert rec["source_hash"] == bench.kernel_hash()


def test_valu_summary_fractions(tmp_path):
    # one dispatch of 1 ms at 2 GHz (GRBM_GUI_ACTIVE summed over 8 XCDs):
    # half the VALU issue slots used, VALU busy a quarter of the time
    cycles = 2.0e9 * 1e-3
    name = "void rlb::(anonymous namespace)::k_step_tubes<float, 256, false>(rlb::TubeRound)"
    fields = ["Dispatch_Id", "Grid_Size", "Workgroup_Size", "Kernel_Name", "Counter_Name",
              "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    vals = {"SQ_INSTS_VALU": 0.5 * bench.CU_NUM * cycles,
            "SQ_ACTIVE_INST_VALU": 0.25 * bench.CU_NUM * cycles,
            "SQ_INSTS_LDS": 0.1 * bench.CU_NUM * cycles,
            "GRBM_GUI_ACTIVE": bench.XCC_NUM * cycles}
    with open(tmp_path / "c.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for c, v in vals.items():
            w.writerow({"Dispatch_Id": 7, "Grid_Size": 65536, "Workgroup_Size": 256,
                        "Kernel_Name": name, "Counter_Name": c, "Counter_Value": v,
                        "Start_Timestamp": 1000, "End_Timestamp": 1000 + 1000000})
    text = bench.valu_summary(str(tmp_path / "c.csv"), "cmd")
    row = [l for l in text.splitlines() if l.startswith("| `k_step_tubes")]
    assert len(row) == 1
    cells = [c.strip() for c in row[0].split("|")[1:-1]]
    assert cells[3] == "1" and cells[4] == "1000.0" and cells[5] == "2.00"
    assert cells[7] == "0.500" and cells[8] == "0.250" and cells[9] == "0.200"
    assert cells[10] == f"{0.5 * 2.0 / 2.4:.3f}"  # the same issues over 2.4 GHz cycles


def test_d2q9_traffic_names_both_corrected_kernels(tmp_path):
    n = 64
    cells = n * n
    one = 2 * 18 * 4 * cells
    kib = 1024.0
    fetch = [(COPY, "131072", "FETCH_SIZE", (1 << 29) / kib)]
    write = [(COPY, "131072", "WRITE_SIZE", (1 << 30) / kib)]
    kern = {
        "void rlb::(anonymous namespace)::k_d2q9_lattice<float, 128, 2, 1, false, true, false, "
        "true>(...)": 1.0,
        "void rlb::(anonymous namespace)::k_d2q9_lattice_c7<float, 64, 8, false, false, "
        "true>(...)": 1.25,
        "void rlb::(anonymous namespace)::k_d2q9_lattice_c7<float, 64, 8, true, false, "
        "true>(...)": 9.0,  # fused diagnostics: not priced
    }
    for k, r in kern.items():
        fetch.append((k, str(cells), "FETCH_SIZE", r * one / 2 / 2 / kib))
        write.append((k, str(cells), "WRITE_SIZE", r * one / 2 / kib))
    _write(tmp_path / "f.csv", fetch)
    _write(tmp_path / "w.csv", write)
    out = bench.d2q9_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), n=n)["kernels"]
    assert sorted(out) == ["k_d2q9_lattice<float,128,2,1>+c7", "k_d2q9_lattice<float,64,8,1>+c7"]
    assert abs(out["k_d2q9_lattice<float,128,2,1>+c7"]["ratio_to_one_step"] - 1.0) < 1e-12
    assert abs(out["k_d2q9_lattice<float,64,8,1>+c7"]["ratio_to_one_step"] - 1.25) < 1e-12


def test_d2q9_tile_rounds_priced_per_cell_update(tmp_path):
    """A tile-round launch advances H steps: its bytes and VALU instructions
    per cell update divide by the cells and by H, which is recovered from the
    number of tiles in the launch grid."""
    n = 4096
    cells = n * n
    kib = 1024.0
    # 32 x 32 window, H = 3: owned 26 x 26, ceil(4096 / 26) = 158 tiles a side
    tiles = 158 * 158
    k = ("void rlb::(anonymous namespace)::k_d2q9_tiles<float, 32, 32, 512, false, "
         "false>(rlb::TileRound)")
    fetch = [(COPY, "131072", "FETCH_SIZE", (1 << 29) / kib),
             (k, str(tiles * 512), "FETCH_SIZE", 56.0 * cells * 3 / 2 / 2 / kib)]
    write = [(COPY, "131072", "WRITE_SIZE", (1 << 30) / kib),
             (k, str(tiles * 512), "WRITE_SIZE", 56.0 * cells * 3 / 2 / kib)]
    _write(tmp_path / "f.csv", fetch)
    _write(tmp_path / "w.csv", write)
    out = bench.d2q9_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), n=n)["kernels"]
    rec = out["k_d2q9_tiles<float,32,32>/h3"]
    assert rec["steps_per_launch"] == 3
    assert abs(rec["bytes_per_cell_update"] - 56.0) < 1e-9
    _write(tmp_path / "v.csv", [(k, str(tiles * 512), "SQ_INSTS_VALU", 7.0 * cells * 3)])
    v = bench.valu_record(str(tmp_path / "v.csv"), n=n)["kernels"]
    assert abs(v["k_d2q9_tiles<float,32,32>/h3"]["valu_per_cell_update"] - 7.0) < 1e-12


def test_graph_shape_counts_the_kernel_nodes():
    assert bench.graph_shape("k_step_tubes<float,256>/h8", 3000) == {
        "graph_launches": 1, "kernel_nodes": 375, "steps_per_node": 8}
    assert bench.graph_shape("k_d2q9_strips<double,256>/h8", 400)["kernel_nodes"] == 50
    assert bench.graph_shape("k_step_members<float,512,1>", 3000) == {
        "graph_launches": 1, "kernel_nodes": 1, "steps_per_node": 3000}


def test_more_than_one_gpu_is_refused_before_any_device_work():
    import os
    import subprocess
    import sys
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(here, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def test_adjoint_trace_summary(tmp_path):
    """Reverse steps, recomputation kernels, their overlap and the sweeps of
    a synthetic kernel trace (two sweeps, every other step overlapped)."""
    import csv
    p = tmp_path / "run_kernel_trace.csv"
    with open(p, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp",
                    "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"])
        t = 0
        for i in range(10):
            w.writerow(["void rlb::k_adj_step<float, true>(x)", t, t + 15000, 512, 512, 1])
            if i % 2 == 0:
                w.writerow(["void rlb::k_gstep<float>(x)", t + 5000, t + 14000, 512, 512, 1])
            t += 16000
        w.writerow(["void rlb::k_adj_step<float, true>(x)", 0, 1, 64, 64, 1])  # other grid
        t += 5_000_000
        for i in range(5):
            w.writerow(["void rlb::k_adj_step<float, true>(x)", t, t + 15000, 512, 512, 1])
            t += 15500
    md = bench.adjoint_trace(str(p), "cmd", steps=10)
    assert "| `k_adj_step` (reverse step) | 15 | 15.00 | 15.00 |" in md
    assert "| `k_gstep` (recomputation) | 5 | 9.00 | 9.00 |" in md
    assert "5 of 15 (33.3 %)" in md
    assert "| 0 | 10 |" in md and "| 1 | 5 |" in md


def test_adjoint_traffic_summary(tmp_path):
    """Byte counters of a synthetic PMC pair: the copy sets the scale, only
    the reverse-sweep kernels on the lattice's grid are priced, against 57
    (reverse step) and 38 (recomputation) FP32 values per cell."""
    import csv
    cells = 4096
    rows = {"FETCH_SIZE": [], "WRITE_SIZE": []}
    # copy: 1 GiB each way, counters read half (fetch) and all (write)
    rows["FETCH_SIZE"].append(("copyBuffer", 131072, (1 << 30) / 2 / 1024))
    rows["WRITE_SIZE"].append(("copyBuffer", 131072, (1 << 30) / 1024))
    # a checkpoint copy of one state does not count towards the calibration
    rows["FETCH_SIZE"].append(("copyBuffer", 131072, 1e3))
    rows["WRITE_SIZE"].append(("copyBuffer", 131072, 1e3))
    adj = "void rlb::(anonymous namespace)::k_adj_step<float, true>(float const*, float*)"
    gst = "void rlb::(anonymous namespace)::k_gstep<float>(float const*, float*)"
    for _ in range(3):
        rows["FETCH_SIZE"].append((adj, cells, 38 * 4 * cells / 2 / 1024))
        rows["WRITE_SIZE"].append((adj, cells, 19 * 4 * cells * 1.1 / 1024))
        rows["FETCH_SIZE"].append((gst, cells, 19 * 4 * cells / 2 / 1024))
        rows["WRITE_SIZE"].append((gst, cells, 19 * 4 * cells / 1024))
    rows["FETCH_SIZE"].append((gst, 64, 1e9))  # another grid
    rows["WRITE_SIZE"].append((gst, 64, 1e9))
    paths = []
    for c, rs in rows.items():
        p = tmp_path / f"{c}.csv"
        with open(p, "w", newline="") as fh:
            w = csv.writer(fh)
            w.writerow(["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
            for k, g, v in rs:
                w.writerow([k, g, c, v])
        paths.append(str(p))
    md = bench.adjoint_traffic(paths[0], paths[1], "cmd", cells=cells)
    assert "FETCH_SIZE x 2.0000, WRITE_SIZE x 1.0000" in md
    # (38 + 19 * 1.1) / 57 = 1.0333
    assert "| `k_adj_step<float, true>` | 3 | 6.2259e+05 | 3.4243e+05 | 1.0333 |" in md
    assert "| `k_gstep<float>` | 3 | 3.1130e+05 | 3.1130e+05 | 1.0000 |" in md
