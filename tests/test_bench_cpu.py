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
