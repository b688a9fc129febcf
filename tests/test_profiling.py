"""Host logic of the rocprofv3 summaries behind the roofline report (no GPU)."""
import csv
import json

from paper_1111_5059_amd import profiling

FIELDS = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]
HOP = "void dwf::hop_kernel<dwf::P16, 32, 1, false, false, 3, false, false, false>(dwf::HopArgs<dwf::P16>, int, int)"


def write(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for d, g, name, v in rows:
            w.writerow({"Dispatch_Id": d, "Grid_Size": g, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": v})


def test_short_name_strips_namespace_and_arguments():
    assert profiling.short_name(HOP) == "hop_kernel<dwf::P16, 32, 1, false, false, 3, false, false, false>"
    assert profiling.short_name("void dwf::fifth_kernel<dwf::P64, 32>(dwf::CHalf<dwf::P64>)") == \
        "fifth_kernel<dwf::P64, 32>"
    assert profiling.short_name("__amd_rocclr_copyBuffer") is None


def test_calibration_uses_the_last_of_the_largest_copies(tmp_path):
    """A solver copy of the same grid size earlier in the run must not be taken for the 1 GiB
    calibration copy at the end; kernel figures are averaged over dispatches and scaled."""
    copy = "__amd_rocclr_copyBuffer"
    fetch, write_ = tmp_path / "f.csv", tmp_path / "w.csv"
    # KiB per dispatch: the calibration copy reads 2^19 KiB (half of 1 GiB), writes 2^20 KiB
    write(fetch, "FETCH_SIZE", [(1, 1024, copy, 1.5), (5, 131072, copy, 1327132.0), (6, 1000, HOP, 100.0),
                                (7, 1000, HOP, 300.0), (9, 131072, copy, 524288.0)])
    write(write_, "WRITE_SIZE", [(5, 131072, copy, 2654264.0), (6, 1000, HOP, 50.0), (7, 1000, HOP, 50.0),
                                 (9, 131072, copy, 1048576.0)])
    out = tmp_path / "t.json"
    profiling.main(["traffic", str(fetch), str(write_), str(1 << 30), str(out)])
    d = json.loads(out.read_text())
    assert d["fetch_scale"] == 2.0 and d["write_scale"] == 1.0
    k = d["kernels"]["hop_kernel<dwf::P16, 32, 1, false, false, 3, false, false, false>"]
    assert k["dispatches"] == 2
    assert k["fetch_bytes_per_launch"] == 200.0 * 1024 * 2.0
    assert k["write_bytes_per_launch"] == 50.0 * 1024
    assert k["hbm_bytes_per_launch"] == k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]
