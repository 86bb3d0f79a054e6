"""Host logic of the profile summaries: HBM traffic of a phase from FETCH_SIZE
and WRITE_SIZE counters, each scaled by what it reads for the copy kernel of
known size; several kernels of one phase add up."""
import csv

from paper_2208_09132_amd import profiling as pf


def _counters(path, name, rows):
    path.mkdir()
    with open(path / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for kernel, values in rows.items():
            for v in values:
                w.writerow({"Kernel_Name": kernel, "Counter_Name": name, "Counter_Value": v})


def test_phase_traffic_sums_its_kernels_with_copy_calibration(tmp_path):
    copy = "void cdg::k_to_f64<double>(cdg::Problem, void const*, double*)"
    a, b = "void cdg::k_face_values_z<float>(cdg::Problem)", "void cdg::k_face_reduce<3, float>(cdg::Problem)"
    copy_bytes = 1024.0 * 1000
    # the copy's FETCH_SIZE reads half its bytes (factor 2), WRITE_SIZE all (factor 1)
    _counters(tmp_path / "f", "FETCH_SIZE", {copy: [500, 500], a: [100, 300], b: [50]})
    _counters(tmp_path / "w", "WRITE_SIZE", {copy: [1000], a: [40], b: [7, 9]})
    out = tmp_path / "t.md"
    pf.write_pmc(str(tmp_path / "f"), str(tmp_path / "w"), str(out), [r"k_face_values_z", r"k_face_reduce"],
                 "t", ["cmd"], units_per_launch=10.0, algo_bytes_per_unit=8.0, copy_bytes=copy_bytes)
    rec = pf.load_record(str(out))
    assert rec["digest"] == pf.source_digest()
    assert rec["fetch_factor"] == 2.0 and rec["write_factor"] == 1.0
    assert rec["fetch_bytes"] == (200 + 50) * 1024.0 * 2.0
    assert rec["write_bytes"] == (40 + 8) * 1024.0
    assert rec["traffic_bytes"] == rec["fetch_bytes"] + rec["write_bytes"]
    assert [k["kernel"] for k in rec["kernels"]] == [a, b]
    assert rec["algorithmic_bytes"] == 80.0
