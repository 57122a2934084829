"""Host logic of the measurement: the work model's pair counts against their
closed forms, the byte model's ordering of the RK4 stage variants, and the
rocprofv3 CSV readers on synthetic files of known content.  No GPU."""
import csv
import json

import pytest

from paper_2312_07874_amd import perfmodel as pm
from paper_2312_07874_amd import profiling as prof


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("p", range(1, 11))
def test_distinct_pair_counts_match_the_closed_forms(dim, p):
    """Each unordered pair of a collapsed-coordinate line once, plus the facet
    correction pairs: (q+1)^2 (q+3) per triangle, (q+1)^3 (2.5 q + 4) per
    tetrahedron (lines of q+1 nodes: q(q+1)/2 pairs each; triangles 2 (q+1)
    lines and 3 (q+1)^2 facet pairs; tetrahedra 3 (q+1)^2 lines and
    3 (q+1)^3 + (q+1)^4 facet pairs)."""
    q = p
    v2, v1, fc, nif = pm.pair_counts(dim, p)
    got = v2 + v1 + fc
    want = (q + 1) ** 2 * (q + 3) if dim == 2 else int(round((q + 1) ** 3 * (2.5 * q + 4)))
    assert got == want
    assert nif == (3 * (q + 1) if dim == 2 else 4 * (q + 1) ** 2)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("p", range(1, 11))
def test_stage_byte_models_are_ordered(dim, p):
    """The plain residual's K2 < the RK4 stage kernel that forms the stage
    combination < that one plus a separate K1; fusing the next projection into
    the stage kernel saves the stage input's write and read."""
    plain, rk, fused, k1 = pm.k2_bytes(dim, p), pm.k2_rk_bytes(dim, p), pm.k2_next_bytes(dim, p), pm.k1_bytes(dim, p)
    assert plain < rk < fused < rk + k1


def _write_csv(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


_PMC = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
        "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
        "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _pmc_rows(counter, values):
    """K1 first, four stage kernels, a plain residual's K2 and the 1 GiB copy
    last (counter values in KiB, as rocprofv3 reports them)."""
    names = (["void esd::k_entropy_projection<2, 4, false>(double const*)"]
             + ["void esd::k_rhs<2, 4, 0, true>(double const*, double*)"] * 4
             + ["void esd::k_rhs<2, 4, 0, false>(double const*, double*)", "__amd_rocclr_copyBuffer"])
    rows = []
    for d, (n, v) in enumerate(zip(names, values), start=1):
        rows.append([d, d, "Agent 1", 1, 1, 1, 1, 1, n, 256, 0, 0, 100, 0, 32, counter, v, 0, 1])
    return rows


def test_traffic_reader_takes_the_stage_kernels_and_the_copy_scale(tmp_path, monkeypatch):
    fetch = [9.0, 100.0, 120.0, 120.0, 100.0, 7.0, 1 << 19]       # copy: FETCH reads half of 1 GiB
    write = [5.0, 40.0, 40.0, 40.0, 20.0, 3.0, 1 << 20]            # copy: WRITE reads all of it
    fcsv, wcsv = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_csv(fcsv, _PMC, _pmc_rows("FETCH_SIZE", fetch))
    _write_csv(wcsv, _PMC, _pmc_rows("WRITE_SIZE", write))
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(prof, "TRAFFIC_FILE", str(out))
    prof.traffic("vortex_tri_M64_p4", str(fcsv), str(wcsv))
    rec = json.load(open(out))["workloads"]["vortex_tri_M64_p4"]
    assert rec["kernel"] == "esd::k_rhs<2, 4, 0, true>"
    assert rec["fetch_kib_per_stage"] == [100.0, 120.0, 120.0, 100.0]
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["read_bytes_per_launch"] == pytest.approx(110.0 * 1024 * 2.0)
    assert rec["write_bytes_per_launch"] == pytest.approx(35.0 * 1024)
    # the fused stage kernel is priced with its own byte model, 8192 triangles
    assert rec["algorithmic_bytes_per_launch"] == pm.k2_next_bytes(2, 4) * 8192


def test_traffic_reader_rejects_a_run_without_the_calibration_copy(tmp_path, monkeypatch):
    rows = [r for r in _pmc_rows("FETCH_SIZE", [1.0] * 7) if "copyBuffer" not in r[8]]
    fcsv = tmp_path / "f.csv"
    _write_csv(fcsv, _PMC, rows)
    monkeypatch.setattr(prof, "TRAFFIC_FILE", str(tmp_path / "t.json"))
    with pytest.raises(SystemExit):
        prof.traffic("vortex_tri_M64_p4", str(fcsv), str(fcsv))


def test_stats_groups_launches_by_block(tmp_path, capsys):
    hdr = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id", "Kernel_Id", "Kernel_Name",
           "Correlation_Id", "Start_Timestamp", "End_Timestamp", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
           "Accum_VGPR_Count", "SGPR_Count", "Workgroup_Size_X", "Workgroup_Size_Y", "Workgroup_Size_Z",
           "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
    k2 = "void esd::k_rhs<3, 6, 0, false>(double const*)"
    rows = []
    for i, (bs, dur) in enumerate([(256, 2000), (256, 4000), (512, 9000), (256, 3000)]):
        rows.append(["KERNEL_DISPATCH", "Agent 1", 1, 0, 1, i, 1, k2, i, 1000 * i, 1000 * i + dur,
                     0, 0, 100, 0, 32, bs, 1, 1, bs, 1, 1])
    rows.append(["KERNEL_DISPATCH", "Agent 1", 1, 0, 1, 9, 2, "__amd_rocclr_copyBuffer", 9, 0, 5, 0, 0, 8, 0, 32,
                 512, 1, 1, 512, 1, 1])
    t = tmp_path / "trace.csv"
    _write_csv(t, hdr, rows)
    prof.stats(str(t))
    out = capsys.readouterr().out
    assert "| `esd::k_rhs<3, 6, 0, false>` | 256 | 3 | 3.00 |" in out
    assert "| `esd::k_rhs<3, 6, 0, false>` | 512 | 1 | 9.00 |" in out
    assert "copyBuffer" not in out
