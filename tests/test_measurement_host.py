"""Host logic of the measurement: the work model's pair counts against their
closed forms, the byte model's ordering of the RK4 stage variants, and the
rocprofv3 CSV readers on synthetic files of known content, and that the
stand-alone measurement programs still cross-compile for gfx950.  No GPU."""
import csv
import json
import os
import shutil
import subprocess

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
    3 (q+1)^3 + (q+1)^4 facet pairs); a pair on an eta_1 line belongs to every
    S^l, one on the last line family to one."""
    q = p
    vol, fc, nif = pm.pair_counts(dim, p)
    got = sum(n for n, _ in vol) + fc
    want = (q + 1) ** 2 * (q + 3) if dim == 2 else int(round((q + 1) ** 3 * (2.5 * q + 4)))
    assert got == want
    assert [t for _, t in vol] == list(range(dim, 0, -1))
    assert nif == (3 * (q + 1) if dim == 2 else 4 * (q + 1) ** 2)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("p", range(1, 11))
def test_stage_byte_models_are_ordered(dim, p):
    """The plain residual's K2 < the RK4 stage kernel that forms the stage
    combination < that one plus a separate K1; fusing the next projection into
    the stage kernel saves the stage input's write and read; the library's
    layout moves at least the single-pass minimum."""
    plain, rk, fused, k1 = pm.k2_bytes(dim, p), pm.k2_rk_bytes(dim, p), pm.k2_next_bytes(dim, p), pm.k1_bytes(dim, p)
    assert plain < rk < fused < rk + k1
    assert pm.layout_bytes(dim, p) >= pm.min_bytes(dim, p)


def test_minimum_bytes_match_the_stated_figures():
    """8 [N_c (2 N_p + 2 N_f N_qf) + (d^2 + 1) N_q + d N_f N_qf]: tetrahedra
    23.2 KB at p = 4, 54.5 KB at p = 6, 179.7 KB at p = 10; triangles 3.2 KB at
    p = 4, 8.3 KB at p = 8."""
    assert pm.min_bytes(3, 4) == 8 * (5 * (2 * 35 + 2 * 100) + 10 * 125 + 3 * 100)
    assert abs(pm.min_bytes(3, 6) / 1e3 - 54.5) < 0.1 and abs(pm.min_bytes(3, 10) / 1e3 - 179.7) < 0.1
    assert abs(pm.min_bytes(2, 4) / 1e3 - 3.16) < 0.01 and abs(pm.min_bytes(2, 8) / 1e3 - 8.28) < 0.01


def test_flop_model_components():
    """The weighted counts: a division, square root, logarithm and exponential
    cost more than one flop; the residual's flops grow with the degree; the
    volume pairs of a tetrahedron at p = 6 are the distinct pairs times the
    flux and its direction and accumulation."""
    w = pm.weights()
    assert all(w[k] > 1 for k in ("div", "sqrt", "log", "exp"))
    prev = 0
    for p in range(2, 11):
        f = pm.residual_flops(3, p, 0, 1)
        assert f["total"] == f["k1"] + f["k2"] and f["total"] > prev
        prev = f["total"]
    f = pm.residual_flops(3, 6, 0, 0)
    Q = 7
    n = Q * Q * Q * (Q - 1) // 2
    assert f["volume_pairs"] == sum(n * (f["flux_per_pair"] + 9 * t - 3 + 10) for t in (3, 2, 1))


def _write_csv(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


_PMC = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
        "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
        "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _pmc_rows(counter, values):
    """Two residuals (K1, K2) of a single-degree plan and the 1 GiB copy last
    (counter values in KiB, as rocprofv3 reports them)."""
    names = (["void esd::k_entropy_projection<2, 4, false>(double const*)",
              "void esd::k_rhs<2, 4, 0, false>(double const*, double*)"] * 2 + ["__amd_rocclr_copyBuffer"])
    rows = []
    for d, (n, v) in enumerate(zip(names, values), start=1):
        rows.append([d, d, "Agent 1", 1, 1, 1, 1, 1, n, 256, 0, 0, 100, 0, 32, counter, v, 0, 1])
    return rows


def test_traffic_reader_sums_k2_per_residual_and_takes_the_copy_scale(tmp_path, monkeypatch):
    fetch = [9.0, 100.0, 7.0, 120.0, 1 << 19]       # copy: FETCH reads half of 1 GiB
    write = [5.0, 40.0, 3.0, 30.0, 1 << 20]         # copy: WRITE reads all of it
    fcsv, wcsv = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_csv(fcsv, _PMC, _pmc_rows("FETCH_SIZE", fetch))
    _write_csv(wcsv, _PMC, _pmc_rows("WRITE_SIZE", write))
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(prof, "TRAFFIC_FILE", str(out))
    prof.traffic("vortex_tri_M64_p4", str(fcsv), str(wcsv))
    rec = json.load(open(out))["workloads"]["vortex_tri_M64_p4"]
    assert rec["fetch_kib_per_residual"] == [100.0, 120.0]
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["read_bytes_per_residual"] == pytest.approx(110.0 * 1024 * 2.0)
    assert rec["write_bytes_per_residual"] == pytest.approx(35.0 * 1024)
    assert rec["min_bytes_per_residual"] == pm.min_bytes(2, 4) * 8192
    monkeypatch.setattr(prof, "kernel_source_hash", lambda: json.load(open(out))["kernel_source_sha256"])
    assert prof.measured_traffic("vortex_tri_M64_p4") == pytest.approx(110.0 * 1024 * 2.0 + 35.0 * 1024)


def test_batched_k2_dispatches_are_summed_per_residual():
    rows = [(1, "void esd::k_entropy_projection<3, 2, false>(x)", 1.0),
            (2, "void esd::k_entropy_projection<3, 3, false>(x)", 2.0),
            (3, "void esd::k_mixed_exterior<3, 2>(x)", 0.5),
            (4, "void esd::k_rhs<3, 2, 0, false>(x)", 10.0),
            (5, "void esd::k_rhs<3, 3, 0, false>(x)", 20.0),
            (6, "void esd::k_entropy_projection<3, 2, false>(x)", 1.0),
            (7, "void esd::k_rhs<3, 2, 0, false>(x)", 11.0),
            (8, "void esd::k_rhs<3, 3, 0, false>(x)", 21.0)]
    assert prof._per_residual(rows, prof.K2_PREFIX) == [30.0, 32.0]
    assert prof._per_residual(rows, prof.K1_PREFIX) == [3.0, 1.0]


def test_per_residual_sums_split_at_dispatch_id_gaps():
    """Counters taken on K2 alone (--kernel-include-regex): consecutive rows of
    different residuals are split where the dispatch ids jump."""
    rows = [(4, "void esd::k_rhs<3, 2, 0, false>(x)", 10.0),
            (5, "void esd::k_rhs<3, 3, 0, false>(x)", 20.0),
            (9, "void esd::k_rhs<3, 2, 0, false>(x)", 11.0),
            (10, "void esd::k_rhs<3, 3, 0, false>(x)", 21.0)]
    assert prof._per_residual(rows, prof.K2_PREFIX) == [30.0, 32.0]


def test_stats_picks_the_plain_right_hand_side(tmp_path, capsys):
    """Kernel-trace summary: per-residual K2 sums take k_rhs<..., false, false[, false]>
    only (not the fused-stage, dense or deterministic variants)."""
    path = tmp_path / "trace.csv"
    rows = [("void esd::k_rhs<3, 6, 0, false, false, false>(double const*)", 256, 0, 2000),
            ("void esd::k_rhs<3, 6, 0, false, false, false>(double const*)", 256, 0, 2000),
            ("void esd::k_rhs<3, 6, 0, true, false, false>(double const*)", 256, 0, 9000),
            ("void esd::k_rhs<3, 6, 0, false, false, true>(double const*)", 256, 0, 7000),
            ("void esd::k_entropy_projection<3, 6, false>(double const*)", 128, 0, 500)]
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Workgroup_Size_X", "Start_Timestamp", "End_Timestamp"])
        for r in rows:
            w.writerow(r)
    prof.stats(str(path))
    out = capsys.readouterr().out
    assert "K1 0.001 ms, mixed-degree interface 0.000 ms, K2 0.002 ms" in out


MEASURE = os.path.join(os.path.dirname(prof.__file__), "measure")


@pytest.mark.parametrize("src", ["probe_fp64_ops.hip", "transform_mfma.hip"])
def test_measurement_programs_compile_for_gfx950(src, tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not installed")
    cmd = [hipcc, "-O3", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-c", os.path.join(MEASURE, src), "-o", str(tmp_path / "m.o")]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
