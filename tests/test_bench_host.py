"""Host-side behaviour of bench.py that needs no GPU: the one-GPU contract
(--gpus above 1 exits with a message), the algorithmic byte counts the
roofline uses, and the mixed-precision error report."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_algorithmic_bytes():
    ne, ned, nn = 4_000_000, 6_000_000, 2_000_000
    assert bench.algorithmic_bytes("k_stage", ne, ned, nn, "fp64") == 315.0 * ne
    assert bench.algorithmic_bytes("k_stage", ne, ned, nn, "mixed") == 207.0 * ne
    assert bench.algorithmic_bytes("k_rhs2", ne, ned, nn, "fp64") == 548.0 * ne
    assert bench.algorithmic_bytes("k_forcing", ne, ned, nn) == 40.0 * nn
    assert bench.algorithmic_bytes("k_vbounds", ne, ned, nn, "fp64") == 56.0 * nn + 36.0 * ne


def test_roofline_fraction_from_kernel_times():
    kernels = {"k_stage": {"avg_us": 400.0, "launches": 10, "total_ms": 4.0},
               "k_forcing": {"avg_us": 30.0, "launches": 5, "total_ms": 0.15}}
    r = bench.roofline(kernels, 1_000_000, 1_500_000, 500_000, "fp64", with_traffic=False)
    assert r["kernel"] == "k_stage" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["achieved"] - 315e6 / 400e-6 / 1e9) < 0.1
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-4


def test_mixed_error_report():
    rng = np.random.default_rng(1)
    wf = rng.normal(size=(3, 3, 50))
    wm = wf.copy()
    wm[0, 2, 7] += 1e-6  # mode 2 of zeta: vertex values change by -1e-6, -1e-6, +2e-6
    e = bench.mixed_error(wm, wf)
    assert abs(e["zeta_vertex_max_m"] - 2e-6) < 1e-15 and e["zeta_mean_max_m"] == 0.0 and e["q_mean_max_m2s"] == 0.0


def test_mixed_roofline_uses_207_bytes_and_reports_the_built_count():
    kernels = {"k_stage": {"avg_us": 300.0, "launches": 10, "total_ms": 3.0}}
    r = bench.roofline(kernels, 1_000_000, 1_500_000, 500_000, "mixed", with_traffic=False)
    assert r["bytes_per_launch"] == 207_000_000
    assert abs(r["frac"] - 207e6 / 300e-6 / 8e12) < 1e-4
    assert r["as_built"]["bytes_per_element_stage"] == 217.0
    assert abs(r["as_built"]["frac"] - 217e6 / 300e-6 / 8e12) < 1e-4


def test_cpu_model_is_named():
    assert bench.cpu_model() != ""


def test_ensemble_bytes_and_kernel_names():
    """the fused stage of an ensemble of both orders carries the p = 1
    stage of its p = 1 elements and the p = 2 right-hand side of the rest"""
    ne = {1: 1000, 2: 3000}
    b = bench.algorithmic_bytes("k_stage12", ne, 0, 0, "mixed")
    assert b == bench.B_ALG_MIXED * 1000 + bench.B_ALG_P2[("k_rhs2", "mixed")] * 3000
    assert bench.algorithmic_bytes("k_pp2", ne, 0, 0, "mixed") == bench.B_ALG_P2[("k_pp2", "mixed")] * 3000
    assert bench.algorithmic_bytes("k_forcing", ne, 0, 500, "mixed") == 40.0 * 500
    assert bench.kernel_key("void dgswe::k_stage12<float, 1, 2, false>(dgswe::DevMesh, ...)") == ("k_stage12", "mixed")
    assert bench.kernel_key("void dgswe::k_stage<256, 2, double, 0, false, false>(...)") == ("k_stage", "fp64")
    assert bench.kernel_key("void dgswe::k_rhs2<double, 3, false>(...)") == ("k_rhs2", "fp64")


def test_roofline_of_a_p1_only_ensemble():
    """a p = 1 ensemble (element counts per order) keeps the as-built mixed
    figure of the stage kernel"""
    k = {"k_stage": {"avg_us": 100.0, "total_ms": 1.0, "launches": 10}}
    r = bench.roofline(k, {1: 1_000_000, 2: 0}, 0, 0, "mixed", with_traffic=False)
    assert r["kernel"] == "k_stage" and r["bytes_per_launch"] == int(bench.B_ALG_MIXED * 1_000_000)
    assert r["as_built"]["bytes_per_launch"] == int(bench.B_ALG_MIXED_AS_BUILT * 1_000_000)


def _pmc_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w") as fh:
        fh.write("Dispatch_Id,Grid_Size,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (grid, name, val) in enumerate(rows):
            fh.write(f'{i},{grid},"{name}",X,{val}\n')


def test_summarize_pmc_calibrates_and_keeps_the_ensemble_sized_launches(tmp_path, monkeypatch):
    """the counters scale by the 2 GiB copy of the same run; in the ensemble
    run only the largest grid of each kernel counts (the autotuner's
    single-member launches and the persistent grids are smaller)"""
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    copy = "__amd_rocclr_copyBuffer"
    st = "void dgswe::k_stage<256, 2, double, 0, false, false>(dgswe::DevMesh)"
    st1 = "void dgswe::k_stage<256, 2, double, 1, false, false>(dgswe::DevMesh)"
    sp = "void dgswe::k_stage1pp2<float, 0, 2, false>(dgswe::DevMesh)"
    spp = "void dgswe::k_stage1pp2<float, 0, 2, true>(dgswe::DevMesh)"
    kib = 2 * 1024 ** 2  # a 2 GiB copy in KiB
    for tag, f in (("FETCH_SIZE", 0.5), ("WRITE_SIZE", 1.0)):
        _pmc_csv(tmp_path / "pmc" / tag, [(1 << 20, copy, kib * f), (1000, st, 100.0), (1000, st1, 300.0)])
        _pmc_csv(tmp_path / "pmc" / "ensemble" / tag,
                 [(1 << 20, copy, kib * f), (5000, sp, 1000.0), (5000, sp, 3000.0), (800, spp, 7.0), (64, sp, 9.0)])
    md = tmp_path / "out" / "k_stage.md"
    md.parent.mkdir()
    bench.summarize_pmc(str(tmp_path / "pmc"), None, str(md))
    rec = json.loads((tmp_path / "traffic.json").read_text())
    assert rec["calibration"]["FETCH_SIZE"]["factor"] == 2.0 and rec["calibration"]["WRITE_SIZE"]["factor"] == 1.0
    k = rec["kernels"]["k_stage"]["fp64"]
    assert k["dispatches"] == [2, 2] and k["bytes_per_launch"] == round(200.0 * 1024 * 2 + 200.0 * 1024)
    assert k["grid_size"] == 1000
    e = rec["ensemble"]["k_stage1pp2"]["mixed"]
    assert e["grid_size"] == 5000 and e["dispatches"] == [2, 2]
    assert e["bytes_per_launch"] == round(2000.0 * 1024 * 2 + 2000.0 * 1024)
    assert (tmp_path / "out" / "ensemble_64_members_mixed.md").exists()
    assert (tmp_path / "out" / "k_rhs2_k_pp2_hurricane_4M_p2.md").exists()


def test_summarize_counters_tabulates_the_largest_grid(tmp_path):
    """per-wave counts and time shares from the two counter runs, for the
    4M-mesh launches only"""
    name = "void dgswe::k_rhs2<double, 3, false, false>(dgswe::DevMesh)"
    c1 = {"SQ_WAVES": 100, "SQ_WAVE_CYCLES": 1000, "SQ_INSTS_VALU": 4000, "SQ_INSTS_VMEM_RD": 50,
          "SQ_ACTIVE_INST_VALU": 300, "SQ_WAIT_INST_ANY": 200, "SQ_ACTIVE_INST_LDS": 40}
    c2 = {"TCC_HIT_sum": 60, "TCC_MISS_sum": 40, "SQ_INSTS_LDS": 1300, "SQ_ACTIVE_INST_ANY": 450, "SQ_WAIT_ANY": 350,
          "SQ_LDS_BANK_CONFLICT": 10}
    for tag, cs in (("c1", c1), ("c2", c2)):
        os.makedirs(tmp_path / tag)
        with open(tmp_path / tag / "run_counter_collection.csv", "w") as fh:
            fh.write("Dispatch_Id,Grid_Size,Kernel_Name,Counter_Name,Counter_Value\n")
            for k, v in cs.items():
                fh.write(f'1,5000,"{name}",{k},{v}\n')
                fh.write(f'2,64,"{name}",{k},{v * 7}\n')  # a small launch: ignored
    md = tmp_path / "c.md"
    bench.summarize_counters(str(tmp_path), ("k_rhs2",), "t", str(md))
    row = [l for l in md.read_text().splitlines() if l.startswith("| `k_rhs2")][0]
    cells = [x.strip() for x in row.strip("|").split("|")]
    assert cells[1:] == ["1", "100", "40", "13", "0", "45.0", "30.0", "4.0", "20.0", "35.0", "25", "60.0",
                         f"{40 * 128 / 1e9:.3f} GB"]
