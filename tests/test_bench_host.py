"""bench.py's host logic on the CPU: the algorithmic byte model behind the
roofline figures, the mapping of kernel names onto bench kinds, the
rocprofv3 summary (calibrated HBM traffic per launch) that the bench reads
back while the library's sources are unchanged, and the bookkeeping of its
timing windows."""
import csv
import os

import bench

SLAB = "eo_slab_64x64x130"


def test_byte_model_of_the_step_passes():
    """Per fluid site, K = 2: the LB pass moves 19 populations in and out,
    two concentrations in, two increments out, phi (FP64), the velocity and
    the flag word; the ion pass three concentration arrays, the velocity,
    the FP64 source and the flag word, the mixed form also the low words of
    its concentration pairs, plus the potential history of the extrapolated
    start (48 B) or the kept copy of phi (16 B)."""
    assert bench.bytes_per_cell("fluid", "fp32", 2) == 2 * 19 * 4 + 2 * 2 * 4 + 8 + 12 + 4 == 192
    assert bench.bytes_per_cell("fluid", "fp64", 2) == 2 * 19 * 8 + 2 * 2 * 8 + 8 + 24 + 4 == 372
    assert bench.bytes_per_cell("ions", "fp64", 2) == 3 * 2 * 8 + 24 + 8 + 4 + 16 == 100
    assert bench.bytes_per_cell("ions", "fp32", 2, extrap=True) == \
        3 * 2 * 4 + 2 * 2 * 4 + 12 + 8 + 4 + 48 == 112
    # the last Jacobi sweep on the finest level also adds e to phi (FP64 in + out)
    for form in ("fp32", "fp64"):
        assert (bench.bytes_per_cell("mg_smooth0_phi", form, 2)
                == bench.bytes_per_cell("mg_smooth0", form, 2) + 16)
    # kernels with no byte model: the one-work-group coarse end, the charge
    assert bench.bytes_per_cell("mg_small", "fp32", 2) is None
    assert bench.bytes_per_cell("charge", "fp64", 2) is None


def test_kernel_names_map_onto_bench_kinds():
    n = 64 * 64 * 130
    c = bench._classify
    assert c("void lbe::k_fluid_f32_ring<2, true>(lbe::Lattice, ...)", 1000, n) == ("fp32-mg", "fluid")
    assert c("void lbe::k_ions_f64_tiled<2, true>(lbe::Lattice)", 1000, n) == ("fp64-mg", "ions")
    # a finest-level ring launch covers RING_ZRUN planes per work-item
    assert c("void lbe::k_jacobi_ring<float, true>(int)", n // bench.RING_ZRUN, n) == \
        ("fp32-mg", "mg_smooth0_phi")
    assert c("void lbe::k_jacobi<double, false>(int)", n // 8, n) == ("fp64-mg", "mg_smooth")
    # a kernel without a precision in its name takes the form of the one before it
    assert c("void lbe::k_charge(lbe::Lattice)", 10, n, "fp32-mg") == ("fp32-mg", "charge")
    assert c("void lbe::k_ctl_reset(lbe::SolveCtl*, double)", 1, n, "fp32-mg") is None


def _write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_rocprof_summary_is_calibrated_and_read_back(tmp_path, monkeypatch):
    """Synthetic rocprofv3 CSV output: a 256 MiB copy that FETCH_SIZE reads as
    half its bytes and WRITE_SIZE as all of them sets the factors 2 and 1;
    two LB-pass launches and one converged (empty) launch, whose counters
    stay under 4 KiB and are left out of the mean.  The summary's traffic
    line is read back by the bench while its sources line matches the
    library's sources, and ignored otherwise."""
    root = tmp_path / "prof"
    fluid = "void lbe::k_fluid_f32<2, 256, false>(lbe::Lattice, lbe::Phys)"
    n = 64 * 64 * 130
    _write_csv(str(root / "trace" / "trace_kernel_stats.csv"), [
        {"Name": fluid, "Calls": 2, "TotalDurationNs": 60000, "AverageNs": 30000,
         "MinNs": 29000, "MaxNs": 31000}])
    _write_csv(str(root / "trace" / "trace_kernel_trace.csv"), [
        {"Kernel_Name": fluid, "Start_Timestamp": 1000 + 40000 * i,
         "End_Timestamp": 31000 + 40000 * i, "Grid_Size": n} for i in range(2)])
    for counter, sub, cal_kib, vals in (("FETCH_SIZE", "fetch", 131072, (50000, 52000, 2)),
                                        ("WRITE_SIZE", "write", 262144, (40000, 40000, 1))):
        rows = [{"Dispatch_Id": 1, "Kernel_Name": "void copy_calibration(float*)",
                 "Counter_Name": counter, "Counter_Value": cal_kib, "Grid_Size": 1 << 26}]
        rows += [{"Dispatch_Id": 2 + i, "Kernel_Name": fluid, "Counter_Name": counter,
                  "Counter_Value": v, "Grid_Size": n} for i, v in enumerate(vals)]
        _write_csv(str(root / sub / f"{sub}_counter_collection.csv"), rows)
    text = bench.summarize_rocprof(str(root), SLAB)
    fetch = 51000 * 1024 * 2.0
    write = 40000 * 1024 * 1.0
    assert f"traffic fp32-mg fluid {int(round(fetch))} {int(round(write))}" in text
    assert f"sources {bench.sources_hash()}" in text

    prof = tmp_path / "repo" / "profiles"
    prof.mkdir(parents=True)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path / "repo"))
    (prof / f"step_traffic_{SLAB}.txt").write_text(text)
    assert bench.load_traffic(SLAB) == {("fp32-mg", "fluid"): fetch + write}
    (prof / f"step_traffic_{SLAB}.txt").write_text(
        text.replace(f"sources {bench.sources_hash()}", "sources 0000000000000000"))
    assert bench.load_traffic(SLAB) == {}


class _FakeContext:
    """Stands in for lbe.Lbe in the window bookkeeping: each step adds one
    Poisson iteration, a replayed window with one unit fails after its
    steps as lbe_step_chunk does."""

    def __init__(self):
        self.step_no, self.iters = 1000, 0

    def totals(self):
        return {"step": self.step_no, "poisson_total": self.iters}

    def step(self, n):
        self.step_no += n
        self.iters += n

    def step_chunk(self, n, units):
        self.step_no += n
        self.iters += 2 * n
        if units < 2:
            raise bench.lbe.LbeError(bench.lbe.ENOCONV, "Poisson not converged")


def test_timing_windows_count_steps_and_keep_replay_errors(monkeypatch):
    monkeypatch.setattr(bench, "sync", lambda: None)
    g = _FakeContext()
    el, first, it, err = bench.time_window(g, 32)
    assert first == 1000 and it == 1.0 and err is None and el >= 0.0
    el, first, it, err = bench.time_window(g, 32, chunk_units=3)
    assert first == 1032 and it == 2.0 and err is None
    el, first, it, err = bench.time_window(g, 32, chunk_units=1)
    assert first == 1064 and it == 2.0 and "not converged" in err
    assert g.totals()["step"] == 1096
