"""CPU: the rocprofv3 summary helpers (kernel short names, traffic scaling)."""
import csv
import json

from paper_2411_11468_amd import profiling


def test_short_names():
    cases = {
        "void lpa::k_hub_part<long, 16383, 1024>(lpa::HubArgs)": "hub_part",
        "void lpa::k_sweep_block_pipe<long, 16383, 1024, 4>(lpa::SweepArgs)": "sweep_block16383",
        "void lpa::k_sweep_block<long, 2047, 256, 4, false>(lpa::SweepArgs)": "sweep_block2047",
        "void lpa::k_sweep_group<long, 127, 16, false>(lpa::SweepArgs)": "sweep_wave127",
        "void lpa::k_sweep_wave_pipe<long, 1023, 4, 4>(lpa::SweepArgs)": "sweep_wave1023",
        "void lpa::k_sweep_lane4<long>(lpa::SweepArgs)": "sweep_small4",
        "void lpa::k_sweep_small16x2<long>(lpa::SweepArgs)": "sweep_small16",
        "void lpa::k_sweep_small<long, 16, true>(lpa::SweepArgs)": "sweep_small16",
        "void lpa::k_sweep_direct<long, 1, 256, false, true>(lpa::SweepArgs)": "direct_small4",
        "void lpa::k_sweep_direct<long, 16, 256, false, false>(lpa::SweepArgs)": "direct_g16",
        "void lpa::k_sweep_direct<long, 4, 256, true, false>(lpa::SweepArgs)": "direct_small16",
        "void lpa::k_sweep_direct<int, 8, 256, false, false>(lpa::SweepArgs)": "direct_wave127",
        "void lpa::k_sweep_direct2<long, 8, 256>(lpa::SweepArgs)": "direct_wave127",
        "void lpa::k_sweep_direct<long, 256, 256, false, false>(lpa::SweepArgs)": "direct_g256",
        "void lpa::(anonymous namespace)::k_tv_wave<long, double, 1023>(lpa::SweepArgs)":
            "tv_sweep",
        "lpa::k_frontier(long, unsigned char*, unsigned char const*, lpa::ListPtrs)": "frontier",
        "void lpa::(anonymous namespace)::k_fill<float>(float*, float, long)": "fill",
        "lpa::k_init(long, int const*, int const*, int*, unsigned char*, lpa::DevStats*)": "init",
        "__amd_rocclr_copyBuffer": "__amd_rocclr_copyBuffer",
    }
    for kernel, name in cases.items():
        assert profiling.short_name(kernel) == name, kernel


def _counter_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Grid_Size", "Kernel_Name",
                                          "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, r in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Grid_Size": r.pop("grid", 256), **r})


def test_traffic_scaling(tmp_path):
    # the reference copies (1 GiB each, the trailing copy dispatches: one
    # untimed, three timed) read half their bytes per the counter (scale 2)
    # and write all of them (scale 1); a larger upload copy earlier in the
    # run does not enter the scale; a sweep kernel's two dispatches are
    # averaged
    gib = float(1 << 30)
    kib = gib / 1024
    copy = "__amd_rocclr_copyBuffer"
    hub = "void lpa::k_hub_part<long, 16383, 1024>(lpa::HubArgs)"

    def run(counter, upload, hub_vals, ref):
        rows = [{"Kernel_Name": copy, "Counter_Name": counter, "Counter_Value": upload,
                 "grid": 999}]
        rows += [{"Kernel_Name": hub, "Counter_Name": counter, "Counter_Value": v}
                 for v in hub_vals]
        rows += [{"Kernel_Name": copy, "Counter_Name": counter, "Counter_Value": ref,
                  "grid": 131072} for _ in range(4)]
        return rows

    fetch = run("FETCH_SIZE", 4 * kib, [100.0, 300.0], kib / 2)
    write = run("WRITE_SIZE", 8 * kib, [10.0, 30.0], kib)
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(fp, fetch)
    _counter_csv(wp, write)
    t = profiling.traffic_json(str(fp), str(wp), gib, "cmd")
    json.dumps(t)
    assert abs(t["fetch_scale"] - 2.0) < 1e-9 and abs(t["write_scale"] - 1.0) < 1e-9
    assert t["copy_dispatches"] == [3, 3]
    hp = t["kernels"]["hub_part"]
    assert hp["dispatches"] == 2
    assert abs(hp["bytes_per_dispatch"] - 1024.0 * (200.0 * 2.0 + 20.0)) < 1e-6
    assert t["sources"] == profiling.source_hash()
