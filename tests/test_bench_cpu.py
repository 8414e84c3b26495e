"""CPU checks of bench.py: every workload's JSON record builds from stubbed
timings (so a name error in a record cannot hide until a GPU run), carries
the fields of the benchmark contract, and a request for more than one GPU is
refused with a message."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CONTRACT = {"metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
            "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
            "roofline", "cpu_baseline"}


def _check(rec):
    text = json.dumps(rec)
    back = json.loads(text)
    assert CONTRACT <= set(back), CONTRACT - set(back)
    assert back["n_gpus"] == 1 and back["value"] > 0
    assert "workload" in back["config"]
    return back


def _cpu_stub():
    return {"value": 0.02, "unit": "TFLOP/s", "cores": 16, "kind": "oracle", "sample": "stub",
            "host": bench.cpu_info(), "dd_reference": {"value": 1e-4},
            "host_blas_fp64": {"value": 1.0}}


def test_single_record_ozaki1_and_ozaki2():
    wl = {"name": "illcond_zgemm_16384", "seed": 1004, "desc": "stub"}
    roof = bench.roofline_record(21 * 8.0 * 16384 ** 3, 290.0, "k_ozgemm", None)
    assert 0 < roof["frac"] < 1 and roof["bound"] == "mfma" and roof["unit"] == "TFLOP/s"
    native = {"kernel": "k_native", "ms_per_call": 1000.0, "calls": 3, "tflops": 35.0,
              "frac_of_fp64_peak": 0.45}
    acc = {"err_comp_sampled": 1e-13, "by_slices": {"b8": {"6": {"err_comp": 1e-13}}}}
    rec = bench.single_record(wl, 16384, 16384, 16384, True, "ozaki1", "b8", 6, 20, 5, 300.0,
                              {"scan": 1.0, "split": 2.0, "gemm": 290.0, "recon": 0.0}, roof,
                              _cpu_stub(), native, acc, {"tune_id": 13},
                              {"b8_s6": {"ms_per_step": 300.0}})
    back = _check(rec)
    assert back["config"]["pairs"] == 21 and back["config"]["split"] == "b8"
    assert "recon" not in back["phases_ms"]
    assert abs(back["value"] - 8.0 * 16384 ** 3 / 0.3 / 1e12) < 1e-2
    assert back["speedup_vs_native"] == round(1000.0 / 300.0, 3)
    rec2 = bench.single_record(wl, 2048, 2048, 2048, True, "ozaki2", None, 13, 20, 5, 0.8,
                               {"scan": 0.04, "split": 0.1, "gemm": 0.5, "recon": 0.1},
                               bench.roofline_record(13 * 8.0 * 2048 ** 3, 0.5, "crt", None),
                               None, None, None, None)
    back2 = _check(rec2)
    assert back2["config"]["moduli"] == 13 and "split" not in back2["config"]


def test_batched_selector_lu_records():
    roof = bench.roofline_record(28 * 6.6e10, 0.9, "grouped", None)
    _check(bench.batched_record(512, 7, 6.6e10, [32, 1024], 20, 5, 1.9, 2.0,
                                {"scan": 0.3, "split": 0.6, "gemm": 0.9, "recon": 0.0}, roof,
                                _cpu_stub()))
    res = {"ms_learned": 2.5, "ms_fixed": 2.6}
    rec = bench.selector_record(6.6e10, 20, 1e-11, "w.npz", 0.5, 32.0, res)
    assert json.loads(json.dumps(rec))["selector"] == res
    lu = bench.lu_record(2048, 128, "b8", 6, 5, 2, 10.0, 12.0, 1e-9, {5: 1e-7, 6: 1e-9}, 1e-10)
    assert json.loads(json.dumps(lu))["native_updates"]["ms_per_step"] == 12.0


def test_cpu_info_fields():
    info = bench.cpu_info()
    assert info["nproc"] >= 1 and info["blas_threads"] >= 1


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
