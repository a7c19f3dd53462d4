"""Host logic of bench.py that runs without a GPU: the one-GPU guard, the byte accounting behind the
roofline figures, the traffic record's source check, and the CPU-baseline leg on a tiny lattice."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr or "single MI355X" in res.stderr
    assert res.stdout == ""


def test_compulsory_bytes_per_site():
    # FP64: 8 one-hop matrices of 9 complex doubles, 8 three-hop ones (6 complex stored, or 9), 48 B in and out
    assert bench.dslash_bytes_per_site("f64", long12=True) == 8 * 144 + 8 * 96 + 2 * 48 == 2016
    assert bench.dslash_bytes_per_site("f64", long12=False) == 16 * 144 + 2 * 48
    # FP16: binary16 matrices, one binary32 scale per site for each of the two link kinds, 16 B vectors
    assert bench.dslash_bytes_per_site("f16", long12=True) == 8 * 36 + 8 * 24 + 8 + 2 * 16 == 520
    assert bench.dslash_bytes_per_site("f16", xpay=True, long12=True) == 536
    assert bench.dslash_bytes_per_site("f32", long12=True) == 8 * 72 + 8 * 48 + 2 * 24


def test_traffic_record_follows_the_kernel_source(tmp_path, monkeypatch):
    """A counter summary is used only while the kernel sources hash to the value recorded with it, the
    long-link storage matches and it holds the launch shape of the run (checked on a copy of the sources,
    so that the test does not depend on whether the committed record was taken on the current kernels)."""
    import hashlib

    rec = json.load(open(os.path.join(ROOT, "profiles", "dslash_f16_28x28x28x96_traffic.json")))
    shape = dict(wg=64, rhs_per_lane=1, lds_stage=0, tile_order=0, t_chunks=1)
    other = dict(shape, wg=128)
    root = tmp_path / "root"
    (root / "profiles").mkdir(parents=True)
    h = hashlib.sha256()
    for f in rec["source_files"]:
        dst = root / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        data = open(os.path.join(ROOT, f), "rb").read()
        dst.write_bytes(data)
        h.update(data)
    mine = dict(rec, source_sha256=h.hexdigest(), traffic_bytes_per_launch={"l12:64,1,0,0,1": 123.0})
    (root / "profiles" / "dslash_f16_28x28x28x96_traffic.json").write_text(json.dumps(mine))
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.measured_traffic("f16", (28, 28, 28, 96), True, 1, shape) == 123.0
    assert bench.measured_traffic("f16", (28, 28, 28, 96), True, 1, other) is None  # shape not counted
    assert bench.measured_traffic("f16", (28, 28, 28, 96), False, 1, shape) is None
    assert bench.measured_traffic("f16", (4, 4, 4, 4), True, 1, shape) is None  # no record for this lattice
    changed = root / rec["source_files"][0]
    changed.write_bytes(changed.read_bytes() + b"\n// changed\n")
    assert bench.measured_traffic("f16", (28, 28, 28, 96), True, 1, shape) is None


def test_cpu_baseline_leg_on_a_tiny_lattice():
    from stag_inputs import fat_field, gaussian_source, random_su3_field

    dims = (4, 4, 4, 4)
    fat = fat_field(dims, 1)
    lng = random_su3_field(dims, 2)
    b = gaussian_source(dims, 3)[0]
    cb = bench.cpu_baseline(fat, lng, b, dims, 0.1, 100)
    assert cb["kind"] == "oracle" and cb["cores"] == 1 and cb["unit"] == "s"
    assert cb["per_iteration_s"] > 0 and np.isclose(cb["value"], 100 * cb["per_iteration_s"])


@pytest.mark.parametrize("argv", [["--workload", "9"], ["--prec", "f64"]])
def test_bad_arguments_are_rejected(argv):
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, capture_output=True, text=True,
                         timeout=120)
    assert res.returncode != 0


def test_long_link_storage_per_leg():
    """auto: 18 reals only for a mixed-precision leg whose lattices all have a multiple of 8 RHS (8 per lane);
    12 reals for FP64 and for the batched and single-RHS legs; the flags force either."""
    from types import SimpleNamespace

    auto = SimpleNamespace(long_links="auto")
    assert bench.long12_for(auto, "f16", [8]) is False
    assert bench.long12_for(auto, "f16", [16, 8]) is False
    assert bench.long12_for(auto, "f16", [4, 12, 8]) is True
    assert bench.long12_for(auto, "f16", 1) is True
    assert bench.long12_for(auto, "f64", [8]) is True
    assert bench.long12_for(SimpleNamespace(long_links="12"), "f16", [8]) is True
    assert bench.long12_for(SimpleNamespace(long_links="18"), "f64", 1) is False


@pytest.mark.parametrize("window", [1, 2, 5])
def test_break_even_stall_keeps_pace_with_mixed_precision(window):
    """The stall ratio asks each flexible-CG window to cut ||r|| as much as the mixed-precision CG does in
    the same time: windows at exactly that ratio, for as long as the mixed-precision solve takes, reach its
    tolerance.  A dearer network application or a longer window spans more mixed-precision progress, so
    it must cut more (a smaller ratio)."""
    mp_s, iters, t_net, tol = 6.0, 1000, 0.11, 1e-10
    win, ratio = bench.break_even_stall(mp_s, iters, t_net, tol, window)
    assert win == window and 0.0 < ratio < 1.0
    t_window = window * (mp_s / iters + t_net)
    assert ratio ** (mp_s / t_window) == pytest.approx(tol, rel=1e-9)
    assert bench.break_even_stall(mp_s, iters, 2 * t_net, tol, window)[1] < ratio
    assert bench.break_even_stall(mp_s, iters, t_net, tol, window + 1)[1] < ratio
