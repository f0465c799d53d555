"""Host-side pieces of bench.py: the kernel code hash that decides whether the
committed HBM-traffic counters still describe the step kernel, and the
refusal of more than one GPU."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_code_hash_ignores_comments_only():
    b = _bench()
    src = "int f(int x)\n{\n    return x + 1;   // add one\n}\n"
    assert b.code_hash(src) == b.code_hash("// header\nint f(int x)\n{\n\n    return x + 1;\n}\n/* end */\n")
    assert b.code_hash(src) != b.code_hash(src.replace("x + 1", "x + 2"))
    assert b.code_hash(src) != b.code_hash(src.replace("return x", "return  x"))


def test_traffic_record_matches_current_kernel():
    """The committed counters carry the code hash of the kernel they were
    taken on; bench.py reports them only while it matches."""
    b = _bench()
    t = b.measured_traffic("cavity256_f64")
    if t is not None:
        assert t > 0
    assert b.measured_traffic("no such workload") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_unknown_section_is_refused():
    """Checked before anything touches the GPU."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--sections", "cavity256,nope"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "unknown sections: ['nope']" in r.stderr
    b = _bench()
    assert set(b.SECTIONS) == {"cavity256", "converge", "serving", "cylinder", "cylinder200k", "original", "large",
                               "converge_cylinder", "serving_narrow"}
    # the long sections run only when named, so the default run stays short
    assert set(b.SECTIONS) - set(b.DEFAULT_SECTIONS) == {"converge_cylinder", "cylinder", "serving_narrow"}
    assert b.CONVERGE_CASES == ("cavity256_re1000", "cylinder200k_re40")
    assert b.SERVING_TRACE["cavity_n"] == (64, 1024) and b.SERVING_TRACE["cylinder_cells"] == (10_000, 1_000_000)


def test_cpu_model_is_named():
    assert _bench()._cpu_model()


@pytest.mark.parametrize("opt", ["--schedule", "--batch-schedule", "--cylinder-schedule"])
def test_malformed_schedule_is_refused(opt):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), opt, "32"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and f"{opt} takes two integers" in r.stderr


def test_traffic_requires_the_recorded_schedule(tmp_path, monkeypatch):
    b = _bench()
    rec = {"w": {"kernel_code_sha1": b.kernel_hash(), "schedule": {"tile_cells": 32, "block_threads": 128},
                 "bytes_per_launch": 123}}
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(rec))
    monkeypatch.setattr(b, "TRAFFIC", str(p))
    assert b.measured_traffic("w", {"tile_cells": 32, "block_threads": 128}) == 123
    assert b.measured_traffic("w", {"tile_cells": 16, "block_threads": 64}) is None
    assert b.measured_traffic("w") == 123


def test_converge_stopping_rule():
    """FP64 stops at the tolerance or the cap; the FP32 deviation form with
    FP64; the FP32 non-equilibrium form runs on to the tolerance, up to 1.5
    times FP64's steps; a non-finite residual stops every form."""
    done = _bench().converge_done
    assert done("f64", 9e-9, 1000, False, 0, 1e-8, 10**6)
    assert not done("f64", 2e-8, 1000, False, 0, 1e-8, 10**6)
    assert done("f64", 2e-8, 10**6, False, 0, 1e-8, 10**6)
    assert not done("fp32dev", 4e-8, 2000, False, 1000, 1e-8, 10**6)
    assert done("fp32dev", 4e-8, 2000, True, 2000, 1e-8, 10**6)
    assert not done("fp32neq", 2e-8, 2000, True, 2000, 1e-8, 10**6)
    assert not done("fp32neq", 2e-8, 2999, True, 2000, 1e-8, 10**6)
    assert done("fp32neq", 2e-8, 3000, True, 2000, 1e-8, 10**6)
    assert done("fp32neq", 9e-9, 2100, True, 2000, 1e-8, 10**6)
    assert all(done(p, float("nan"), 1, False, 0, 1e-8, 10**6) for p in ("f64", "fp32dev", "fp32neq"))
