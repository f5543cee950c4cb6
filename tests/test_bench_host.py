"""Host-side logic of bench.py (CPU): the one-GPU refusal, the argument
defaults the headline line depends on, and the rule that a stored traffic
figure is reported only while the sources it was measured on are unchanged."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def parse(argv):
    old = sys.argv
    sys.argv = ["bench.py", *argv]
    try:
        return bench.parse()
    finally:
        sys.argv = old


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_defaults():
    a = parse([])
    assert (a.gpus, a.n, a.prec) == (1, 11, "f32x6")
    assert a.steps > 0 and a.warmup >= 0
    assert a.settle_ms == 200.0
    assert not (a.no_variants or a.no_long or a.no_batched or a.no_cpu_baseline)


def test_headline_only_drops_every_side_record():
    a = parse(["--headline-only", "--settle-ms", "0"])
    assert a.no_variants and a.no_long and a.no_batched and a.no_cpu_baseline
    assert a.settle_ms == 0.0


@pytest.mark.parametrize("kernel", sorted(bench.TRAFFIC))
def test_traffic_needs_matching_sources(kernel, monkeypatch):
    rec = dict(bench.TRAFFIC[kernel])
    assert "paper_2207_05341_amd/build.py" in rec["sources"]  # build flags change the kernels too
    # a record whose hash matches the sources is reported, any other is not
    rec["sources_sha256"] = bench.sources_sha256(rec["sources"])
    monkeypatch.setitem(bench.TRAFFIC, kernel, rec)
    assert bench.traffic_of(kernel) == rec["bytes"]
    monkeypatch.setitem(bench.TRAFFIC, kernel, dict(rec, sources_sha256="0" * 64))
    assert bench.traffic_of(kernel) is None
    assert bench.traffic_of("no_such_kernel") is None
