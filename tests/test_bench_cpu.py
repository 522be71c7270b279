"""Host logic of bench.py and the committed rocprofv3 summaries (CPU only).

The summaries under profiles/ are what the benchmark's `roofline.traffic`
is read from, so their arithmetic is checked here: HBM bytes are the raw
FETCH_SIZE / WRITE_SIZE KiB per dispatch times the copy-kernel calibration,
the traffic ratio is those bytes over the algorithmic bytes of the workload,
and a summary is used only for the kernel kind and sources it was taken on.
"""
import glob
import json
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1004_0480_amd import workloads as W  # noqa: E402

PMC = sorted(glob.glob(os.path.join(ROOT, "profiles", "*_pmc.json")))
TRACES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*_trace.md")))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_bytes_per_cell():
    # one read and one write of every stored species; the front model's two
    # passes add the FP32 chemical potential (written, read) and C read again
    assert bench.alg_bytes_per_cell("brusselator256", "f32") == 16
    assert bench.alg_bytes_per_cell("brusselator256", "bf16") == 8
    assert bench.alg_bytes_per_cell("diffusion512", "f32") == 8
    assert bench.alg_bytes_per_cell("pollutant512", "f32") == 32
    assert bench.alg_bytes_per_cell("front384", "f32") == 36
    assert bench.alg_bytes_per_cell("front384", "bf16") == 12 + 8 + 2
    # the one-pass front step moves each species once each way
    assert bench.alg_bytes_per_cell("front384", "f32", one_pass=True) == 24
    assert bench.alg_bytes_per_cell("front384", "bf16", one_pass=True) == 12
    assert bench.alg_bytes_per_cell("t1_turing192", "f32") == 16


def test_traffic_is_read_only_for_its_sources_and_kernel_kind(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "profiles", "diffusion512_lds_kernel_pmc.json")
    rec = json.load(open(src))
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    shutil.copy(src, tmp_path / "diffusion512_lds_kernel_pmc.json")
    d = rec["source_digest"]
    assert bench.measured_traffic("diffusion512", d, 4)["traffic_over_algorithmic"] == \
        rec["traffic_over_algorithmic"]
    assert bench.measured_traffic("diffusion512", "0" * 16, 4) is None    # other sources
    assert bench.measured_traffic("diffusion512", d, 3) is None           # other kind
    assert bench.measured_traffic("diffusion512_19pt", d, 4) is None      # other workload
    # a summary whose kernel is not of the kind its file name says is ignored
    bad = dict(rec, kernel=rec["kernel"].replace("lds_kernel", "block_kernel"))
    (tmp_path / "diffusion512_lds_kernel_pmc.json").write_text(json.dumps(bad))
    assert bench.measured_traffic("diffusion512", d, 4) is None


def test_kernel_source_digest_tracks_the_kernel_sources(tmp_path, monkeypatch):
    d = bench.kernel_source_digest()
    assert len(d) == 16 and int(d, 16) >= 0
    csrc = tmp_path / "paper_1004_0480_amd" / "csrc"
    shutil.copytree(os.path.join(ROOT, "paper_1004_0480_amd", "csrc"), csrc)
    from paper_1004_0480_amd import build
    monkeypatch.setattr(build, "CSRC", str(csrc))
    assert bench.kernel_source_digest() == d
    (csrc / "rd_device.hpp").write_text((csrc / "rd_device.hpp").read_text() + "\n")
    assert bench.kernel_source_digest() != d


@pytest.mark.parametrize("path", PMC, ids=[os.path.basename(p) for p in PMC])
def test_committed_pmc_summary_arithmetic(path):
    rec = json.load(open(path))
    base = os.path.basename(path)[:-len("_pmc.json")]
    kind = next(k for k in bench.KERNEL_NAMES.values() if base.endswith(k))
    workload = base[:-len(kind) - 1]
    stencil = 19 if workload.endswith("_19pt") else 7
    workload = workload.replace("_19pt", "")
    names = rec["kernel"] if isinstance(rec["kernel"], list) else [rec["kernel"]]
    assert all(kind in n for n in names)
    assert ("%d-point Laplacian" % stencil) in rec["workload"]
    # calibration: the copy kernel moves COPY_PROBE_BYTES each way
    assert rec["read_scale"] == pytest.approx(bench.COPY_PROBE_BYTES / (rec["copy_fetch_kib_raw"] * 1024.0))
    assert rec["write_scale"] == pytest.approx(bench.COPY_PROBE_BYTES / (rec["copy_write_kib_raw"] * 1024.0))
    rd = wr = 0.0
    for k in rec["per_kernel"]:
        assert k["hbm_read_bytes"] == pytest.approx(k["fetch_kib_raw"] * 1024.0 * rec["read_scale"])
        assert k["hbm_write_bytes"] == pytest.approx(k["write_kib_raw"] * 1024.0 * rec["write_scale"])
        rd += k["hbm_read_bytes"]
        wr += k["hbm_write_bytes"]
    assert rec["hbm_read_bytes_per_launch_set"] == pytest.approx(rd)
    assert rec["hbm_write_bytes_per_launch_set"] == pytest.approx(wr)
    cells = int(np.prod(W.DEFAULT_SHAPES[workload]))
    one_pass = all("fch_kernel" in n for n in names)
    alg = bench.alg_bytes_per_cell(workload, "f32", one_pass) * cells
    assert rec["algorithmic_bytes_per_launch_set"] == alg
    assert rec["traffic_over_algorithmic"] == pytest.approx((rd + wr) / alg)
    # a step kernel cannot move less than it must read and write
    assert 0.99 < rec["traffic_over_algorithmic"] < 1.5
    assert "rocprofv3 --pmc FETCH_SIZE" in rec["command"] and "bench.py" in rec["command"]


@pytest.mark.parametrize("path", TRACES, ids=[os.path.basename(p) for p in TRACES])
def test_committed_trace_summary_names_its_command_and_kernel(path):
    text = open(path).read()
    assert "rocprofv3 --kernel-trace --stats" in text and "bench.py" in text
    kind = next(k for k in bench.KERNEL_NAMES.values() if os.path.basename(path).endswith(k + "_trace.md"))
    rows = [l for l in text.splitlines() if l.startswith("| `") and kind in l]
    assert rows, "no %s row" % kind
    calls, avg = rows[0].split("|")[2:4]
    assert int(calls) >= 100 and 1.0 < float(avg) < 10000.0


def test_every_summary_has_a_kind_the_bench_knows():
    assert PMC and TRACES
    for p in PMC + TRACES:
        b = os.path.basename(p)
        assert any(("_%s_" % k) in b for k in bench.KERNEL_NAMES.values()), b


def test_cpu_sample_keeps_the_workload_or_its_lowest_planes():
    """The CPU baseline's sample: the whole grid when it is small enough, else
    the lowest z planes of the same problem (wind and sources cut to them)."""
    w = W.make_workload("pollutant512", shape=(16, 12, 10))
    same, where = bench.cpu_sample(w, 10 ** 6)
    assert same is w and where == "whole grid"
    sub, where = bench.cpu_sample(w, 12 * 10 * 5)
    assert sub.shape == (5, 12, 10) and "5 of 16" in where
    assert len(sub.spec.wind) == 5 and np.array_equal(sub.spec.wind, w.spec.wind[:5])
    assert np.all(sub.spec.sources[0] < 5 * 12 * 10)
    for a, b in zip(sub.fields, w.fields):
        assert np.array_equal(a, b[:5])
