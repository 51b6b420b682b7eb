"""Host-side checks of bench.py: the one-GPU contract and the roofline bookkeeping."""

import os
import subprocess
import sys

import bench
from tests.conftest import ROOT


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_per_site():
    # 40 stored 3x3 complex links + 12 complex in and 12 out per right-hand side
    assert bench.stencil_bytes_per_site(8, 8) == 6144
    assert bench.stencil_bytes_per_site(4, 4) == 3072
    assert bench.stencil_bytes_per_site(4, 2) == 1632
    assert bench.stencil_bytes_per_site(8, 8, 12) == 720 * 8 + 48 * 12 * 8


def test_counter_traffic_is_tied_to_the_stencil_sources():
    # the committed counter summary is used only while the stencil sources hash to its digest
    traffic = bench.measured_traffic()
    if not os.path.exists(bench.TRAFFIC_FILE):
        assert traffic is None
        return
    with open(bench.TRAFFIC_FILE) as f:
        txt = f.read()
    sha = [ln.split("=", 1)[1].strip() for ln in txt.splitlines() if ln.startswith("kernel_src_sha")][0]
    if sha == bench.kernel_source_digest():
        V = 1
        for v in bench.L_BENCH:
            V *= v
        assert traffic is not None and traffic > bench.stencil_bytes_per_site(8, 8) * V
    else:
        assert traffic is None


def test_gate_reads_the_stored_oracle_outputs():
    # every stored 32^3x64 oracle output is a point source of the benchmark's batch
    for c in bench.golden_cases(bench.L_BENCH):
        assert str(c["source_kind"]) == "point" and 0 <= int(c["source_arg"]) < bench.NSRC
        assert float(c["tol"]) <= 1e-13 and int(c["kl_n"]) == bench.KL_N
        assert tuple(int(v) for v in c["L"]) == bench.L_BENCH
