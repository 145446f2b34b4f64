"""Host-side pieces of the measurement tooling (no GPU): the bench refuses
more than one GPU, and the rocprofv3 summary maps kernel names and grid
sizes onto tree levels."""
import os
import subprocess
import sys

from paper_1810_00204_amd import rocprof_summary as rs
from paper_1810_00204_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_short_kernel_names():
    assert rs.short_name("void qv::k_node<8, true>(qv::DevModel, qv::LevelArgs, qv::TreeArgs)") \
        == "k_node<8, true>"
    assert rs.short_name("qv::k_stats(qv::DevModel, qv::LevelArgs)") == "k_stats"
    assert rs.short_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_level_grids_of_the_64x64_workload():
    prob = wl.make_rect(seed=0)
    g = rs.level_grids("rect64")
    K, A = prob.A * prob.n, prob.A
    for d in range(prob.D):
        assert g[("k_node", K ** d * A * rs.NODE_BLOCK)] == d
    # level 0 also carries the leaf band's sort workgroup
    assert g[("k_node", (A + 1) * rs.NODE_BLOCK)] == 0
    # the last level: one workgroup per (parent, band); 64 x 64 is one band
    assert g[("k_leaf_parent", K ** (prob.D - 1) * rs.NODE_BLOCK)] == prob.D - 1
