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


def test_level_grids_of_the_512x512_workload():
    """Level 1 of the 512x512 plan runs the leaf kernel over its parents'
    bands (the basis inner level) and its completion per (parent, action);
    the last level runs the leaf kernel over 32 bands of every slot and its
    completion per parent."""
    prob = wl.make_large(seed=0)
    g = rs.level_grids("large512")
    K = prob.A * prob.n
    bands = (prob.H + 8192 // prob.W - 1) // (8192 // prob.W)
    assert bands == 32
    assert g[("k_leaf_parent", K * bands * rs.NODE_BLOCK)] == 1
    assert g[("k_inner_finish", K * prob.A * rs.BLOCK)] == 1
    assert g[("k_leaf_parent", K ** 2 * bands * rs.NODE_BLOCK)] == 2
    assert g[("k_leaf_finish", K ** 2 * rs.NODE_BLOCK)] == 2


def test_shape_cache_round_trip(tmp_path):
    from paper_1810_00204_amd.planner import ShapeCache, batch_key
    probs = [wl.make_small(seed=1, W=12, H=9, D=2), wl.make_small(seed=2, W=20, H=20, D=3)]
    k = batch_key(probs, 3, 0, "gfx950", "abc")
    assert k == batch_key(probs, 3, 0, "gfx950", "abc")
    # everything the launches' work depends on changes the key
    assert k != batch_key(probs, 2, 0, "gfx950", "abc")
    assert k != batch_key(probs, 3, 1, "gfx950", "abc")
    assert k != batch_key(probs, 3, 0, "other", "abc")
    assert k != batch_key(probs, 3, 0, "gfx950", "abd")
    assert k != batch_key(probs[::-1], 3, 0, "gfx950", "abc")
    deeper = [wl.make_small(seed=1, W=12, H=9, D=3), probs[1]]
    assert k != batch_key(deeper, 3, 0, "gfx950", "abc")
    path = str(tmp_path / "shapes.json")
    c = ShapeCache(path)
    assert c.get(k) is None                      # no file yet
    c.put(k, 4096, 2, 5.25)
    assert c.get(k) == (4096, 2, 5.25)
    k2 = batch_key(deeper, 3, 0, "gfx950", "abc")
    ShapeCache(path).put(k2, 512, 1, 1.5)        # merged, not replaced
    assert c.get(k) == (4096, 2, 5.25) and c.get(k2) == (512, 1, 1.5)
    with open(path, "w") as f:                   # a damaged file reads as empty
        f.write("{not json")
    assert c.get(k) is None
    c.put(k, 256, 4, 2.0)
    assert c.get(k) == (256, 4, 2.0)
