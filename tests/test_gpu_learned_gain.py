"""What the trained network gains over the method without it: on a clustered
128^3 box drawn with a seed held out of training (2001; the network was
trained on seeds 1001-1020), the learned seed (features + MLP) and the plain
seed (geometric pre-walk) each run the relative walk at the largest alpha
whose 99th-percentile force error against FP64 direct summation is <= 1e-3
(a sqrt(2) grid refined by bisection); the learned step must be faster, and the ratio is
printed.  The step and the calibration are bench.py's own."""
import types

import pytest
import torch

pytestmark = pytest.mark.gpu


def test_learned_seed_beats_prewalk_at_equal_p99():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import bench
    import paper_2010_03567_amd.g4hip as g
    args = types.SimpleNamespace(rcut=7.0, leaf=32, group=64, keys="morton", sr_table=0, no_learned=False,
                                 err_sample=10000)
    ctx = g.Context()
    case = bench.TreePMCase(g, ctx, args, 128 ** 3, 2001)
    assert case.learned is not None, "no trained weights for 128^3, leaf 32"
    res = {v: case.variant(v, steps=5, warmup=2) for v in ("plain", "learned")}
    for v, r in res.items():
        assert "ms_per_step" in r, (v, r)
        assert r["errors_vs_direct"]["p99"] <= bench.ERR_BOUND, (v, r["errors_vs_direct"])
    ratio = res["plain"]["ms_per_step"] / res["learned"]["ms_per_step"]
    print(f"held-out 128^3: plain {res['plain']['ms_per_step']:.2f} ms/step at alpha {res['plain']['alpha']}, "
          f"learned {res['learned']['ms_per_step']:.2f} ms/step at alpha {res['learned']['alpha']}: {ratio:.2f}x")
    assert ratio > 1.1
    case.free()
