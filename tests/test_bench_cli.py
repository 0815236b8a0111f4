"""Host-side behaviour of bench.py that needs no GPU: the single-GPU refusal and
the FLOP accounting it reports against."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    """--gpus above 1 prints one JSON line with the reason and exits with status 2."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


def test_walk_flop_counts_are_additive():
    """The reported FLOPs are the per-interaction units times the interaction
    counts, with no term for the opening decisions."""
    sys.path.insert(0, ROOT)
    from paper_2010_03567_amd import flops
    assert flops.walk_flops_algorithmic("treepm", 1, 0) == flops.P2M_ALG["treepm"] == 85
    assert flops.walk_flops_algorithmic("treepm", 0, 1) == flops.P2P_ALG["treepm"] == 44
    assert flops.walk_flops_algorithmic("newton", 3, 5) == 3 * 60 + 5 * 19
    assert flops.fmm_flops_algorithmic(1, 0, 0, 0, 0) == 44
    assert flops.fmm_flops_algorithmic(0, 2, 3, 4, 5) == 2 * 120 + 3 * 275 + 4 * 100 + 5 * 40
