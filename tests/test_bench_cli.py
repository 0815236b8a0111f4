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
    """walk_flops is the per-event counts times the event numbers (no hidden terms)."""
    sys.path.insert(0, ROOT)
    from paper_2010_03567_amd import flops
    assert flops.walk_flops("treepm", "relative", 1, 0, 0) == flops.VISIT[("treepm", "relative")]
    assert flops.walk_flops("treepm", "relative", 0, 1, 0) == flops.P2M["treepm"]
    assert flops.walk_flops("treepm", "relative", 0, 0, 1) == flops.P2P["treepm"]
    assert flops.walk_flops("newton", "geometric", 2, 3, 5) == 2 * 11 + 3 * 46 + 5 * 18
