"""Host-side behaviour of bench.py that needs no GPU: the single-GPU refusal,
the FLOP accounting it reports against and the alpha calibration."""
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


def _fake_case(bound_alpha):
    """A TreePMCase whose p99 grows linearly with alpha and equals the bound
    at bound_alpha (no device, no particles)."""
    sys.path.insert(0, ROOT)
    import bench

    class Fake(bench.TreePMCase):
        def __init__(self):
            self.n = 1
            self.asked = []

        def params(self, variant, alpha, r_cut=None, order=3):
            return alpha

        def errors(self, variant, alpha):
            self.asked.append(alpha)
            return {"p99": bench.ERR_BOUND * alpha / bound_alpha}

    return bench, Fake()


def test_calibration_refines_between_grid_values():
    """The calibrated alpha meets the bound, lies between the passing grid value
    and the failing one above it, and is within one bisection step (in log
    alpha) of the true threshold; no alpha above a failing one is chosen."""
    import math
    bench, c = _fake_case(0.00121)
    alpha, cal = c.calibrate("learned")
    assert cal[alpha]["p99"] <= bench.ERR_BOUND
    assert 0.001 <= alpha < 0.00121 <= 0.0014
    assert math.log(0.00121 / alpha) <= math.log(0.0014 / 0.001) / 2 ** bench.REFINE
    assert all(a not in cal or cal[a]["p99"] > bench.ERR_BOUND for a in bench.ALPHAS if a > alpha)
    assert len(c.asked) == len(set(c.asked)) <= list(bench.ALPHAS).index(0.001) + 1 + bench.REFINE


def test_calibration_edges():
    """A bound met at the top of the grid needs no bisection; one never met
    gives no alpha; a fixed alpha is evaluated once and returned as given."""
    bench, c = _fake_case(1.0)
    assert c.calibrate("plain")[0] == bench.ALPHAS[0] and c.asked == [bench.ALPHAS[0]]
    bench, c = _fake_case(1e-9)
    alpha, cal = c.calibrate("plain")
    assert alpha is None and sorted(cal) == sorted(bench.ALPHAS)
    bench, c = _fake_case(1e-9)
    assert c.calibrate("plain", fixed=0.003)[0] == 0.003 and c.asked == [0.003]
