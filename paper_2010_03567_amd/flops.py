"""Algorithmic floating-point operation counts per interaction (frozen).

Counted from the formulas as the kernels evaluate them: an add, multiply or
compare-free min/max of floats counts 1, a fused multiply-add counts 2, a
hardware transcendental (rsqrt, rcp, exp2) counts 1; integer differences and
int-to-float conversions count 0.  "visit" is the per-lane cost of looking at
one node: the relative vector to the centre of mass, r^2, rsqrt and the
opening test (for TreePM also the nearest-edge distance against r_cut).  A
particle-node interaction is counted beyond the visit that precedes it; a
particle-particle interaction is counted whole.
"""

# one-sided walk, p = 3 (force only)
VISIT = {("newton", "geometric"): 15, ("newton", "relative"): 19,
         ("treepm", "geometric"): 27, ("treepm", "relative"): 31}
P2M = {"newton": 46, "treepm": 91}
P2P = {"newton": 18, "treepm": 40}


def walk_flops(kernel: str, criterion: str, n_visit: int, n_p2m: int, n_p2p: int) -> float:
    return (VISIT[(kernel, criterion)] * float(n_visit) + P2M[kernel] * float(n_p2m) + P2P[kernel] * float(n_p2p))
