"""Algorithmic floating-point operation counts per interaction (frozen).

Counted from the formulas as the kernels evaluate them: an add, multiply,
subtract or max of floats counts 1, a fused multiply-add counts 2, a hardware
transcendental (rsqrt, rcp, exp2) counts 1; integer differences,
int-to-float conversions and compares count 0.

* visit: the per-lane cost of looking at one node: relative vector to the
  centre of mass (3), r^2 (5), rsqrt (1), the opening test (geometric 2,
  relative 7: l^3, r^5, M l^3, alpha|a| r^5) and, for the short-range
  kernel, the nearest-edge distance against r_cut (15).
* p2m: a particle-node interaction beyond the visit that precedes it:
  g_1..g_3 of the kernel (Newtonian 6; short-range 47 including exp and the
  Hastings erfc: rcp + 4 FMA) and the quadrupole force M D1 + Q2:D3 / 2 (40).
* p2p: a whole particle-particle interaction: relative vector (3), r^2 (5),
  rsqrt (1), 1/r^2 (1), kernel factor (Newtonian 1; short-range 24),
  m K (1), accumulation (3 FMA = 6).
"""

VISIT = {("newton", "geometric"): 11, ("newton", "relative"): 16,
         ("treepm", "geometric"): 26, ("treepm", "relative"): 31}
P2M = {"newton": 46, "treepm": 87}
P2P = {"newton": 18, "treepm": 40}
MLP_FORWARD = 64 * 8 * 2 + 64 * 64 * 2 + 64 * 2 + 128 * 5  # per particle (FMA = 2, SiLU = 5)


def walk_flops(kernel: str, criterion: str, n_visit: int, n_p2m: int, n_p2p: int) -> float:
    return (VISIT[(kernel, criterion)] * float(n_visit) + P2M[kernel] * float(n_p2m) + P2P[kernel] * float(n_p2p))
