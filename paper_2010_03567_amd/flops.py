"""Algorithmic floating-point operation counts per interaction (frozen).

The roofline fractions are reported at these per-interaction units, counted
from the formulas of the interactions themselves (a fused multiply-add counts
2, a transcendental 1), independent of how a kernel schedules them:

* P2P_ALG: one particle-particle interaction: separation, r^2, 1/r, the
  softened kernel factor and the accumulation (Newtonian ~19); the TreePM
  short-range factor adds ~25 (erfc, exp and the polynomial around them).
* P2M_ALG: one particle-node interaction at p = 3 (monopole + quadrupole
  force, -G [M D1 + Q2:D3 / 2]) with Newtonian g_n; the same ~25 for the
  short-range g_n.
* FMM_ALG: symmetric node-node interaction (field expansions to order 3 in
  both nodes) ~275, particle-node pair (M2P + P2L) ~120, particle pair 44,
  downward shift per node ~100, evaluation per particle ~40.

The opening decisions are not algorithmic work of the interactions: the
per-lane cost of one criterion evaluation is listed as VISIT_BOOKKEEPING
(relative vector, r^2, the criterion and, for TreePM, the nearest-edge test
against r_cut) and reported beside the fraction, never inside it.
"""

P2P_ALG = {"newton": 19, "treepm": 44}
P2M_ALG = {"newton": 60, "treepm": 85}
FMM_ALG = {"nn": 275, "pn": 120, "pp": 44, "l2l_per_node": 100, "l2p_per_particle": 40}
VISIT_BOOKKEEPING = {("newton", "geometric"): 11, ("newton", "relative"): 16,
                     ("treepm", "geometric"): 26, ("treepm", "relative"): 31}
MLP_FORWARD = 64 * 8 * 2 + 64 * 64 * 2 + 64 * 2 + 128 * 5  # per particle (FMA = 2, SiLU = 5)


def walk_flops_algorithmic(kernel: str, n_p2m: int, n_p2p: int) -> float:
    """FLOPs of the interactions of one walk (decisions not counted)."""
    return P2M_ALG[kernel] * float(n_p2m) + P2P_ALG[kernel] * float(n_p2p)


def fmm_flops_algorithmic(n_pp: int, n_pn: int, n_nn: int, n_nodes: int, n_particles: int) -> float:
    """FLOPs of one FMM call: interactions, downward pass and evaluation."""
    f = FMM_ALG
    return (f["pp"] * float(n_pp) + f["pn"] * float(n_pn) + f["nn"] * float(n_nn)
            + f["l2l_per_node"] * float(n_nodes) + f["l2p_per_particle"] * float(n_particles))
