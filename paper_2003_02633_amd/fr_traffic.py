"""Memory traffic of the flux-reconstruction right-hand side per hexahedral element (§4, Tables
fr_nse and mem_usage): the bytes each of the 12 steps reads and writes, uncompressed and with
every compressible 3-vector stored as one 64-bit code, and the resulting compression ratio.

A quantity is counted per solution point (n_s = (k+1)^3) or per flux point (n_f = 6 (k+1)^2), as
a number of scalars (4 bytes each) and a number of 3-vectors (12 bytes each, 8 bytes compressed).
n_p = 5 equations.

Readings (where the printed table and the listed step data disagree):
  * step 4 (q^s -> w^s) is printed as 2.50 KiB for k = 3, 4 and 5; the listed data are
    2 n_s n_p scalars, which is 2.50 KiB at k = 3 only.  The printed improvements (20.1, 20.6,
    21.0 %) and weighted ratios follow from the listed data, the printed column total from the
    printed rows.  ``as_printed=True`` reproduces the printed row, the default counts the data;
  * step 8 (interface viscous flux) is printed with 43 scalars per flux point, 5 more than its
    listed data; the common interface primitives w^I of step 3 (5 per flux point, needed by the
    interface viscous flux) account for both the printed size and the printed ratio;
  * step 12 counts the interface flux correction F^fc at the solution points (n_s n_p), which
    the printed sizes require (step 11 writes it at the flux points).
The headline improvement is 1 - Gamma of the traffic-weighted average (20.1 %, 20.6 %, 21.0 %).
"""
from __future__ import annotations

from dataclasses import dataclass

NP = 5


@dataclass(frozen=True)
class Qty:
    name: str
    at: str            # "s" (solution points) or "f" (flux points)
    scalars: int = 0   # per point
    vectors: int = 0   # compressible 3-vectors per point


def _q(k: int):
    """the quantities of Table (fr_nse)"""
    return {
        "q_s": Qty("q^s", "s", scalars=NP), "q_f": Qty("q^f", "f", scalars=NP),
        "w_s": Qty("w^s", "s", scalars=NP), "w_I": Qty("w^I", "f", scalars=NP),
        "n_f": Qty("n_f", "f", vectors=1),
        "nFinv": Qty("n.F^I_inv", "f", scalars=NP), "nFvis": Qty("n.F^I_vis", "f", scalars=NP),
        "nFdiff": Qty("n.(F^I_inv - F^I_vis)", "f", scalars=NP),
        "gw_s": Qty("grad w^s", "s", vectors=NP), "gw_c": Qty("grad w^c", "s", vectors=NP),
        "gw_f": Qty("grad w^f", "f", vectors=NP),
        "J_f": Qty("J_f", "f", vectors=3), "detJ_f": Qty("|J_f|", "f", scalars=1),
        "J_s": Qty("J_s", "s", vectors=3), "detJ_s": Qty("|J_s|", "s", scalars=1),
        "F_s": Qty("F^s", "s", vectors=NP), "divF_s": Qty("div F^s", "s", scalars=NP),
        "F_fc_f": Qty("F^fc", "f", scalars=NP), "F_fc_s": Qty("F^fc (at solution points)", "s", scalars=NP),
        "divF_c": Qty("div F^c", "s", scalars=NP),
    }


STEPS = [
    (1, "Interpolate solution to flux points", ["q_s", "q_f"]),
    (2, "Common interface inviscid flux", ["q_f", "n_f", "nFinv"]),
    (3, "Common interface primitives", ["q_f", "w_I"]),
    (4, "Primitives at solution points", ["q_s", "w_s"]),
    (5, "Gradient of primitives", ["w_s", "gw_s"]),
    (6, "Correct gradient of primitives", ["gw_s", "w_I", "gw_c"]),
    (7, "Interpolate gradient to flux points", ["gw_c", "gw_f"]),
    (8, "Common interface viscous flux", ["gw_f", "n_f", "J_f", "detJ_f", "q_f", "w_I", "nFvis"]),
    (9, "Flux at solution points", ["gw_s", "J_s", "detJ_s", "q_s", "F_s"]),
    (10, "Divergence of flux", ["F_s", "divF_s"]),
    (11, "Correction to flux at interfaces", ["F_s", "nFdiff", "F_fc_f"]),
    (12, "Correct divergence of flux", ["F_fc_s", "divF_s", "divF_c"]),
]


def points(k: int):
    return (k + 1) ** 3, 6 * (k + 1) ** 2


def step_bytes(k: int, step: int, as_printed: bool = False):
    """(uncompressed bytes, compressed bytes) of one step for one element of degree k"""
    ns, nf = points(k)
    if as_printed and step == 4:
        ns = points(3)[0]   # the printed row repeats the k = 3 figure
    q = _q(k)
    names = dict((s, n) for s, _, n in STEPS)[step]
    full = comp = 0
    for key in names:
        Q = q[key]
        n = ns if Q.at == "s" else nf
        full += n * (4 * Q.scalars + 12 * Q.vectors)
        comp += n * (4 * Q.scalars + 8 * Q.vectors)
    return full, comp


def table(k: int, as_printed: bool = False):
    """rows (step, description, T KiB, Gamma) and the total (sum T, traffic-weighted Gamma)"""
    rows = []
    tot_f = tot_c = 0
    for s, desc, _ in STEPS:
        f, c = step_bytes(k, s, as_printed)
        rows.append((s, desc, f / 1024.0, c / f))
        tot_f += f
        tot_c += c
    return rows, (tot_f / 1024.0, tot_c / tot_f)


def improvement(k: int, as_printed: bool = False) -> float:
    """predicted fractional reduction of the right-hand side's run time (memory-bound): 1 - Gamma"""
    return 1.0 - table(k, as_printed)[1][1]
