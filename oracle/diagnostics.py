"""Run diagnostics: conserved sums and entropies (Sec. 4).

Test infrastructure only (see ``oracle/__init__``).

  * sum_x u_m (conserved by transport and by every R_omega);
  * total microscopic entropy sum_x Sigma(f), conserved by transport and, with
    the entropy-limited omega, by relaxation (Sec. 4);
  * sum_x S(u), bounded by the initial total microscopic entropy when the
    initial data are at equilibrium (the inequality chain at the end of Sec. 4).
Sums are plain ``math.fsum`` (exactly rounded) so they are independent of order.
"""
import math

import numpy as np

from .systems import kinetic_entropy_sum


def diagnostics(lat, sys, V, f):
    u = f.sum(axis=0)
    micro, ok = kinetic_entropy_sum(lat, sys, V, f)
    return {
        "mass": [math.fsum(u[m].ravel()) for m in range(u.shape[0])],
        "micro_entropy": math.fsum(np.where(ok, micro, 0.0).ravel()),
        "macro_entropy": math.fsum(sys.macro_entropy(u).ravel()),
        "n_outside_domain": int(np.count_nonzero(~ok)),
        "n_inadmissible": int(np.count_nonzero(~sys.admissible(u))),
        "n_nan": int(np.count_nonzero(~np.isfinite(f))),
    }
