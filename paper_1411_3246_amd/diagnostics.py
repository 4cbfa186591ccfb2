"""Post-processing of recorded plasma electron trajectories (radii per slice
from wk_plasma_response_traj), for the discussion of the trajectories behind
the driver in Section III: where the electrons that the drive expels come
back to the axis, and over how wide a range of xi."""
from typing import Dict, Sequence

import numpy as np


def axis_crossings(tr: np.ndarray, xi: np.ndarray, h: float, xi_drive: float,
                   thresholds: Sequence[int] = (2, 4)) -> Dict[str, dict]:
    """tr: (n_xi, n) radii, xi: (n_xi,) slice positions, h: cell size.

    Electrons loaded within r0 <= 2 that the drive expels (their radius grows
    by more than 0.3 behind xi_drive) and that come back to the axis: for
    each threshold m, the number whose radius drops below m cells after its
    largest excursion, and the xi of that first drop (mean, std and the
    10-90 % width)."""
    k0 = int(np.searchsorted(xi, xi_drive))
    r0 = tr[0]
    out = {}
    for m in thresholds:
        cross = []
        for q in np.where(r0 <= 2.0)[0]:
            seg = tr[k0:, q]
            kpk = int(np.argmax(seg))
            if seg[kpk] < r0[q] + 0.3:
                continue
            below = np.where(seg[kpk:] < m * h)[0]
            if len(below):
                cross.append(xi[k0 + kpk + below[0]])
        cross = np.array(cross)
        out[f"below_{m}_cells"] = {
            "electrons": int(len(cross)),
            "xi_mean": float(cross.mean()) if len(cross) else None,
            "xi_std": float(cross.std()) if len(cross) else None,
            "xi_width_10_90": float(np.percentile(cross, 90) - np.percentile(cross, 10)) if len(cross) > 2 else None,
        }
    return out
