"""Error norms for comparing two solutions of the same problem."""
from __future__ import annotations

import numpy as np


def rel_l1(fields, ref, gamma: float = 1.4) -> dict:
    """Relative L1 distance per field between `fields` and `ref`, both
    (rho, ux, uy, uz, p) tuples of arrays.  rho and p are normalised by their
    own reference L1 norm; each velocity component by the L1 norm of the
    reference sound speed sqrt(gamma p / rho), since a component may vanish
    identically."""
    rho, ux, uy, uz, p = (np.asarray(a, dtype=np.float64) for a in fields)
    rr, rux, ruy, ruz, rp = (np.asarray(a, dtype=np.float64) for a in ref)
    a = np.sqrt(gamma * np.abs(rp) / np.abs(rr))
    sa = np.sum(a)
    out = {
        "rho": float(np.sum(np.abs(rho - rr)) / np.sum(np.abs(rr))),
        "ux": float(np.sum(np.abs(ux - rux)) / sa),
        "uy": float(np.sum(np.abs(uy - ruy)) / sa),
        "uz": float(np.sum(np.abs(uz - ruz)) / sa),
        "p": float(np.sum(np.abs(p - rp)) / np.sum(np.abs(rp))),
    }
    return out


def max_rel_l1(fields, ref, gamma: float = 1.4) -> float:
    return max(rel_l1(fields, ref, gamma).values())
