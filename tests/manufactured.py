"""The paper's quadratic manufactured Stokes solution (Section 4.1: velocity
v2, pressure phi2; closed forms in tests/golden/manufactured_fields.json) as
nodal values and the right-hand side of the block system of Section 3.2.
Plain closed-form evaluation; nothing here is shared with the oracle or the
GPU path."""
from __future__ import annotations

import json
import os

import numpy as np

from tests import polytools as PT

HERE = os.path.dirname(os.path.abspath(__file__))


def fields():
    fx = json.load(open(os.path.join(HERE, "golden", "manufactured_fields.json")))
    v = [PT.from_terms(c) for c in fx["v2"]["components"]]
    lap_v = [PT.from_terms(c) for c in fx["v2"]["laplacian"]]
    phi = PT.from_terms(fx["phi2"]["field"])
    grad_phi = [PT.from_terms(g) for g in fx["phi2"]["gradient"]]
    lap_phi = PT.from_terms(fx["phi2"]["laplacian"])
    return v, lap_v, phi, grad_phi, lap_phi


def exact_system(pts, bnd, nrm, nlap_h, nu):
    """Nodal unknowns x (velocity, zero-mean pressure, multiplier 0) and the
    right-hand side: f = -nu Laplacian v2 + grad phi2 (interior velocity),
    v2 (boundary velocity), div f = Laplacian phi2 (interior pressure),
    div f - beta n.f (boundary pressure), 0 (multiplier)."""
    v, lap_v, phi, grad_phi, lap_phi = fields()
    n, d = pts.shape
    V = np.stack([PT.evaluate(c, pts) for c in v], axis=1)
    f = np.stack([-nu * PT.evaluate(lap_v[c], pts) + PT.evaluate(grad_phi[c], pts) for c in range(d)], axis=1)
    div_f = PT.evaluate(lap_phi, pts)  # div f = Laplacian phi since div v = 0
    P = PT.evaluate(phi, pts)
    x = np.concatenate([V.reshape(-1), P - P.mean(), [0.0]])
    b = np.where(bnd[:, None] == 1, V, f).reshape(-1)
    g = np.where(bnd == 1, div_f - nlap_h * np.sum(nrm * f, axis=1), div_f)
    return x, np.concatenate([b, g, [0.0]])
