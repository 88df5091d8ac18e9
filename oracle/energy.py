"""Demagnetising energy from boundary data (oracle; test infrastructure only).

Section 6.2 compares the computed magnetostatic energy with analytic values;
for a uniformly magnetised sphere the demagnetising factor is 1/3 and the
energy density mu0 Ms^2/6.  For uniform M = Ms z the energy needs only the
boundary trace of u = u1 + u2: with H = -grad u inside,

    E_d = -(mu0/2) int_Omega M.H dV = (mu0 Ms/2) int_Omega d_z u dV
        = (mu0 Ms/2) oint u n_z dS,

and u1 = Ms z.  With P1 data on flat triangles (Ms = 1, mu0 = 1):

    E = (1/2) [ V_poly + sum_T A_T n_z,T (u2_a + u2_b + u2_c)/3 ],

V_poly = oint z n_z dS being the polyhedron's volume.  Exact: E = V/6 for a
sphere (u = z/3 inside).
"""
from __future__ import annotations

import numpy as np

from . import geometry


def demag_energy_z(xyz: np.ndarray, tri: np.ndarray, u2: np.ndarray) -> float:
    """E/(mu0 Ms^2) of the uniformly z-magnetised body, from u2 = M z at the nodes."""
    t = np.asarray(tri, dtype=np.int64)
    nrm, area = geometry.triangle_normals_areas(xyz, t)
    vol = geometry.signed_volume(xyz, t)
    mean_u2 = (u2[t[:, 0]] + u2[t[:, 1]] + u2[t[:, 2]]) / 3.0
    return 0.5 * (vol + float(np.sum(area * nrm[:, 2] * mean_u2)))
