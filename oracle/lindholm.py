"""Closed-form double-layer integrals over one flat triangle (oracle; test only).

The entries of K (Section 3, eq. matrix_definition) are

    K_ij = (1/4pi) * integral over the surface of phi_j(y) n(y).(xi_i - y)/|xi_i - y|^3 dS_y,

the normal derivative (with respect to y) of 1/(4 pi |x - y|).  The paper
cites analytic forms for them (Lindholm 1984) without stating them; they are
re-derived here from the definition.  For a triangle T = (r1, r2, r3),
counter-clockwise about its unit normal n, area A, and a point x:

* e_b = r_{b+1} - r_b, s_b = |e_b|, u_b = e_b/s_b (indices mod 3);
* zeta = n.(x - r1): x's height above the plane of T;
* Omega(x) = integral_T n.(x - y)/|x - y|^3 dS, the signed solid angle of T
  seen from x (negative on the inner side), by the Van Oosterom-Strackee form
  Omega = 2 atan2(R1.(R2 x R3), rho1 rho2 rho3 + rho1 R2.R3 + rho2 R3.R1 + rho3 R1.R2),
  R_a = x - r_a, rho_a = |R_a|;
* P_b = integral over edge b of dl/|x - y| = ln((rho_b + rho_{b+1} + s_b)/(rho_b + rho_{b+1} - s_b));
* the hat function of local vertex a is phi_a(y) = s_{a+1} (n x u_{a+1}).(y - r_{a+1})/(2A).

Writing y - r_{a+1} = (y - p) + (p - r_{a+1}) with p the foot of x in the plane
and applying the in-plane divergence theorem to (y - p)/|x - y|^3 gives

    L_a(x) = s_{a+1}/(8 pi A) * [ (n x u_{a+1}).(x - r_{a+1}) * Omega(x)
                                  + zeta * sum_b (u_{a+1}.u_b) P_b ],

the contribution of T to K_ij for the node j at local vertex a, evaluated at
x = xi_i.  Checked against brute-force quadrature, the partition
sum_a L_a = Omega/(4 pi) and Gauss's theorem in tests/test_oracle_lindholm.py.
"""
from __future__ import annotations

import numpy as np


def _dot(a, b):
    return np.einsum("...i,...i->...", a, b)


def solid_angle(x: np.ndarray, r1: np.ndarray, r2: np.ndarray, r3: np.ndarray) -> np.ndarray:
    """Signed solid angle Omega_T(x) (broadcasting over leading axes)."""
    R1, R2, R3 = x - r1, x - r2, x - r3
    p1, p2, p3 = np.linalg.norm(R1, axis=-1), np.linalg.norm(R2, axis=-1), np.linalg.norm(R3, axis=-1)
    num = _dot(R1, np.cross(R2, R3))
    den = p1 * p2 * p3 + p1 * _dot(R2, R3) + p2 * _dot(R3, R1) + p3 * _dot(R1, R2)
    return 2.0 * np.arctan2(num, den)


def weights(x: np.ndarray, r1: np.ndarray, r2: np.ndarray, r3: np.ndarray) -> np.ndarray:
    """L_a(x) for a = 0, 1, 2: array of shape (..., 3).

    Not valid when x is a vertex of T (0 * infinity); callers decide incidence
    by index and drop those pairs (the exact contribution is 0 there, because
    n.(x - y) vanishes on T).
    """
    r = [r1, r2, r3]
    e = [r[(b + 1) % 3] - r[b] for b in range(3)]
    s = [np.linalg.norm(eb, axis=-1) for eb in e]
    u = [e[b] / s[b][..., None] for b in range(3)]
    cr = np.cross(e[0], -e[2])                    # (r2 - r1) x (r3 - r1)
    two_a = np.linalg.norm(cr, axis=-1)
    n = cr / two_a[..., None]
    area = 0.5 * two_a
    rho = [np.linalg.norm(x - r[b], axis=-1) for b in range(3)]
    P = []
    for b in range(3):
        ssum = rho[b] + rho[(b + 1) % 3]
        P.append(np.log1p(2.0 * s[b] / (ssum - s[b])))
    omega = solid_angle(x, r1, r2, r3)
    zeta = _dot(n, x - r1)
    out = []
    for a in range(3):
        op = (a + 1) % 3                           # edge opposite vertex a
        eta = np.cross(n, u[op])                   # inward in-plane normal of that edge
        term1 = _dot(eta, x - r[op]) * omega
        term2 = zeta * sum(_dot(u[op], u[b]) * P[b] for b in range(3))
        out.append(s[op] / (8.0 * np.pi * area) * (term1 + term2))
    return np.stack(out, axis=-1)
