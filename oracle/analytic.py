"""Closed-form point-source solutions used to pin the oracle (test infrastructure only).

Homogeneous, unbounded, isotropic elastic full space (density rho, P speed a, S speed b);
source at the origin, receiver at x (m), r = |x|, direction cosines g = x / r.

Point force (Stokes' solution, Aki & Richards 2002 eq. 4.23): a force F (N, a vector)
with time history X(t) gives the displacement

    u_i = 1/(4 pi rho) (3 g_i g_j - d_ij) / r^3  int_{r/a}^{r/b} tau X(t - tau) dtau F_j
        + 1/(4 pi rho a^2) g_i g_j / r  X(t - r/a) F_j
        - 1/(4 pi rho b^2) (g_i g_j - d_ij) / r  X(t - r/b) F_j

(near field, far-field P, far-field S).  The particle velocity is the same expression
with X replaced by its time derivative.

Moment tensor (Aki & Richards 2002 eq. 4.29): a moment tensor M_pq with time history
m(t) gives

    u_n = 1/(4 pi rho) A^N_npq / r^4  int_{r/a}^{r/b} tau m(t - tau) dtau M_pq
        + 1/(4 pi rho a^2) A^IP_npq / r^2  m(t - r/a) M_pq
        - 1/(4 pi rho b^2) A^IS_npq / r^2  m(t - r/b) M_pq
        + 1/(4 pi rho a^3) A^FP_npq / r  m'(t - r/a) M_pq
        - 1/(4 pi rho b^3) A^FS_npq / r  m'(t - r/b) M_pq

    A^N  = 15 g_n g_p g_q - 3 g_n d_pq - 3 g_p d_nq - 3 g_q d_np
    A^IP =  6 g_n g_p g_q -   g_n d_pq -   g_p d_nq -   g_q d_np
    A^IS =  6 g_n g_p g_q -   g_n d_pq -   g_p d_nq - 2 g_q d_np
    A^FP =    g_n g_p g_q
    A^FS =  (g_n g_p - d_np) g_q

(near, intermediate and far fields).  It equals minus the x_q derivative of the force
solution for a force along p with history m, contracted with M_pq; the tests check
this, and that M = M0 I reduces to the explosion below.

Explosion (M = M0 I, moment rate M0 s(t)): the radial velocity

    v_r(r, t) = M0 / (4 pi rho a^2) * ( s(tau) / r^2 + s'(tau) / (a r) ),  tau = t - r / a.

Time histories here are Ricker pulses and their antiderivatives, so the near-field
integrals have closed forms: with G1' = g and G2' = G1,

    int_A^B tau g(t - tau) dtau = [ -tau G1(t - tau) - G2(t - tau) ]_{tau=A}^{tau=B}.
"""
from __future__ import annotations

import numpy as np


def ricker(t, f0):
    """Ricker wavelet r(t) = (1 - 2 (pi f0 t)^2) exp(-(pi f0 t)^2)."""
    a = (np.pi * f0 * np.asarray(t)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def ricker_dot(t, f0):
    """Time derivative of the Ricker wavelet."""
    t = np.asarray(t)
    b = (np.pi * f0) ** 2
    a = b * t * t
    return np.exp(-a) * (-4.0 * b * t - 2.0 * b * t * (1.0 - 2.0 * a))


def ricker_int(t, f0):
    """Antiderivative of the Ricker wavelet: t exp(-(pi f0 t)^2)."""
    t = np.asarray(t)
    return t * np.exp(-(np.pi * f0 * t) ** 2)


def ricker_int2(t, f0):
    """Antiderivative of ricker_int: -exp(-(pi f0 t)^2) / (2 (pi f0)^2)."""
    b = (np.pi * f0) ** 2
    return -np.exp(-b * np.asarray(t) ** 2) / (2.0 * b)


class History:
    """A time history g(t) = shape(t - t0) with its derivative and two antiderivatives,
    built from the Ricker family: order 0 = Ricker, -1 = its antiderivative, +1 = its
    derivative."""

    _CHAIN = (ricker_int2, ricker_int, ricker, ricker_dot)

    def __init__(self, f0, t0, order=0):
        if order not in (-1, 0, 1):
            raise ValueError("order must be -1, 0 or 1")
        self.f0, self.t0, self.k = f0, t0, order + 2  # index of g in _CHAIN

    def _at(self, idx, t):
        return self._CHAIN[idx](np.asarray(t) - self.t0, self.f0)

    def g(self, t):
        return self._at(self.k, t)

    def dg(self, t):
        if self.k + 1 >= len(self._CHAIN):
            raise ValueError("no derivative of this order")
        return self._at(self.k + 1, t)

    def G1(self, t):
        return self._at(self.k - 1, t)

    def G2(self, t):
        if self.k - 2 < 0:
            raise ValueError("no second antiderivative of this order")
        return self._at(self.k - 2, t)


def near_integral(h: History, t, A, B):
    """int_A^B tau g(t - tau) dtau in closed form (integration by parts)."""
    t = np.asarray(t)
    return (-B * h.G1(t - B) - h.G2(t - B)) - (-A * h.G1(t - A) - h.G2(t - A))


def _geom(x):
    x = np.asarray(x, dtype=np.float64)
    r = float(np.linalg.norm(x))
    return r, x / r


def force_field(x, t, F, rho, a, b, h: History):
    """Aki & Richards 4.23: field [3, nt] at x for a force F (3-vector) with history g of
    ``h`` (displacement for the force's own history; velocity when ``h`` is its time
    derivative)."""
    r, g = _geom(x)
    F = np.asarray(F, dtype=np.float64)
    d = np.eye(3)
    gg = np.outer(g, g)
    near = (3.0 * gg - d) @ F / r ** 3
    fp = gg @ F / (a * a * r)
    fs = (gg - d) @ F / (b * b * r)
    t = np.asarray(t, dtype=np.float64)
    out = (near[:, None] * near_integral(h, t, r / a, r / b)[None, :]
           + fp[:, None] * h.g(t - r / a)[None, :]
           - fs[:, None] * h.g(t - r / b)[None, :])
    return out / (4.0 * np.pi * rho)


def moment_field(x, t, M, rho, a, b, h: History):
    """Aki & Richards 4.29: field [3, nt] at x for a symmetric moment tensor M (3x3, or
    the six values Mxx Myy Mzz Mxy Mxz Myz) with history g of ``h``.  With g the moment
    rate this is the particle velocity."""
    M = np.asarray(M, dtype=np.float64)
    if M.shape == (6,):
        xx, yy, zz, xy, xz, yz = M
        M = np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])
    r, g = _geom(x)
    d = np.eye(3)
    ggg = np.einsum("n,p,q->npq", g, g, g)
    g_dpq = np.einsum("n,pq->npq", g, d)  # g_n d_pq
    g_dnq = np.einsum("p,nq->npq", g, d)  # g_p d_nq
    g_dnp = np.einsum("q,np->npq", g, d)  # g_q d_np
    AN = 15.0 * ggg - 3.0 * g_dpq - 3.0 * g_dnq - 3.0 * g_dnp
    AIP = 6.0 * ggg - g_dpq - g_dnq - g_dnp
    AIS = 6.0 * ggg - g_dpq - g_dnq - 2.0 * g_dnp
    AFP = ggg
    AFS = np.einsum("np,q->npq", np.outer(g, g) - d, g)
    c = lambda A: np.einsum("npq,pq->n", A, M)
    t = np.asarray(t, dtype=np.float64)
    out = (c(AN)[:, None] / r ** 4 * near_integral(h, t, r / a, r / b)[None, :]
           + c(AIP)[:, None] / (a * a * r * r) * h.g(t - r / a)[None, :]
           - c(AIS)[:, None] / (b * b * r * r) * h.g(t - r / b)[None, :]
           + c(AFP)[:, None] / (a ** 3 * r) * h.dg(t - r / a)[None, :]
           - c(AFS)[:, None] / (b ** 3 * r) * h.dg(t - r / b)[None, :])
    return out / (4.0 * np.pi * rho)


def explosion_vr(r, t, m0, rho, vp, f0, t0):
    """Radial particle velocity of an explosion whose moment rate is m0 * ricker(t - t0)."""
    tau = np.asarray(t) - r / vp - t0
    return m0 / (4.0 * np.pi * rho * vp * vp) * (ricker(tau, f0) / r ** 2 + ricker_dot(tau, f0) / (vp * r))
