"""Closed-form point-source solutions used to pin the oracle (test infrastructure only).

Homogeneous, unbounded, isotropic elastic full space; source at the origin.

Explosion (moment tensor M0 * I, moment-rate history M0 * s(t)): the displacement
potential gives the radial velocity

    v_r(r, t) = M0 / (4 pi rho vp^2) * ( s(tau) / r^2 + s'(tau) / (vp r) ),  tau = t - r / vp

(Aki & Richards 2002, the isotropic case of eq. 4.29: near-field 1/r^2 term plus the
far-field 1/r term).  All other velocity components vanish.
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


def explosion_vr(r, t, m0, rho, vp, f0, t0):
    """Radial particle velocity of an explosion whose moment rate is m0 * ricker(t - t0)."""
    tau = np.asarray(t) - r / vp - t0
    return m0 / (4.0 * np.pi * rho * vp * vp) * (ricker(tau, f0) / r ** 2 + ricker_dot(tau, f0) / (vp * r))
