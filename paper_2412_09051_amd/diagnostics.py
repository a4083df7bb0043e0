"""Diagnostics of the temporal mixing layer (Sec. 4.4), computed from nodal moment fields.

These functions analyse what the library has computed (density and velocity per node,
the nodal quadrature volumes); they are not part of the time step.  They take numpy
arrays or torch tensors (on any device) shaped [Nz][Ny][Nx], y the cross-stream axis.
"""
from __future__ import annotations

import numpy as np

# Extent of the self-similar stage, tau = t du / dtheta0, per convective Mach number
# (Tab. 3: tau_min and tau_max).
MIX_WINDOW = {0.3: (350.0, 550.0), 0.7: (450.0, 700.0), 0.9: (800.0, 1100.0), 1.2: (1400.0, 2000.0)}


def momentum_thickness(rho, ux, V, du, area_xz, rho0=1.0):
    """Momentum thickness (Sec. 4.4, the delta_theta display):
        delta_theta = 1 / (rho0 du^2) int <rho> (du/2 - u~)(du/2 + u~) dy,
    with <.> the plane average over x and z and u~ = <rho u_x> / <rho> the Favre average.
    The plane averages and the y integral use the nodal quadrature volumes V (the
    integrals of the nodal Lagrange functions): summing V over a node plane gives that
    plane's y weight times the plane's area, area_xz = L_x L_z."""
    A = (V * rho).sum(axis=(0, 2))
    B = (V * rho * ux).sum(axis=(0, 2))
    Wy = V.sum(axis=(0, 2))
    rbar = A / Wy
    ut = B / A
    wy = Wy / area_xz
    return float((wy * rbar * (0.5 * du - ut) * (0.5 * du + ut)).sum() / (rho0 * du ** 2))


def window_rate(tau, theta, window):
    """Growth rate d(delta_theta)/d(tau) fitted by least squares over the samples whose tau
    lies inside window = (tau_min, tau_max); None if fewer than three samples do."""
    tau = np.asarray(tau, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    sel = (tau >= window[0]) & (tau <= window[1])
    if sel.sum() < 3:
        return None
    return float(np.polyfit(tau[sel], theta[sel], 1)[0])
