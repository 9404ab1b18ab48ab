"""Closed-form Green's functions used to pin the discrete operator (test infrastructure).

Convention: (Delta + k^2) G = delta with time dependence e^{-i omega t}, so the
outgoing free-space solution is G = -exp(i k r)/(4 pi r).

Linear velocity gradient (the paper validates its FD and FE schemes against an
analytic solution in c = c0 + alpha z, FD-vs-FE section and Table 1): with
Z = z + c0/alpha the medium is c = alpha Z and the equation maps to the
Helmholtz equation of hyperbolic space, whose outgoing Green's function gives
    G(x, xs) = -exp(i mu sigma) / (4 pi sqrt(Z Zs) sinh sigma),
    cosh sigma = 1 + |x - xs|^2 / (2 Z Zs)  (sinh(sigma/2) = |x - xs|/(2 sqrt(Z Zs))),  mu = sqrt((omega/alpha)^2 - 1/4).
Near the source sigma ~ r/sqrt(Z Zs) and G -> -1/(4 pi r).
"""
from __future__ import annotations

import numpy as np


def green_homogeneous(r, k):
    return -np.exp(1j * k * r) / (4.0 * np.pi * r)


def green_linear_gradient(x, y, z, xs, ys, zs, omega, c0, alpha):
    Z = z + c0 / alpha
    Zs = zs + c0 / alpha
    r = np.sqrt((x - xs) ** 2 + (y - ys) ** 2 + (z - zs) ** 2)
    # cosh sigma = 1 + 2 sinh^2(sigma/2): the half-angle form avoids cancellation near the source
    sig = 2.0 * np.arcsinh(r / (2.0 * np.sqrt(Z * Zs)))
    mu = np.sqrt((omega / alpha) ** 2 - 0.25)
    return -np.exp(1j * mu * sig) / (4.0 * np.pi * np.sqrt(Z * Zs) * np.sinh(sig))
