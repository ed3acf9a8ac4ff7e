"""Oracle: constant-medium closed forms.  TEST INFRASTRUCTURE ONLY.

Sec. 1 states the 3D point-source solution for kappa = 1 and the choice tau = r that
makes the amplitude smooth.  With the source on the right of eq. Helmholtz as +delta,
Delta u + w^2 u = delta(x - x0) has the outgoing (exp(-i w r)) solution
    3D: u = -exp(-i w r) / (4 pi r),            a = u exp(i w r) = -1 / (4 pi r)
    2D: u = (i/4) H0^(2)(w r),                  a = (i/4) H0^(2)(w r) exp(i w r)
(the paper prints +1/(4 pi r); the sign follows from the +delta source).
"""
import numpy as np
from scipy.special import hankel2


def amplitude_3d(r):
    return -1.0 / (4.0 * np.pi * np.asarray(r, dtype=np.float64))


def amplitude_2d(r, omega):
    r = np.asarray(r, dtype=np.float64)
    return 0.25j * hankel2(0, omega * r) * np.exp(1j * omega * r)


def wavefield_3d(r, omega):
    return amplitude_3d(r) * np.exp(-1j * omega * np.asarray(r))


def wavefield_2d(r, omega):
    return 0.25j * hankel2(0, omega * np.asarray(r, dtype=np.float64))
