"""Oracle (test infrastructure only): the two-dimensional variable-coefficient
heat problems T1 and T2 of the stencil appendix, on the periodic square
[0, 2pi]^2, advanced with 3-node Gauss-Lobatto SDC and 4 sweeps, time step
0.4 / ((dx^-2 + dy^-2) max(a, b)) rounded down so that an integer number of
steps reaches t = 1."""
import math

import numpy as np

from . import heat2d
from .sdc import gauss_lobatto, sdc_run

EPS_T1 = 0.1
EPS_T2 = 0.9


def grid(n):
    x = 2 * np.pi * np.arange(n) / n
    Y, X = np.meshgrid(x, x, indexing="ij")
    return X, Y


def t1_coeffs(n):
    X, Y = grid(n)
    a = 1.0 + EPS_T1 * np.cos(X) * np.cos(Y)
    return X, Y, a, a.copy()


def t2_coeffs(n):
    X, Y = grid(n)
    a = 1.0 + EPS_T2 * np.cos(2 * X) * np.sin(2 * Y + np.pi / 3)
    b = 1.0 + EPS_T2 * np.cos(2 * X + np.pi / 3) * np.sin(2 * Y)
    return X, Y, a, b


def time_step(n, amax):
    dx = 2 * np.pi / n
    dt = 0.4 / ((2.0 / dx ** 2) * amax)
    nsteps = math.ceil(1.0 / dt - 1e-12)
    return 1.0 / nsteps, nsteps


def run(problem, n, m47, m48, t_end=1.0):
    dx = 2 * np.pi / n
    if problem == "T1":
        X, Y, a, b = t1_coeffs(n)
        src = 1.0 + 4.0 * EPS_T1 * np.cos(X) * np.cos(Y)
        base = np.sin(X) * np.sin(Y)

        def f(u, t):
            return heat2d(a, b, u, dx, m47, m48) + src * math.exp(-t) * base
        amax = 1.0 + EPS_T1
    else:
        X, Y, a, b = t2_coeffs(n)

        def f(u, t):
            return heat2d(a, b, u, dx, m47, m48)
        amax = max(a.max(), b.max())
    dt, nsteps = time_step(n, amax)
    u0 = np.sin(X) * np.sin(Y)
    u = sdc_run(f, u0, 0.0, dt, gauss_lobatto(3), 4, nsteps)
    return u, X, Y
