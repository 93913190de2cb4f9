"""Textbook formulas used as independent pins of the oracle.

These are the standard single-relaxation-time (BGK) forms of the lattice
Boltzmann method with Guo's forcing (Guo, Zheng & Shi, Phys. Rev. E 65,
046308, 2002), written in population space.  The MRT operator of the method
must reduce to them when every relaxation rate is equal.
"""
import numpy as np

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])


def feq9(rho, ux, uy):
    eu = EX * ux + EY * uy
    usq = ux * ux + uy * uy
    return W9 * rho * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * usq)


def geq5(T, ux, uy, a=-2.0):
    w0 = (1 - a) / 5
    wk = (4 + a) / 20
    out = np.empty(5)
    out[0] = w0 * T
    for k in range(1, 5):
        out[k] = wk * T + 0.5 * T * (EX[k] * ux + EY[k] * uy)
    return out


def guo_force9(ux, uy, Fx, Fy):
    """Guo's forcing term F_i = w_i [3 (e_i - u) + 9 (e_i . u) e_i] . F."""
    eu = EX * ux + EY * uy
    return W9 * ((3 * (EX - ux) + 9 * eu * EX) * Fx + (3 * (EY - uy) + 9 * eu * EY) * Fy)


def bgk_guo_collide(f, s, Fx, Fy):
    rho = f.sum()
    ux = ((EX * f).sum() + 0.5 * Fx) / rho
    uy = ((EY * f).sum() + 0.5 * Fy) / rho
    return f - s * (f - feq9(rho, ux, uy)) + (1 - 0.5 * s) * guo_force9(ux, uy, Fx, Fy), (rho, ux, uy)
