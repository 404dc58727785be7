"""A minimal micromagnetic evaluation loop around the demagnetizing field.

Test infrastructure: only the tests, the package smoke check and the
benchmark's CPU baseline use this module.

Paper:
  * Sec. 2, Eq. 1: the LLG equation dm/dt = -gamma m x H_eff + alpha m x dm/dt
    with gamma = mu0 g_rel |gamma_e| and gamma_e = -g mu_B / hbar.  Solved for
    dm/dt it reads dm/dt = -gamma/(1 + alpha^2) [m x H + alpha m x (m x H)].
  * Appendix A, Table 1, "Direct Exchange": H = (2A / (mu0 Ms)) lap(m) with the
    homogeneous Neumann condition dm/dn = 0; "Demagnetizing Field" as in
    conv.py; the applied (Zeeman) field adds H_ext.
  * Sec. 7: the benchmark evaluates demagnetizing, exchange and applied fields
    with the RK4 method, four evaluations per time step.
  * Sec. 6: for two sublattices the demagnetizing field is that of
    (M_A + M_B) / 2.

Readings: the Laplacian is the 6-point finite-difference one, where a missing
neighbour at the mesh surface is replaced by the cell itself (the discrete
dm/dn = 0); m is renormalized to unit length after each RK4 step, not inside
it; g_rel = 1 and g = 2.00231930436 (CODATA), so gamma = 2.2128e5 m/(A s).
FP64 throughout.
"""
import math

import numpy as np

from .conv import MU0, fft_conv

G_E = 2.00231930436
MU_B = 9.2740100783e-24
HBAR = 1.054571817e-34
GAMMA = MU0 * G_E * MU_B / HBAR          # m / (A s)


def laplacian_neumann(m, h, pbc=(False, False, False)):
    """6-point Laplacian of each component of m [3, nz, ny, nx] with the
    homogeneous Neumann condition (ghost cell = boundary cell), or periodic
    neighbours along the axes flagged in pbc (x, y, z)."""
    m = np.asarray(m, np.float64)
    out = np.zeros_like(m)
    for ax, hh, per in zip((3, 2, 1), h, pbc):          # x, y, z array axes
        if m.shape[ax] == 1:
            continue
        if per:
            fwd, bwd = np.roll(m, -1, axis=ax), np.roll(m, 1, axis=ax)
        else:
            fwd = np.concatenate([np.take(m, range(1, m.shape[ax]), axis=ax),
                                  np.take(m, [m.shape[ax] - 1], axis=ax)], axis=ax)
            bwd = np.concatenate([np.take(m, [0], axis=ax),
                                  np.take(m, range(0, m.shape[ax] - 1), axis=ax)], axis=ax)
        out += (fwd - 2.0 * m + bwd) / (hh * hh)
    return out


def exchange_field(m, Ms, A, h, pbc=(False, False, False)):
    """H_ex = (2 A / (mu0 Ms)) lap(m)  (A/m)."""
    return 2.0 * A / (MU0 * Ms) * laplacian_neumann(m, h, pbc)


def effective_field(m, Ms, A, Hext, h, Nfull=None, pbc=(False, False, False)):
    """H_eff = H_demag[Ms m] + H_ex + H_ext (Nfull: the tensor to convolve
    with, e.g. the image-summed one of periodic boundaries)."""
    He = fft_conv(Ms * np.asarray(m, np.float64), h, Nfull)
    He += exchange_field(m, Ms, A, h, pbc)
    He += np.asarray(Hext, np.float64).reshape(3, 1, 1, 1)
    return He


def llg_rhs(m, H, alpha, gamma=GAMMA):
    """dm/dt of Eq. 1 solved for dm/dt."""
    mxH = np.cross(m, H, axis=0)
    return -gamma / (1.0 + alpha * alpha) * (mxH + alpha * np.cross(m, mxH, axis=0))


def rk4_step(m, dt, Ms, A, alpha, Hext, h, gamma=GAMMA, Nfull=None, pbc=(False, False, False)):
    """One classical RK4 step of the LLG equation (four field evaluations),
    then renormalization of m."""
    m = np.asarray(m, np.float64)
    f = lambda x: llg_rhs(x, effective_field(x, Ms, A, Hext, h, Nfull, pbc), alpha, gamma)
    k1 = f(m)
    k2 = f(m + 0.5 * dt * k1)
    k3 = f(m + 0.5 * dt * k2)
    k4 = f(m + dt * k3)
    out = m + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return out / np.linalg.norm(out, axis=0, keepdims=True)


def single_spin(theta0, phi0, H, alpha, t, gamma=GAMMA):
    """Closed-form motion of one moment in a static field H along +z (no other
    torque): the azimuth advances at gamma' H and tan(theta/2) decays as
    exp(-alpha gamma' H t), with gamma' = gamma / (1 + alpha^2).  Returns the
    unit vector at time t."""
    gp = gamma / (1.0 + alpha * alpha)
    th = 2.0 * math.atan(math.tan(theta0 / 2.0) * math.exp(-alpha * gp * H * t))
    ph = phi0 + gp * H * t
    return np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])


def two_sublattice_demag(mA, mB, MsA, MsB, h, Nfull=None):
    """Demagnetizing field of (M_A + M_B) / 2 (Sec. 6)."""
    M = 0.5 * (MsA * np.asarray(mA, np.float64) + MsB * np.asarray(mB, np.float64))
    return fft_conv(M, h, Nfull)


def total_energy(m, Ms, A, Hext, h, Nfull=None):
    """Demagnetizing + exchange + Zeeman energy (J) of the discrete system:
    E = -mu0 V sum [ (1/2) M.H_d + (1/2) M.H_ex + M.H_ext ]."""
    V = h[0] * h[1] * h[2]
    M = Ms * np.asarray(m, np.float64)
    Hd = fft_conv(M, h, Nfull)
    Hx = exchange_field(m, Ms, A, h)
    Hz = np.asarray(Hext, np.float64).reshape(3, 1, 1, 1)
    return -MU0 * V * float(np.sum(M * (0.5 * Hd + 0.5 * Hx + Hz)))
