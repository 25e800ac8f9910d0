"""Closed forms and reference solutions the paper fixes (section 4).

TEST INFRASTRUCTURE ONLY (used to pin the oracle; never by the product).

All flat-interface quantities are in the paper's dimensionless variables
(tilde omitted): y is the distance into the liquid, t the scaled time.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize, special


# --- section 4.1: expanding sphere (and its circle analogue) -------------
def expansion_gamma(t, K, dim=3, gamma0=1.0):
    """Insoluble Gamma on an interface expanding with u = K r e_r: the area
    grows as exp((dim-1) K t), so Gamma = Gamma0 exp(-(dim-1) K t)
    (section 4.1 gives the dim = 3 case, exp(-2 K t))."""
    return gamma0 * np.exp(-(dim - 1) * K * np.asarray(t))


# --- section 4.2: rotating circle ---------------------------------------
def rotation_gamma(theta, t, omega, pe):
    """Gamma on a circle in solid rotation at angular velocity omega with
    surface Peclet number Pe = omega d^2 / D_s: 2 + sin(theta - omega t)
    exp(-4 omega t / Pe) (counter-clockwise rotation; the time variable of
    the advection-diffusion equation on the circle is omega t)."""
    return 2.0 + np.sin(theta - omega * t) * np.exp(-4.0 * omega * t / pe)


# --- section 4.3.1: constant adsorption flux (Henry) ---------------------
def henry_bulk(y, t, Da):
    """Bulk profile for dGamma/dt = Da F_s with F(y,0) = 1 on y > 0."""
    y = np.asarray(y, dtype=float)
    s = math.sqrt(t)
    a = y / (2 * s)
    # exp(Da (y + Da t)) erfc(a + Da s) written with erfcx for stability
    return special.erf(a) + np.exp(-a * a) * special.erfcx(a + Da * s)


def henry_gamma(t, Da):
    t = np.asarray(t, dtype=float)
    s = np.sqrt(t)
    return (special.erfcx(Da * s) - 1.0 + 2.0 * Da * s / math.sqrt(math.pi)) / Da


# --- section 4.3.2: pure desorption --------------------------------------
def desorption_gamma(t, Bi):
    return np.exp(-Bi * np.asarray(t))


def desorption_bulk(y, t, Bi):
    """F(y,t) = Bi/sqrt(pi) e^{-Bi t} int_0^t exp(Bi tau - y^2/(4 tau))/sqrt(tau) dtau."""
    def one(yv):
        # substitute tau = s^2 to remove the 1/sqrt(tau) singularity
        g = lambda s: 2.0 * math.exp(Bi * s * s - yv * yv / (4 * s * s)) if s > 0 else (
            2.0 if yv == 0 else 0.0)
        val, _ = integrate.quad(g, 0.0, math.sqrt(t), limit=200, epsabs=1e-13, epsrel=1e-12)
        return Bi / math.sqrt(math.pi) * math.exp(-Bi * t) * val
    return np.array([one(float(v)) for v in np.atleast_1d(y)])


# --- section 4.3.3: Langmuir --------------------------------------------
def langmuir_gamma_eq(Da, Bi):
    """Equilibrium coverage with an undepleted bulk: Da / (Da + Bi)."""
    return Da / (Da + Bi)


def langmuir_1d_reference(Da, Bi, t_out, length=4.0, n=800, F0=1.0, G0=0.0,
                          saturation=True):
    """Sharp-interface 1D reference of section 4.3.3: F_t = F_yy on
    0 < y < length with dGamma/dt = Da F(0)(1 - Gamma) - Bi Gamma supplied
    by the bulk at y = 0 (F_y(0) = dGamma/dt) and no flux at y = length.
    Second-order finite volumes in y, implicit BDF in time (scipy).
    saturation=False drops the (1 - Gamma) factor (the constant adsorption
    flux law of section 4.3.1), which the closed form there checks.
    Returns (Gamma(t_out), F(y_cells, t_out[-1]), y_cells)."""
    h = length / n
    y = (np.arange(n) + 0.5) * h

    def rhs(_t, z):
        F = z[:n]
        G = z[n]
        # wall value at y = 0 by linear extrapolation of the first two cells
        F0w = 1.5 * F[0] - 0.5 * F[1]
        J = Da * F0w * ((1.0 - G) if saturation else 1.0) - Bi * G
        dF = np.empty(n)
        flux = np.empty(n + 1)          # diffusive flux -F_y (towards +y) at faces
        flux[1:n] = -(F[1:] - F[:-1]) / h
        flux[0] = -J                    # J leaves the bulk towards -y, into the interface
        flux[n] = 0.0
        dF[:] = -(flux[1:] - flux[:-1]) / h
        return np.concatenate([dF, [J]])

    z0 = np.concatenate([np.full(n, F0), [G0]])
    sol = integrate.solve_ivp(rhs, (0.0, float(np.max(t_out))), z0, method="BDF",
                              t_eval=np.atleast_1d(t_out), rtol=1e-9, atol=1e-12)
    return sol.y[n], sol.y[:n, -1], y


def closed_box_langmuir(phi_sum, delta_sum, total, k_a, k_d, gamma_inf):
    """Equilibrium of a closed box with uniform c and Gamma: the total
    surfactant c * sum(phi) + Gamma * sum(delta) (cell sums times the cell
    volume) equals the initial total, and adsorption balances desorption,
    k_a c (Gamma_inf - Gamma) = k_d Gamma.  Returns (c_eq, Gamma_eq)."""
    def gam(c):
        return gamma_inf * k_a * c / (k_a * c + k_d)

    f = lambda c: c * phi_sum + gam(c) * delta_sum - total
    c = optimize.brentq(f, 0.0, total / phi_sum * 1.0000001 + 1e-30, xtol=1e-15, rtol=1e-15)
    return c, gam(c)


# --- section 2.3 / 2.5 helpers ------------------------------------------
def planar_delta_column_sum(offset, h, eps, chi_max):
    """Sum over a column of cells of phi(1-phi)/eps * h for a planar signed
    distance chi = -(y - offset) sampled at cell centres, unclamped, plus the
    clamp contribution handled by the caller.  Used only as a convenience for
    the P1 pin (the integral of |grad phi| across a planar interface is 1)."""
    k = np.arange(-4000, 4001)
    chi = -((k + 0.5) * h - offset)
    chi = np.clip(chi, -chi_max, chi_max)
    ph = 1.0 / (1.0 + np.exp(chi / eps))
    return float(np.sum(ph * (1 - ph) / eps) * h)
