"""Brute-force reference for the oracle pins: no splitting, no Romberg.

Integrates Hamilton's equations of the general Hamiltonian of §2.1
(eq. generalH)

    H = -(1 + hX) Ps - (q/p0)(1 + hX) A_s + Pt/β0,

together with the spin equation dS/ds = Ω × S (eq. t-bmt.s), with an
adaptive 8th-order Runge–Kutta method (scipy's DOP853) at tolerances near
double-precision round-off.  Hamilton's equations are written here directly
from H, term by term:

    X'  =  (1 + hX) Px/Ps          Px' = h Ps - ∂V/∂X
    Y'  =  (1 + hX) Py/Ps          Py' = -∂V/∂Y
    T'  = -(1 + hX)(1/β0 + Pt)/Ps + 1/β0,    Pt' = 0

with V = -(q/p0)(1 + hX) A_s:  sector bend V = (η/2)(1 + hX)^2, quadrupole
V = (k1/2)(X^2 - Y^2), sextupole V = (k2/6)(X^3 - 3 X Y^2).

Thin multipoles are the limit of a kick flow over a unit pseudo-length with
no drift term: X, Y fixed, Px and Py changing linearly, the spin precessing
about the integrated Ω evaluated along the changing momenta.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.integrate import solve_ivp


def _omega(X, Px, Py, Pt, h, b, beam):
    b0 = beam.beta0
    P = math.sqrt(1.0 + 2.0 * Pt / b0 + Pt * Pt)
    Ps = math.sqrt(1.0 + 2.0 * Pt / b0 + Pt * Pt - Px * Px - Py * Py)
    u = np.array([Px, Py, Ps]) / P
    gamma = beam.gamma0 * (1.0 + b0 * Pt)
    a1, a2 = 1.0 + beam.G * gamma, beam.G * (gamma - 1.0)
    ub = float(u @ b)
    om = -(1.0 + h * X) / Ps * (a1 * b - a2 * ub * u)
    om[1] += h
    return om


def _rhs_thick(kind, par, beam):
    b0 = beam.beta0
    h = par.get("h", 0.0)
    eta = par.get("eta", 1.0)
    k1 = par.get("k1", 0.0)
    k2 = par.get("k2", 0.0)

    def f(s, y):
        X, Px, Y, Py, T, Pt, Sx, Sy, Sz = y
        Ps = math.sqrt(1.0 + 2.0 * Pt / b0 + Pt * Pt - Px * Px - Py * Py)
        w = 1.0 + h * X
        if kind == "sbend":
            dVx, dVy = eta * h * w, 0.0
            b = np.array([0.0, eta * h, 0.0])
        elif kind == "quad":
            dVx, dVy = k1 * X, -k1 * Y
            b = np.array([k1 * Y, k1 * X, 0.0])
        elif kind == "sext":
            dVx, dVy = 0.5 * k2 * (X * X - Y * Y), -k2 * X * Y
            b = np.array([k2 * X * Y, 0.5 * k2 * (X * X - Y * Y), 0.0])
        else:  # drift
            dVx = dVy = 0.0
            b = np.zeros(3)
        om = _omega(X, Px, Py, Pt, h, b, beam)
        S = np.array([Sx, Sy, Sz])
        dS = np.cross(om, S)
        return [w * Px / Ps, h * Ps - dVx, w * Py / Ps, -dVy,
                -w * (1.0 / b0 + Pt) / Ps + 1.0 / b0, 0.0, dS[0], dS[1], dS[2]]
    return f


def _rhs_thin(k1l, k2l, X, Y, beam):
    # integrated field of the thin multipole at the (fixed) position
    b = np.array([k1l * Y + k2l * X * Y, k1l * X + 0.5 * k2l * (X * X - Y * Y), 0.0])
    dPx = -(k1l * X + 0.5 * k2l * (X * X - Y * Y))
    dPy = k1l * Y + k2l * X * Y

    def f(t, y):
        Xs, Px, Ys, Py, T, Pt, Sx, Sy, Sz = y
        om = _omega(X, Px, Py, Pt, 0.0, b, beam)
        dS = np.cross(om, np.array([Sx, Sy, Sz]))
        return [0.0, dPx, 0.0, dPy, 0.0, 0.0, dS[0], dS[1], dS[2]]
    return f


def _rhs_solenoid(ks, profile, beam):
    """Hamilton's equations of eq. Hsolenoid with the vector potential of
    eq. Asol scaled by a longitudinal profile S(s), and the spin in the field
    b = (-X/2 ks S', -Y/2 ks S', ks S) (div b = 0), û from the kinetic
    momentum (eq. mgVSol)."""
    b0 = beam.beta0

    def f(s, y):
        X, Px, Y, Py, T, Pt, Sx, Sy, Sz = y
        S, dS = profile(s)
        eta = 0.5 * ks * S
        kx, ky = Px + eta * Y, Py - eta * X
        P2 = 1.0 + 2.0 * Pt / b0 + Pt * Pt
        Ps = math.sqrt(P2 - kx * kx - ky * ky)
        P = math.sqrt(P2)
        b = np.array([-0.5 * X * ks * dS, -0.5 * Y * ks * dS, ks * S])
        u = np.array([kx, ky, Ps]) / P
        gamma = beam.gamma0 * (1.0 + b0 * Pt)
        a1, a2 = 1.0 + beam.G * gamma, beam.G * (gamma - 1.0)
        om = -(1.0 / Ps) * (a1 * b - a2 * float(u @ b) * u)
        dSv = np.cross(om, np.array([Sx, Sy, Sz]))
        return [kx / Ps, eta * ky / Ps, ky / Ps, -eta * kx / Ps,
                -(1.0 / b0 + Pt) / Ps + 1.0 / b0, 0.0, dSv[0], dSv[1], dSv[2]]
    return f


def track_solenoid(L, ks, eps, beam, z, s, rtol=1e-13, atol=1e-16):
    """A solenoid whose field rises linearly over [0, eps], stays at ks up to
    L and falls linearly over [L, L + eps] (field integral ks L); eps = 0
    integrates the body alone."""
    y = np.concatenate([np.asarray(z, float), np.asarray(s, float)])
    if eps == 0.0:
        pieces = [(0.0, L, lambda t: (1.0, 0.0))]
    else:
        pieces = [(0.0, eps, lambda t: (t / eps, 1.0 / eps)),
                  (eps, L, lambda t: (1.0, 0.0)),
                  (L, L + eps, lambda t: ((L + eps - t) / eps, -1.0 / eps))]
    for a, b, prof in pieces:
        sol = solve_ivp(_rhs_solenoid(ks, prof, beam), (a, b), y, method="DOP853",
                        rtol=rtol, atol=atol)
        y = sol.y[:, -1]
    return y[:6].copy(), y[6:].copy()


def track_element(e, beam, z, s, rtol=1e-13, atol=1e-16):
    """Brute-force map of one element (workloads.Element) on one particle."""
    y0 = np.concatenate([np.asarray(z, float), np.asarray(s, float)])
    if e.kind == "snake":
        hp = e.snake_phi / 2.0
        ax = np.array([math.sin(e.snake_mu), 0.0, math.cos(e.snake_mu)])
        S = np.asarray(s, float)
        # Rodrigues' rotation formula
        th = e.snake_phi
        Sr = S * math.cos(th) + np.cross(ax, S) * math.sin(th) + ax * (ax @ S) * (1 - math.cos(th))
        del hp
        return np.asarray(z, float).copy(), Sr
    if e.kind == "marker":
        return np.asarray(z, float).copy(), np.asarray(s, float).copy()
    if e.kind == "thin":
        f = _rhs_thin(e.k1l, e.k2l, z[0], z[2], beam)
        L = 1.0
    else:
        par = {}
        if e.kind == "sbend":
            par = {"h": e.angle / e.L, "eta": e.eta}
            kind = "sbend"
        elif e.kind == "quad":
            par = {"k1": e.k1}
            kind = "quad"
        else:
            kind = "drift"
        f = _rhs_thick(kind, par, beam)
        L = e.L
    sol = solve_ivp(f, (0.0, L), y0, method="DOP853", rtol=rtol, atol=atol)
    y = sol.y[:, -1]
    return y[:6].copy(), y[6:].copy()


def track_line(elements, beam, z, s, **kw):
    z = np.asarray(z, float).copy()
    s = np.asarray(s, float).copy()
    for e in elements:
        z, s = track_element(e, beam, z, s, **kw)
    return z, s


def track_prot(phi, beam, z, rtol=1e-13, atol=1e-16):
    """Flow of H = -X Ps over the frame angle φ (no spin)."""
    b0 = beam.beta0

    def f(t, y):
        X, Px, Y, Py, T, Pt = y
        Ps = math.sqrt(1.0 + 2.0 * Pt / b0 + Pt * Pt - Px * Px - Py * Py)
        return [X * Px / Ps, Ps, X * Py / Ps, 0.0, -X * (1.0 / b0 + Pt) / Ps, 0.0]
    sol = solve_ivp(f, (0.0, phi), np.asarray(z, float), method="DOP853", rtol=rtol, atol=atol)
    return sol.y[:, -1].copy()


def _rhs_rect_dipole(fb, profile, beam):
    """A dipole field b_y = fb f(z) in a Cartesian frame, with the lowest-order
    fringe vector potential of eq. vecArb: a_z = -fb f X, a_x = -fb f' Y²/2,
    so b = (0, fb f, fb f' Y); spin with û from the kinetic momentum."""
    b0 = beam.beta0

    def f(s, y):
        X, Px, Y, Py, T, Pt, Sx, Sy, Sz = y
        F, dF = profile(s)
        ax = -fb * dF * Y * Y / 2.0
        kx = Px - ax
        P2 = 1.0 + 2.0 * Pt / b0 + Pt * Pt
        Ps = math.sqrt(P2 - kx * kx - Py * Py)
        b = np.array([0.0, fb * F, fb * dF * Y])
        u = np.array([kx, Py, Ps]) / math.sqrt(P2)
        gamma = beam.gamma0 * (1.0 + b0 * Pt)
        a1, a2 = 1.0 + beam.G * gamma, beam.G * (gamma - 1.0)
        om = -(1.0 / Ps) * (a1 * b - a2 * float(u @ b) * u)
        dS = np.cross(om, np.array([Sx, Sy, Sz]))
        return [kx / Ps, -fb * F, Py / Ps, -kx * fb * dF * Y / Ps,
                -(1.0 / b0 + Pt) / Ps + 1.0 / b0, 0.0, dS[0], dS[1], dS[2]]
    return f


def track_rbend(L, angle, eta, eps, beam, z, s, rtol=1e-13, atol=1e-16, asym=0.0):
    """Rectangular bend whose faces meet the design orbit at phe = angle/2 +
    asym (entrance) and phx = asym - angle/2 (exit): frame rotation by phe, a
    dipole field rising linearly over [0, eps], flat to L, falling over
    [L, L + eps], X referred to the exit point of the hard-edge design circle
    (radius rho = L/(sin phe - sin phx), exit X = rho (cos phx - cos phe)),
    frame rotation by -phx; spin components turned with each frame rotation;
    T referred to the design arc rho·angle."""
    phe, phx = angle / 2 + asym, asym - angle / 2
    rho = L / (math.sin(phe) - math.sin(phx))
    fb = eta / rho
    zz = track_prot(phe, beam, z, rtol, atol)
    S = np.asarray(s, float)

    def roty(S, a):          # active rotation about ŷ by a
        c, sn = math.cos(a), math.sin(a)
        return np.array([c * S[0] + sn * S[2], S[1], -sn * S[0] + c * S[2]])
    S = roty(S, phe)
    y = np.concatenate([zz, S])
    pieces = [(0.0, eps, lambda t: (t / eps, 1.0 / eps)),
              (eps, L, lambda t: (1.0, 0.0)),
              (L, L + eps, lambda t: ((L + eps - t) / eps, -1.0 / eps))]
    for a, b, prof in pieces:
        sol = solve_ivp(_rhs_rect_dipole(fb, prof, beam), (a, b), y, method="DOP853",
                        rtol=rtol, atol=atol)
        y = sol.y[:, -1]
    y = y.copy()
    y[0] -= rho * (math.cos(phx) - math.cos(phe))
    zz = track_prot(-phx, beam, y[:6], rtol, atol)
    S = roty(y[6:], -phx)
    larc = rho * angle
    zz[4] += (larc - (L + eps)) / beam.beta0
    return zz, S


def _rhs_fringed(h, b1, k1, profile, beam):
    """A dipole b1 = b1/(Bρ)0 (in a frame of curvature h) or a quadrupole
    k1 (h = 0) scaled by a longitudinal profile F(s), from the vector
    potential
        a_x = -b1 F' Y²/2 - (k1/4) F' X Y²,   a_y = (k1/4) F' X² Y,
        (1 + hX) a_s = -b1 F (X + hX²/2) - (k1/2) F (X² - Y²),
    whose curl inside a linear ramp (F'' = 0) is
        b = (k1 F Y, b1 F + k1 F X, b1 F' Y + k1 F' X Y):
    the longitudinal field of the fringe to lowest order.  Hamilton's
    equations of H = -(1 + hX) Ps - (1 + hX) a_s + Pt/β0 with Ps from the
    kinetic momenta (Px - a_x, Py - a_y); the spin precesses about Ω of
    eq. t-bmt.s with û along the kinetic momentum."""
    b0 = beam.beta0
    assert h == 0.0 or k1 == 0.0

    def f(s, y):
        X, Px, Y, Py, T, Pt, Sx, Sy, Sz = y
        F, dF = profile(s)
        w = 1.0 + h * X
        ax = -b1 * dF * Y * Y / 2.0 - 0.25 * k1 * dF * X * Y * Y
        ay = 0.25 * k1 * dF * X * X * Y
        kx, ky = Px - ax, Py - ay
        P2 = 1.0 + 2.0 * Pt / b0 + Pt * Pt
        Ps = math.sqrt(P2 - kx * kx - ky * ky)
        dax_dx, day_dx = -0.25 * k1 * dF * Y * Y, 0.5 * k1 * dF * X * Y
        dax_dy, day_dy = -b1 * dF * Y - 0.5 * k1 * dF * X * Y, 0.25 * k1 * dF * X * X
        dwas_dx = -b1 * F * w - k1 * F * X
        dwas_dy = k1 * F * Y
        b = np.array([k1 * F * Y, b1 * F + k1 * F * X, b1 * dF * Y + k1 * dF * X * Y])
        u = np.array([kx, ky, Ps]) / math.sqrt(P2)
        gamma = beam.gamma0 * (1.0 + b0 * Pt)
        a1, a2 = 1.0 + beam.G * gamma, beam.G * (gamma - 1.0)
        om = -(w / Ps) * (a1 * b - a2 * float(u @ b) * u)
        om[1] += h
        dS = np.cross(om, np.array([Sx, Sy, Sz]))
        return [w * kx / Ps,
                h * Ps + w * (kx * dax_dx + ky * day_dx) / Ps + dwas_dx,
                w * ky / Ps,
                w * (kx * dax_dy + ky * day_dy) / Ps + dwas_dy,
                -w * (1.0 / b0 + Pt) / Ps + 1.0 / b0, 0.0, dS[0], dS[1], dS[2]]
    return f


def track_fringed(e, eps, beam, z, s, rtol=1e-13, atol=1e-16):
    """A sector bend or quadrupole (workloads.Element) whose field rises
    linearly over [-eps/2, eps/2] about the entrance face and falls over
    [L - eps/2, L + eps/2] about the exit face, so the field integral is
    that of the hard-edge magnet.  A bend's curved frame covers [0, L]; the
    outer halves of its ramps lie in straight frames.  Compare with the
    hard-edge magnet between two drifts of eps/2."""
    L = e.L
    if e.kind == "sbend":
        h, b1, k1 = e.angle / L, e.eta * e.angle / L, 0.0
    else:
        h, b1, k1 = 0.0, 0.0, e.k1
    rise = lambda t: ((t + eps / 2) / eps, 1.0 / eps)
    flat = lambda t: (1.0, 0.0)
    fall = lambda t: ((L + eps / 2 - t) / eps, -1.0 / eps)
    pieces = [(-eps / 2, 0.0, 0.0, rise), (0.0, eps / 2, h, rise), (eps / 2, L - eps / 2, h, flat),
              (L - eps / 2, L, h, fall), (L, L + eps / 2, 0.0, fall)]
    y = np.concatenate([np.asarray(z, float), np.asarray(s, float)])
    for a, b, hh, prof in pieces:
        sol = solve_ivp(_rhs_fringed(hh, b1, k1, prof, beam), (a, b), y, method="DOP853",
                        rtol=rtol, atol=atol)
        y = sol.y[:, -1]
    return y[:6].copy(), y[6:].copy()
