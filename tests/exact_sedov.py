"""Self-similar solution of the point-explosion (Sedov blast-wave) problem, for the checks of the
Sedov runs (the paper compares its 1D run with Sedov's exact solution, Sec. 4.2.2, and runs a 2D
version on an unstructured disk, Sec. 4.3.2).  Test infrastructure only.

A strong shock at r = R(t) runs into gas at rest (density rho0, pressure 0) after the energy E
is released at the origin; geometry j = 1 (planar, the blast at the centre of a line, both sides
counted), 2 (cylindrical), 3 (spherical).  With lam = r/R and

    u = R' f(lam),  rho = rho0 g(lam),  p = rho0 R'^2 h(lam),  R = (E / (alpha rho0))^(1/(j+2)) t^delta,

delta = 2/(j+2), the Euler equations in radial symmetry (continuity, momentum, and constant
entropy p/rho^gamma along particle paths) become, with a = (1 - delta)/delta and D = f - lam,

    D g' + g f' + (j-1) g f / lam = 0
    D f' + h'/g = a f
    D (h'/h - gamma g'/g) = 2 a,

integrated here from the strong-shock (Rankine-Hugoniot) values at lam = 1,
f = h = 2/(gamma+1), g = (gamma+1)/(gamma-1), towards the centre (down to lam = 1e-3; closer in,
the values at that point are used: the density there is below 1e-5 of the undisturbed one).
alpha follows from the energy, E = sigma_j rho0 R'^2 R^j int_0^1 (g f^2/2 + h/(gamma-1)) lam^(j-1) dlam with sigma = 2, 2 pi, 4 pi,
i.e. alpha = sigma_j delta^2 I.

Independent of the ODE system above, the energy inside every sphere lam = const is constant in
time, which gives the algebraic integral (the flux of energy through such a surface vanishes)

    (g f^2/2 + h/(gamma-1)) (f - lam) + h f = 0,

used by the tests as a check on the integration.
"""
import math

import numpy as np
from scipy.integrate import solve_ivp


class Sedov:
    def __init__(self, j, gamma=1.4, E=1.0, rho0=1.0, lam_min=1e-3):
        self.j, self.gamma, self.E, self.rho0 = j, gamma, E, rho0
        g_ = gamma
        self.delta = 2.0 / (j + 2)
        a = (1.0 - self.delta) / self.delta

        def rhs(lam, y):
            f, g, h = y
            D = f - lam
            fp = (a * f * D - (h / g) * (2 * a - g_ * (j - 1) * f / lam)) / (D * D - g_ * h / g)
            gp = -g * (fp + (j - 1) * f / lam) / D
            hp = h * (2 * a / D + g_ * gp / g)
            return [fp, gp, hp]

        y1 = [2.0 / (g_ + 1), (g_ + 1) / (g_ - 1), 2.0 / (g_ + 1)]
        lam = np.concatenate([np.linspace(1.0, 0.05, 2000), np.geomspace(0.05, lam_min, 400)[1:]])
        sol = solve_ivp(rhs, (1.0, lam_min), y1, t_eval=lam, method="DOP853", rtol=1e-11, atol=1e-14)
        assert sol.success, sol.message
        self.lam = sol.t[::-1].copy()
        self.f, self.g, self.h = (v[::-1].copy() for v in sol.y)
        w = self.g * self.f ** 2 / 2 + self.h / (g_ - 1)
        integrand = w * self.lam ** (j - 1)
        # below lam_min the integrand is taken constant times lam^(j-1) (the pressure tends to a
        # constant at the centre, the density to zero); the ODEs are singular there
        I = np.trapezoid(integrand, self.lam) + w[0] * self.lam[0] ** j / j
        sigma = {1: 2.0, 2: 2.0 * math.pi, 3: 4.0 * math.pi}[j]
        self.alpha = sigma * self.delta ** 2 * I

    def radius(self, t):
        return (self.E / (self.alpha * self.rho0)) ** (1.0 / (self.j + 2)) * t ** self.delta

    def energy_integral_residual(self):
        """max over lam of |(g f^2/2 + h/(gamma-1)) (f - lam) + h f|, relative to the shock values."""
        f, g, h, lam = self.f, self.g, self.h, self.lam
        r = (g * f ** 2 / 2 + h / (self.gamma - 1)) * (f - lam) + h * f
        return float(np.abs(r).max() / (2.0 / (self.gamma + 1)) ** 2)

    def state(self, r, t):
        """(rho, u, p) at distances r >= 0 from the centre at time t > 0 (u radial, outwards)."""
        r = np.abs(np.asarray(r, dtype=np.float64))
        R = self.radius(t)
        Rd = self.delta * R / t
        lam = r / R
        inside = lam < 1.0
        li = np.clip(lam, self.lam[0], 1.0)
        rho = np.where(inside, self.rho0 * np.interp(li, self.lam, self.g), self.rho0)
        u = np.where(inside, Rd * np.interp(li, self.lam, self.f), 0.0)
        p = np.where(inside, self.rho0 * Rd ** 2 * np.interp(li, self.lam, self.h), 0.0)
        return rho, u, p
