"""Exact solution of the 1D Riemann problem for the Euler equations (ideal gas).

Test infrastructure: the textbook construction (two-rarefaction / two-shock pressure function,
Newton iteration for the star pressure, then sampling of the self-similar solution in x/t), as in
E. F. Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4.  Used to pin the
oracle on 1D Riemann problems.
"""
import math

import numpy as np


class ExactRiemann:
    def __init__(self, left, right, gamma=1.4):
        self.g = g = gamma
        self.rl, self.ul, self.pl = left
        self.rr, self.ur, self.pr = right
        self.cl = math.sqrt(g * self.pl / self.rl)
        self.cr = math.sqrt(g * self.pr / self.rr)
        if 2.0 / (g - 1) * (self.cl + self.cr) <= self.ur - self.ul:
            raise ValueError("vacuum is generated")
        self.ps, self.us = self._star()

    def _fk(self, p, rk, pk, ck):
        g = self.g
        if p > pk:
            A = 2.0 / ((g + 1) * rk)
            B = (g - 1) / (g + 1) * pk
            q = math.sqrt(A / (p + B))
            return (p - pk) * q, q * (1 - 0.5 * (p - pk) / (p + B))
        r = p / pk
        f = 2 * ck / (g - 1) * (r ** ((g - 1) / (2 * g)) - 1)
        df = 1.0 / (rk * ck) * r ** (-(g + 1) / (2 * g))
        return f, df

    def _star(self):
        du = self.ur - self.ul
        # two-rarefaction guess
        g = self.g
        z = (g - 1) / (2 * g)
        p = ((self.cl + self.cr - 0.5 * (g - 1) * du) / (self.cl / self.pl ** z + self.cr / self.pr ** z)) ** (1 / z)
        p = max(p, 1e-14)
        for _ in range(100):
            fl, dfl = self._fk(p, self.rl, self.pl, self.cl)
            fr, dfr = self._fk(p, self.rr, self.pr, self.cr)
            pn = p - (fl + fr + du) / (dfl + dfr)
            pn = max(pn, 1e-3 * p)
            if abs(pn - p) <= 1e-15 * 0.5 * (pn + p):
                p = pn
                break
            p = pn
        fl, _ = self._fk(p, self.rl, self.pl, self.cl)
        fr, _ = self._fk(p, self.rr, self.pr, self.cr)
        return p, 0.5 * (self.ul + self.ur) + 0.5 * (fr - fl)

    def sample(self, s):
        """Primitive (rho, u, p) at x/t = s."""
        g, ps, us = self.g, self.ps, self.us
        if s <= us:
            rk, uk, pk, ck, sgn = self.rl, self.ul, self.pl, self.cl, -1.0
        else:
            rk, uk, pk, ck, sgn = self.rr, self.ur, self.pr, self.cr, 1.0
        if ps > pk:  # shock
            S = uk + sgn * ck * math.sqrt((g + 1) / (2 * g) * ps / pk + (g - 1) / (2 * g))
            if (s - S) * sgn >= 0:
                return rk, uk, pk
            r = rk * (ps / pk + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pk + 1)
            return r, us, ps
        # rarefaction
        head = uk + sgn * ck
        cs = ck * (ps / pk) ** ((g - 1) / (2 * g))
        tail = us + sgn * cs
        if (s - head) * sgn >= 0:
            return rk, uk, pk
        if (s - tail) * sgn <= 0:
            return rk * (ps / pk) ** (1 / g), us, ps
        c = 2 / (g + 1) * (ck - sgn * (g - 1) / 2 * (uk - s))
        u = 2 / (g + 1) * (-sgn * ck + (g - 1) / 2 * uk + s)
        return rk * (c / ck) ** (2 / (g - 1)), u, pk * (c / ck) ** (2 * g / (g - 1))

    def cell_averages(self, x0, x1, n, t, xjump, sub=64):
        """Cell averages of the conserved variables on n uniform cells at time t."""
        h = (x1 - x0) / n
        out = np.zeros((n, 3))
        for i in range(n):
            xs = x0 + (i + (np.arange(sub) + 0.5) / sub) * h
            acc = np.zeros(3)
            for x in xs:
                r, u, p = self.sample((x - xjump) / t)
                acc += [r, r * u, p / (self.g - 1) + 0.5 * r * u * u]
            out[i] = acc / sub
        return out
