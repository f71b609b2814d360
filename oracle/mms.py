"""Manufactured solution and its forcing (oracle).

The paper's forms carry no forcing but note that forcing terms are easily
added (Sec. 2); the workloads here are manufactured solutions built from a
stream function, so the velocity is divergence free and u.n = 0 on the
boundary.  Pressure sign reading: the momentum equation u_t + R (u.grad)u
+ grad(phi) - lap(u) = f is tested as -(phi, div psi) (see assembly), so the
forcing is f = u_t + R (u.grad)u - lap(u) + grad(p) for the exact (u, p).
Derivatives are written out by hand from the product form of each mode.
"""
import numpy as np

PI = np.pi


class MMS:
    def __init__(self, psi_ab, psi_coef, p_ab, p_coef, reynolds):
        self.psi_ab = np.asarray(psi_ab, dtype=float).reshape(-1, 2)
        self.psi_coef = np.asarray(psi_coef, dtype=float).reshape(-1, 3)
        self.p_ab = np.asarray(p_ab, dtype=float).reshape(-1, 2)
        self.p_coef = np.asarray(p_coef, dtype=float).reshape(-1, 3)
        self.R = float(reynolds)

    def _psi_derivs(self, t, x, y):
        """Dict of stream-function derivatives at broadcastable (t, x, y)."""
        t, x, y = np.broadcast_arrays(np.asarray(t, float), np.asarray(x, float),
                                      np.asarray(y, float))
        keys = ["x", "y", "xx", "xy", "yy", "xt", "yt", "xxx", "xxy", "xyy", "yyy"]
        d = {k: np.zeros(t.shape) for k in keys}
        for (a, b), (c, w, th) in zip(self.psi_ab, self.psi_coef):
            A, B = a * PI, b * PI
            sx, cx = np.sin(A * x), np.cos(A * x)
            sy, cy = np.sin(B * y), np.cos(B * y)
            tau, taut = np.cos(w * t + th), -w * np.sin(w * t + th)
            d["x"] += c * A * cx * sy * tau
            d["y"] += c * B * sx * cy * tau
            d["xx"] += -c * A * A * sx * sy * tau
            d["yy"] += -c * B * B * sx * sy * tau
            d["xy"] += c * A * B * cx * cy * tau
            d["xt"] += c * A * cx * sy * taut
            d["yt"] += c * B * sx * cy * taut
            d["xxx"] += -c * A ** 3 * cx * sy * tau
            d["xxy"] += -c * A * A * B * sx * cy * tau
            d["xyy"] += -c * A * B * B * cx * sy * tau
            d["yyy"] += -c * B ** 3 * sx * cy * tau
        return d

    def velocity(self, t, x, y):
        d = self._psi_derivs(t, x, y)
        return d["y"], -d["x"]

    def pressure(self, t, x, y):
        t, x, y = np.broadcast_arrays(np.asarray(t, float), np.asarray(x, float),
                                      np.asarray(y, float))
        p = np.zeros(t.shape)
        for (al, be), (dd, w, th) in zip(self.p_ab, self.p_coef):
            p += dd * np.cos(al * PI * x) * np.cos(be * PI * y) * np.cos(w * t + th)
        return p

    def pressure_grad(self, t, x, y):
        t, x, y = np.broadcast_arrays(np.asarray(t, float), np.asarray(x, float),
                                      np.asarray(y, float))
        px = np.zeros(t.shape)
        py = np.zeros(t.shape)
        for (al, be), (dd, w, th) in zip(self.p_ab, self.p_coef):
            tau = np.cos(w * t + th)
            px += -dd * al * PI * np.sin(al * PI * x) * np.cos(be * PI * y) * tau
            py += -dd * be * PI * np.cos(al * PI * x) * np.sin(be * PI * y) * tau
        return px, py

    def forcing(self, t, x, y):
        d = self._psi_derivs(t, x, y)
        ux, uy = d["y"], -d["x"]
        # velocity gradient: dux/dx = psi_xy, dux/dy = psi_yy, duy/dx = -psi_xx, duy/dy = -psi_xy
        conv_x = ux * d["xy"] + uy * d["yy"]
        conv_y = ux * (-d["xx"]) + uy * (-d["xy"])
        lap_x = d["xxy"] + d["yyy"]
        lap_y = -(d["xxx"] + d["xyy"])
        px, py = self.pressure_grad(t, x, y)
        fx = d["yt"] + self.R * conv_x - lap_x + px
        fy = -d["xt"] + self.R * conv_y - lap_y + py
        return fx, fy


class Chorin:
    """The Chorin test problem (Sec. 2, Definition of the Chorin test problem):
    on the unit square the velocity

        u = (-cos(pi x) sin(pi y), sin(pi x) cos(pi y)) exp(-2 pi^2 t)

    with full Dirichlet data from u, initial value u(0).  Its pressure, in the
    sign convention above (strong form + grad p), is
    p = -(R / 4) (cos(2 pi x) + cos(2 pi y)) exp(-4 pi^2 t): the printed
    pressure carries a factor pi and the opposite sign (the sign is the one
    the printed weak form implies); with this p the pair solves the equations
    with no forcing (u_t = lap u, R (u.grad)u = -grad p), so the forcing is
    zero.  The velocity does not depend on R."""

    def __init__(self, reynolds):
        self.R = float(reynolds)

    @staticmethod
    def _fields(t, x, y):
        t, x, y = np.broadcast_arrays(np.asarray(t, float), np.asarray(x, float),
                                      np.asarray(y, float))
        return t, x, y

    def velocity(self, t, x, y):
        t, x, y = self._fields(t, x, y)
        e = np.exp(-2.0 * PI * PI * t)
        return -np.cos(PI * x) * np.sin(PI * y) * e, np.sin(PI * x) * np.cos(PI * y) * e

    def pressure(self, t, x, y):
        t, x, y = self._fields(t, x, y)
        return -0.25 * self.R * (np.cos(2 * PI * x) + np.cos(2 * PI * y)) * np.exp(-4.0 * PI * PI * t)

    def pressure_grad(self, t, x, y):
        t, x, y = self._fields(t, x, y)
        e = np.exp(-4.0 * PI * PI * t)
        return 0.5 * PI * self.R * np.sin(2 * PI * x) * e, 0.5 * PI * self.R * np.sin(2 * PI * y) * e

    def forcing(self, t, x, y):
        t, x, y = self._fields(t, x, y)
        return np.zeros(t.shape), np.zeros(t.shape)


class Cavity:
    """The lid-driven cavity (Sec. 2, Definition of the lid-driven cavity):
    velocity (1, 0) on the top side of the unit square, zero on the bottom,
    left and right sides, no forcing, zero initial velocity.  Readings: the
    two top corners belong to the no-slip sides (zero), and the lid is at
    speed 1 from the first slab on (the initial value is zero everywhere, the
    lid included).  There is no exact solution; ``velocity`` gives the
    boundary data."""

    def __init__(self, reynolds):
        self.R = float(reynolds)

    def velocity(self, t, x, y):
        t, x, y = np.broadcast_arrays(np.asarray(t, float), np.asarray(x, float),
                                      np.asarray(y, float))
        lid = (y > 1.0 - 1e-12) & (x > 1e-12) & (x < 1.0 - 1e-12)
        return np.where(lid, 1.0, 0.0), np.zeros(t.shape)

    def initial_velocity(self, x, y):
        x = np.asarray(x, float)
        return np.zeros(x.shape), np.zeros(x.shape)

    def forcing(self, t, x, y):
        t, x, y = np.broadcast_arrays(np.asarray(t, float), np.asarray(x, float),
                                      np.asarray(y, float))
        return np.zeros(t.shape), np.zeros(t.shape)


def make_flow(prob):
    """The flow of a problem: the manufactured modes, the Chorin problem
    (prob.flow == 1) or the lid-driven cavity (prob.flow == 2)."""
    flow = getattr(prob, "flow", 0)
    if flow == 1:
        return Chorin(prob.reynolds)
    if flow == 2:
        return Cavity(prob.reynolds)
    return MMS(prob.psi_ab, prob.psi_coef, prob.p_ab, prob.p_coef, prob.reynolds)
