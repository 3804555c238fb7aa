"""Closed-form volume potentials on the unit cube B_0 = [-1/2,1/2]^3 under
1/(4 pi r), used as references by the volume tests."""
import numpy as np
from scipy.special import erf


def cube_potential(x):
    """(1/4 pi) int_{[-1/2,1/2]^3} dy / |x - y| (closed form of the Newtonian
    potential of a rectangular box: sum over the 8 corners of
    XY ln(Z+R) + YZ ln(X+R) + ZX ln(Y+R) - X^2/2 atan(YZ/(XR)) - ...)."""
    def F(X, Y, Z):
        R = np.sqrt(X * X + Y * Y + Z * Z)

        def lg(a, b, c):
            with np.errstate(divide="ignore", invalid="ignore"):
                v = a * b * np.log(c + R)
            return np.where(np.abs(a * b) > 0, v, 0.0)

        def at(a, b, c):
            with np.errstate(divide="ignore", invalid="ignore"):
                v = 0.5 * a * a * np.arctan(b * c / (a * R))
            return np.where(np.abs(a) > 0, v, 0.0)
        return lg(X, Y, Z) + lg(Y, Z, X) + lg(Z, X, Y) - at(X, Y, Z) - at(Y, Z, X) - at(Z, X, Y)
    s = 0.0
    for i in (0, 1):
        for j in (0, 1):
            for k in (0, 1):
                X = (0.5 if i else -0.5) - x[:, 0]
                Y = (0.5 if j else -0.5) - x[:, 1]
                Z = (0.5 if k else -0.5) - x[:, 2]
                s = s + (-1) ** (3 - i - j - k) * F(X, Y, Z)
    return s / (4 * np.pi)


def gauss_box_potential(x, c, sig):
    """(1/4 pi) int_{[-1/2,1/2]^3} exp(-|y-c|^2/sig^2) / |x-y| dy through
    1/r = (2/sqrt pi) int_0^inf exp(-r^2 t^2) dt: each axis is then a Gaussian
    integral over [-1/2,1/2] in closed form (erf), and the t integral is a
    trapezoidal rule in u = log t on [-30, 30]."""
    u = np.linspace(-30.0, 30.0, 6001)
    t = np.exp(u)
    out = np.zeros(len(x))
    for n in range(len(x)):
        prod = np.ones_like(t)
        for d in range(3):
            a = 1.0 / sig ** 2 + t ** 2
            b = (c[d] / sig ** 2 + x[n, d] * t ** 2) / a
            prod *= (np.exp(-(x[n, d] - c[d]) ** 2 * t ** 2 / (1 + sig ** 2 * t ** 2)) * np.sqrt(np.pi)
                     / (2 * np.sqrt(a)) * (erf(np.sqrt(a) * (0.5 - b)) - erf(np.sqrt(a) * (-0.5 - b))))
        out[n] = np.sum(prod * t) * (u[1] - u[0]) * 2 / np.sqrt(np.pi) / (4 * np.pi)
    return out


def gauss_mixture_potential(x, sig, cen, amp):
    """sum_i a_i (box-restricted Gaussian potential of centre c_i, width s_i)."""
    out = np.zeros(len(x))
    for s, c, a in zip(sig, cen, amp):
        out += a * gauss_box_potential(x, np.asarray(c, dtype=np.float64), float(s))
    return out
