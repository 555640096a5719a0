"""Analytic maps X = T^{-1} from the computational square (-1,1)^2 onto physical domains.

These are *inputs* to the solver (the method takes the map T as given, paper Sec. 2,
"Setup phase"): each map returns physical coordinates and the exact Jacobian
dX/d(xi,eta) at arbitrary computational points.  No part of the discretisation lives here.

Maps provided
-------------
* identity            : X(xi,eta) = (xi,eta)          (Sec. 4.1, identity-map coefficient problems)
* affine              : X = A (xi,eta)^T + c          (tests)
* quarter_annulus     : inverse of the analytic T of Sec. 4.1 "Quarter annulus"
* star                : R o Phi, Phi the conformal square->disk map, R a radial star
                        deformation with boundary radius 1 + sum_k a_k cos(k theta + phi_k)
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.special as sps

# Half side of the square that the disk is sent to by F(w) = int_0^w dt / sqrt(1 + t^4):
# F(1) = Gamma(1/4)^2 / (8 sqrt(pi)) (a lemniscate constant).
CONFORMAL_A = math.gamma(0.25) ** 2 / (8.0 * math.sqrt(math.pi))


class Map:
    """Base class: ``__call__(xi, eta) -> (x, y)`` and ``jacobian(xi, eta) -> (J11, J12, J21, J22)``
    with J11 = dx/dxi, J12 = dx/deta, J21 = dy/dxi, J22 = dy/deta."""

    name = "map"

    def __call__(self, xi, eta):
        raise NotImplementedError

    def jacobian(self, xi, eta):
        raise NotImplementedError


class Identity(Map):
    name = "identity"

    def __call__(self, xi, eta):
        return np.array(xi, dtype=np.float64, copy=True), np.array(eta, dtype=np.float64, copy=True)

    def jacobian(self, xi, eta):
        o = np.ones(np.broadcast(xi, eta).shape)
        z = np.zeros_like(o)
        return o, z, z, o.copy()


@dataclass
class Affine(Map):
    """X = A @ (xi,eta) + c with det A > 0 (a constant-tensor test map)."""

    A: np.ndarray
    c: np.ndarray = None
    name = "affine"

    def __post_init__(self):
        self.A = np.asarray(self.A, dtype=np.float64)
        self.c = np.zeros(2) if self.c is None else np.asarray(self.c, dtype=np.float64)
        if np.linalg.det(self.A) <= 0:
            raise ValueError("affine map must preserve orientation")

    def __call__(self, xi, eta):
        A, c = self.A, self.c
        return A[0, 0] * xi + A[0, 1] * eta + c[0], A[1, 0] * xi + A[1, 1] * eta + c[1]

    def jacobian(self, xi, eta):
        sh = np.broadcast(xi, eta).shape
        return tuple(np.full(sh, v) for v in (self.A[0, 0], self.A[0, 1], self.A[1, 0], self.A[1, 1]))


class QuarterAnnulus(Map):
    """Inverse of the quarter-annulus map of Sec. 4.1: theta in [pi/2, pi], r in [r2, r1] = [1/2, 1].

    T(x,y) = (2 (|x| - r2)/(r1 - r2) - 1, (4/pi) atan2(y,x) - 3), so
    r = r2 + (xi + 1)(r1 - r2)/2 and theta = pi (eta + 3)/4.
    """

    name = "quarter_annulus"

    def __init__(self, r_inner: float = 0.5, r_outer: float = 1.0):
        self.r2, self.r1 = float(r_inner), float(r_outer)

    def _polar(self, xi, eta):
        r = self.r2 + (np.asarray(xi) + 1.0) * (self.r1 - self.r2) / 2.0
        th = math.pi * (np.asarray(eta) + 3.0) / 4.0
        return r, th

    def __call__(self, xi, eta):
        r, th = self._polar(xi, eta)
        return r * np.cos(th), r * np.sin(th)

    def jacobian(self, xi, eta):
        r, th = self._polar(xi, eta)
        dr = (self.r1 - self.r2) / 2.0
        dth = math.pi / 4.0
        c, s = np.cos(th), np.sin(th)
        return c * dr, -r * s * dth, s * dr, r * c * dth


def _sd_complex(x, y, m=0.5):
    """Jacobi sd = sn/dn at the complex argument x + i y (parameter m), from the real-argument
    values at x (parameter m) and y (complementary parameter 1-m) via Jacobi's imaginary
    transformation and the addition theorem."""
    s, c, d, _ = sps.ellipj(x, m)
    s1, c1, d1, _ = sps.ellipj(y, 1.0 - m)
    delta = c1 * c1 + m * s * s * s1 * s1
    sn = (s * d1 + 1j * c * d * s1 * c1) / delta
    dn = (d * c1 * d1 - 1j * m * s * c * s1) / delta
    return sn / dn


def conformal_square_to_disk(xi, eta):
    """w = F^{-1}(a (xi + i eta)) with F(w) = int_0^w dt/sqrt(1+t^4) and a = F(1).

    F(w) = e^{i pi/4} sl^{-1}(e^{-i pi/4} w) with sl the lemniscate sine, and
    sl(u) = sd(sqrt(2) u | m=1/2)/sqrt(2); hence w = (1+i)/2 * sd((1-i) a z | 1/2).
    Returns (w, dw/dz) with dw/dz = a sqrt(1 + w^4)."""
    xi = np.asarray(xi, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    a = CONFORMAL_A
    w = 0.5 * (1 + 1j) * _sd_complex(a * (xi + eta), a * (eta - xi))
    dw = a * np.sqrt(1.0 + w ** 4)
    return w, dw


class Star(Map):
    """Star-shaped domain X = R o Phi.

    Phi : square -> unit disk is conformal (so it alone contributes an isotropic metric);
    R(w) = (1 + h(w)) w with h(w) = sum_{k=1..K} a_k Re(e^{i phi_k} w^k), whose boundary radius is
    1 + sum_k a_k cos(k theta + phi_k).  With a_k <= 0.05/k the radial derivative of |R| stays
    >= 1 - 0.05 sum_k (1 + 1/k) > 0.46, so R is a diffeomorphism of the closed disk.
    """

    name = "star"

    def __init__(self, amps, phases):
        self.a = np.asarray(amps, dtype=np.float64)
        self.phi = np.asarray(phases, dtype=np.float64)
        self.k = np.arange(1, len(self.a) + 1)

    @classmethod
    def random(cls, rng: np.random.Generator, K: int = 8, amp: float = 0.05):
        k = np.arange(1, K + 1)
        return cls(rng.uniform(0.0, amp / k), rng.uniform(0.0, 2 * math.pi, size=K))

    def boundary_radius(self, theta):
        theta = np.asarray(theta, dtype=np.float64)
        return 1.0 + np.sum(self.a[:, None] * np.cos(self.k[:, None] * theta.ravel()[None, :]
                                                     + self.phi[:, None]), axis=0).reshape(theta.shape)

    def _h(self, w):
        h = np.zeros(w.shape)
        hw = np.zeros(w.shape, dtype=np.complex128)  # dh/dw as a holomorphic-part derivative
        wk = np.ones_like(w)
        for idx in range(len(self.a)):
            k = idx + 1
            e = np.exp(1j * self.phi[idx])
            hw += self.a[idx] * e * k * wk          # d/dw of a e w^k uses w^{k-1}
            wk = wk * w
            h += self.a[idx] * np.real(e * wk)
        return h, hw

    def __call__(self, xi, eta):
        w, _ = conformal_square_to_disk(xi, eta)
        h, _ = self._h(w)
        p = (1.0 + h) * w
        return p.real, p.imag

    def jacobian(self, xi, eta):
        w, dw = conformal_square_to_disk(xi, eta)
        h, hw = self._h(w)
        # h = Re(g(w)) with g holomorphic: dh/dx = Re g', dh/dy = -Im g'
        hx, hy = hw.real, -hw.imag
        u, v = w.real, w.imag
        # J_R = (1+h) I + (u,v)^T grad h
        R11 = 1.0 + h + u * hx
        R12 = u * hy
        R21 = v * hx
        R22 = 1.0 + h + v * hy
        # J_Phi = [[Re f', -Im f'], [Im f', Re f']]
        P11, P12, P21, P22 = dw.real, -dw.imag, dw.imag, dw.real
        return (R11 * P11 + R12 * P21, R11 * P12 + R12 * P22,
                R21 * P11 + R22 * P21, R21 * P12 + R22 * P22)
