"""Closed-form elliptic measures used to pin the oracle (K = I special cases).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

* Disk: the Poisson kernel quoted in the introduction (harmonic measure of the unit ball,
  density (1-|x|^2)/(sigma(dB)|x-y|^d)), integrated in closed form over arcs.
* Ball: the same kernel in 3D, integrated in closed form over zonal bands for poles on the axis.
* Annulus: the series representation mentioned next to it in the introduction, obtained by
  separation of variables (Fourier modes r^n, r^-n, log r).
"""
from __future__ import annotations

import numpy as np


def _F(t, rho):
    """Antiderivative in the angle of the unit-disk Poisson kernel (1-rho^2)/(2pi(1-2rho cos t+rho^2)),
    normalised so that F(-pi) = -1/2, F(pi) = 1/2 (t in [-pi, pi])."""
    c = (1.0 + rho) / (1.0 - rho)
    return np.arctan2(c * np.sin(t / 2), np.cos(t / 2)) / np.pi


def disk_arc_measure(x, R, th1, th2):
    """mu_x(arc [th1, th2]) for the disk of radius R centred at 0 (0 <= th2 - th1 <= 2 pi)."""
    x = np.asarray(x, float) / R
    rho = np.hypot(x[0], x[1])
    phi = np.arctan2(x[1], x[0])
    t1 = np.mod(th1 - phi + np.pi, 2 * np.pi) - np.pi
    t2 = t1 + (th2 - th1)
    if t2 <= np.pi:
        return float(_F(t2, rho) - _F(t1, rho))
    return float((0.5 - _F(t1, rho)) + (_F(t2 - 2 * np.pi, rho) + 0.5))


def disk_H(x_obs, R, M):
    """Exact H[i, j] = mu_{x_i}(arc j) for M equal arcs counted counter-clockwise from angle 0."""
    H = np.zeros((len(x_obs), M))
    for i, x in enumerate(x_obs):
        for j in range(M):
            H[i, j] = disk_arc_measure(x, R, 2 * np.pi * j / M, 2 * np.pi * (j + 1) / M)
    return H


def disk_density(x, y, R=1.0):
    """Poisson kernel density d mu_x / d sigma at y on the circle of radius R (introduction)."""
    x, y = np.asarray(x, float), np.asarray(y, float)
    return (R * R - x @ x) / (2 * np.pi * R * np.sum((x - y) ** 2))


def ball_band_above(a, c):
    """mu_x({z >= c}) on the unit sphere for the pole x = (0, 0, a), 0 <= a < 1."""
    if a == 0.0:
        return (1.0 - c) / 2.0
    return ((1 - a * a) / (2 * a)) * (1.0 / (1.0 - a) - 1.0 / np.sqrt(1 - 2 * a * c + a * a))


def ball_density(x, y):
    """Poisson kernel of the unit ball in 3D: (1 - |x|^2) / (4 pi |x - y|^3)."""
    x, y = np.asarray(x, float), np.asarray(y, float)
    return (1 - x @ x) / (4 * np.pi * np.sum((x - y) ** 2) ** 1.5)


def ball_cells_axis(a, nz, nphi):
    """mu_x of the equal-area (z, phi) cells (band iz counted from z = 1) for x = (0, 0, a):
    the band measure split evenly over the nphi sectors by rotational symmetry."""
    edges = 1 - 2 * np.arange(nz + 1) / nz
    above = np.array([ball_band_above(a, c) for c in edges])
    band = above[1:] - above[:-1]
    return np.repeat(band / nphi, nphi)


def annulus_inner_mass(rho, r_in, r_out):
    """Total harmonic measure of the inner circle from radius rho (K = I)."""
    return np.log(r_out / rho) / np.log(r_out / r_in)


def annulus_arc_measures(x, r_in, r_out, m_out, m_in, tol=1e-18, n_max=100000):
    """mu_x of the m_out outer arcs then the m_in inner arcs of the concentric annulus (K = I).

    Density in the angle (separation of variables):
      outer: (1/2pi) [ log(rho/r_in)/log(r_out/r_in)
                       + sum_n 2 cos n(th-phi) (rho^n - r_in^2n rho^-n)/(r_out^n - r_in^2n r_out^-n) ]
      inner: (1/2pi) [ log(r_out/rho)/log(r_out/r_in)
                       + sum_n 2 cos n(th-phi) (r_out^2n rho^-n - rho^n)/(r_out^2n r_in^-n - r_in^n) ]
    Arc integrals of cos n(th - phi) are taken exactly."""
    x = np.asarray(x, float)
    rho = np.hypot(x[0], x[1])
    phi = np.arctan2(x[1], x[0])
    L = np.log(r_out / r_in)
    out = []
    for m, outer in ((m_out, True), (m_in, False)):
        e = 2 * np.pi * np.arange(m + 1) / m
        mass = np.full(m, (np.log(rho / r_in) if outer else np.log(r_out / rho)) / L / m)
        n = 1
        while n < n_max:
            if outer:
                coef = (rho ** n - r_in ** (2 * n) * rho ** -n) / (r_out ** n - r_in ** (2 * n) * r_out ** -n)
            else:
                lr = n * np.log(r_in / rho)
                coef = (np.exp(lr) - np.exp(n * np.log(r_in * rho / r_out ** 2))) / (1 - (r_in / r_out) ** (2 * n))
            sinv = np.sin(n * (e - phi))
            mass += coef * (sinv[1:] - sinv[:-1]) / (n * np.pi)
            if abs(coef) < tol:
                break
            n += 1
        out.append(mass)
    return np.concatenate(out)
