"""Pins for oracle.special: the Green's function and the self-cell integral.

Each value is fixed by something other than the oracle itself: published Bessel
values (Abramowitz & Stegun tables), the Wronskian identity, mpmath's
independent arbitrary-precision Hankel function, and direct 2-D quadrature of the
singular cell integral.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy import integrate
from scipy.special import hankel1

from oracle import special

EULER = 0.5772156649015329


def test_green_published_values():
    # G(r) * 4 / i = H0(kappa r); at kappa r = 1: J0(1) + i Y0(1) (A&S Table 9.1)
    g = special.green(0.1, 10.0)
    h0 = g * 4 / 1j
    assert abs(h0.real - 0.7651976865579666) < 1e-15
    assert abs(h0.imag - 0.08825696421567696) < 1e-15


def test_green_first_zeros():
    # first zeros of J0 and Y0 (A&S Table 9.5)
    assert abs(hankel1(0, 2.404825557695773).real) < 1e-15
    assert abs(special.green(0.8935769662791675, 1.0).real) < 1e-15   # Re G = -Y0/4


def test_green_wronskian():
    z = np.linspace(0.05, 200.0, 777)
    j0, y0 = hankel1(0, z).real, hankel1(0, z).imag
    j1, y1 = hankel1(1, z).real, hankel1(1, z).imag
    assert np.max(np.abs((j1 * y0 - j0 * y1) * z * math.pi / 2 - 1.0)) < 1e-12


def test_green_small_argument_limit():
    z = 1e-6
    g = special.green(z, 1.0)
    # Y0(z) ~ (2/pi)(ln(z/2) + gamma) as z -> 0, J0 -> 1
    assert abs(g.imag - 0.25) < 1e-12
    assert abs(-4 * g.real - (2 / math.pi) * (math.log(z / 2) + EULER)) < 1e-10


@pytest.mark.parametrize("z", [0.3, 2.0, 7.1, 13.7, 31.0, 226.0])
def test_green_against_mpmath(z):
    ref = complex(mpmath.hankel1(0, z)) * 0.25j
    got = special.green(z, 1.0)
    assert abs(got - ref) <= 2e-15 * abs(ref)


@pytest.mark.parametrize("h,kappa", [(1 / 16, 10.0), (2 / 256, 40.0), (2 / 512, 80.0), (0.2, 3.0)])
def test_self_cell_vs_2d_quadrature(h, kappa):
    w = special.self_cell(h, kappa)

    def part(fn):
        val, _ = integrate.dblquad(lambda y, x: fn(0.25j * hankel1(0, kappa * math.hypot(x, y))),
                                   0.0, h / 2, 0.0, h / 2, epsabs=1e-17, epsrel=1e-13)
        return 4.0 * val

    ref = part(np.real) + 1j * part(np.imag)
    assert abs(w - ref) <= 1e-13 * abs(ref)


def test_self_cell_small_cell_expansion():
    # For kappa h -> 0, (i/4) H0(kappa r) ~ i/4 - (1/(2 pi)) (ln(kappa r / 2) + gamma);
    # int over the square of ln|y| is h^2 (ln(h/2) + (ln 2)/2 + pi/4 - 3/2)... evaluated numerically here.
    h, kappa = 1e-3, 1.0
    w = special.self_cell(h, kappa)
    lnint, _ = integrate.dblquad(lambda y, x: math.log(math.hypot(x, y)), 0, h / 2, 0, h / 2,
                                 epsabs=1e-20, epsrel=1e-12)
    lnint *= 4
    approx = 0.25j * h * h - (1 / (2 * math.pi)) * (lnint + h * h * (math.log(kappa / 2) + EULER))
    assert abs(w - approx) <= 1e-6 * abs(w)
