"""Pins of the oracle's observables (channel probabilities, cross sections).

* The trapezoidal cross section of P = 1 is pi b_max^2 exactly: the
  integrand P b is linear in b, which the rule integrates exactly, and the
  [0, b_1] interval must be included (dropping it, or the factor 2 pi, fails).
* For P = exp(-b^2) on a uniform b grid the error of the rule is its
  Euler-Maclaurin leading term, 2 pi (h^2 / 12) (f'(b_max) - f'(0)) with
  f = P b: checked to 2% at two spacings (a missing half-weight at either
  end, or a wrong spacing, changes the O(h) or O(h^2) term).
* Channel membership reproduces the state counts of the basis recipe (one
  ground state, the other bound states, the wave-packet bins; on two centres
  the projectile's bound states and bins).
"""
import math

import numpy as np

from oracle import observables as O
from oracle.radial import BasisSpec, build_basis


def test_constant_probability_exact():
    rng = np.random.default_rng(3)
    b = rng.uniform(0.05, 12.0, 37)
    s = O.cross_section(b, np.ones_like(b))
    assert abs(s - math.pi * b.max() ** 2) <= 1e-13 * s


def test_gaussian_euler_maclaurin():
    for n in (200, 400):
        bmax = 8.0
        b = bmax * np.arange(1, n + 1) / n
        h = bmax / n
        br = b[::-1]   # the order of the paths does not matter
        s = O.cross_section(br, np.exp(-br * br))
        exact = math.pi * (1.0 - math.exp(-bmax * bmax))
        fp0, fpe = 1.0, math.exp(-bmax * bmax) * (1.0 - 2.0 * bmax * bmax)
        lead = 2.0 * math.pi * h * h / 12.0 * (fpe - fp0)   # T - I = (h^2/12)(f'(b) - f'(a)) + O(h^4)
        assert abs((s - exact) / lead - 1.0) < 0.02, (n, s - exact, lead)


def test_channel_counts_one_centre():
    bas = build_basis(BasisSpec(n_max=3, l_max=2, n_bins=8, k_max=3.0, n_r=300))
    c = O.channel_probabilities(np.ones(bas.n_states), bas.eps)
    # bound: n = 1 (1 state), n = 2 (1 + 3), n = 3 (1 + 3 + 5); bins: 8 per l and m
    assert c[O.ELASTIC] == 1 and c[O.EXCITATION] == 13 and c[O.TARGET_CONT] == 8 * 9
    assert c[O.CAPTURE] == 0 and c[O.PROJ_CONT] == 0 and c[O.TOTAL] == bas.n_states == 86


def test_channel_counts_two_centre():
    t = build_basis(BasisSpec(n_max=3, l_max=2, n_bins=1, k_max=1.5, n_r=200, r_max=40.0))
    p = build_basis(BasisSpec(n_max=2, l_max=1, n_bins=2, k_max=1.5, n_r=200, r_max=40.0))
    P = np.arange(1, t.n_states + p.n_states + 1, dtype=np.float64)
    c = O.channel_probabilities(np.ones_like(P), t.eps, p.eps)
    assert c[O.ELASTIC] == 1 and c[O.EXCITATION] == 13 and c[O.TARGET_CONT] == 9
    assert c[O.CAPTURE] == 5 and c[O.PROJ_CONT] == 2 * 4 and c[O.TOTAL] == P.size
    w = O.channel_probabilities(P, t.eps, p.eps)
    assert w[O.TOTAL] == P.sum() and np.isclose(w[:5].sum(), P.sum(), rtol=1e-15)
