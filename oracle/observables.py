"""Observables at the end of the paths: channel probabilities and cross sections.

Test infrastructure only (see ``oracle/__init__.py``).

Paper anchors
-------------
* Sec. II, after Algorithm 1: the solution vector at z_max gives the
  observables (cross sections of the reaction processes), and a collision
  calculation runs 30 to 50 paths at different impact parameters.
* Sec. III: a one-centre expansion gives only the total electron loss; the
  two-centre expansion separates electron capture from ionisation.

Readings (the paper names these observables but does not write them out)
------------------------------------------------------------------------
* P_i = |X_i|^2 of every state at the last grid point.
* Channels by the centre a state is expanded about and the sign of its
  energy (bound eigenstates have eps < 0, wave-packet pseudostates eps > 0):
    ELASTIC      the target ground state (state 0)
    EXCITATION   the other target states with eps < 0
    TARGET_CONT  target states with eps > 0 (target continuum)
    CAPTURE      projectile states with eps < 0 (two-centre only)
    PROJ_CONT    projectile states with eps > 0 (two-centre only)
    TOTAL        every state
  Ionisation (two-centre) is TARGET_CONT + PROJ_CONT; electron loss
  (one-centre) is TARGET_CONT.
* Cross section of a channel: sigma = 2 pi int_0^inf P(b) b db, by the
  trapezoidal rule in b over the sorted impact parameters of one batch
  (paths with the same basis and speed); the interval [0, b_1] uses the
  integrand's value 0 at b = 0, and nothing is added beyond the largest b.
"""
from __future__ import annotations

import math

import numpy as np

ELASTIC, EXCITATION, TARGET_CONT, CAPTURE, PROJ_CONT, TOTAL = range(6)
N_CHANNELS = 6


def channel_of_states(eps_target: np.ndarray, eps_projectile: np.ndarray | None = None) -> np.ndarray:
    """Channel index of every state (target states first, then projectile states)."""
    t = np.where(np.asarray(eps_target) < 0.0, EXCITATION, TARGET_CONT)
    t[0] = ELASTIC
    if eps_projectile is None:
        return t
    p = np.where(np.asarray(eps_projectile) < 0.0, CAPTURE, PROJ_CONT)
    return np.concatenate([t, p])


def channel_probabilities(P: np.ndarray, eps_target: np.ndarray,
                          eps_projectile: np.ndarray | None = None) -> np.ndarray:
    """Sum of P_i over the states of each channel, and the total: [N_CHANNELS]."""
    ch = channel_of_states(eps_target, eps_projectile)
    out = np.zeros(N_CHANNELS)
    for i, p in enumerate(np.asarray(P, dtype=np.float64)):
        out[ch[i]] += p
        out[TOTAL] += p
    return out


def cross_section(b: np.ndarray, P: np.ndarray) -> float:
    """2 pi int_0^inf P(b) b db by the trapezoidal rule over the sorted b
    (integrand 0 at b = 0, nothing beyond the largest b)."""
    order = np.argsort(b, kind="stable")
    bs = np.concatenate([[0.0], np.asarray(b, dtype=np.float64)[order]])
    f = np.concatenate([[0.0], np.asarray(P, dtype=np.float64)[order] * bs[1:]])
    total = 0.0
    for i in range(bs.size - 1):
        total += 0.5 * (bs[i + 1] - bs[i]) * (f[i] + f[i + 1])
    return 2.0 * math.pi * total
