"""Statistics on amplitudes: XEB, Porter-Thomas check, relative L2 error.

* ``xeb``: linear cross-entropy fidelity 2^n <p_I(x)> - 1 over the given
  bitstrings' ideal probabilities (paper §2).
* ``collision_xeb``: the same expectation taken exactly over the ideal
  distribution itself, 2^n sum_x p(x)^2 - 1; it is 1 for an exact
  Porter-Thomas distribution (paper §2 XEB of the ideal output).
* ``porter_thomas_ks``: Kolmogorov-Smirnov distance between the values N p
  and the unit exponential law, whose density e^{-x} is the Porter-Thomas
  form N e^{-Np} written for x = N p (paper §A.4).
* ``rel_l2``: ||a - ref||_2 / ||ref||_2 over a whole vector.
* ``frugal_acceptance`` / ``frugal_xeb``: frugal rejection sampling (paper
  §3, after Markov et al. 2018) accepts a candidate bitstring x, drawn
  uniformly, with probability min(1, N p(x) / M); the accepted ones follow
  q(x) proportional to min(p(x), M / N).  These give, from the ideal
  probabilities of every bitstring, the acceptance probability of one
  candidate, sum_x min(1, N p / M) / N, and the XEB of the accepted
  samples, N sum_x q(x) p(x) - 1.

Pins (tests/test_oracle_misc.py, test_oracle_statevector.py): uniform
probabilities give XEB 0 and exact exponential quantiles give KS distance
~0; a two-point distribution with hand-computed XEB; the 20-qubit random
circuit gives collision XEB within a statistical window of 1; the frugal
XEB tends to the collision XEB as M grows and is 0 when M is below every
N p (uniform acceptance), with a hand-computed two-point case.
"""

from __future__ import annotations

import math

import numpy as np


def xeb(amps, n_qubits: int) -> float:
    p = np.abs(np.asarray(amps, dtype=np.complex128)) ** 2
    return float((2.0 ** n_qubits) * p.mean() - 1.0)


def collision_xeb(amps_all, n_qubits: int) -> float:
    p = np.abs(np.asarray(amps_all, dtype=np.complex128)) ** 2
    return float((2.0 ** n_qubits) * np.sum(p * p) - 1.0)


def frugal_acceptance(probs_all, m: float) -> float:
    p = np.asarray(probs_all, dtype=np.float64)
    n = p.size
    return float(np.minimum(1.0, n * p / m).mean())


def frugal_xeb(probs_all, m: float) -> float:
    p = np.asarray(probs_all, dtype=np.float64)
    n = p.size
    q = np.minimum(p, m / n)
    return float(n * np.sum(q * p) / np.sum(q) - 1.0)


def porter_thomas_ks(probs, n_states: int) -> float:
    x = np.sort(np.asarray(probs, dtype=np.float64) * n_states)
    m = len(x)
    cdf = 1.0 - np.exp(-x)
    upper = np.arange(1, m + 1) / m - cdf
    lower = cdf - np.arange(0, m) / m
    return float(max(upper.max(), lower.max()))


def rel_l2(a, ref) -> float:
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    ref = np.asarray(ref, dtype=np.complex128).reshape(-1)
    den = math.sqrt(float(np.sum(np.abs(ref) ** 2)))
    num = math.sqrt(float(np.sum(np.abs(a - ref) ** 2)))
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return num / den


def cancellation(per_slice) -> np.ndarray:
    """kappa[b] = sum_s |T_s[b]| / |sum_s T_s[b]| for a [slices, entries] array."""
    t = np.asarray(per_slice, dtype=np.complex128)
    return np.abs(t).sum(axis=0) / np.maximum(np.abs(t.sum(axis=0)), 1e-300)
