"""Seeded random-circuit generator for the grid circuit family of paper §2.

A circuit is plain data: a list of moments, each either a layer of named
single-qubit gates (one per qubit) or a layer of qubit pairs that each get an
fSim(theta, phi) gate.  Gate matrices are *not* defined here; each consumer
derives them from the names.

Readings of the paper taken here (the figure that fixes the layout is not
available):

* Grid "RxC" means R rows and C columns; site (r, c) gets qubit index
  r*C + c, renumbered row-major after dead sites are removed.
* Coupler patterns on the grid: A = horizontal pairs (r,c)-(r,c+1) with r+c
  even, B = horizontal with r+c odd, C = vertical (r,c)-(r+1,c) with r+c even,
  D = vertical with r+c odd.  Each pattern is a matching and together they
  cover every coupler exactly once.
* Cycle k (0-based) uses pattern "ABCDCDAB"[k mod 8] (paper §2).
* The first single-qubit layer draws uniformly from {sqrt(X), sqrt(Y),
  sqrt(W)}; every later layer (including the final one before measurement)
  draws uniformly from the two gates different from the one the same qubit
  received in the previous layer (paper §2).
* The per-cycle Z rotations of the device are omitted and every pair uses the
  same (theta, phi); qubits without a partner in a two-qubit layer idle.
"""

from __future__ import annotations

import math

import numpy as np

GATE_1Q_NAMES = ("sqrt_x", "sqrt_y", "sqrt_w")
PATTERN_SEQUENCE = "ABCDCDAB"


def grid_sites(rows: int, cols: int, dead=()):
    """Return (sites, index): live sites in row-major order and site->qubit."""
    dead = {tuple(d) for d in dead}
    sites = [(r, c) for r in range(rows) for c in range(cols) if (r, c) not in dead]
    index = {s: i for i, s in enumerate(sites)}
    return sites, index


def coupler_pattern(rows: int, cols: int, letter: str, dead=()):
    """Qubit pairs of coupler pattern ``letter`` (A, B, C or D) on the grid."""
    _, index = grid_sites(rows, cols, dead)
    pairs = []
    for r in range(rows):
        for c in range(cols):
            parity = (r + c) % 2
            if letter in "AB":
                if parity != (0 if letter == "A" else 1):
                    continue
                other = (r, c + 1)
            elif letter in "CD":
                if parity != (0 if letter == "C" else 1):
                    continue
                other = (r + 1, c)
            else:
                raise ValueError(f"unknown coupler pattern {letter!r}")
            if (r, c) in index and other in index:
                pairs.append((index[(r, c)], index[other]))
    return pairs


def make_circuit(rows: int, cols: int, cycles: int, seed: int, dead=(),
                 theta: float = math.pi / 2, phi: float = math.pi / 6) -> dict:
    """Draw one random circuit of the grid family (paper §2) from ``seed``."""
    sites, _ = grid_sites(rows, cols, dead)
    n = len(sites)
    rng = np.random.Generator(np.random.PCG64(seed))
    moments = []
    prev = None
    for layer in range(cycles + 1):
        if prev is None:
            choice = rng.integers(0, 3, size=n)
        else:
            # pick one of the two gates different from the previous one, in
            # the fixed order of GATE_1Q_NAMES with the previous gate removed
            pick = rng.integers(0, 2, size=n)
            choice = np.array([[g for g in range(3) if g != p][k]
                               for p, k in zip(prev, pick)])
        moments.append({"kind": "1q",
                        "gates": [GATE_1Q_NAMES[int(g)] for g in choice]})
        prev = choice
        if layer < cycles:
            letter = PATTERN_SEQUENCE[layer % len(PATTERN_SEQUENCE)]
            moments.append({"kind": "2q", "pattern": letter,
                            "pairs": [list(p) for p in
                                      coupler_pattern(rows, cols, letter, dead)]})
    return {
        "n_qubits": n,
        "rows": rows,
        "cols": cols,
        "dead": [list(d) for d in dead],
        "cycles": cycles,
        "seed": seed,
        "theta": theta,
        "phi": phi,
        "moments": moments,
    }


def block_qubits(rows: int, cols: int, r_range, c_range, dead=()):
    """Qubit indices of the sites in a rectangular block, ascending."""
    _, index = grid_sites(rows, cols, dead)
    out = [index[(r, c)] for r in r_range for c in c_range if (r, c) in index]
    return sorted(out)
