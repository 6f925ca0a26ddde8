"""Seeded random tensors and bitstrings.

Two kinds of randomness live here:

* Small tensors and bitstrings are drawn with numpy's PCG64 generator on the
  host and handed to both sides as data.
* Stems of up to 2^30 entries are too large to draw on the host for every
  test, so their entries come from a counter-based generator that anyone can
  evaluate at any index: SplitMix64 (Steele, Lea and Flood, "Fast splittable
  pseudorandom number generators", OOPSLA 2014).  Each side implements it on
  its own from that definition; entry values are exactly representable in
  float32, so both sides see bit-identical inputs.

Entry recipe for the counter-based stem (complex entry ``i``, seed ``seed``):
words w_j = splitmix64(seed, 4*i + j) for j = 0..3.  Each 64-bit word gives two
22-bit integers (bits 42..63 and bits 10..31).  re = (a0 + a1 + a2 + a3) - 2^23
from the four integers of w0, w1; im likewise from w2, w3.  The value is that
integer times 2^-scale_log2.  The sum of four uniforms is an Irwin-Hall(4)
variable: a bell-shaped, zero-mean stand-in for a Gaussian with variance
4 * (2^44 / 12) per component before scaling.
"""

from __future__ import annotations

import numpy as np

MASK64 = np.uint64(0xFFFFFFFFFFFFFFFF)
SPLITMIX_GAMMA = np.uint64(0x9E3779B97F4A7C15)
SPLITMIX_M1 = np.uint64(0xBF58476D1CE4E5B9)
SPLITMIX_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counter: np.ndarray) -> np.ndarray:
    """SplitMix64 output number ``counter`` (0-based) of the stream ``seed``.

    State after k+1 steps is seed + (k+1)*gamma (mod 2^64); the output is the
    published mixing function of that state.
    """
    with np.errstate(over="ignore"):
        c = np.asarray(counter, dtype=np.uint64)
        z = np.uint64(seed) + (c + np.uint64(1)) * SPLITMIX_GAMMA
        z = (z ^ (z >> np.uint64(30))) * SPLITMIX_M1
        z = (z ^ (z >> np.uint64(27))) * SPLITMIX_M2
        z = z ^ (z >> np.uint64(31))
    return z


def counter_stem_default_scale(rank: int) -> int:
    """Power-of-two exponent that gives the counter stem a norm close to 1.

    Per component the integer sum has variance 4 * 2^44 / 12 = 2^44 / 3, so a
    complex entry has E|z|^2 = 2^45 / 3 ~ 2^43.4.  Unit total norm over 2^rank
    entries needs E|z|^2 * 2^(-2e) = 2^-rank, i.e. e ~ (43.4 + rank) / 2.
    """
    return int(round((43.415 + rank) / 2.0))


def counter_stem_entries(seed: int, index: np.ndarray, scale_log2: int) -> np.ndarray:
    """Complex128 values of the counter-based stem at flat indices ``index``."""
    idx = np.asarray(index, dtype=np.uint64)
    parts = []
    for j in range(4):
        w = splitmix64(seed, idx * np.uint64(4) + np.uint64(j))
        hi = (w >> np.uint64(42)).astype(np.int64)
        lo = ((w >> np.uint64(10)) & np.uint64(0x3FFFFF)).astype(np.int64)
        parts.append(hi + lo)
    re = parts[0] + parts[1] - (1 << 23)
    im = parts[2] + parts[3] - (1 << 23)
    scale = 2.0 ** (-scale_log2)
    return (re.astype(np.float64) * scale) + 1j * (im.astype(np.float64) * scale)


def random_bitstrings(n_bits: int, count: int, seed: int) -> list[int]:
    """``count`` independent uniform ``n_bits``-bit integers (bit 0 = MSB qubit)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        bits = rng.integers(0, 2, size=n_bits)
        v = 0
        for b in bits:
            v = (v << 1) | int(b)
        out.append(v)
    return out


def split_open_prefix(n_qubits: int, open_qubits, seed: int) -> dict:
    """Seeded assignment of the closed qubits for a 2^len(open) amplitude batch.

    Returns {"open": sorted open qubits, "closed": the other qubits ascending,
    "closed_bits": one uniform bit per closed qubit}.
    """
    open_q = sorted(int(q) for q in open_qubits)
    closed = [q for q in range(n_qubits) if q not in set(open_q)]
    rng = np.random.Generator(np.random.PCG64(seed))
    bits = [int(b) for b in rng.integers(0, 2, size=len(closed))]
    return {"open": open_q, "closed": closed, "closed_bits": bits}


def _column_normalised_branch(rng, s: int, f: int) -> np.ndarray:
    """Complex Gaussian [2^s x 2^f] matrix with unit-L2 columns."""
    k, n = 1 << s, 1 << f
    b = rng.standard_normal((k, n)) + 1j * rng.standard_normal((k, n))
    b /= np.linalg.norm(b, axis=0, keepdims=True)
    return b


def random_isolated_stem(n_rank: int, n_steps: int, seed: int, *,
                         lo: int | None = None, hi: int | None = None,
                         s_range=(4, 8), r_range=(6, 14),
                         shared="random") -> dict:
    """Shapes, labels and branch values of an isolated stem chain.

    The stem starts with labels 0..n_rank-1 (C order, label 0 slowest) and
    stays between ``lo`` and ``hi`` address bits (default n_rank-2..n_rank).
    At each step s shared labels are drawn uniformly from s_range, then the
    branch rank r uniformly from the values that keep the next stem between
    lo and hi (and within r_range, with r >= s); an s with no valid r is
    redrawn.  ``shared="random"`` picks a uniform s-subset of the current
    labels; ``shared="fastest"`` takes the s fastest-varying labels.  Branch
    entries are complex Gaussian with every column (fixed free index)
    normalised to unit L2 norm over the shared labels, which keeps the stem's
    per-entry magnitude stationary.

    The initial stem's values are not drawn here: they come from the
    counter-based generator (seed ``seed``, scale
    ``counter_stem_default_scale(n_rank)``).
    """
    lo = n_rank - 2 if lo is None else lo
    hi = n_rank if hi is None else hi
    rng = np.random.Generator(np.random.PCG64(seed))
    labels = list(range(n_rank))
    next_label = n_rank
    steps = []
    for _ in range(n_steps):
        R = len(labels)
        while True:
            s = int(rng.integers(s_range[0], s_range[1] + 1))
            r_lo = max(r_range[0], s, lo - R + 2 * s)
            r_hi = min(r_range[1], hi - R + 2 * s)
            if r_lo <= r_hi and s <= R:
                break
        r = int(rng.integers(r_lo, r_hi + 1))
        if shared == "random":
            pos = sorted(int(p) for p in rng.choice(R, size=s, replace=False))
            shared_labels = [labels[p] for p in pos]
        elif shared == "fastest":
            shared_labels = labels[R - s:]
        else:
            raise ValueError(shared)
        # the shared labels appear in the branch in a random order
        shared_labels = [shared_labels[int(p)] for p in rng.permutation(s)]
        new_labels = list(range(next_label, next_label + (r - s)))
        next_label += r - s
        mat = _column_normalised_branch(rng, s, r - s)
        data = mat.reshape((2,) * r).astype(np.complex64)
        steps.append({"labels": shared_labels + new_labels, "data": data})
        labels = [x for x in labels if x not in set(shared_labels)] + new_labels
    return {
        "stem_labels": list(range(n_rank)),
        "stem_seed": seed,
        "stem_scale_log2": counter_stem_default_scale(n_rank),
        "branches": steps,
        "final_labels": labels,
        "n_labels": next_label,
    }
