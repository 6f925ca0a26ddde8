"""Frugal rejection sampling from batches of amplitudes (paper §3).

A batch is the 2^k amplitudes of the k open qubits for one random
assignment (prefix) of the other qubits, computed by one contraction of a
plan whose closed qubits are projected labels; many prefixes go through
one ``stem_contract`` call as its batch entries.  Following the frugal
rejection sampling the paper adopts (Markov et al. 2018), a candidate
bitstring x is accepted with probability min(1, N p(x) / M), N = 2^n, and
the accepted bitstrings follow q(x) proportional to min(p(x), M / N).
Random numbers are drawn by the caller and passed in.

Two readings of "a batch yields a sample": ``all`` keeps every accepted
candidate (correct marginals, samples of one batch share their prefix),
``first`` keeps the first accepted candidate of each batch in a given
random visiting order (at most one sample per prefix).

The XEB of the produced samples, 2^n <|a(x)|^2> - 1 over them, runs on the
GPU in FP64 (``stem_xeb_f64``).
"""

from __future__ import annotations

import numpy as np

from .stem import stem_xeb_f64


def accept(probs: np.ndarray, n_qubits: int, m: float, u: np.ndarray) -> np.ndarray:
    """Acceptance mask of candidates with ideal probabilities ``probs``
    given uniforms ``u`` of the same shape."""
    return u < np.minimum(1.0, (2.0 ** n_qubits) * np.asarray(probs) / m)


def first_accepted(acc: np.ndarray, order: np.ndarray) -> np.ndarray:
    """Per batch (row), the first accepted column in the visiting order
    ``order[b]`` (a permutation of the columns), or -1."""
    out = np.full(acc.shape[0], -1, dtype=np.int64)
    for b in range(acc.shape[0]):
        hit = np.nonzero(acc[b, order[b]])[0]
        if len(hit):
            out[b] = int(order[b][hit[0]])
    return out


def bitstrings(open_qubits, proj_qubits, n_qubits: int, batch_assign, open_index) -> np.ndarray:
    """Integer bitstrings (qubit 0 most significant) of (prefix, open index)
    pairs: projected qubits from the prefix (first projected qubit = most
    significant prefix bit), open qubits from the open index likewise."""
    batch_assign = np.asarray(batch_assign, dtype=np.int64)
    open_index = np.asarray(open_index, dtype=np.int64)
    x = np.zeros(np.broadcast(batch_assign, open_index).shape, dtype=np.int64)
    for j, q in enumerate(proj_qubits):
        bit = (batch_assign >> (len(proj_qubits) - 1 - j)) & 1
        x |= bit << (n_qubits - 1 - q)
    for j, q in enumerate(open_qubits):
        bit = (open_index >> (len(open_qubits) - 1 - j)) & 1
        x |= bit << (n_qubits - 1 - q)
    return x


def sample(plan, n_qubits: int, open_qubits, proj_qubits, prefixes, m: float, rng,
           mode: str = "all", n_slices: int | None = None) -> dict:
    """Contract the batches of ``prefixes`` (projected assignments) with
    ``plan`` and run frugal rejection sampling on them.

    Returns the produced bitstrings, their amplitudes (device complex128),
    the acceptance rate and the FP64 XEB of the produced samples.
    """
    import torch

    prefixes = np.asarray(prefixes, dtype=np.uint64)
    amps = plan.contract(0, n_slices, proj=prefixes)          # [B][2^k] complex128
    probs = np.abs(amps.cpu().numpy()) ** 2
    u = rng.random(probs.shape)
    acc = accept(probs, n_qubits, m, u)
    if mode == "first":
        order = np.argsort(rng.random(probs.shape), axis=1)
        pick = first_accepted(acc, order)
        rows = np.nonzero(pick >= 0)[0]
        cols = pick[rows]
    elif mode == "all":
        rows, cols = np.nonzero(acc)
    else:
        raise ValueError("mode must be 'all' or 'first'")
    out = {"candidates": int(probs.size), "acceptance": float(acc.mean()),
           "bitstrings": bitstrings(open_qubits, proj_qubits, n_qubits,
                                    prefixes[rows].astype(np.int64), cols),
           "n_samples": int(len(rows))}
    if len(rows):
        idx = torch.from_numpy(rows * probs.shape[1] + cols).to(amps.device)
        chosen = amps.reshape(-1)[idx].contiguous()
        out["amplitudes"] = chosen
        out["xeb"] = float(stem_xeb_f64(chosen, n_qubits)[0].item())
    else:
        out["xeb"] = float("nan")
    return out
