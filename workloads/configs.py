"""The five synthetic workloads, as plain parameters (no arithmetic).

Each stands in for a workload of the paper's Sycamore experiments (§2,
§5, §A.4), whose circuit files are not available: seeded grid circuits of
the same gate family and pattern sequence, a 64-amplitude batch (6 open
qubits, paper §3), and slicing to a per-slice width the hardware holds.
"""

from __future__ import annotations

from .circuits import block_qubits

# Grid rows x cols, cycles, circuit seed, open block (rows, cols), prefix seed,
# sliced-label count of the planner.
CIRCUIT_CONFIGS = {
    "c1_4x5_m8": dict(rows=4, cols=5, cycles=8, seed=1, dead=(),
                      open_rows=range(0, 2), open_cols=range(2, 5), prefix_seed=1001,
                      n_sliced=0, bitstring_seed=1001, sample_seed=2001),
    "c2_5x6_m14": dict(rows=5, cols=6, cycles=14, seed=2, dead=(),
                       open_rows=range(0, 2), open_cols=range(3, 6), prefix_seed=1002,
                       n_sliced=10, slice_sample_seed=2002, max_branch_rank=12),
}

# 53 qubits (6x9 grid without site (0, 4)), 20 cycles: one slice at the
# full per-slice width, and candidate slicing sets for the runtime models.
# Planner: linear stem order over order_trials seeded trials, greedy slicing
# to max_width, then slicing again with local optimisation over windows of
# local_window tensors; candidates from the randomised greedy slicer
# (uniform among the 3 best picks) with candidate_seed.
C5_53Q_M20 = dict(rows=6, cols=9, cycles=20, seed=5, dead=((0, 4),),
                  open_rows=range(0, 2), open_cols=range(6, 9), prefix_seed=1005,
                  max_width=30, order_trials=256, order_seed=0, local_window=4,
                  candidate_seed=5000, n_candidates=1000)

# Eight 40-qubit circuits (5x8 grid) of uneven width run as one batch: the
# first 512 slices of each.
BATCH_5X8 = dict(rows=5, cols=8, cycles=(10, 11, 12, 13, 14, 10, 12, 14),
                 widths=(20, 21, 22, 23, 24, 21, 22, 24), circuit_seed0=400,
                 prefix_seed0=1400, open_rows=range(0, 2), open_cols=range(5, 8),
                 slices_each=512)

# Isolated stem at its real shape: 2^30 complex64 stem, 40 steps; branch
# shapes and values from workloads.tensors.random_isolated_stem.
ISOLATED_STEM = dict(n_rank=30, n_steps=40, seed=3)


def open_qubits(cfg: dict) -> list[int]:
    return block_qubits(cfg["rows"], cfg["cols"], cfg["open_rows"], cfg["open_cols"],
                        cfg.get("dead", ()))


def circuit_case(cfg: dict, cycles: int | None = None, seed: int | None = None,
                 prefix_seed: int | None = None):
    """(circuit, open qubits, closed {qubit: bit}) of a grid workload."""
    from .circuits import make_circuit
    from .tensors import split_open_prefix

    dead = cfg.get("dead", ())
    circ = make_circuit(cfg["rows"], cfg["cols"], cfg["cycles"] if cycles is None else cycles,
                        cfg["seed"] if seed is None else seed, dead=dead)
    oq = open_qubits(cfg)
    pre = split_open_prefix(circ["n_qubits"], oq,
                            cfg["prefix_seed"] if prefix_seed is None else prefix_seed)
    return circ, oq, dict(zip(pre["closed"], pre["closed_bits"]))
