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
                       n_sliced=10, slice_sample_seed=2002),
}

# Isolated stem at its real shape: 2^30 complex64 stem, 40 steps; branch
# shapes and values from workloads.tensors.random_isolated_stem.
ISOLATED_STEM = dict(n_rank=30, n_steps=40, seed=3)


def open_qubits(cfg: dict) -> list[int]:
    return block_qubits(cfg["rows"], cfg["cols"], cfg["open_rows"], cfg["open_cols"],
                        cfg.get("dead", ()))
