"""Seeded synthetic workloads (inputs only, none of the method's arithmetic).

The paper measures random lattice circuits from the random-circuit
literature; their instance files are not available, so these seeded
synthetic workloads of the same shapes stand in for them:

  4x5-d10    20 qubits, 4x5 lattice, depth 10 (small full-state case)
  5x6-d20    30 qubits, 5x6 lattice, depth 20 (full 2^30 state, 8 GiB)
  6x6m2-d30  34 qubits, 6x6 lattice minus sites (0,0) and (5,5), depth 30
  7x7-d16    49 qubits, 7x7 lattice, depth 16, split after column 3
  5x6-d16    30 qubits, 5x6 lattice, depth 16, split after column 2 (full check)
  uneven     512 circuits, n ~ U{14..26}, depth ~ U{8..24}

Both the GPU path and the CPU oracle take their lattice, depth, seed and the
sampled bitstrings from here; each side builds the circuit with its own
generator.
"""
from __future__ import annotations

import math

import numpy as np

CIRCUIT_SEED_BASE = 0x5EED0000
BITSTRING_SEED_BASE = 0xB1750000

WORKLOADS = {
    "4x5-d10": dict(rows=4, cols=5, absent=(), depth=10, seed=CIRCUIT_SEED_BASE + 1, n=20),
    "5x6-d20": dict(rows=5, cols=6, absent=(), depth=20, seed=CIRCUIT_SEED_BASE + 2, n=30),
    "6x6m2-d30": dict(rows=6, cols=6, absent=((0, 0), (5, 5)), depth=30,
                      seed=CIRCUIT_SEED_BASE + 3, n=34),
    "7x7-d16": dict(rows=7, cols=7, absent=(), depth=16, seed=CIRCUIT_SEED_BASE + 4, n=49),
    # reduced-size split case: cut after column 2 gives 10 cut CZs, 2^10 branch pairs
    "5x6-d16": dict(rows=5, cols=6, absent=(), depth=16, seed=CIRCUIT_SEED_BASE + 6, n=30),
}


def present_mask(spec) -> list:
    """Row-major list of 0/1 site flags of a workload lattice."""
    rows, cols = spec["rows"], spec["cols"]
    m = [[1] * cols for _ in range(rows)]
    for r, c in spec["absent"]:
        m[r][c] = 0
    return [x for row in m for x in row]


def present_grid(spec) -> list:
    rows, cols = spec["rows"], spec["cols"]
    flat = present_mask(spec)
    return [flat[r * cols:(r + 1) * cols] for r in range(rows)]


def bitstrings(n: int, m: int, seed: int) -> np.ndarray:
    """m distinct bitstrings drawn uniformly from [0, 2^n), sorted (uint64)."""
    rng = np.random.default_rng(seed)
    if m > (1 << n):
        raise ValueError("more bitstrings than basis states")
    out = set()
    while len(out) < m:
        k = m - len(out)
        draw = rng.integers(0, 1 << n, size=2 * k, dtype=np.uint64) if n < 64 else None
        for x in draw.tolist():
            out.add(x)
            if len(out) == m:
                break
    return np.array(sorted(out), dtype=np.uint64)


def lattice_for_qubits(n: int):
    """floor(sqrt(n)) rows, ceil(n/rows) columns, first n sites row-major."""
    rows = max(1, math.isqrt(n))
    cols = -(-n // rows)
    present = [1 if i < n else 0 for i in range(rows * cols)]
    return rows, cols, present


def uneven_batch(count: int = 512, seed: int = CIRCUIT_SEED_BASE + 5,
                 n_range=(14, 26), d_range=(8, 24)):
    """(n, depth, circuit seed) for `count` circuits of uneven size."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    ds = rng.integers(d_range[0], d_range[1] + 1, size=count)
    seeds = rng.integers(0, 2 ** 63, size=count, dtype=np.uint64)
    return [(int(a), int(b), int(c)) for a, b, c in zip(ns, ds, seeds)]


def column_cut_mask(rows: int, cols: int, after_col: int) -> int:
    """Qubit mask of the sites in columns 0..after_col of a full lattice."""
    m = 0
    for r in range(rows):
        for c in range(cols):
            if c <= after_col:
                m |= 1 << (r * cols + c)
    return m
