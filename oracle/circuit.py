"""Oracle-side random lattice circuit generator (test infrastructure only).

This module is part of the CPU oracle.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path has
its own generator written in C++ and the two are compared gate by gate.

What it follows
---------------
* Section 2 (preliminaries): the universal random circuit family lives on a
  2D grid, uses the gates H, X^1/2, Y^1/2, T and CZ, CZ only between lattice
  neighbours and at positions that are fixed per layer; the single-qubit gates
  are random.
* Section 1, footnote on depth: the opening layer of Hadamards is "layer 0"
  and is not counted in the depth; depth d means layers 1..d after it.
* Section 2.1.2 (the 49-qubit partition discussion) and Table "28qubit" fix
  the concrete rule set through the printed numbers (see the readings below).

Readings taken where the paper defers to an uncited source
----------------------------------------------------------
R3  qubit q = row-major rank of lattice site (r, c) among the present sites.
R4  eight CZ pattern classes on a rows x cols grid:
      Hab: horizontal bonds (r,c)-(r,c+1) with c = a and r = b (mod 2)
      Vab: vertical bonds   (r,c)-(r+1,c) with r = a and c = b (mod 2)
    bonds touching an absent site are dropped.
R5  layer t >= 1 uses ORDER[(t-1) mod 8] with
      ORDER = H00, H01, V10, V11, H10, V01, V00, H11.
    This order reproduces the gate counts of Table "28qubit" (4x7 lattice),
    the 3 + 4 cut CZs behind f(7)=24 and f(8)=28 of Section 2.1.2 and the
    remark that qubits 0, 2, 4, 6 carry single-qubit gates at layer 40.
R6  at layer t >= 1 qubit q receives a single-qubit gate iff q took part in a
    CZ at layer t-1 and takes part in none at layer t (CZ(0) is empty, so
    layer 1 holds CZs only).  Within a layer the CZs come first (sorted by
    their smaller then larger qubit), then the single-qubit gates in
    increasing q.
R7  the single-qubit gate type is drawn i.i.d. uniform over {T, SX, SY}
    (this is what the probability 1-(2/3)^4 = 65/81 of the "lucky circuit"
    remark assumes).  Draws come from SplitMix64 (Steele, Lea and Flood,
    OOPSLA 2014): one 64-bit output r per gate, in gate order, type index
    floor((r >> 32) * 3 / 2^32) mapped 0 -> T, 1 -> SX, 2 -> SY.
R16 "6x6 minus two corner sites" removes sites (0,0) and (5,5).
R17 an arbitrary qubit count n uses R = floor(sqrt(n)) rows,
    C = ceil(n / R) columns, and keeps the first n sites in row-major order.
"""
from __future__ import annotations

import math

MASK64 = (1 << 64) - 1

# Gate names used throughout the oracle.  Single-qubit: H T SX SY Z P0 P1 TDG
# SXDG SYDG; two-qubit: CZ.
ONE_QUBIT = ("H", "T", "SX", "SY", "Z", "P0", "P1", "TDG", "SXDG", "SYDG")
DIAGONAL = ("T", "Z", "P0", "P1", "TDG", "CZ")

ORDER = (("H", 0, 0), ("H", 0, 1), ("V", 1, 0), ("V", 1, 1),
         ("H", 1, 0), ("V", 0, 1), ("V", 0, 0), ("H", 1, 1))


class SplitMix64:
    """SplitMix64 as published by Steele, Lea and Flood (2014)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)


class Lattice:
    """rows x cols grid with a presence mask; qubit = row-major rank (R3)."""

    def __init__(self, rows: int, cols: int, present=None):
        self.rows, self.cols = rows, cols
        if present is None:
            present = [[True] * cols for _ in range(rows)]
        self.present = [[bool(present[r][c]) for c in range(cols)] for r in range(rows)]
        self.qubit = {}
        q = 0
        for r in range(rows):
            for c in range(cols):
                if self.present[r][c]:
                    self.qubit[(r, c)] = q
                    q += 1
        self.n = q

    @staticmethod
    def for_qubits(n: int) -> "Lattice":
        """R17: floor(sqrt(n)) rows, first n sites in row-major order."""
        rows = max(1, math.isqrt(n))
        cols = -(-n // rows)
        pres = [[r * cols + c < n for c in range(cols)] for r in range(rows)]
        return Lattice(rows, cols, pres)

    def pattern(self, cls) -> list:
        """CZ pairs (q0 < q1) of one pattern class (R4), sorted."""
        orient, a, b = cls
        out = []
        for r in range(self.rows):
            for c in range(self.cols):
                if orient == "H":
                    if c % 2 != a or r % 2 != b or c + 1 >= self.cols:
                        continue
                    s0, s1 = (r, c), (r, c + 1)
                else:
                    if r % 2 != a or c % 2 != b or r + 1 >= self.rows:
                        continue
                    s0, s1 = (r, c), (r + 1, c)
                if s0 in self.qubit and s1 in self.qubit:
                    q0, q1 = self.qubit[s0], self.qubit[s1]
                    out.append((min(q0, q1), max(q0, q1)))
        return sorted(out)


def layer_pattern(t: int):
    """Pattern class of layer t >= 1 (R5)."""
    return ORDER[(t - 1) % 8]


def random_circuit(lattice: Lattice, depth: int, seed: int) -> list:
    """Gate list [(name, q0, q1, layer)] for a lattice circuit of the given depth.

    Layer 0 is H on every qubit; layers 1..depth follow R4-R7.  q1 is -1 for
    single-qubit gates.
    """
    rng = SplitMix64(seed)
    gates = [("H", q, -1, 0) for q in range(lattice.n)]
    prev = set()
    for t in range(1, depth + 1):
        pairs = lattice.pattern(layer_pattern(t))
        cur = set()
        for q0, q1 in pairs:
            gates.append(("CZ", q0, q1, t))
            cur.update((q0, q1))
        for q in range(lattice.n):
            if q in prev and q not in cur:
                r = rng.next()
                k = ((r >> 32) * 3) >> 32
                gates.append((("T", "SX", "SY")[k], q, -1, t))
        prev = cur
    return gates


def gate_count_excluding_layer0(gates) -> int:
    return sum(1 for g in gates if g[3] > 0)


# --- gate matrices ------------------------------------------------------------
# Reading R1: the paper names the gates but prints no matrices.  Standard
# definitions: H = [[1,1],[1,-1]]/sqrt2; T = diag(1, e^{i pi/4});
# X^1/2 and Y^1/2 are the principal square roots of X and Y,
# sqrt(X) = [[1+i, 1-i], [1-i, 1+i]]/2, sqrt(Y) = [[1+i, -1-i], [1+i, 1+i]]/2.
# Entries are (row, col) with row/col = value of the acted-on bit.

def gate_matrix(name: str):
    """2x2 complex matrix [[a, b], [c, d]] of a single-qubit gate, as Python complex."""
    s = 1.0 / math.sqrt(2.0)
    w = complex(math.cos(math.pi / 4), math.sin(math.pi / 4))
    m = {
        "H": [[s, s], [s, -s]],
        "T": [[1, 0], [0, w]],
        "TDG": [[1, 0], [0, w.conjugate()]],
        "SX": [[0.5 + 0.5j, 0.5 - 0.5j], [0.5 - 0.5j, 0.5 + 0.5j]],
        "SY": [[0.5 + 0.5j, -0.5 - 0.5j], [0.5 + 0.5j, 0.5 + 0.5j]],
        "Z": [[1, 0], [0, -1]],
        "P0": [[1, 0], [0, 0]],
        "P1": [[0, 0], [0, 1]],
    }
    if name in m:
        return [[complex(x) for x in row] for row in m[name]]
    if name in ("SXDG", "SYDG"):
        a = gate_matrix(name[:2])
        return [[a[0][0].conjugate(), a[1][0].conjugate()],
                [a[0][1].conjugate(), a[1][1].conjugate()]]
    raise ValueError(f"unknown single-qubit gate {name}")


def inverse_circuit(gates) -> list:
    """Adjoint circuit: reversed order, each gate replaced by its adjoint."""
    inv = {"H": "H", "T": "TDG", "TDG": "T", "SX": "SXDG", "SXDG": "SX",
           "SY": "SYDG", "SYDG": "SY", "Z": "Z", "CZ": "CZ"}
    return [(inv[g[0]], g[1], g[2], g[3]) for g in reversed(gates)]


# --- Named workloads ----------------------------------------------------------

def config_lattice(name: str) -> Lattice:
    if name == "4x5":
        return Lattice(4, 5)
    if name == "5x6":
        return Lattice(5, 6)
    if name == "6x6-2":
        pres = [[True] * 6 for _ in range(6)]
        pres[0][0] = False
        pres[5][5] = False
        return Lattice(6, 6, pres)
    if name == "7x7":
        return Lattice(7, 7)
    raise ValueError(name)
