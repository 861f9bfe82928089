"""Python face of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It drives the plain complex128 C simulator in ``ref.c`` (built
into ``liboracle.so`` beside it by ``oracle/build.py``) and adds the plain
Python pieces: the Schmidt split of cut CZ gates and the FP64 branch combine.

Passages followed
-----------------
* Section 2 (preliminaries), single-qubit pair rule and CZ sign rule: see
  ``ref.c``.
* Section 2 (preliminaries), CZ decomposition: CU = P0 (x) I + P1 (x) U, so a
  CZ whose two qubits lie on opposite sides of a cut is replaced by the
  projector P_l on the side-A qubit and Z^l on the side-B qubit, one branch
  per l in {0, 1}; Fig. 2: the output is the sum over branches of the tensor
  product of the two half states.
* Section 2.1.1 (Fig. 4 and the 49-qubit remark on the final layer): a cut CZ
  after which neither of its qubits sees a non-diagonal gate is diagonal on
  the output, so it is folded exactly into the output phase (-1)^{x_a x_b}
  instead of doubling the branch count.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import circuit as C

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build
            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.oref_run.argtypes = [dp, ctypes.c_int, ctypes.c_int64, ip, ip, dp]
        L.oref_run.restype = None
        L.oref_norm2.argtypes = [dp, ctypes.c_int64]
        L.oref_norm2.restype = ctypes.c_double
        L.oref_zero_state.argtypes = [dp, ctypes.c_int]
        L.oref_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _encode(gates):
    """Gate list -> (q0, q1, mats) arrays for ``oref_run``."""
    g = len(gates)
    q0 = np.empty(g, np.int32)
    q1 = np.empty(g, np.int32)
    mats = np.zeros((g, 8), np.float64)
    for i, (name, a, b, _layer) in enumerate(gates):
        q0[i] = a
        if name == "CZ":
            q1[i] = b
        else:
            q1[i] = -1
            m = C.gate_matrix(name)
            mats[i] = [m[0][0].real, m[0][0].imag, m[0][1].real, m[0][1].imag,
                       m[1][0].real, m[1][0].imag, m[1][1].real, m[1][1].imag]
    return q0, q1, mats


def zero_state(n: int) -> np.ndarray:
    psi = np.empty(1 << n, np.complex128)
    lib().oref_zero_state(_dptr(psi.view(np.float64)), n)
    return psi


def run(psi: np.ndarray, n: int, gates) -> np.ndarray:
    """Apply ``gates`` in order to ``psi`` (complex128, modified in place)."""
    assert psi.dtype == np.complex128 and psi.size == (1 << n) and psi.flags.c_contiguous
    if not gates:
        return psi
    q0, q1, mats = _encode(gates)
    ip = ctypes.POINTER(ctypes.c_int32)
    lib().oref_run(_dptr(psi.view(np.float64)), n, len(gates),
                   q0.ctypes.data_as(ip), q1.ctypes.data_as(ip), _dptr(mats))
    return psi


def simulate(gates, n: int) -> np.ndarray:
    """psi = U_G ... U_1 |0...0> in complex128 (Task 1: the complete state)."""
    return run(zero_state(n), n, gates)


def norm2(psi: np.ndarray) -> float:
    """Neumaier-compensated sum of |psi_i|^2."""
    a = np.ascontiguousarray(psi, np.complex128)
    return lib().oref_norm2(_dptr(a.view(np.float64)), a.size)


def threads() -> int:
    return lib().oref_threads()


# --- Schmidt split of cut CZ gates ------------------------------------------

def _non_diagonal(name):
    return name not in C.DIAGONAL


def split_circuit(gates, n: int, side_a):
    """Cut the circuit between qubit set ``side_a`` and its complement.

    Returns a dict with
      qa, qb      : sorted global qubit lists of the two halves
      cuts        : crossing CZs that become branches, [(a, b, layer)], a in A
      folded      : crossing CZs folded into the output phase, [(a, b, layer)]
      half(l)     : function of a branch tuple l -> (gates_A, gates_B) in the
                    halves' local qubit numbering
    """
    A = sorted(set(side_a))
    Aset = set(A)
    B = [q for q in range(n) if q not in Aset]
    loc = {q: i for i, q in enumerate(A)}
    loc.update({q: i for i, q in enumerate(B)})
    # A crossing CZ folds iff no non-diagonal gate follows on either qubit.
    last_nd = {}
    for i, g in enumerate(gates):
        if _non_diagonal(g[0]):
            last_nd[g[1]] = i
    items = []  # per gate: ("A", g) / ("B", g) / ("cut", j) / ("fold",)
    cuts, folded = [], []
    for i, (name, q0, q1, layer) in enumerate(gates):
        if name == "CZ" and ((q0 in Aset) != (q1 in Aset)):
            a, b = (q0, q1) if q0 in Aset else (q1, q0)
            if last_nd.get(a, -1) < i and last_nd.get(b, -1) < i:
                folded.append((a, b, layer))
                items.append(("fold",))
            else:
                items.append(("cut", len(cuts)))
                cuts.append((a, b, layer))
        elif q0 in Aset:
            items.append(("A", (name, loc[q0], loc[q1] if q1 >= 0 else -1, layer)))
        else:
            items.append(("B", (name, loc[q0], loc[q1] if q1 >= 0 else -1, layer)))

    def half(l):
        assert len(l) == len(cuts)
        ga, gb = [], []
        for it in items:
            if it[0] == "A":
                ga.append(it[1])
            elif it[0] == "B":
                gb.append(it[1])
            elif it[0] == "cut":
                a, b, layer = cuts[it[1]]
                bit = l[it[1]]
                ga.append(("P1" if bit else "P0", loc[a], -1, layer))
                if bit:
                    gb.append(("Z", loc[b], -1, layer))
        return ga, gb

    return {"qa": A, "qb": B, "cuts": cuts, "folded": folded, "half": half}


def sub_index(x: int, qubits) -> int:
    """Bits of x at the listed qubits, packed in order (bit i <- qubit qubits[i])."""
    v = 0
    for i, q in enumerate(qubits):
        v |= ((x >> q) & 1) << i
    return v


def fold_sign(x: int, folded) -> int:
    s = 1
    for a, b, _ in folded:
        if (x >> a) & 1 and (x >> b) & 1:
            s = -s
    return s


def combine(a_tab, b_tab, signs=None):
    """out[x] = s(x) * sum_l a_tab[l, x] * b_tab[l, x] in FP64.

    Each product is formed in double precision from the stored values and the
    branch sum is exact up to the final rounding (math.fsum), separately for
    the real and imaginary parts.
    """
    a = np.asarray(a_tab)
    b = np.asarray(b_tab)
    nb, m = a.shape
    out = np.empty(m, np.complex128)
    for x in range(m):
        re, im = [], []
        for l in range(nb):
            ar, ai = float(a[l, x].real), float(a[l, x].imag)
            br, bi = float(b[l, x].real), float(b[l, x].imag)
            re.append(ar * br)
            re.append(-(ai * bi))
            im.append(ar * bi)
            im.append(ai * br)
        s = 1.0 if signs is None else float(signs[x])
        out[x] = complex(s * math.fsum(re), s * math.fsum(im))
    return out


def split_amplitudes(gates, n: int, side_a, xs, branches=None):
    """Amplitudes psi[x] of the full circuit through the Schmidt split.

    Runs every half for every branch (or the listed ``branches``) with the
    plain simulator and combines with ``combine``.  Returns (amps, info).
    """
    info = split_circuit(gates, n, side_a)
    c = len(info["cuts"])
    if branches is None:
        branches = range(1 << c)
    nA, nB = len(info["qa"]), len(info["qb"])
    xa = [sub_index(x, info["qa"]) for x in xs]
    xb = [sub_index(x, info["qb"]) for x in xs]
    at, bt = [], []
    for br in branches:
        l = tuple((br >> j) & 1 for j in range(c))
        ga, gb = info["half"](l)
        sa = simulate(ga, nA)
        sb = simulate(gb, nB)
        at.append(sa[xa])
        bt.append(sb[xb])
    signs = [fold_sign(x, info["folded"]) for x in xs]
    return combine(np.array(at), np.array(bt), signs), info
