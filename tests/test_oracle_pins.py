"""Pins for the CPU oracle: checks against what the paper and mathematics fix.

Each test pins the oracle (generator, simulator, split/combine) to something
other than itself: numbers printed in the paper, a known-answer vector of a
published generator, dense Kronecker-product brute force, closed forms,
invariants, and exact identities.
"""
import cmath
import itertools
import math
import random

import numpy as np
import pytest

from oracle import circuit as C
from oracle import sim

# ----------------------------------------------------------------------------
# Generator pins
# ----------------------------------------------------------------------------


def test_splitmix64_known_answer():
    # Reference outputs of SplitMix64 (Steele, Lea, Flood 2014) from state 0.
    r = C.SplitMix64(0)
    assert [r.next() for _ in range(3)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


@pytest.mark.parametrize("seed", [0, 1, 0x5EED0000])
def test_table_28qubit_gate_counts(seed):
    # Table "28qubit": 28-qubit circuits, gates (layer 0 not counted) at
    # depths 18/26/34/42/50 are 258/375/492/609/726.  4 x 7 lattice.
    lat = C.Lattice(4, 7)
    got = [C.gate_count_excluding_layer0(C.random_circuit(lat, d, seed))
           for d in (18, 26, 34, 42, 50)]
    assert got == [258, 375, 492, 609, 726]


def _swap_count_two_halves(gates, n=28, nloc=14):
    """Two-half schedule of Section 2.4: local qubits are 0..13 or 14..27.

    Gates are applied in order while they are diagonal or act only on local
    qubits and no earlier gate on their qubits is pending; when stuck, the
    halves swap.
    """
    diag = set(C.DIAGONAL)
    done = [False] * len(gates)
    local = set(range(nloc))
    swaps = 0
    while True:
        progress = True
        while progress:
            progress = False
            blocked = set()
            for i, g in enumerate(gates):
                if done[i]:
                    continue
                qs = [g[1]] + ([g[2]] if g[2] >= 0 else [])
                ok = all(q not in blocked for q in qs) and (
                    g[0] in diag or all(q in local for q in qs))
                if ok:
                    done[i] = True
                    progress = True
                else:
                    blocked.update(qs)
        if all(done):
            return swaps
        local = set(range(n)) - local
        swaps += 1


def test_table_28qubit_swap_counts():
    # Table "28qubit": 3/4/5/6/7 swaps at depths 18/26/34/42/50 with 14
    # global qubits, diagonal T and CZ applied on any qubit (Section 2.4).
    lat = C.Lattice(4, 7)
    for seed in range(20):
        got = [_swap_count_two_halves(C.random_circuit(lat, d, seed))
               for d in (18, 26, 34, 42, 50)]
        assert got == [3, 4, 5, 6, 7], (seed, got)


def test_7x7_cut_counts():
    # Section 2.1.2: the upper splitting line starts beneath the third row;
    # f(1) = 21, f(7) = 21 + 3 = 24, f(8) = 21 + 3 + 4 = 28, and for the lower
    # part g(1) = 28, g(8) = 35.  f(t) counts cuts in layers < t.
    lat = C.Lattice(7, 7)
    gates = C.random_circuit(lat, 8, 0)
    upper = set(range(21))
    cuts_by_layer = {}
    for name, a, b, layer in gates:
        if name == "CZ" and ((a in upper) != (b in upper)):
            cuts_by_layer[layer] = cuts_by_layer.get(layer, 0) + 1
    f = lambda t: 21 + sum(v for k, v in cuts_by_layer.items() if k < t)
    g = lambda t: 28 + sum(v for k, v in cuts_by_layer.items() if k < t)
    assert f(1) == 21 and f(7) == 24 and f(8) == 28
    assert g(1) == 28 and g(8) == 35
    assert cuts_by_layer == {6: 3, 7: 4}


def test_layer40_single_qubit_positions():
    # Section 2.1.2 ("lucky circuit"): at layer 40 of a 7x7 circuit the
    # qubits 0, 2, 4, 6 carry single-qubit gates.
    gates = C.random_circuit(C.Lattice(7, 7), 40, 3)
    at40 = {a for name, a, b, layer in gates if layer == 40 and b < 0}
    assert {0, 2, 4, 6} <= at40


def test_gate_draw_distribution():
    # The lucky-circuit probability p = 1 - (2/3)^4 = 65/81 assumes the four
    # single-qubit gates on qubits 0,2,4,6 at layer 40 are independent with
    # P(T) = 1/3.
    lat = C.Lattice(7, 7)
    hits, trials, n_t, n_1q = 0, 1500, 0, 0
    for seed in range(trials):
        gates = C.random_circuit(lat, 40, 1000 + seed)
        at40 = {a: name for name, a, b, layer in gates if layer == 40 and b < 0}
        hits += any(at40[q] == "T" for q in (0, 2, 4, 6))
        if seed < 200:
            for name, a, b, layer in gates:
                if layer > 0 and b < 0:
                    n_1q += 1
                    n_t += name == "T"
    p = hits / trials
    sigma = math.sqrt(65 / 81 * 16 / 81 / trials)
    assert abs(p - 65 / 81) < 4 * sigma
    assert abs(n_t / n_1q - 1 / 3) < 0.01


def test_single_qubit_gate_placement_rule():
    # A single-qubit gate goes on q at layer t iff q was in a CZ at t-1 and is
    # not in one at t; no qubit gets two gates in one layer.
    lat = C.Lattice(5, 6)
    gates = C.random_circuit(lat, 20, 7)
    cz = {}
    for name, a, b, layer in gates:
        if name == "CZ":
            cz.setdefault(layer, set()).update((a, b))
    for t in range(1, 21):
        one = sorted(a for name, a, b, layer in gates if layer == t and b < 0)
        want = sorted(cz.get(t - 1, set()) - cz.get(t, set()))
        assert one == want
    assert sum(1 for g in gates if g[3] == 0 and g[0] == "H") == 30


# ----------------------------------------------------------------------------
# Simulator pins
# ----------------------------------------------------------------------------

def _dense_unitary(gates, n):
    """Brute force: product of the n-qubit matrices I^{n-k-1} (x) U (x) I^{k}."""
    dim = 1 << n
    U = np.eye(dim, dtype=np.complex128)
    for name, a, b, _ in gates:
        if name == "CZ":
            d = np.array([-1.0 if ((i >> a) & 1 and (i >> b) & 1) else 1.0
                          for i in range(dim)])
            G = np.diag(d).astype(np.complex128)
        else:
            u = np.array(C.gate_matrix(name), dtype=np.complex128)
            G = np.kron(np.kron(np.eye(1 << (n - a - 1)), u), np.eye(1 << a))
        U = G @ U
    return U


def _random_gate_list(n, count, rng):
    names = ["H", "T", "SX", "SY", "Z", "TDG", "SXDG", "SYDG", "CZ", "P0", "P1"]
    out = []
    for _ in range(count):
        name = rng.choice(names)
        if name == "CZ":
            a, b = rng.sample(range(n), 2)
            out.append(("CZ", a, b, 0))
        else:
            out.append((name, rng.randrange(n), -1, 0))
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_bruteforce_dense(n):
    rng = random.Random(100 + n)
    gates = _random_gate_list(n, 40, rng) if n > 1 else [
        (nm, 0, -1, 0) for nm in ["H", "T", "SX", "SY", "Z", "TDG", "SXDG", "SYDG"]]
    got = sim.simulate(gates, n)
    e0 = np.zeros(1 << n, np.complex128)
    e0[0] = 1
    want = _dense_unitary(gates, n) @ e0
    assert np.max(np.abs(got - want)) < 1e-12


def test_bruteforce_lattice_circuit():
    lat = C.Lattice(2, 5)
    gates = C.random_circuit(lat, 12, 5)
    got = sim.simulate(gates, lat.n)
    e0 = np.zeros(1 << lat.n, np.complex128)
    e0[0] = 1
    want = _dense_unitary(gates, lat.n) @ e0
    assert np.max(np.abs(got - want)) < 1e-12


def test_bruteforce_detects_transposed_matrix(monkeypatch):
    # A planted mistake in the oracle (sqrt(Y) transposed) must fail the
    # brute-force comparison: the pin has teeth.
    gates = [("H", 0, -1, 0), ("SY", 0, -1, 0), ("SY", 1, -1, 0), ("CZ", 0, 1, 0)]
    want = _dense_unitary(gates, 2)[:, 0]
    orig = C.gate_matrix

    def bad(name):
        m = orig(name)
        if name == "SY":
            return [[m[0][0], m[1][0]], [m[0][1], m[1][1]]]
        return m
    monkeypatch.setattr(C, "gate_matrix", bad)
    got = sim.simulate(gates, 2)
    assert np.max(np.abs(got - want)) > 0.1


def test_gate_identities():
    # sqrt(X)^2 = X and sqrt(Y)^2 = Y exactly (principal roots); T^2 = S; H^2 = I.
    m = lambda nm: np.array(C.gate_matrix(nm))
    assert np.allclose(m("SX") @ m("SX"), [[0, 1], [1, 0]], atol=1e-15)
    assert np.allclose(m("SY") @ m("SY"), [[0, -1j], [1j, 0]], atol=1e-15)
    assert np.allclose(m("T") @ m("T"), [[1, 0], [0, 1j]], atol=1e-15)
    assert np.allclose(m("H") @ m("H"), np.eye(2), atol=1e-15)
    for nm in ("H", "T", "SX", "SY"):
        u = m(nm)
        assert np.allclose(u.conj().T @ u, np.eye(2), atol=1e-15)


# X^1/2 and Y^1/2 (Section 2, the gate set of the random circuits) are the
# principal square roots: X and Y have eigenvalues +1 and -1, and the
# principal root maps them to +1 and +i.  The matrices below are built from
# numpy's eigendecomposition of X and Y, independently of the oracle's
# literal constants; the adjoints SXDG/SYDG are their conjugate transposes.
# Both the oracle's matrices and its simulator path are compared, the latter
# column by column from |0> and |1> = H Z H |0>.
_PAULI = {"SX": np.array([[0, 1], [1, 0]], np.complex128),
          "SY": np.array([[0, -1j], [1j, 0]], np.complex128)}


def _principal_root(p):
    lam, vec = np.linalg.eigh(p)
    root = np.array([1.0 if l > 0 else 1j for l in lam.real])
    return vec @ np.diag(root) @ vec.conj().T


def _root_deviation():
    worst = 0.0
    for nm, p in _PAULI.items():
        want = _principal_root(p)
        assert np.allclose(want @ want, p, atol=1e-14)
        for name, w in ((nm, want), (nm + "DG", want.conj().T)):
            got = np.array(C.gate_matrix(name), np.complex128)
            worst = max(worst, float(np.max(np.abs(got - w))))
            for col, prep in ((0, []), (1, [("H", 0, -1, 0), ("Z", 0, -1, 0), ("H", 0, -1, 0)])):
                psi = sim.simulate(prep + [(name, 0, -1, 0)], 1)
                worst = max(worst, float(np.max(np.abs(psi - w[:, col]))))
    return worst


def test_sqrt_gates_are_principal_roots():
    assert _root_deviation() < 1e-14
    # eigenvalues {1, +i}: the adjoint roots have {1, -i} and are the wrong choice
    for nm in ("SX", "SY"):
        ev = sorted(np.linalg.eigvals(np.array(C.gate_matrix(nm), np.complex128)), key=lambda z: z.imag)
        assert np.allclose(ev, [1, 1j], atol=1e-14)


@pytest.mark.parametrize("swap", [("SX", "SXDG"), ("SY", "SYDG")])
def test_sqrt_root_pin_detects_adjoint_swap(monkeypatch, swap):
    # A planted mistake in the oracle (a root replaced by its adjoint, which
    # also squares to the Pauli matrix and is unitary) must fail the pin.
    table = {swap[0]: swap[1], swap[1]: swap[0]}
    mats = {nm: C.gate_matrix(nm) for nm in ("H", "T", "TDG", "Z", "P0", "P1", "SX", "SY", "SXDG", "SYDG")}
    monkeypatch.setattr(C, "gate_matrix", lambda name: mats[table.get(name, name)])
    assert _root_deviation() > 0.5


@pytest.mark.parametrize("n", [1, 7, 16])
def test_layer0_uniform(n):
    psi = sim.simulate([("H", q, -1, 0) for q in range(n)], n)
    assert np.max(np.abs(psi - 2.0 ** (-n / 2))) < 1e-15


@pytest.mark.parametrize("n,seed", [(6, 1), (12, 2), (16, 3)])
def test_closed_form_graph_state(n, seed):
    # H on all qubits followed by diagonal gates only:
    # alpha_x = 2^{-n/2} * w^{#T(x) - #TDG(x)} * (-1)^{#CZ(x) + #Z(x)}.
    rng = random.Random(seed)
    gates = [("H", q, -1, 0) for q in range(n)]
    for _ in range(5 * n):
        nm = rng.choice(["T", "TDG", "Z", "CZ", "CZ"])
        if nm == "CZ":
            a, b = rng.sample(range(n), 2)
            gates.append(("CZ", a, b, 1))
        else:
            gates.append((nm, rng.randrange(n), -1, 1))
    psi = sim.simulate(gates, n)
    x = np.arange(1 << n)
    k = np.zeros(1 << n, np.int64)
    sign = np.zeros(1 << n, np.int64)
    for nm, a, b, _ in gates[n:]:
        bit = (x >> a) & 1
        if nm == "T":
            k += bit
        elif nm == "TDG":
            k -= bit
        elif nm == "Z":
            sign += bit
        elif nm == "CZ":
            sign += bit & ((x >> b) & 1)
    want = 2.0 ** (-n / 2) * np.exp(1j * np.pi / 4 * k) * (-1.0) ** sign
    assert np.max(np.abs(psi - want)) < 1e-14


def test_product_state():
    # Single-qubit gates only keep a product state: alpha_x = prod_q v_q[x_q].
    n = 12
    rng = random.Random(9)
    gates = [(rng.choice(["H", "T", "SX", "SY", "TDG"]), rng.randrange(n), -1, 0)
             for _ in range(60)]
    vs = [np.array([1, 0], np.complex128) for _ in range(n)]
    for nm, a, _, _ in gates:
        vs[a] = np.array(C.gate_matrix(nm)) @ vs[a]
    want = np.array([1.0 + 0j])
    for q in range(n):  # qubit q is index bit q: kron(v_q, lower)
        want = np.kron(vs[q], want)
    psi = sim.simulate(gates, n)
    assert np.max(np.abs(psi - want)) < 1e-14


def test_unitarity_inverse_returns_to_zero():
    lat = C.Lattice(3, 5)
    gates = C.random_circuit(lat, 16, 11)
    psi = sim.simulate(gates, lat.n)
    assert abs(sim.norm2(psi) - 1) < 1e-13
    sim.run(psi, lat.n, C.inverse_circuit(gates))
    e0 = np.zeros_like(psi)
    e0[0] = 1
    assert np.max(np.abs(psi - e0)) < 1e-13


def test_task2_amplitude_from_two_half_sweeps():
    # Section 2.2, Task 2: alpha_x = <x|U|+>.  Split in time, U = U2 U1:
    # alpha_x = <U2^dagger x | U1 +>, two sweeps of half the depth and an inner
    # product; against the amplitude of the full forward sweep.
    lat = C.Lattice(4, 4)
    gates = C.random_circuit(lat, 14, 0x7A5C)
    n = lat.n
    full = sim.simulate(gates, n)
    h = 7
    first = [g for g in gates if g[3] < h]
    second = [g for g in gates if g[3] >= h]
    psi1 = sim.simulate(first, n)
    rng = random.Random(5)
    for x in [0, (1 << n) - 1] + [rng.randrange(1 << n) for _ in range(6)]:
        phi = np.zeros(1 << n, np.complex128)
        phi[x] = 1
        sim.run(phi, n, C.inverse_circuit(second))
        alpha = np.vdot(phi, psi1)
        assert abs(alpha - full[x]) < 1e-13, x


def test_porter_thomas_deep_circuit():
    # Section 3 (Fig. 10): output probabilities of deep random circuits follow
    # Porter-Thomas: N * sum p^2 -> 2 and N*p ~ Exp(1).
    lat = C.Lattice(4, 5)
    psi = sim.simulate(C.random_circuit(lat, 40, 0x5EED0001), lat.n)
    p = np.abs(psi) ** 2
    N = p.size
    assert 1.9 <= N * np.sum(p ** 2) <= 2.1
    # KS distance of N p against Exp(1) on a deterministic sample of 4096.
    s = np.sort(N * p[:: N // 4096])
    ecdf = np.arange(1, s.size + 1) / s.size
    ks = np.max(np.abs(ecdf - (1 - np.exp(-s))))
    assert ks < 0.03


def test_shallow_circuit_not_porter_thomas():
    # Depth 10 on 4x5 is far from Porter-Thomas: many exact zeros.
    lat = C.Lattice(4, 5)
    psi = sim.simulate(C.random_circuit(lat, 10, 0x5EED0001), lat.n)
    p = np.abs(psi) ** 2
    assert p.size * np.sum(p ** 2) > 3.0
    assert np.mean(p < 1e-30) > 0.2


def test_neumaier_norm():
    rng = np.random.default_rng(4)
    v = rng.standard_normal(10000) + 1j * rng.standard_normal(10000)
    want = math.fsum(list((v.real ** 2 + v.imag ** 2)))
    assert abs(sim.norm2(v) - want) <= 1e-15 * want
    # Ill-conditioned for naive left-to-right summation.
    w = np.array([1e8] + [1e-4] * 100000, np.complex128)
    exact = math.fsum([1e16] + [1e-8] * 100000)
    assert abs(sim.norm2(w) - exact) <= 2e-16 * exact


# ----------------------------------------------------------------------------
# Split / combine pins
# ----------------------------------------------------------------------------

def test_split_identity_full_state():
    # CU = P0 (x) I + P1 (x) U: the branch sum equals the unsplit state
    # exactly (Section 2, Fig. 2).
    lat = C.Lattice(3, 4)
    n = lat.n
    gates = C.random_circuit(lat, 12, 21)
    side_a = [q for q in range(n) if q % 4 < 2]  # vertical cut after column 1
    xs = list(range(1 << n))
    amps, info = sim.split_amplitudes(gates, n, side_a, xs)
    want = sim.simulate(gates, n)
    assert len(info["cuts"]) + len(info["folded"]) == sum(
        1 for g in gates if g[0] == "CZ" and ((g[1] in side_a) != (g[2] in side_a)))
    assert np.max(np.abs(amps - want)) < 1e-13


def test_split_folds_final_layer():
    # Crossing CZs of the final layer fold into the output phase (Fig. 6
    # caption: final-layer CZs are diagonal on the output).
    lat = C.Lattice(3, 4)
    n = lat.n
    for depth in range(1, 12):
        gates = C.random_circuit(lat, depth, 3)
        side_a = [q for q in range(n) if q % 4 < 2]
        info = sim.split_circuit(gates, n, side_a)
        for a, b, layer in info["folded"]:
            assert layer <= depth
        last = [c for c in info["cuts"] + info["folded"] if c[2] == depth]
        assert all(c in info["folded"] for c in last)


def _paper_4qubit_example():
    """The 4-qubit example of Section 2.1.1 (Fig. 3, eqs. (1)-(3)).

    Part A holds qubits 0, 1, part B qubits 2, 3.  The two cut CZs act on
    (2, 1); part C acts on qubits 1, 2 only.  X and Y are read as sqrt(X) and
    sqrt(Y) and the H pair of part B as H^2 H^3.
    """
    full = [("H", 0, -1, 0), ("H", 1, -1, 0), ("H", 2, -1, 0), ("H", 3, -1, 0),
            ("CZ", 2, 1, 1), ("CZ", 2, 3, 1), ("T", 1, -1, 2), ("T", 2, -1, 2),
            ("CZ", 2, 1, 3), ("SY", 1, -1, 4), ("CZ", 0, 1, 4), ("SX", 0, -1, 5),
            ("SX", 3, -1, 5)]
    part_c = [("SX", 2, -1, 6), ("CZ", 1, 2, 7), ("SX", 2, -1, 8), ("SY", 1, -1, 8)]
    return full, part_c


def test_paper_4qubit_example_and_zero_invariant():
    full, part_c = _paper_4qubit_example()
    direct = sim.simulate(full + part_c, 4)
    # A = {0, 1}; B = {2, 3}.  Both cut CZs have qubit 2 on side B; the
    # projector goes to the control side (qubit 2), Z^l to qubit 1.
    info = sim.split_circuit(full, 4, [2, 3])
    assert len(info["cuts"]) == 2 and info["folded"] == []
    psi_in = np.zeros(16, np.complex128)
    for l1 in (0, 1):
        for l2 in (0, 1):
            gb, ga = info["half"]((l1, l2))   # side "A" of the split is {2, 3}
            xi = sim.simulate(gb, 2)          # local bits: qubit 2 -> 0, qubit 3 -> 1
            phi = sim.simulate(ga, 2)         # local bits: qubit 0 -> 0, qubit 1 -> 1
            # Implicit decomposition: after the last projector on qubit 2 no
            # gate acts on it in part B, so xi_{i2, i3, l1, l2 != i2} = 0.
            for i in range(4):
                if (i & 1) != l2:
                    assert abs(xi[i]) < 1e-15
            psi_in += np.kron(xi, phi)        # eq. (1): sum of tensor products
    out = sim.run(psi_in.copy(), 4, part_c)   # eq. (2)
    assert np.max(np.abs(out - direct)) < 1e-14
    # eq. (3): part C touches only qubits 1 and 2, so it is block diagonal over
    # (i0, i3): apply it to each 2-qubit block separately.
    blocks = np.zeros(16, np.complex128)
    for i0 in (0, 1):
        for i3 in (0, 1):
            idx = [i0 | (j1 << 1) | (j2 << 2) | (i3 << 3) for j2 in (0, 1) for j1 in (0, 1)]
            sub = psi_in[idx].copy()
            local = [(nm, {1: 0, 2: 1}[a], {1: 0, 2: 1}.get(b, -1), t) for nm, a, b, t in part_c]
            sim.run(sub, 2, local)
            blocks[idx] = sub
    assert np.max(np.abs(blocks - direct)) < 1e-14


def test_combine_exact_on_integers():
    rng = np.random.default_rng(2)
    a = rng.integers(-50, 50, (64, 8)) + 1j * rng.integers(-50, 50, (64, 8))
    b = rng.integers(-50, 50, (64, 8)) + 1j * rng.integers(-50, 50, (64, 8))
    signs = rng.choice([-1, 1], 8)
    got = sim.combine(a, b, signs)
    want = signs * np.sum(a * b, axis=0)
    assert np.array_equal(got, want)


# ----------------------------------------------------------------------------
# Three-part partition (Section 2.1.1 eqs. (2)-(3); Section 2.1.2 Algorithm 1)
# ----------------------------------------------------------------------------

from oracle import partition as PT  # noqa: E402


def _line_sequences(lat, r0, gates, t_s, offs, upper):
    """Every legal, non-decreasing sequence of one line's offsets (brute force)."""
    depth, cz = PT._layers(gates)
    cross = PT.upper_crosses if upper else PT.lower_crosses
    positions = [p for p in itertools.product(*[range(m + 1) for m in offs])]
    seqs = [[]]
    for t in range(t_s, depth + 1):
        nxt = []
        for s in seqs:
            prev = s[-1] if s else tuple([0] * lat.cols)
            for p in positions:
                if all(a >= b for a, b in zip(p, prev)) and not cross(lat, r0, p, cz[t]):
                    nxt.append(s + [p])
        seqs = nxt
    return seqs


def _brute_force_best(lat, gates, r0, max_move):
    """Smallest 2^f + 2^g + 2^c over all separation layers and line sequences.

    The objective separates: f depends on the upper line only, g on the lower
    one, c on both final positions; free cuts are recounted per sequence from
    the enter layers, independently of the dynamic programme.
    """
    depth, _ = PT._layers(gates)
    site = PT._sites(lat)
    up_max, dn_max = PT.max_offsets(lat, r0, max_move)
    nA = sum(1 for q in range(lat.n) if site[q][0] < r0)
    nB = lat.n - nA
    best = None
    for t_s in range(1, depth + 2):
        cuts = PT.cuts_before(lat, gates, r0, t_s)
        K = len(cuts)

        def side_values(upper, offs):
            vals = []
            for seq in _line_sequences(lat, r0, gates, t_s, offs, upper):
                fin = seq[-1] if seq else tuple([0] * lat.cols)
                enter = {}
                for q in range(lat.n):
                    r, c = site[q]
                    enter[q] = depth + 1
                    for k, p in enumerate(seq):
                        inside = (r0 - p[c] <= r < r0) if upper else (r0 <= r < r0 + p[c])
                        if inside:
                            enter[q] = t_s + k
                            break
                not_free = 0
                for gi, a, b, _t in cuts:
                    q = a if upper else b
                    if not PT.free_after(gates, gi, q, enter[q]):
                        not_free += 1
                cnt = 0
                for q in range(lat.n):
                    r, c = site[q]
                    if (r0 - fin[c] <= r < r0) if upper else (r0 <= r < r0 + fin[c]):
                        cnt += 1
                vals.append((not_free, cnt))
            return vals

        for nfa, ca in side_values(True, up_max):
            for nfb, cb in side_values(False, dn_max):
                obj = 2 ** (nA + nfa) + 2 ** (nB + nfb) + 2 ** (ca + cb)
                best = obj if best is None else min(best, obj)
    return best


@pytest.mark.parametrize("rows,cols,depth,seed,r0,mm", [
    (2, 3, 6, 1, 1, 1), (3, 3, 5, 2, 1, 2), (3, 3, 6, 3, 2, 1), (3, 2, 8, 4, 1, 2), (2, 4, 7, 5, 1, 1)])
def test_partition_dp_matches_brute_force(rows, cols, depth, seed, r0, mm):
    lat = C.Lattice(rows, cols)
    gates = C.random_circuit(lat, depth, seed)
    s = PT.plan(lat, gates, r0, mm)
    assert s["objective"] == _brute_force_best(lat, gates, r0, mm)
    ev = PT.evaluate(lat, gates, s)          # the scheme is legal and scores what it claims
    assert ev["objective"] == s["objective"]
    assert (ev["f"], ev["g"], ev["c"]) == (s["f"], s["g"], s["c"])


def test_partition_evaluate_rejects_illegal_schemes():
    lat = C.Lattice(3, 3)
    gates = C.random_circuit(lat, 6, 7)
    depth = 6
    # the lines at the initial position after t_s = 1 cut the vertical CZs of
    # layer 3 (pattern V10 joins rows 1-2 in column 0 and 2)
    zero = [(0, 0, 0)] * depth
    with pytest.raises(ValueError):
        PT.evaluate(lat, gates, {"r0": 2, "t_s": 1, "ups": zero, "dns": zero})
    # offsets that shrink again
    ups = [(1, 1, 1)] * 2 + [(0, 1, 1)] + [(1, 1, 1)] * 3
    with pytest.raises(ValueError):
        PT.evaluate(lat, gates, {"r0": 2, "t_s": 1, "ups": ups, "dns": [(1, 1, 1)] * depth})


@pytest.mark.parametrize("rows,cols,depth,seed,r0", [(3, 4, 8, 77, 1), (3, 4, 8, 77, 2), (4, 4, 9, 11, 2),
                                                     (4, 3, 10, 12, 1)])
def test_partition_state_equals_direct_simulation(rows, cols, depth, seed, r0):
    """eqs. (2)-(3): U_C sum_l phi_l (x) xi_l is the circuit's output state."""
    lat = C.Lattice(rows, cols)
    gates = C.random_circuit(lat, depth, seed)
    direct = sim.simulate(gates, lat.n)
    schemes = [PT.plan(lat, gates, r0, 3)]
    # no part C: the plain two-part split with every crossing CZ cut
    schemes.append({"r0": r0, "t_s": depth + 1, "ups": [], "dns": []})
    for s in schemes:
        psi = PT.partition_state(lat, gates, s)
        assert np.max(np.abs(psi - direct)) < 1e-13


def test_partition_detects_a_dropped_part_c_gate():
    lat = C.Lattice(3, 4)
    gates = C.random_circuit(lat, 8, 77)
    s = PT.plan(lat, gates, 1, 3)
    ev, ga, gb, gc = PT.parts(lat, gates, s)
    assert any(g[0] not in PT.DIAGONAL for g in gc)
    # the same method with one non-diagonal gate of part C left out no longer
    # reproduces the state: part C's gates are really applied after the combine
    drop = next(i for i, g in enumerate(gates) if g in gc and g[0] not in PT.DIAGONAL)
    direct = sim.simulate(gates[:drop] + gates[drop + 1:], lat.n)
    psi = PT.partition_state(lat, gates, s)
    assert np.max(np.abs(psi - direct)) > 1e-3


def test_implicit_decomposition_identity():
    """A cut free on side B: xi_l = [x_b = l] xi' (the projector is absorbed)."""
    lat = C.Lattice(3, 4)
    gates = C.random_circuit(lat, 8, 77)
    s = PT.plan(lat, gates, 1, 3)
    ev, ga, gb, gc = PT.parts(lat, gates, s)
    free = [x for x in ev["cuts"] if x["free_b"]]
    assert free
    x = free[0]
    qb = ev["qb"]
    loc = {q: i for i, q in enumerate(qb)}
    others = [c for c in ev["cuts"] if c is not x]
    for l in (0, 1):
        with_p, without = [], []
        for g in gb:
            if g[0] == "CUT":
                if g[1] == x["gate"]:
                    with_p.append(("P1" if l else "P0", x["b"], -1, x["layer"]))
                else:  # other cuts: branch 0
                    c = next(c for c in others if c["gate"] == g[1])
                    with_p.append(("P0", c["b"], -1, c["layer"]))
                    without.append(("P0", c["b"], -1, c["layer"]))
            else:
                with_p.append(g)
                without.append(g)
        lb = [(g[0], loc[g[1]], loc[g[2]] if g[2] >= 0 else -1, g[3]) for g in with_p]
        lw = [(g[0], loc[g[1]], loc[g[2]] if g[2] >= 0 else -1, g[3]) for g in without]
        xi = sim.simulate(lb, len(qb))
        xi0 = sim.simulate(lw, len(qb))
        idx = np.arange(xi.size)
        mask = ((idx >> loc[x["b"]]) & 1) == l
        assert np.max(np.abs(xi - np.where(mask, xi0, 0))) < 1e-14


def test_paper_4qubit_example_partition_sizes():
    """Fig. 3 example as a 4 x 1 lattice (qubit r at row r), lines after row 1.

    The paper gives S_A = 16 and S_C = 4, and S_B = 8 by absorbing the second
    cut (no gate at all follows it on qubit 2 in part B).  Only diagonal gates
    (CZ^{2,3}, T^2) follow the first cut on qubit 2, so that projector commutes
    to the end of part B as well: S_B = 4 here (xi_{l1,l2} = 0 unless
    l1 = l2 = x_2, which the zero-invariant test above shows for l2).
    """
    full, part_c = _paper_4qubit_example()
    gates = full + part_c
    lat = C.Lattice(4, 1)
    scheme = {"r0": 2, "t_s": 4, "ups": [(0,), (1,), (1,), (1,), (1,)],
              "dns": [(1,), (1,), (1,), (1,), (1,)]}
    ev = PT.evaluate(lat, gates, scheme)
    assert len(ev["cuts"]) == 2
    assert 2 ** ev["f"] == 16 and 2 ** ev["c"] == 4 and 2 ** ev["g"] == 4
    assert [(x["free_a"], x["free_b"]) for x in ev["cuts"]] == [(False, True), (False, True)]
    _, ga, gb, gc = PT.parts(lat, gates, scheme)
    assert sorted((g[0], g[1]) for g in gc) == sorted((g[0], g[1]) for g in part_c)
    psi = PT.partition_state(lat, gates, scheme)
    assert np.max(np.abs(psi - sim.simulate(gates, 4))) < 1e-14
