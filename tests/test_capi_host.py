"""Host-side checks of the C-ABI library (no GPU needed).

The library must load and export every entry point of include/qsv.h; the
C++ circuit generator and split must agree gate by gate with the oracle's
independent generator; argument errors must return a status; the pass
planner's grouping must respect gate semantics; and the host emulation of
the pass programs must reproduce the oracle state.
"""
import os
import re

import numpy as np
import pytest

from oracle import circuit as OC
from oracle import sim
from paper_1804_04797_amd import qsv, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_header_symbol():
    hdr = open(os.path.join(ROOT, "include", "qsv.h")).read()
    names = set(re.findall(r"^(?:qsv_status|void|const char \*)\s*\**\s*(\w+)\s*\(", hdr, re.M))
    assert names, "no declarations parsed"
    L = qsv.lib()
    for nm in sorted(names):
        assert hasattr(L, nm), nm
    assert names == set(qsv.EXPORTS)


def _to_oracle(gates):
    out = []
    for g in gates:
        name = qsv.KIND_NAME[int(g["kind"])]
        out.append((name, int(g["q0"]), int(g["q1"]) if name == "CZ" else -1, int(g["layer"])))
    return out


def _oracle_lattice(spec):
    return OC.Lattice(spec["rows"], spec["cols"], workloads.present_grid(spec))


@pytest.mark.parametrize("name", list(workloads.WORKLOADS))
def test_generator_matches_oracle(name):
    spec = workloads.WORKLOADS[name]
    c = qsv.circuit_create(spec["rows"], spec["cols"], workloads.present_mask(spec),
                           spec["depth"], spec["seed"])
    n, d, ng = c.info()
    lat = _oracle_lattice(spec)
    want = OC.random_circuit(lat, spec["depth"], spec["seed"])
    assert n == lat.n == spec["n"] and d == spec["depth"] and ng == len(want)
    assert _to_oracle(c.gates()) == want


@pytest.mark.parametrize("rows,cols,depth,seed", [(4, 7, 50, 1), (3, 3, 40, 9), (1, 6, 12, 3),
                                                  (7, 7, 40, 3), (2, 2, 9, 0)])
def test_generator_matches_oracle_more(rows, cols, depth, seed):
    c = qsv.circuit_create(rows, cols, None, depth, seed)
    want = OC.random_circuit(OC.Lattice(rows, cols), depth, seed)
    assert _to_oracle(c.gates()) == want


def test_generator_uneven_lattices():
    for n, d, s in workloads.uneven_batch(24):
        rows, cols, pres = workloads.lattice_for_qubits(n)
        c = qsv.circuit_create(rows, cols, pres, d, s)
        lat = OC.Lattice.for_qubits(n)
        assert _to_oracle(c.gates()) == OC.random_circuit(lat, d, s)


def test_explicit_gate_list_roundtrip():
    g = np.zeros(3, qsv.GATE_DTYPE)
    g[0] = (qsv.KIND["H"], 0, 0, 0, 0, 0)
    g[1] = (qsv.KIND["CZ"], 0, 1, 0, 1, 0)
    g[2] = (qsv.KIND["T"], 1, 0, 0, 2, 0)
    c = qsv.circuit_create(1, 2, None, gates=g)
    assert c.info() == (2, 2, 3)
    assert np.array_equal(c.gates(), g)


def test_error_statuses():
    with pytest.raises(qsv.QsvError) as e:
        qsv.circuit_create(0, 5, None, 3, 1)
    assert e.value.status == 1
    g = np.zeros(1, qsv.GATE_DTYPE)
    g[0] = (qsv.KIND["H"], 9, 0, 0, 0, 0)
    with pytest.raises(qsv.QsvError) as e:
        qsv.circuit_create(2, 2, None, gates=g)
    assert e.value.status == 2
    g[0] = (99, 0, 0, 0, 0, 0)
    with pytest.raises(qsv.QsvError) as e:
        qsv.circuit_create(2, 2, None, gates=g)
    assert e.value.status == 1
    c = qsv.circuit_create(2, 3, None, 4, 1)
    with pytest.raises(qsv.QsvError) as e:
        qsv.circuit_split(c, 0)
    assert e.value.status == 1
    with pytest.raises(qsv.QsvError) as e:
        qsv.circuit_split(c, 1 << 40)
    assert e.value.status == 2
    # state pointer checks happen before any device call
    with pytest.raises(qsv.QsvError) as e:
        qsv.sv_apply_fused(0, c)
    assert e.value.status == 1
    with pytest.raises(qsv.QsvError) as e:
        qsv.sv_init(8, 5, 0)          # misaligned pointer
    assert e.value.status == 1
    with pytest.raises(qsv.QsvError) as e:
        qsv.sv_init(256, 40, 0)       # n too large
    assert e.value.status == 2
    with pytest.raises(qsv.QsvError) as e:
        qsv.sv_apply_fused(256, c, opts={"reg_qubits": 7, "thread_qubits": 8,
                                         "low_qubits": 0, "plain": 0})
    assert e.value.status == 5


@pytest.mark.parametrize("after_col", [1, 2])
def test_split_matches_oracle(after_col):
    rows, cols, depth, seed = 3, 4, 12, 21
    c = qsv.circuit_create(rows, cols, None, depth, seed)
    mask = workloads.column_cut_mask(rows, cols, after_col)
    ha, hb, ceff, folded = qsv.circuit_split(c, mask)
    side_a = [q for q in range(rows * cols) if (mask >> q) & 1]
    info = sim.split_circuit(OC.random_circuit(OC.Lattice(rows, cols), depth, seed),
                             rows * cols, side_a)
    assert ceff == len(info["cuts"])
    assert folded == [(a, b) for a, b, _ in info["folded"]]
    # PB/ZB with branch bit j must equal the oracle's P_l / Z^l for every l
    ga, gb = ha.gates(), hb.gates()
    for br in range(min(1 << ceff, 64)):
        l = tuple((br >> j) & 1 for j in range(ceff))
        oa, ob = info["half"](l)
        mine_a, mine_b = [], []
        for g in ga:
            k = qsv.KIND_NAME[int(g["kind"])]
            if k == "PB":
                k = "P1" if l[int(g["arg"])] else "P0"
            mine_a.append((k, int(g["q0"]), int(g["q1"]) if k == "CZ" else -1, int(g["layer"])))
        for g in gb:
            k = qsv.KIND_NAME[int(g["kind"])]
            if k == "ZB":
                if not l[int(g["arg"])]:
                    continue
                k = "Z"
            mine_b.append((k, int(g["q0"]), int(g["q1"]) if k == "CZ" else -1, int(g["layer"])))
        assert mine_a == oa and mine_b == ob


def _random_explicit(n, count, seed, kinds=("H", "T", "SX", "SY", "CZ", "TDG", "SXDG", "SYDG",
                                            "Z", "P0", "P1")):
    rng = np.random.default_rng(seed)
    g = np.zeros(count, qsv.GATE_DTYPE)
    for i in range(count):
        k = kinds[rng.integers(len(kinds))]
        q0 = int(rng.integers(n))
        q1 = q0
        while k == "CZ" and q1 == q0:
            q1 = int(rng.integers(n))
        g[i] = (qsv.KIND[k], q0, q1 if k == "CZ" else 0, 0, i // 4, 0)
    return g


SHAPES = [None, dict(reg_qubits=3, thread_qubits=4, low_qubits=3, plain=0),
          dict(reg_qubits=4, thread_qubits=6, low_qubits=5, plain=0),
          dict(reg_qubits=2, thread_qubits=3, low_qubits=2, plain=0)]


@pytest.mark.parametrize("shape", SHAPES)
def test_plan_respects_dependencies(shape):
    spec = workloads.WORKLOADS["4x5-d10"]
    c = qsv.circuit_create(spec["rows"], spec["cols"], None, 24, 77)
    info = qsv.sv_plan_info(c, opts=shape)
    gates = _to_oracle(c.gates())
    pog, oip = info["pass_of_gate"], info["order_in_pass"]
    assert (pog >= 0).all()
    # every non-diagonal gate runs in a pass where its qubit is resident
    for i, g in enumerate(gates):
        if g[0] not in OC.DIAGONAL:
            assert (info["resident"][pog[i]] >> g[1]) & 1
    # executing in (pass, position) order gives the in-order state
    order = sorted(range(len(gates)), key=lambda i: (pog[i], oip[i]))
    re = sim.simulate([gates[i] for i in order], 20)
    ref = sim.simulate(gates, 20)
    assert np.max(np.abs(re - ref)) < 1e-12
    assert 1 <= info["n_passes"] <= 25


OOP_SHAPES = [(4, 6, 5), (3, 6, 4), (2, 3, 2), (3, 4, 3), (4, 7, 4), (5, 8, 4), (4, 6, 3), (6, 9, 4)]


@pytest.mark.parametrize("name", ["4x5-d10", "5x6-d16"])
def test_emulated_out_of_place_plans(name):
    """Out-of-place plans write every pass under a new qubit-to-bit map (the
    next pass's qubits at the low bits) into the other buffer; emulated with
    the device's buffer schedule, against the oracle.  A plan with an odd
    pass count falls back to the in-place plan when the first pass reads the
    state, so the shapes cover both cases."""
    spec = workloads.WORKLOADS[name]
    rows, cols = spec["rows"], spec["cols"]
    depth = spec["depth"] if rows * cols <= 20 else 8
    c = qsv.circuit_create(rows, cols, None, depth, spec["seed"])
    n = rows * cols
    if n > 20:  # a 20-qubit sub-lattice keeps the emulation quick
        c = qsv.circuit_create(4, 5, None, 12, spec["seed"])
        n = 20
    ref = sim.simulate(_to_oracle(c.gates()), n)
    even = 0
    for sh in OOP_SHAPES:
        for oop in (1, -1):
            o = dict(reg_qubits=sh[0], thread_qubits=sh[1], low_qubits=sh[2], plain=0, jit=1,
                     out_of_place=oop)
            psi = np.zeros(1 << n, np.complex64)
            psi[0] = 1
            qsv.sv_debug_emulate(psi, c, opts=o)
            assert np.max(np.abs(psi - ref)) < 1e-6, (sh, oop)
            if oop == 1 and qsv.sv_plan_info(c, opts=o)["n_passes"] % 2 == 0:
                even += 1
    assert even >= 1  # at least one shape ran the two-buffer schedule


@pytest.mark.parametrize("shape", SHAPES)
def test_emulated_plan_matches_oracle(shape):
    spec = workloads.WORKLOADS["4x5-d10"]
    c = qsv.circuit_create(spec["rows"], spec["cols"], None, spec["depth"], spec["seed"])
    psi = np.zeros(1 << 20, np.complex64)
    psi[0] = 1
    qsv.sv_debug_emulate(psi, c, opts=shape)
    ref = sim.simulate(_to_oracle(c.gates()), 20)
    assert np.max(np.abs(psi - ref)) < 1e-6
    p64 = psi.astype(np.complex128)
    fid = abs(np.vdot(ref, p64)) ** 2 / (np.vdot(p64, p64).real * np.vdot(ref, ref).real)
    assert 1 - fid < 1e-9
    assert abs(np.vdot(p64, p64).real - 1) < 1e-5


def test_emulated_explicit_gates_all_kinds():
    n = 12
    g = _random_explicit(n, 300, 5)
    c = qsv.circuit_create(3, 4, None, gates=g)
    for shape in SHAPES:
        psi = np.zeros(1 << n, np.complex64)
        psi[0] = 1
        qsv.sv_debug_emulate(psi, c, opts=shape)
        ref = sim.simulate(_to_oracle(c.gates()), n)
        assert np.max(np.abs(psi - ref)) < 1e-5


def test_emulated_layer_ranges_compose():
    spec = workloads.WORKLOADS["4x5-d10"]
    c = qsv.circuit_create(spec["rows"], spec["cols"], None, 16, 3)
    psi = np.zeros(1 << 20, np.complex64)
    psi[0] = 1
    for lb, le in ((0, 3), (3, 4), (4, 11), (11, -1)):
        qsv.sv_debug_emulate(psi, c, layer_begin=lb, layer_end=le)
    ref = sim.simulate(_to_oracle(c.gates()), 20)
    assert np.max(np.abs(psi - ref)) < 1e-6


def test_emulated_split_branches():
    rows, cols, depth, seed = 3, 4, 10, 4
    n = rows * cols
    c = qsv.circuit_create(rows, cols, None, depth, seed)
    mask = workloads.column_cut_mask(rows, cols, 1)
    ha, hb, ceff, folded = qsv.circuit_split(c, mask)
    na, nb = ha.n, hb.n
    qa = [q for q in range(n) if (mask >> q) & 1]
    qb = [q for q in range(n) if not (mask >> q) & 1]
    opts = dict(reg_qubits=2, thread_qubits=3, low_qubits=2, plain=0)
    total = np.zeros(1 << n, np.complex128)
    xs = np.arange(1 << n)
    xa = np.array([sim.sub_index(int(x), qa) for x in xs])
    xb = np.array([sim.sub_index(int(x), qb) for x in xs])
    for br in range(1 << ceff):
        A = np.zeros(1 << na, np.complex64); A[0] = 1
        B = np.zeros(1 << nb, np.complex64); B[0] = 1
        qsv.sv_debug_emulate(A, ha, branch=br, opts=opts)
        qsv.sv_debug_emulate(B, hb, branch=br, opts=opts)
        total += A[xa].astype(np.complex128) * B[xb]
    sign = np.array([sim.fold_sign(int(x), [(a, b, 0) for a, b in folded]) for x in xs])
    total *= sign
    ref = sim.simulate(OC.random_circuit(OC.Lattice(rows, cols), depth, seed), n)
    assert np.max(np.abs(total - ref)) < 1e-5


@pytest.mark.parametrize("k", [4, 5, 6, 7])
def test_dense_blocks_emulated_match_oracle(k):
    """Dense-block plan (FP64 block matrices rounded to complex64) applied on
    the host reproduces the oracle state."""
    spec = workloads.WORKLOADS["4x5-d10"]
    c = qsv.circuit_create(spec["rows"], spec["cols"], None, spec["depth"], spec["seed"])
    psi = np.zeros(1 << 20, np.complex64)
    psi[0] = 1
    nb = qsv.sv_debug_emulate_dense(psi, c, k)
    assert 1 <= nb <= len(c.gates())
    ref = sim.simulate(_to_oracle(c.gates()), 20)
    assert np.max(np.abs(psi - ref)) < 1e-5


def test_dense_blocks_all_gate_kinds():
    n = 12
    g = _random_explicit(n, 200, 17)
    c = qsv.circuit_create(3, 4, None, gates=g)
    psi = np.zeros(1 << n, np.complex64)
    psi[0] = 1
    qsv.sv_debug_emulate_dense(psi, c, 5)
    ref = sim.simulate(_to_oracle(c.gates()), n)
    assert np.max(np.abs(psi - ref)) < 1e-5


@pytest.mark.parametrize("shape", [None, dict(reg_qubits=4, thread_qubits=8, low_qubits=4, plain=0),
                                   dict(reg_qubits=3, thread_qubits=4, low_qubits=3, plain=0)])
def test_compiled_pass_source_compiles(shape):
    """The generated straight-line pass kernels (complex64 and complex128
    instantiations, with generated initial state and norm epilogue) compile
    for gfx950 (hipRTC runs without a device)."""
    spec = workloads.WORKLOADS["4x5-d10"]
    c = qsv.circuit_create(spec["rows"], spec["cols"], None, spec["depth"], spec["seed"])
    nbytes, secs = qsv.sv_debug_jit_compile(c, layer_begin=1, opts=shape)
    assert nbytes > 1000


@pytest.mark.parametrize("name,shape", [("6x6m2-d30", (5, 8, 4)), ("5x6-d20", (5, 9, 5))])
def test_exchange_layouts_checked_for_the_headline_plans(name, shape):
    """Every exchange layout of the 34- and 30-qubit sweeps' plans (one tile
    per workgroup staged in halves or whole, persistent, sampling, batched)
    passes the generator's injectivity check (no fall-back to plain weights,
    else QSV_EINTERNAL), and the sources compile."""
    spec = dict(workloads.WORKLOADS[name])
    c = qsv.circuit_create(spec["rows"], spec["cols"], workloads.present_mask(spec), spec["depth"], spec["seed"])
    o = dict(reg_qubits=shape[0], thread_qubits=shape[1], low_qubits=shape[2], plain=0, jit=1, out_of_place=0)
    nbytes, _ = qsv.sv_debug_jit_compile(c, layer_begin=1, opts=o)
    assert nbytes > 1000


def test_circuit_inverse_matches_oracle():
    """circuit_inverse: reversed order, adjoint kinds, mirrored layers, against
    the oracle generator's adjoint of the same circuit."""
    spec = workloads.WORKLOADS["5x6-d16"]
    c = qsv.circuit_create(spec["rows"], spec["cols"], None, spec["depth"], spec["seed"])
    inv = qsv.circuit_inverse(c)
    fwd = _to_oracle(c.gates())
    want = OC.inverse_circuit(fwd)
    got = _to_oracle(inv.gates())
    top = max(g[3] for g in fwd)
    assert [g[:3] for g in got] == [g[:3] for g in want]
    assert [g[3] for g in got] == [top - g[3] for g in want]
    assert inv.info()[0] == c.info()[0]


# --- three-part partition (host side) ----------------------------------------

from oracle import partition as OPT  # noqa: E402


def _branch_gates(gates, branch):
    """Library branch gates (PB / ZB with bit `arg`) as plain oracle gates for one branch."""
    out = []
    for g in gates:
        name = qsv.KIND_NAME[int(g["kind"])]
        q0, t = int(g["q0"]), int(g["layer"])
        if name in ("PB", "ZB"):
            bit = (branch >> int(g["arg"])) & 1
            if name == "PB":
                out.append(("P1" if bit else "P0", q0, -1, t))
            elif bit:
                out.append(("Z", q0, -1, t))
            continue
        out.append((name, q0, int(g["q1"]) if name == "CZ" else -1, t))
    return out


PART_CASES = [(3, 4, 8, 77, 1), (3, 4, 8, 77, 2), (4, 5, 10, 5, 2), (4, 5, 10, 5, 3), (3, 5, 12, 9, 1),
              (4, 4, 12, 21, 2)]


@pytest.mark.parametrize("rows,cols,depth,seed,r0", PART_CASES)
def test_partition_plan_matches_oracle(rows, cols, depth, seed, r0):
    lat = OC.Lattice(rows, cols)
    gates = OC.random_circuit(lat, depth, seed)
    c = qsv.circuit_create(rows, cols, None, depth, seed)
    want = OPT.plan(lat, gates, r0, 2)
    p = qsv.circuit_partition_plan(c, rows, cols, None, r0, 2)
    info = qsv.circuit_partition_info(p)
    # the optimum is unique, the scheme reaching it need not be
    assert info["objective"] == want["objective"]
    ups, dns = qsv.circuit_partition_offsets(p)
    ev = OPT.evaluate(lat, gates, {"r0": r0, "t_s": info["t_s"], "ups": ups.tolist(), "dns": dns.tolist()})
    assert (ev["f"], ev["g"], ev["c"]) == (info["f"], info["g"], info["n_c"])
    assert info["cuts"] == len(ev["cuts"])
    fa = sum(1 for x in ev["cuts"] if x["free_a"] and not x["free_b"])
    fb = sum(1 for x in ev["cuts"] if x["free_b"] and not x["free_a"])
    both = sum(1 for x in ev["cuts"] if x["free_a"] and x["free_b"])
    assert info["folded"] == both
    assert info["explicit_bits"] == info["cuts"] - fa - fb - both
    assert info["sel_a"] <= fa and info["sel_b"] <= fb


@pytest.mark.parametrize("rows,cols,depth,seed,r0", PART_CASES[:4])
def test_partition_parts_reproduce_state(rows, cols, depth, seed, r0):
    """The library's part circuits, run per branch with the oracle simulator and
    combined with the documented branch layout, give the circuit's state."""
    lat = OC.Lattice(rows, cols)
    gates = OC.random_circuit(lat, depth, seed)
    n = lat.n
    c = qsv.circuit_create(rows, cols, None, depth, seed)
    p = qsv.circuit_partition_plan(c, rows, cols, None, r0, 2)
    info = qsv.circuit_partition_info(p)
    A, B, Cc, qa, qb = qsv.circuit_partition_parts(p)
    na, nb, eb = info["n_a"], info["n_b"], info["explicit_bits"]
    ka, kb = info["sel_a"], info["sel_b"]
    phi = [sim.simulate(_branch_gates(A.gates(), i), na) for i in range(info["branches_a"])]
    xi = [sim.simulate(_branch_gates(B.gates(), i), nb) for i in range(info["branches_b"])]
    xs = np.arange(1 << n)
    xa = np.zeros_like(xs)
    xb = np.zeros_like(xs)
    for i, q in enumerate(qa):
        xa |= ((xs >> int(q)) & 1) << i
    for i, q in enumerate(qb):
        xb |= ((xs >> int(q)) & 1) << i
    u = xb >> (nb - kb)   # B selector qubits pick A's extra branch bits
    w = xa >> (na - ka)   # A selector qubits pick B's extra branch bits
    ev = OPT.evaluate(lat, gates, {"r0": r0, "t_s": info["t_s"],
                                   "ups": qsv.circuit_partition_offsets(p)[0].tolist(),
                                   "dns": qsv.circuit_partition_offsets(p)[1].tolist()})
    sign = np.ones(1 << n)
    for x in ev["cuts"]:
        if x["free_a"] and x["free_b"]:
            sign *= np.where(((xs >> x["a"]) & 1) & ((xs >> x["b"]) & 1), -1.0, 1.0)
    PA = np.array(phi)
    PB = np.array(xi)
    psi = np.zeros(1 << n, np.complex128)
    for e in range(1 << eb):
        psi += PA[e | (u << eb), xa] * PB[e | (w << eb), xb]
    psi *= sign
    cg = _to_oracle(Cc.gates())
    sim.run(psi, n, cg)
    direct = sim.simulate(gates, n)
    assert np.max(np.abs(psi - direct)) < 1e-13


def test_partition_create_checks_the_scheme():
    rows, cols, depth, seed = 3, 4, 8, 77
    c = qsv.circuit_create(rows, cols, None, depth, seed)
    p = qsv.circuit_partition_plan(c, rows, cols, None, 1, 2)
    info = qsv.circuit_partition_info(p)
    ups, dns = qsv.circuit_partition_offsets(p)
    q = qsv.circuit_partition_create(c, rows, cols, None, 1, info["t_s"], ups, dns)
    assert qsv.circuit_partition_info(q) == info
    # no part C at all: every crossing CZ is cut
    q2 = qsv.circuit_partition_create(c, rows, cols, None, 1, depth + 1, [], [])
    assert qsv.circuit_partition_info(q2)["n_c"] == 0
    with pytest.raises(qsv.QsvError):   # lines at rest cut later CZs
        qsv.circuit_partition_create(c, rows, cols, None, 1, 1, np.zeros((depth, cols)), np.zeros((depth, cols)))
    if len(ups) > 1 and ups[-1].any():
        bad = ups.copy()
        bad[-1] = 0                      # offsets that shrink
        with pytest.raises(qsv.QsvError):
            qsv.circuit_partition_create(c, rows, cols, None, 1, info["t_s"], bad, dns)
    with pytest.raises(qsv.QsvError):   # lattice does not match the circuit
        qsv.circuit_partition_plan(c, rows, cols + 1, None, 1, 2)
    with pytest.raises(qsv.QsvError):   # r0 outside 1..rows-1
        qsv.circuit_partition_plan(c, rows, cols, None, rows, 2)


def test_partition_simulate_rejects_small_blocks():
    """Blocks of fewer than 2^7 rows are refused before any device work."""
    c = qsv.circuit_create(4, 5, None, 10, 5)
    p = qsv.circuit_partition_plan(c, 4, 5, None, 1, 2)  # part A: 5 qubits
    assert qsv.circuit_partition_info(p)["n_a"] < 7
    ws = qsv.sv_partition_workspace_bytes(p)
    with pytest.raises(qsv.QsvError) as e:
        qsv.sv_partition_simulate(p, 1 << 20, ws, 1 << 30, stream=0)
    assert e.value.status == 5  # QSV_EUNSUPPORTED


def test_partition_with_absent_sites():
    """Lattice with two absent sites (qubits renumbered over the present ones):
    the planner matches the oracle's optimum and its parts reproduce the state."""
    rows, cols, depth, seed, r0 = 4, 4, 10, 31, 2
    grid = [[True] * cols for _ in range(rows)]
    grid[0][0] = False
    grid[3][2] = False
    pres = np.array(grid, np.uint8)
    lat = OC.Lattice(rows, cols, grid)
    gates = OC.random_circuit(lat, depth, seed)
    c = qsv.circuit_create(rows, cols, pres, depth, seed)
    assert _to_oracle(c.gates()) == gates
    want = OPT.plan(lat, gates, r0, 2)
    p = qsv.circuit_partition_plan(c, rows, cols, pres, r0, 2)
    info = qsv.circuit_partition_info(p)
    assert info["objective"] == want["objective"]
    ups, dns = qsv.circuit_partition_offsets(p)
    ev = OPT.evaluate(lat, gates, {"r0": r0, "t_s": info["t_s"], "ups": ups.tolist(), "dns": dns.tolist()})
    assert (ev["f"], ev["g"], ev["c"]) == (info["f"], info["g"], info["n_c"])
    A, B, Cc, qa, qb = qsv.circuit_partition_parts(p)
    assert sorted(list(qa) + list(qb)) == list(range(lat.n))
    assert all(lat.qubit[(r, k)] in qa for (r, k) in lat.qubit if r < r0)


def test_apply_fused_from_argument_checks():
    """Overlapping or misaligned buffers are refused before any device work."""
    c = qsv.circuit_create(4, 5, None, 6, 3)
    base = 1 << 32
    size = 8 << 20  # 2^20 complex64
    for src, dst in [(base, base + size // 2), (base + size // 2, base)]:
        with pytest.raises(qsv.QsvError) as e:
            qsv.sv_apply_fused_from(src, dst, c, stream=0)
        assert e.value.status == 1  # QSV_EINVAL
    with pytest.raises(qsv.QsvError) as e:
        qsv.sv_apply_fused_from(base + 8, base + 2 * size, c, stream=0)
    assert e.value.status == 1


@pytest.mark.parametrize("rows,cols,depth,seed,r0", [(3, 4, 8, 77, 1), (4, 5, 10, 5, 2)])
def test_partition_plan_without_moves(rows, cols, depth, seed, r0):
    """max_move = 0: the lines cannot leave the initial row, so part C stays
    empty and only the separation layer is chosen; same optimum as the oracle."""
    lat = OC.Lattice(rows, cols)
    gates = OC.random_circuit(lat, depth, seed)
    c = qsv.circuit_create(rows, cols, None, depth, seed)
    want = OPT.plan(lat, gates, r0, 0)
    info = qsv.circuit_partition_info(qsv.circuit_partition_plan(c, rows, cols, None, r0, 0))
    assert info["objective"] == want["objective"] and info["n_c"] == 0 == want["c"]


def test_sampler_argument_checks():
    """Bitstrings >= 2^n and an empty set are refused before any device work."""
    c = qsv.circuit_create(4, 5, None, 6, 3)
    with pytest.raises(qsv.QsvError) as e:
        qsv.sv_sampler_create(c, np.array([1, 1 << 20], np.uint64))
    assert e.value.status == 2  # QSV_ERANGE
    with pytest.raises(qsv.QsvError) as e:
        qsv.sv_sampler_create(c, np.array([], np.uint64))
    assert e.value.status == 2
    # the multi-branch run refuses a missing sampler, branch list or output on the host
    br = np.array([0, 1], np.uint64)
    assert qsv.lib().sv_sampler_run_branches(None, 256, 512, br.ctypes.data, 2, 1024, None, 0, None) == 1
    assert qsv.lib().sv_sampler_run_branches(None, 256, 512, None, 2, 1024, None, 0, None) == 1
    assert qsv.lib().sv_sampler_run_branches(None, 256, 512, br.ctypes.data, 2, None, None, 0, None) == 1


# --- branch stages (prefix sharing among the branches of a split half) -------

STAGE_CASES = [(3, 4, 14, 21, 1, 0), (3, 4, 14, 21, 1, 1), (4, 4, 16, 5, 1, 0), (3, 5, 16, 9, 2, 1),
               (4, 5, 12, 3, 2, 0)]


@pytest.mark.parametrize("rows,cols,depth,seed,after_col,side", STAGE_CASES)
def test_branch_stages_reproduce_every_branch(rows, cols, depth, seed, after_col, side):
    c = qsv.circuit_create(rows, cols, None, depth, seed)
    ha, hb, ceff, _ = qsv.circuit_split(c, workloads.column_cut_mask(rows, cols, after_col))
    h = (ha, hb)[side]
    n = h.n
    full = h.gates()
    levels = qsv.circuit_branch_levels(h)
    L = len(levels)
    assert L >= 2
    # the level masks partition the branch bits; each level's PB / ZB gates sit in one layer
    assert sum(levels) == (1 << ceff) - 1 and all(a & b == 0 for i, a in enumerate(levels)
                                                  for b in levels[i + 1:])
    stages = [qsv.circuit_branch_stage(h, k, k + 1).gates() for k in range(L + 1)]
    assert sum(len(s) for s in stages) == len(full)
    for k, s in enumerate(stages):
        bb = [int(g["arg"]) for g in s if qsv.KIND_NAME[int(g["kind"])] in ("PB", "ZB")]
        assert sum(1 << b for b in set(bb)) == (levels[k - 1] if k else 0)
        # original order kept: s is a subsequence of the whole gate list
        it = iter(full.tobytes()[i * full.itemsize:(i + 1) * full.itemsize] for i in range(len(full)))
        assert all(any(x == y for y in it) for x in (s.tobytes()[i * s.itemsize:(i + 1) * s.itemsize]
                                                       for i in range(len(s))))
    # the stage order really moves gates (the check below is not vacuous)
    assert np.concatenate(stages).tobytes() != full.tobytes()
    groupings = [list(range(L + 2)), [0, 1, L + 1], [0, L, L + 1], [0, L + 1]]
    rng = np.random.default_rng(seed)
    for br in sorted({0, (1 << ceff) - 1} | {int(x) for x in rng.integers(0, 1 << ceff, 6)}):
        want = sim.simulate(_branch_gates(full, br), n)
        for grp in groupings:
            gates = []
            for a, b in zip(grp, grp[1:]):
                gates += _branch_gates(qsv.circuit_branch_stage(h, a, b if b <= L else -1).gates(), br)
            got = sim.simulate(gates, n)
            assert np.max(np.abs(got - want)) < 1e-12, (br, grp)


def test_branch_stages_without_branches_and_bad_ranges():
    c = qsv.circuit_create(3, 3, None, 8, 4)
    assert qsv.circuit_branch_levels(c) == []
    assert qsv.circuit_branch_stage(c, 0, -1).gates().tobytes() == c.gates().tobytes()
    ha, _, _, _ = qsv.circuit_split(qsv.circuit_create(3, 4, None, 14, 21),
                                    workloads.column_cut_mask(3, 4, 1))
    L = len(qsv.circuit_branch_levels(ha))
    for lb, le in [(1, 1), (2, 1), (-1, 1), (0, L + 2)]:
        with pytest.raises(qsv.QsvError) as e:
            qsv.circuit_branch_stage(ha, lb, le)
        assert e.value.status == 1


def test_tune_set_applies_to_plans():
    """sv_tune_set makes later calls without options plan with the given
    shape; it is keyed by circuit content and layer range; null arguments are
    refused."""
    c = qsv.circuit_create(5, 6, None, 20, 0x7E57)  # a circuit no other test tunes
    o = dict(reg_qubits=5, thread_qubits=9, low_qubits=5, plain=0, jit=1)
    want = qsv.sv_plan_info(c, 1, -1, o)["resident"]
    qsv.sv_tune_set(c, o, layer_begin=1)
    assert qsv.sv_plan_info(c, 1, -1)["resident"] == want
    same = qsv.circuit_create(5, 6, None, 20, 0x7E57)  # same content
    assert qsv.sv_plan_info(same, 1, -1)["resident"] == want
    assert qsv.lib().sv_tune_set(None, 0, -1, None) == 1



def test_workspace_bytes():
    # sv_workspace_bytes: the second state buffer when the options run out
    # of place (n >= 24 by default with compiled passes), plus the FP64
    # partial sums (16 bytes per 2^11-amplitude tile, at least 1 MiB)
    c30 = qsv.circuit_create(5, 6, None, 6, 1)
    part30 = 16 * max(1 << (30 - 11), 65536)
    assert qsv.sv_workspace_bytes(c30, 1) == (8 << 30) + part30
    assert qsv.sv_workspace_bytes(c30, 1, opts={"out_of_place": -1}) == part30
    assert qsv.sv_workspace_bytes(c30, 1, opts={"jit": -1}) == part30
    assert qsv.sv_workspace_bytes(c30, 1, opts={"plain": 1}) == part30
    c20 = qsv.circuit_create(4, 5, None, 6, 1)
    assert qsv.sv_workspace_bytes(c20, 1) == 16 * 65536
    assert qsv.sv_workspace_bytes(c20, 1, opts={"jit": 1, "out_of_place": 1}) == (8 << 20) + 16 * 65536
    with pytest.raises(qsv.QsvError) as e:
        qsv.sv_workspace_bytes(c20, -1)
    assert e.value.status == 1


@pytest.mark.parametrize("seed,workers", [(1, 1), (2, 3), (3, 64), (4, 512)])
def test_persistent_batch_schedule(seed, workers):
    # The persistent batch launch's work-item order and waiting rule (host
    # emulation): uneven entries with different pass counts, every item run
    # once, never before its entry's earlier passes, and no stall for any
    # number of workgroups, including one.
    rng = np.random.default_rng(seed)
    n = rng.integers(11, 17, size=40)
    passes = rng.integers(0, 5, size=40)
    items = qsv.sv_debug_batch_schedule(n, passes, 11, workers, seed)
    assert items == int(sum(int(p) << (int(q) - 11) for q, p in zip(n, passes)))


def test_persistent_batch_schedule_detects_a_broken_rule():
    # a planted wrong rule (an item may start one tile early) must fail the
    # check; edge cases: one entry, entries with zero passes; a tile larger
    # than a state is refused
    rng = np.random.default_rng(9)
    n = rng.integers(11, 15, size=20)
    passes = rng.integers(1, 4, size=20)
    with pytest.raises(qsv.QsvError):
        qsv.sv_debug_batch_schedule(n, passes, 11, 64, 5, planted_early_start=True)
    assert qsv.sv_debug_batch_schedule([11], [3], 11, 2) == 3
    assert qsv.sv_debug_batch_schedule([12, 11], [0, 2], 11, 4) == 2
    with pytest.raises(qsv.QsvError):
        qsv.sv_debug_batch_schedule([10], [1], 11, 2)


def test_whole_state_tile_plans():
    """A state of 2^14 amplitudes or fewer fits one tile: its plan on that
    tile has every qubit resident and a single pass for these depths."""
    for n, d in [(11, 9), (12, 14), (13, 20), (14, 24)]:
        rows, cols, pres = workloads.lattice_for_qubits(n)
        c = qsv.circuit_create(rows, cols, pres, d, 5)
        R, T = {11: (4, 7), 12: (5, 7), 13: (5, 8), 14: (5, 9)}[n]
        info = qsv.sv_plan_info(c, 1, -1, dict(reg_qubits=R, thread_qubits=T, low_qubits=5, plain=0, jit=-1))
        assert info["n_passes"] == 1, (n, info["n_passes"])


def test_jit_code_object_disk_cache(tmp_path):
    # QSV_JIT_CACHE: the first process compiles and stores the code objects,
    # a second process loads them (no compile) and gets the same code size
    import subprocess
    import sys
    prog = (
        "import sys, time; sys.path.insert(0, %r)\n"
        "from paper_1804_04797_amd import qsv, workloads\n"
        "spec = workloads.WORKLOADS['4x5-d10']\n"
        "c = qsv.circuit_create(spec['rows'], spec['cols'], None, spec['depth'], spec['seed'])\n"
        "o = dict(reg_qubits=4, thread_qubits=7, low_qubits=4, plain=0, jit=1)\n"
        "t = time.time(); b, _ = qsv.sv_debug_jit_compile(c, 1, -1, o); print(b, time.time() - t)\n"
    ) % ROOT
    env = dict(os.environ, QSV_JIT_CACHE=str(tmp_path))
    r1 = subprocess.run([sys.executable, "-c", prog], env=env, capture_output=True, text=True, timeout=600)
    assert r1.returncode == 0, r1.stderr
    files = sorted(p.name for p in tmp_path.iterdir())
    assert files and all(f.startswith("qsv_") and f.endswith(".co") for f in files)
    r2 = subprocess.run([sys.executable, "-c", prog], env=env, capture_output=True, text=True, timeout=600)
    assert r2.returncode == 0, r2.stderr
    b1, t1 = r1.stdout.split()
    b2, t2 = r2.stdout.split()
    assert b1 == b2
    assert float(t2) < 0.5 * float(t1)
    assert sorted(p.name for p in tmp_path.iterdir()) == files
