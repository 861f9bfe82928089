"""GPU tests of batched execution: the size classes (a whole state in one
tile for 2^14 amplitudes or fewer, the batch's tile shape below 2^21, compiled
kernels from 2^21) against the oracle.  The persistent launch over (pass
round, entry, tile) work items is switched off (its tests are skipped with
the reason); asking for it is refused."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import circuit as OC  # noqa: E402
from oracle import sim  # noqa: E402
from paper_1804_04797_amd import qsv, workloads  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = 1e-5
TOL_SCALED = 1e-4


def _items(spec, seed0):
    items = []
    for i, (n, d) in enumerate(spec):
        rows, cols, pres = workloads.lattice_for_qubits(n)
        seed = seed0 + i
        items.append((qsv.circuit_create(rows, cols, pres, d, seed),
                      OC.random_circuit(OC.Lattice.for_qubits(n), d, seed), n))
    return items


def _refs(items):
    out = []
    for _, gates, n in items:
        psi = np.full(1 << n, 2.0 ** (-n / 2), np.complex128)
        out.append(sim.run(psi, n, [g for g in gates if g[3] >= 1]))
    return out


def _check(st, ref, n):
    got = st.cpu().numpy().astype(np.complex128)
    d = float(np.max(np.abs(got - ref)))
    assert d <= TOL and d * 2 ** (n / 2) <= TOL_SCALED, (n, d)


def _batch(items, env=None):
    old = {}
    for k, v in (env or {}).items():
        old[k] = os.environ.get(k)
        os.environ[k] = v
    try:
        return qsv.sv_batch_create([c for c, _, _ in items])
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.skip(reason="this case did not finish on the device when the batch ran it with the persistent launch "
                         "(a 120 s timeout in sv_batch_status); that launch is now refused, but the case stays off "
                         "the device until the cause is found; test_batch_whole_state_tiles_replayed covers the "
                         "whole-state class with per-round launches")
def test_batch_every_size_class_replayed():
    """11..14 qubits (whole state in one tile), 15 and 18 (batch tile), 21 and
    22 (compiled kernels at the default and at a tuned tile shape): every
    state against the oracle, over three replays with eager work between."""
    items = _items([(11, 9), (12, 14), (13, 20), (14, 24), (15, 12), (18, 16), (21, 10), (22, 12)], 0xB47C)
    qsv.sv_tune_set(items[7][0], dict(reg_qubits=4, thread_qubits=7, low_qubits=4, plain=0, jit=1), layer_begin=1)
    b = _batch(items)
    states = [torch.empty(1 << n, dtype=torch.complex64, device=DEV) for _, _, n in items]
    refs = _refs(items)
    for rep in range(3):
        qsv.sv_batch_run(b, states, init_plus=True)
        qsv.sv_batch_status(b)
        for st, ref, (_, _, n) in zip(states, refs, items):
            _check(st, ref, n)
        for st in states:
            st.zero_()
        torch.cuda.synchronize()


def test_batch_whole_state_tiles_replayed():
    """States of 11..14 qubits (each on one tile that holds it whole) beside
    15- and 17-qubit states on the batch tile, per-round launches: every
    state against the oracle over two replays with eager work between."""
    items = _items([(11, 9), (12, 14), (13, 20), (14, 24), (14, 9), (15, 12), (17, 10)], 0x1D5)
    b = _batch(items)
    states = [torch.empty(1 << n, dtype=torch.complex64, device=DEV) for _, _, n in items]
    refs = _refs(items)
    for rep in range(2):
        print(f"replay {rep}", flush=True)
        qsv.sv_batch_run(b, states, init_plus=True)
        qsv.sv_batch_status(b)
        for st, ref, (_, _, n) in zip(states, refs, items):
            _check(st, ref, n)
        for st in states:
            st.zero_()
        torch.cuda.synchronize()


def test_batch_21_and_22_qubit_entries():
    """The compiled class's lower edge: states of 21 and 22 qubits (compiled
    kernels from 2^21 amplitudes), one at the default tile shape and one at a
    shape set with sv_tune_set, beside 16- and 13-qubit states of the generic
    classes; every state against the oracle."""
    items = _items([(21, 10), (22, 12), (16, 10), (13, 12)], 0x2122)
    qsv.sv_tune_set(items[1][0], dict(reg_qubits=4, thread_qubits=7, low_qubits=4, plain=0, jit=1), layer_begin=1)
    b = _batch(items)
    states = [torch.empty(1 << n, dtype=torch.complex64, device=DEV) for _, _, n in items]
    qsv.sv_batch_run(b, states, init_plus=True)
    qsv.sv_batch_status(b)
    for st, ref, (_, _, n) in zip(states, _refs(items), items):
        _check(st, ref, n)


PERSISTENT_OFF = ("the persistent batch launch is switched off: its first two runs on the device did not "
                  "finish (a run killed for silence, then a 120 s test timeout in sv_batch_status) and the "
                  "cause is not yet found")


@pytest.mark.skip(reason=PERSISTENT_OFF)
@pytest.mark.parametrize("count,nrange,seed", [(40, (11, 19), 3), (7, (15, 20), 4)])
def test_persistent_launch_matches_round_launches(count, nrange, seed):
    """The persistent launch (work items in order, per-entry counters) gives
    the per-round launches' states bit for bit (same tile arithmetic), and
    both match the oracle."""
    rng = np.random.default_rng(seed)
    spec = [(int(rng.integers(nrange[0], nrange[1] + 1)), int(rng.integers(6, 20))) for _ in range(count)]
    items = _items(spec, 0x9E5 + seed)
    bp = _batch(items)
    br = _batch(items, {"QSV_BATCH_PERSISTENT": "0"})
    sp = [torch.empty(1 << n, dtype=torch.complex64, device=DEV) for _, _, n in items]
    sr = [torch.empty_like(x) for x in sp]
    qsv.sv_batch_run(bp, sp, init_plus=True)
    qsv.sv_batch_run(br, sr, init_plus=True)
    qsv.sv_batch_status(bp)
    qsv.sv_batch_status(br)
    for a, b in zip(sp, sr):
        assert torch.equal(a, b)
    for st, ref, (_, _, n) in zip(sp, _refs(items), items):
        _check(st, ref, n)


@pytest.mark.skip(reason=PERSISTENT_OFF)
def test_persistent_wait_gives_up_on_abort_and_recovers():
    """With the abort flag set from the host, the waits of a persistent
    launch give up at once (every workgroup still drains); sv_batch_status
    reports it and clears the flag, and the next run is correct again."""
    items = _items([(20, 16)], 0xAB0)
    b = _batch(items)
    st = [torch.empty(1 << 20, dtype=torch.complex64, device=DEV)]
    qsv.sv_batch_run(b, st, init_plus=True)
    qsv.sv_batch_status(b)
    qsv.sv_batch_abort(b)
    qsv.sv_batch_run(b, st, init_plus=True)
    with pytest.raises(qsv.QsvError) as e:
        qsv.sv_batch_status(b)
    assert e.value.status == 6
    qsv.sv_batch_run(b, st, init_plus=True)
    qsv.sv_batch_status(b)
    _check(st[0], _refs(items)[0], 20)


def test_persistent_launch_is_refused():
    items = _items([(16, 8)], 0x5EF)
    with pytest.raises(qsv.QsvError) as e:
        _batch(items, {"QSV_BATCH_PERSISTENT": "1"})
    assert e.value.status == 5
