"""GPU tests of the boundary's ownership rules: sweeps take a caller-owned
workspace (sv_workspace_bytes) for the second state buffer of out-of-place
passes and the FP64 partial sums, and the library keeps none of its own.
Two out-of-place sweeps in flight at once on two streams, each with its own
workspace, must both match the oracle.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import circuit as OC  # noqa: E402
from oracle import sim  # noqa: E402
from paper_1804_04797_amd import qsv  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
OOP = {"reg_qubits": 5, "thread_qubits": 8, "low_qubits": 4, "jit": 1, "out_of_place": 1}


def _oracle_state(rows, cols, depth, seed):
    gates = OC.random_circuit(OC.Lattice(rows, cols), depth, seed)
    return sim.simulate(gates, rows * cols)


def test_two_streams_out_of_place_own_workspaces():
    rows, cols, depth = 4, 6, 14
    seeds = (11, 12)
    circs = [qsv.circuit_create(rows, cols, None, depth, s) for s in seeds]
    n = rows * cols
    states = [torch.empty(1 << n, dtype=torch.complex64, device=DEV) for _ in seeds]
    wss = [qsv.alloc_workspace(c, 0, -1, OOP) for c in circs]
    assert all(w.numel() == qsv.sv_workspace_bytes(circs[0], 0, -1, OOP) for w in wss)
    assert wss[0].numel() >= 8 << n
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for rep in range(2):  # the second round replays the same plans
        for a, c, w, s in zip(states, circs, wss, streams):
            with torch.cuda.stream(s):
                qsv.sv_init(a, n, qsv.INIT_ZERO, stream=s)
                qsv.sv_apply_fused(a, c, opts=OOP, workspace=w, stream=s)
        torch.cuda.synchronize()
        for a, seed in zip(states, seeds):
            ref = _oracle_state(rows, cols, depth, seed)
            got = a.cpu().numpy().astype(np.complex128)
            d = float(np.max(np.abs(got - ref)))
            assert d <= 1e-5 and d * 2 ** (n / 2) <= 1e-4, (rep, seed, d)


def test_forced_out_of_place_needs_the_workspace():
    # a sweep whose first pass generates the state runs out of place with any
    # pass count, so forcing it needs the second buffer in the workspace
    c = qsv.circuit_create(4, 6, None, 10, 3)
    n = 24
    a = torch.empty(1 << n, dtype=torch.complex64, device=DEV)
    qsv.sv_init(a, n, qsv.INIT_ZERO)
    before = a.clone()
    small = torch.empty(1 << 20, dtype=torch.uint8, device=DEV)
    for ws in (small, False):
        with pytest.raises(qsv.QsvError) as e:
            qsv.sv_simulate(a, c, init_kind=qsv.INIT_PLUS, layer_begin=1, opts=OOP, workspace=ws)
        assert e.value.status == 1
        with pytest.raises(qsv.QsvError) as e:
            qsv.sv_apply_fused_from(before, a, c, layer_begin=1, opts=OOP, workspace=ws)
        assert e.value.status == 1
    torch.cuda.synchronize()
    assert torch.equal(a, before)  # nothing was enqueued
    # automatic mode without room for the second buffer runs in place
    auto = dict(OOP, out_of_place=0)
    qsv.sv_simulate(a, c, init_kind=qsv.INIT_PLUS, layer_begin=1, opts=auto, workspace=False)
    b = torch.empty_like(a)
    qsv.sv_simulate(b, c, init_kind=qsv.INIT_PLUS, layer_begin=1, opts=OOP)
    torch.cuda.synchronize()
    assert float((a - b).abs().max()) <= 1e-6


def test_norm_needs_a_workspace():
    c = qsv.circuit_create(4, 6, None, 8, 4)
    n = 24
    a = torch.empty(1 << n, dtype=torch.complex64, device=DEV)
    nrm = torch.zeros(1, dtype=torch.float64, device=DEV)
    for jit in (-1, 1):
        with pytest.raises(qsv.QsvError) as e:
            qsv.sv_simulate(a, c, init_kind=qsv.INIT_PLUS, layer_begin=1, opts={"jit": jit},
                            norm_out=nrm, workspace=False)
        assert e.value.status == 1
        qsv.sv_simulate(a, c, init_kind=qsv.INIT_PLUS, layer_begin=1, opts={"jit": jit}, norm_out=nrm)
        torch.cuda.synchronize()
        assert abs(nrm.item() - 1.0) < 1e-5


@pytest.mark.parametrize("nbytes", [16, 16 * 2047, 16 * (1 << 20) + 48, 1 << 28])
def test_stream_copy_exact(nbytes):
    g = torch.Generator().manual_seed(nbytes % 1000)
    src = torch.randint(0, 256, (nbytes + 32,), dtype=torch.uint8, generator=g).to(DEV)
    dst = torch.zeros(nbytes + 32, dtype=torch.uint8, device=DEV)
    qsv.sv_stream_copy(src, dst, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert int(dst[nbytes:].abs().sum()) == 0  # nothing past the end
    with pytest.raises(qsv.QsvError):
        qsv.sv_stream_copy(src, dst, nbytes + 8)
    with pytest.raises(qsv.QsvError):
        qsv.sv_stream_copy(src, src[16:], 64)


def test_amplitudes_refuse_out_of_range_bitstrings():
    """A bitstring >= 2^n: QSV_ERANGE and nothing enqueued (the output keeps
    its contents); in range, the gather returns the state's entries."""
    n = 16
    g = torch.Generator().manual_seed(7)
    st = torch.complex(torch.randn(1 << n, generator=g), torch.randn(1 << n, generator=g)).to(DEV)
    out = torch.full((3,), complex(7.0, -7.0), dtype=torch.complex64, device=DEV)
    bad = torch.tensor([0, 5, 1 << n], dtype=torch.int64, device=DEV)
    with pytest.raises(qsv.QsvError) as e:
        qsv.sv_amplitudes(st, n, bad, out)
    assert e.value.status == 2
    torch.cuda.synchronize()
    assert torch.all(out == complex(7.0, -7.0))
    good = torch.tensor([0, 5, (1 << n) - 1], dtype=torch.int64, device=DEV)
    qsv.sv_amplitudes(st, n, good, out)
    torch.cuda.synchronize()
    assert torch.equal(out.cpu(), st.cpu()[[0, 5, (1 << n) - 1]])


@pytest.mark.parametrize("jit", [1, -1])
def test_simulate_with_out_of_range_bitstring_enqueues_nothing(jit):
    """sv_simulate (compiled and generic path) refuses a bitstring >= 2^n
    before it enqueues anything: the state and the outputs keep their
    contents."""
    c = qsv.circuit_create(4, 5, None, 10, 99)
    n = 20
    opts = {"reg_qubits": 5, "thread_qubits": 8, "low_qubits": 4, "jit": jit}
    amps = torch.full((1 << n,), complex(3.0, 1.0), dtype=torch.complex64, device=DEV)
    out = torch.full((2,), complex(7.0, -7.0), dtype=torch.complex64, device=DEV)
    nrm = torch.full((1,), -1.0, dtype=torch.float64, device=DEV)
    xs = torch.tensor([1, 1 << (n + 3)], dtype=torch.int64, device=DEV)
    with pytest.raises(qsv.QsvError) as e:
        qsv.sv_simulate(amps, c, init_kind=qsv.INIT_PLUS, layer_begin=1, opts=opts, norm_out=nrm,
                        bitstrings=xs, amps_out=out)
    assert e.value.status == 2
    torch.cuda.synchronize()
    assert torch.all(amps == complex(3.0, 1.0))
    assert torch.all(out == complex(7.0, -7.0))
    assert nrm.item() == -1.0


def test_tune_and_code_caches_across_processes(tmp_path):
    """QSV_TUNE_CACHE and QSV_JIT_CACHE: a second process takes the tuned
    options from the file and the compiled kernels from the directory, so its
    set-up (tune + first sweep) is a small fraction of the first one's, with
    the same options and the same amplitudes."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    prog = (
        "import sys, time, json; sys.path.insert(0, %r)\n"
        "import torch\n"
        "from paper_1804_04797_amd import qsv\n"
        "c = qsv.circuit_create(4, 6, None, 14, 31)\n"
        "a = torch.empty(1 << 24, dtype=torch.complex64, device='cuda:0')\n"
        "t = time.time(); o, _ = qsv.sv_tune(a, c, layer_begin=1)\n"
        "qsv.sv_simulate(a, c, init_kind=qsv.INIT_PLUS, layer_begin=1); torch.cuda.synchronize()\n"
        "dt = time.time() - t\n"
        "print(json.dumps({'opts': o, 's': dt, 'a': [float(x) for x in a[:8].abs().cpu()]}))\n"
    ) % root
    env = dict(os.environ, QSV_TUNE_CACHE=str(tmp_path / "tune.txt"), QSV_JIT_CACHE=str(tmp_path))
    outs = []
    for _ in range(2):
        r = subprocess.run([sys.executable, "-c", prog], env=env, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(json.loads([ln for ln in r.stdout.splitlines() if ln.startswith("{")][-1]))
    assert outs[0]["opts"] == outs[1]["opts"]
    assert outs[0]["a"] == outs[1]["a"]
    assert outs[1]["s"] < 0.5 * outs[0]["s"], (outs[0]["s"], outs[1]["s"])
    assert (tmp_path / "tune.txt").read_text().count("\n") == 1
