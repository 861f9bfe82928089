"""Thin ctypes binding of libqsv.so (argument marshalling only).

Every function mirrors the C entry point of the same name in include/qsv.h.
Device buffers may be given as torch tensors (their data_ptr() is used) or as
integer device addresses; `stream` defaults to torch's current stream.  The
library must be built (paper_1804_04797_amd/build.py); importing this module
without it raises, so no code path silently runs without the HIP kernels.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsv.so")

GATE_DTYPE = np.dtype([("kind", "u1"), ("q0", "u1"), ("q1", "u1"), ("arg", "u1"),
                       ("layer", "<u2"), ("reserved", "<u2")])
KIND = {"H": 0, "T": 1, "SX": 2, "SY": 3, "CZ": 4, "P0": 5, "P1": 6, "Z": 7, "TDG": 8,
        "SXDG": 9, "SYDG": 10, "PB": 11, "ZB": 12}
KIND_NAME = {v: k for k, v in KIND.items()}
INIT_ZERO, INIT_PLUS, INIT_BASIS = 0, 1, 2
STATUS = {0: "QSV_OK", 1: "QSV_EINVAL", 2: "QSV_ERANGE", 3: "QSV_ENOMEM", 4: "QSV_EHIP",
          5: "QSV_EUNSUPPORTED", 6: "QSV_EINTERNAL"}

EXPORTS = ["circuit_create", "circuit_destroy", "circuit_info", "circuit_gates",
           "circuit_split", "sv_init", "sv_apply_fused", "sv_apply_plain", "sv_amplitudes",
           "sv_norm_fp64", "sv_branch_combine", "sv_simulate", "sv_simulate_c128", "sv_batch_create", "sv_batch_run",
           "sv_batch_destroy", "sv_plan_info", "sv_debug_emulate", "sv_debug_jit_compile",
           "sv_tune", "sv_apply_dense", "sv_debug_emulate_dense", "qsv_release_device_buffers",
           "circuit_inverse", "sv_inner_product", "sv_branch_combine_full",
           "circuit_partition_plan", "circuit_partition_create", "circuit_partition_info",
           "circuit_partition_offsets", "circuit_partition_parts", "circuit_partition_destroy",
           "sv_partition_workspace_bytes", "sv_partition_simulate", "sv_apply_fused_from",
           "sv_simulate_dot", "sv_sampler_create", "sv_sampler_run", "sv_sampler_destroy", "sv_sampler_run_branches", "sv_sampler_run_subtree",
           "sv_sampler_create_tiles", "sv_sampler_inputs",
           "circuit_branch_levels", "circuit_branch_stage", "sv_tune_set",
           "qsv_last_error", "qsv_version", "sv_norm_fp64_noalloc", "sv_workspace_bytes",
           "sv_stream_copy", "sv_batch_status", "sv_batch_abort", "sv_debug_batch_schedule"]


class QsvError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class FuseOpts(ctypes.Structure):
    _fields_ = [("reg_qubits", ctypes.c_int), ("thread_qubits", ctypes.c_int),
                ("low_qubits", ctypes.c_int), ("plain", ctypes.c_int), ("jit", ctypes.c_int),
                ("out_of_place", ctypes.c_int), ("pass_forms", ctypes.c_uint32)]


class PartitionInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int) for k in ("r0", "t_s", "depth", "cols", "n_a", "n_b", "n_c", "cuts",
                                            "explicit_bits", "sel_a", "sel_b", "folded", "f", "g")] + [
        ("objective", ctypes.c_double), ("branches_a", ctypes.c_uint64), ("branches_b", ctypes.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1804_04797_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, u64, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_int
    st = ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "circuit_create": (st, [i32, i32, vp, i32, u64, vp, sz, P(vp)]),
        "circuit_destroy": (None, [vp]),
        "circuit_info": (st, [vp, P(i32), P(i32), P(sz)]),
        "circuit_gates": (st, [vp, vp, sz, P(sz)]),
        "circuit_split": (st, [vp, u64, P(vp), P(vp), P(i32), vp, vp, sz, P(sz)]),
        "sv_init": (st, [vp, i32, i32, u64, vp]),
        "sv_apply_fused": (st, [vp, vp, u64, i32, i32, vp, vp, sz, vp]),
        "sv_workspace_bytes": (st, [vp, i32, i32, vp, P(sz)]),
        "sv_apply_plain": (st, [vp, vp, u64, i32, i32, vp]),
        "sv_apply_fused_from": (st, [vp, vp, vp, u64, i32, i32, vp, vp, sz, vp]),
        "sv_simulate_dot": (st, [vp, vp, u64, i32, u64, i32, i32, vp, vp, vp, vp, sz, vp]),
        "sv_sampler_create": (st, [vp, i32, i32, vp, vp, sz, P(vp)]),
        "sv_sampler_run": (st, [vp, vp, vp, u64, vp, vp, sz, vp]),
        "sv_sampler_destroy": (None, [vp]),
        "sv_sampler_run_branches": (st, [vp, vp, vp, vp, sz, vp, vp, sz, vp]),
        "sv_sampler_run_subtree": (st, [vp, vp, vp, u64, u64, vp, vp, sz, vp]),
        "sv_sampler_create_tiles": (st, [vp, i32, i32, vp, vp, sz, P(vp)]),
        "sv_sampler_inputs": (st, [vp, vp, sz, P(sz)]),
        "sv_simulate": (st, [vp, vp, u64, i32, u64, i32, i32, vp, vp, vp, sz, vp, i32, vp, sz, vp]),
        "sv_simulate_c128": (st, [vp, vp, u64, i32, u64, i32, i32, vp, vp, sz, vp, vp, sz, vp]),
        "sv_amplitudes": (st, [vp, i32, vp, sz, vp, i32, vp]),
        "sv_norm_fp64": (st, [vp, i32, vp, vp]),
        "sv_norm_fp64_noalloc": (st, [vp, i32, vp, vp]),
        "sv_stream_copy": (st, [vp, vp, sz, vp]),
        "sv_branch_combine": (st, [vp, vp, sz, sz, vp, vp, vp]),
        "sv_batch_create": (st, [vp, vp, sz, vp, P(vp)]),
        "sv_batch_run": (st, [vp, vp, i32, vp, sz, vp, vp]),
        "sv_batch_destroy": (None, [vp]),
        "sv_batch_status": (st, [vp, vp]),
        "sv_batch_abort": (st, [vp]),
        "sv_debug_batch_schedule": (st, [vp, vp, sz, i32, i32, u64, i32, P(u64)]),
        "sv_plan_info": (st, [vp, i32, i32, vp, P(i32), vp, vp, sz, vp, sz]),
        "sv_debug_emulate": (st, [vp, vp, u64, i32, i32, vp]),
        "sv_debug_jit_compile": (st, [vp, i32, i32, vp, P(sz), P(ctypes.c_double)]),
        "qsv_release_device_buffers": (st, []),
        "circuit_inverse": (st, [vp, P(vp)]),
        "circuit_branch_levels": (st, [vp, P(i32), vp, sz]),
        "sv_tune_set": (st, [vp, i32, i32, vp]),
        "circuit_branch_stage": (st, [vp, i32, i32, P(vp)]),
        "sv_inner_product": (st, [vp, vp, i32, vp, vp]),
        "sv_branch_combine_full": (st, [vp, vp, sz, i32, i32, u64, vp, vp, sz, vp, i32, vp]),
        "sv_tune": (st, [vp, vp, i32, i32, vp, sz, vp, P(ctypes.c_double), vp]),
        "sv_apply_dense": (st, [vp, vp, u64, i32, i32, i32, P(i32), vp]),
        "sv_debug_emulate_dense": (st, [vp, vp, u64, i32, i32, i32, P(i32)]),
        "circuit_partition_plan": (st, [vp, i32, i32, vp, i32, i32, P(vp)]),
        "circuit_partition_create": (st, [vp, i32, i32, vp, i32, i32, vp, vp, P(vp)]),
        "circuit_partition_info": (st, [vp, vp]),
        "circuit_partition_offsets": (st, [vp, vp, vp, sz]),
        "circuit_partition_parts": (st, [vp, P(vp), P(vp), P(vp), vp, vp]),
        "circuit_partition_destroy": (None, [vp]),
        "sv_partition_workspace_bytes": (st, [vp, P(sz)]),
        "sv_partition_simulate": (st, [vp, vp, sz, vp, vp]),
        "qsv_last_error": (ctypes.c_char_p, []),
        "qsv_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status):
    if status != 0:
        raise QsvError(status, lib().qsv_last_error().decode())


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take a device pointer of {type(x)}")


def _stream(stream):
    if stream is not None:
        return stream if isinstance(stream, int) else getattr(stream, "cuda_stream", stream)
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


def _nbytes(x):
    if hasattr(x, "numel") and hasattr(x, "element_size"):
        return x.numel() * x.element_size()
    if isinstance(x, np.ndarray):
        return x.nbytes
    raise TypeError(f"cannot size a workspace of {type(x)}")


def _device_present():
    import torch
    return torch.cuda.is_available()


def sv_workspace_bytes(c, layer_begin=0, layer_end=-1, opts=None) -> int:
    b = ctypes.c_size_t()
    _check(lib().sv_workspace_bytes(c, layer_begin, layer_end, _opts(opts), ctypes.byref(b)))
    return b.value


def alloc_workspace(c, layer_begin=0, layer_end=-1, opts=None, device=None):
    """A device buffer of sv_workspace_bytes bytes (torch uint8 tensor)."""
    import torch
    return torch.empty(sv_workspace_bytes(c, layer_begin, layer_end, opts), dtype=torch.uint8,
                       device=device if device is not None else torch.device("cuda", torch.cuda.current_device()))


def _ws(workspace, c, layer_begin, layer_end, opts, stream):
    """(pointer, bytes, keep-alive) of a sweep call's workspace.  None: a
    buffer of sv_workspace_bytes bytes from torch's allocator on the current
    device (kept by the caller's frame for the call; torch reuses it only
    after the work queued on the stream it was allocated for); False: none;
    a tensor or array: its memory; a (pointer, bytes) pair: as given."""
    if workspace is False:
        return None, 0, None
    if workspace is None:
        import torch
        if not torch.cuda.is_available():  # no device: the call fails its own checks
            return None, 0, None
        t = alloc_workspace(c, layer_begin, layer_end, opts)
        if stream is not None and not isinstance(stream, int) and hasattr(stream, "cuda_stream"):
            t.record_stream(stream)
        return t.data_ptr(), _nbytes(t), t
    if isinstance(workspace, tuple):
        return workspace[0], workspace[1], None
    return _ptr(workspace), _nbytes(workspace), workspace


def _opts(opts):
    if opts is None:
        return None
    if isinstance(opts, FuseOpts):
        return ctypes.byref(opts)
    o = FuseOpts(**{"jit": 0, **opts})
    return ctypes.byref(o)


class Circuit:
    """Owning handle of a qsv_circuit."""

    def __init__(self, handle):
        self.handle = ctypes.c_void_p(handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.circuit_destroy(h)
            self.handle = None

    @property
    def _as_parameter_(self):
        return self.handle

    def info(self):
        return circuit_info(self)

    @property
    def n(self):
        return circuit_info(self)[0]

    def gates(self):
        return circuit_gates(self)


def circuit_create(rows, cols, present=None, depth=0, seed=0, gates=None) -> Circuit:
    L = lib()
    pres = None
    if present is not None:
        pres = np.ascontiguousarray(np.asarray(present, dtype=np.uint8).reshape(-1))
    g = None
    ng = 0
    if gates is not None:
        g = np.ascontiguousarray(np.asarray(gates, dtype=GATE_DTYPE))
        ng = g.size
    out = ctypes.c_void_p()
    _check(L.circuit_create(rows, cols, _ptr(pres) if pres is not None else None, depth,
                            ctypes.c_uint64(seed), _ptr(g) if g is not None else None, ng,
                            ctypes.byref(out)))
    return Circuit(out.value)


def circuit_info(c):
    n, d, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
    _check(lib().circuit_info(c, ctypes.byref(n), ctypes.byref(d), ctypes.byref(g)))
    return n.value, d.value, g.value


def circuit_gates(c) -> np.ndarray:
    _, _, ng = circuit_info(c)
    out = np.zeros(ng, GATE_DTYPE)
    k = ctypes.c_size_t()
    _check(lib().circuit_gates(c, _ptr(out), ng, ctypes.byref(k)))
    return out[: k.value]


def circuit_split(c, side_a_mask: int):
    ha, hb = ctypes.c_void_p(), ctypes.c_void_p()
    ceff = ctypes.c_int()
    nf = ctypes.c_size_t()
    cap = 4096
    fa = np.zeros(cap, np.int32)
    fb = np.zeros(cap, np.int32)
    _check(lib().circuit_split(c, ctypes.c_uint64(side_a_mask), ctypes.byref(ha),
                               ctypes.byref(hb), ctypes.byref(ceff), _ptr(fa), _ptr(fb), cap,
                               ctypes.byref(nf)))
    k = min(nf.value, cap)
    return Circuit(ha.value), Circuit(hb.value), ceff.value, list(zip(fa[:k].tolist(),
                                                                        fb[:k].tolist()))


def sv_init(amps, n_qubits, kind=INIT_ZERO, basis=0, stream=None):
    _check(lib().sv_init(_ptr(amps), n_qubits, kind, ctypes.c_uint64(basis), _stream(stream)))


def sv_apply_fused(amps, c, branch=0, layer_begin=0, layer_end=-1, opts=None, stream=None,
                   workspace=None):
    wp, wb, _keep = _ws(workspace, c, layer_begin, layer_end, opts, stream)
    _check(lib().sv_apply_fused(_ptr(amps), c, ctypes.c_uint64(branch), layer_begin, layer_end,
                                _opts(opts), wp, wb, _stream(stream)))


def sv_simulate(amps, c, branch=0, init_kind=INIT_ZERO, basis=0, layer_begin=0, layer_end=-1,
                opts=None, norm_out=None, bitstrings=None, amps_out=None, c128=False,
                stream=None, workspace=None):
    m = 0
    if amps_out is not None:
        m = amps_out.numel() if hasattr(amps_out, "numel") else len(amps_out)
    wp, wb, _keep = _ws(workspace, c, layer_begin, layer_end, opts, stream)
    _check(lib().sv_simulate(_ptr(amps), c, ctypes.c_uint64(branch), init_kind,
                             ctypes.c_uint64(basis), layer_begin, layer_end, _opts(opts),
                             _ptr(norm_out), _ptr(bitstrings), m, _ptr(amps_out),
                             1 if c128 else 0, wp, wb, _stream(stream)))


def sv_simulate_c128(amps, c, branch=0, init_kind=INIT_ZERO, basis=0, layer_begin=0,
                     layer_end=-1, norm_out=None, bitstrings=None, amps_out=None, stream=None,
                     workspace=None):
    m = 0
    if amps_out is not None:
        m = amps_out.numel() if hasattr(amps_out, "numel") else len(amps_out)
    if workspace is None and norm_out is None:
        workspace = False
    if workspace is None and _device_present():  # the norm's partial sums only (in place)
        workspace = alloc_workspace(c, layer_begin, layer_end, {"reg_qubits": 4, "thread_qubits": 8,
                                                               "low_qubits": 4, "jit": -1})
    wp, wb, _keep = _ws(workspace, c, layer_begin, layer_end, None, stream)
    _check(lib().sv_simulate_c128(_ptr(amps), c, ctypes.c_uint64(branch), init_kind,
                                  ctypes.c_uint64(basis), layer_begin, layer_end, _ptr(norm_out),
                                  _ptr(bitstrings), m, _ptr(amps_out), wp, wb, _stream(stream)))


def sv_apply_fused_from(src, dst, c, branch=0, layer_begin=0, layer_end=-1, opts=None, stream=None,
                        workspace=None):
    wp, wb, _keep = _ws(workspace, c, layer_begin, layer_end, opts, stream)
    _check(lib().sv_apply_fused_from(_ptr(src), _ptr(dst), c, ctypes.c_uint64(branch), layer_begin,
                                     layer_end, _opts(opts), wp, wb, _stream(stream)))


def sv_simulate_dot(amps, c, other, out_dev, branch=0, init_kind=INIT_ZERO, basis=0, layer_begin=0,
                    layer_end=-1, opts=None, stream=None, workspace=None):
    """out_dev (device float64[2]) = <U init | other>; amps is a work buffer."""
    wp, wb, _keep = _ws(workspace, c, layer_begin, layer_end, opts, stream)
    _check(lib().sv_simulate_dot(_ptr(amps), c, ctypes.c_uint64(branch), init_kind, ctypes.c_uint64(basis),
                                 layer_begin, layer_end, _opts(opts), _ptr(other), _ptr(out_dev),
                                 wp, wb, _stream(stream)))


def sv_apply_plain(amps, c, branch=0, layer_begin=0, layer_end=-1, stream=None):
    _check(lib().sv_apply_plain(_ptr(amps), c, ctypes.c_uint64(branch), layer_begin, layer_end,
                                _stream(stream)))


def sv_amplitudes(amps, n_qubits, bitstrings, out, c128=False, stream=None):
    m = out.numel() if hasattr(out, "numel") else len(bitstrings)
    _check(lib().sv_amplitudes(_ptr(amps), n_qubits, _ptr(bitstrings), m, _ptr(out),
                               1 if c128 else 0, _stream(stream)))


def sv_norm_fp64(amps, n_qubits, out, stream=None):
    _check(lib().sv_norm_fp64(_ptr(amps), n_qubits, _ptr(out), _stream(stream)))


def sv_stream_copy(src, dst, nbytes, stream=None):
    _check(lib().sv_stream_copy(_ptr(src), _ptr(dst), nbytes, _stream(stream)))


def sv_norm_fp64_noalloc(amps, n_qubits, out, stream=None):
    _check(lib().sv_norm_fp64_noalloc(_ptr(amps), n_qubits, _ptr(out), _stream(stream)))


def sv_branch_combine(a_tab, b_tab, n_branches, m, sign, out, stream=None):
    _check(lib().sv_branch_combine(_ptr(a_tab), _ptr(b_tab), n_branches, m, _ptr(sign),
                                   _ptr(out), _stream(stream)))


class Batch:
    """Owning handle of a qsv_batch; keeps its circuits alive."""

    def __init__(self, handle, circuits):
        self.handle = ctypes.c_void_p(handle)
        self.circuits = list(circuits)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.sv_batch_destroy(h)
            self.handle = None

    @property
    def _as_parameter_(self):
        return self.handle


def sv_batch_create(circuits, branch_ids=None, opts=None) -> Batch:
    arr = (ctypes.c_void_p * len(circuits))(*[c.handle.value for c in circuits])
    br = None
    if branch_ids is not None:
        br = np.ascontiguousarray(np.asarray(branch_ids, dtype=np.uint64))
        assert br.size == len(circuits)
    out = ctypes.c_void_p()
    _check(lib().sv_batch_create(arr, _ptr(br) if br is not None else None, len(circuits),
                                 _opts(opts), ctypes.byref(out)))
    return Batch(out.value, circuits)


def sv_batch_run(batch, amps_list, init_plus=False, bitstrings=None, m=0, amp_table=None,
                 stream=None):
    arr = (ctypes.c_void_p * len(amps_list))(*[_ptr(a) for a in amps_list])
    _check(lib().sv_batch_run(batch, arr, 1 if init_plus else 0, _ptr(bitstrings), m,
                              _ptr(amp_table), _stream(stream)))


def sv_batch_status(batch, stream=None):
    _check(lib().sv_batch_status(batch, _stream(stream)))


def sv_batch_abort(batch):
    _check(lib().sv_batch_abort(batch))


def sv_debug_batch_schedule(n_qubits, passes, tile_qubits, workers, seed=1, planted_early_start=False) -> int:
    """Host emulation of a persistent batch launch's schedule; returns the
    number of work items (raises if the ordering rule is violated)."""
    nq = np.ascontiguousarray(np.asarray(n_qubits, dtype=np.int32))
    pp = np.ascontiguousarray(np.asarray(passes, dtype=np.int32))
    items = ctypes.c_uint64()
    _check(lib().sv_debug_batch_schedule(_ptr(nq), _ptr(pp), nq.size, tile_qubits, workers,
                                         ctypes.c_uint64(seed), 1 if planted_early_start else 0,
                                         ctypes.byref(items)))
    return items.value


def sv_plan_info(c, layer_begin=0, layer_end=-1, opts=None):
    n, _, ng = circuit_info(c)
    npass = ctypes.c_int()
    pog = np.zeros(ng, np.int32)
    oip = np.zeros(ng, np.int32)
    res = np.zeros(4096, np.uint64)
    _check(lib().sv_plan_info(c, layer_begin, layer_end, _opts(opts), ctypes.byref(npass),
                              _ptr(pog), _ptr(oip), ng, _ptr(res), res.size))
    return {"n_passes": npass.value, "pass_of_gate": pog, "order_in_pass": oip,
            "resident": [int(x) for x in res[: npass.value]]}


def sv_debug_emulate(amps_host: np.ndarray, c, branch=0, layer_begin=0, layer_end=-1,
                     opts=None):
    assert amps_host.dtype == np.complex64 and amps_host.flags.c_contiguous
    _check(lib().sv_debug_emulate(_ptr(amps_host), c, ctypes.c_uint64(branch), layer_begin,
                                  layer_end, _opts(opts)))


def sv_debug_jit_compile(c, layer_begin=0, layer_end=-1, opts=None):
    nb = ctypes.c_size_t()
    sec = ctypes.c_double()
    _check(lib().sv_debug_jit_compile(c, layer_begin, layer_end, _opts(opts), ctypes.byref(nb),
                                      ctypes.byref(sec)))
    return nb.value, sec.value


def circuit_inverse(c) -> Circuit:
    out = ctypes.c_void_p()
    _check(lib().circuit_inverse(c, ctypes.byref(out)))
    return Circuit(out.value)


def sv_tune_set(c, opts, layer_begin=0, layer_end=-1):
    _check(lib().sv_tune_set(c, layer_begin, layer_end, _opts(opts)))


def circuit_branch_levels(c) -> list:
    """Branch-bit masks of levels 1..L (see qsv.h)."""
    n = ctypes.c_int()
    bits = np.zeros(64, np.uint64)
    _check(lib().circuit_branch_levels(c, ctypes.byref(n), _ptr(bits), bits.size))
    return [int(x) for x in bits[: n.value]]


def circuit_branch_stage(c, level_begin, level_end=-1) -> Circuit:
    out = ctypes.c_void_p()
    _check(lib().circuit_branch_stage(c, level_begin, level_end, ctypes.byref(out)))
    return Circuit(out.value)


def sv_inner_product(a, b, n_qubits, out_dev, stream=None):
    """<a|b> in FP64 into out_dev (device float64[2] = re, im)."""
    _check(lib().sv_inner_product(_ptr(a), _ptr(b), n_qubits, _ptr(out_dev), _stream(stream)))


COMBINE_OUT_C128, COMBINE_FP32 = 1, 2


def sv_branch_combine_full(a_states, b_states, n_branches, n_a, n_b, side_a_mask, folded_a,
                           folded_b, out_state, flags=0, stream=None):
    """Complete state of a cut circuit from all branch states of both halves
    (folded pairs as returned by circuit_split, host int32 arrays).  flags:
    0 = FP64 products and sums into a complex64 state; COMBINE_OUT_C128 =
    the same into a complex128 state; COMBINE_FP32 = FP32 accumulation."""
    fa = np.ascontiguousarray(np.asarray(folded_a, dtype=np.int32))
    fb = np.ascontiguousarray(np.asarray(folded_b, dtype=np.int32))
    _check(lib().sv_branch_combine_full(_ptr(a_states), _ptr(b_states), n_branches, n_a, n_b,
                                        ctypes.c_uint64(side_a_mask), fa.ctypes.data if fa.size else None,
                                        fb.ctypes.data if fb.size else None, fa.size, _ptr(out_state),
                                        flags, _stream(stream)))


def release_device_buffers():
    """Free the library's device buffers on the current device (the partial
    sums of sv_norm_fp64 / sv_inner_product per stream)."""
    _check(lib().qsv_release_device_buffers())


def sv_tune(amps_scratch, c, layer_begin=0, layer_end=-1, stream=None, workspace=None):
    """Autotune the tile shape; returns (opts dict, best ms)."""
    o = FuseOpts()
    ms = ctypes.c_double()
    wp, wb, _keep = _ws(workspace, c, layer_begin, layer_end, None, stream)
    _check(lib().sv_tune(_ptr(amps_scratch), c, layer_begin, layer_end, wp, wb, ctypes.byref(o),
                         ctypes.byref(ms), _stream(stream)))
    return ({"reg_qubits": o.reg_qubits, "thread_qubits": o.thread_qubits,
             "low_qubits": o.low_qubits, "plain": 0, "jit": o.jit,
             "out_of_place": o.out_of_place, "pass_forms": o.pass_forms}, ms.value)


def sv_apply_dense(amps, c, k, branch=0, layer_begin=0, layer_end=-1, stream=None):
    nb = ctypes.c_int()
    _check(lib().sv_apply_dense(_ptr(amps), c, ctypes.c_uint64(branch), layer_begin, layer_end, k,
                                ctypes.byref(nb), _stream(stream)))
    return nb.value


def sv_debug_emulate_dense(amps_host, c, k, branch=0, layer_begin=0, layer_end=-1):
    assert amps_host.dtype == np.complex64 and amps_host.flags.c_contiguous
    nb = ctypes.c_int()
    _check(lib().sv_debug_emulate_dense(_ptr(amps_host), c, ctypes.c_uint64(branch), layer_begin,
                                        layer_end, k, ctypes.byref(nb)))
    return nb.value


def version() -> str:
    return lib().qsv_version().decode()


class Partition:
    """Owning handle of a qsv_partition (keeps its circuit alive)."""

    def __init__(self, handle, circuit):
        self.handle = handle
        self.circuit = circuit

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.circuit_partition_destroy(self.handle)
            self.handle = None

    @property
    def _as_parameter_(self):
        return ctypes.c_void_p(self.handle)


def _present(present):
    if present is None:
        return None
    return np.ascontiguousarray(np.asarray(present, dtype=np.uint8).reshape(-1))


def circuit_partition_plan(c, rows, cols, present, r0, max_move=3) -> Partition:
    pres = _present(present)
    out = ctypes.c_void_p()
    _check(lib().circuit_partition_plan(c, rows, cols, _ptr(pres) if pres is not None else None, r0,
                                        max_move, ctypes.byref(out)))
    return Partition(out.value, c)


def circuit_partition_create(c, rows, cols, present, r0, t_s, ups, dns) -> Partition:
    pres = _present(present)
    u = np.ascontiguousarray(np.asarray(ups, dtype=np.uint8).reshape(-1))
    d = np.ascontiguousarray(np.asarray(dns, dtype=np.uint8).reshape(-1))
    out = ctypes.c_void_p()
    _check(lib().circuit_partition_create(c, rows, cols, _ptr(pres) if pres is not None else None, r0,
                                          t_s, _ptr(u) if u.size else None, _ptr(d) if d.size else None,
                                          ctypes.byref(out)))
    return Partition(out.value, c)


def circuit_partition_info(p) -> dict:
    info = PartitionInfo()
    _check(lib().circuit_partition_info(p, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in PartitionInfo._fields_}


def circuit_partition_offsets(p):
    """(ups, dns): uint8 arrays of shape (depth + 1 - t_s, cols)."""
    info = circuit_partition_info(p)
    nl = info["depth"] + 1 - info["t_s"]
    ups = np.zeros((nl, info["cols"]), np.uint8)
    dns = np.zeros((nl, info["cols"]), np.uint8)
    _check(lib().circuit_partition_offsets(p, _ptr(ups), _ptr(dns), ups.size))
    return ups, dns


def circuit_partition_parts(p):
    """(A, B, C, qubits_a, qubits_b): the part circuits and the local-to-global maps."""
    info = circuit_partition_info(p)
    a, b, c = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    qa = np.zeros(info["n_a"], np.int32)
    qb = np.zeros(info["n_b"], np.int32)
    _check(lib().circuit_partition_parts(p, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                         _ptr(qa), _ptr(qb)))
    return Circuit(a.value), Circuit(b.value), Circuit(c.value), qa, qb


def sv_partition_workspace_bytes(p) -> int:
    n = ctypes.c_size_t()
    _check(lib().sv_partition_workspace_bytes(p, ctypes.byref(n)))
    return n.value


def sv_partition_simulate(p, workspace, ws_bytes, out_state, stream=None):
    _check(lib().sv_partition_simulate(p, _ptr(workspace), ws_bytes, _ptr(out_state), _stream(stream)))


class Sampler:
    """Owning handle of a qsv_sampler (keeps its circuit alive)."""

    def __init__(self, handle, circuit, m):
        self.handle = handle
        self.circuit = circuit
        self.m = m

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.sv_sampler_destroy(self.handle)
            self.handle = None

    @property
    def _as_parameter_(self):
        return ctypes.c_void_p(self.handle)


def sv_sampler_create(c, bitstrings, layer_begin=0, layer_end=-1, opts=None) -> Sampler:
    xs = np.ascontiguousarray(np.asarray(bitstrings, dtype=np.uint64))
    out = ctypes.c_void_p()
    _check(lib().sv_sampler_create(c, layer_begin, layer_end, _opts(opts), _ptr(xs), xs.size,
                                   ctypes.byref(out)))
    smp = Sampler(out.value, c, xs.size)
    smp.range = (layer_begin, layer_end, opts)
    return smp


def sv_sampler_create_tiles(c, indices, layer_begin=0, layer_end=-1, opts=None) -> Sampler:
    xs = np.ascontiguousarray(np.asarray(indices, dtype=np.uint64))
    out = ctypes.c_void_p()
    _check(lib().sv_sampler_create_tiles(c, layer_begin, layer_end, _opts(opts), _ptr(xs), xs.size,
                                         ctypes.byref(out)))
    smp = Sampler(out.value, c, xs.size)
    smp.range = (layer_begin, layer_end, opts)
    return smp


def sv_sampler_inputs(sampler) -> np.ndarray:
    """Indices of src that a one-pass sampler reads (see qsv.h)."""
    cnt = ctypes.c_size_t()
    _check(lib().sv_sampler_inputs(sampler, None, 0, ctypes.byref(cnt)))
    out = np.empty(cnt.value, np.uint64)
    _check(lib().sv_sampler_inputs(sampler, _ptr(out), out.size, ctypes.byref(cnt)))
    return out


def _sampler_ws(sampler, workspace, stream):
    lb, le, opts = sampler.range
    return _ws(workspace, sampler.circuit, lb, le, opts, stream)


def sv_sampler_run(sampler, src, work, out, branch=0, stream=None, workspace=None):
    wp, wb, _keep = _sampler_ws(sampler, workspace, stream)
    _check(lib().sv_sampler_run(sampler, _ptr(src), _ptr(work), ctypes.c_uint64(branch), _ptr(out),
                                wp, wb, _stream(stream)))


def sv_sampler_run_subtree(sampler, src, work, out, prefix, mask, stream=None, workspace=None):
    wp, wb, _keep = _sampler_ws(sampler, workspace, stream)
    _check(lib().sv_sampler_run_subtree(sampler, _ptr(src), _ptr(work), ctypes.c_uint64(prefix),
                                        ctypes.c_uint64(mask), _ptr(out), wp, wb, _stream(stream)))


def sv_sampler_run_branches(sampler, src, work, out, branches, stream=None, workspace=None):
    br = np.ascontiguousarray(np.asarray(branches, dtype=np.uint64).reshape(-1))
    wp, wb, _keep = _sampler_ws(sampler, workspace, stream)
    _check(lib().sv_sampler_run_branches(sampler, _ptr(src), _ptr(work), _ptr(br), br.size, _ptr(out),
                                         wp, wb, _stream(stream)))
