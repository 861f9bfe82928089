#!/usr/bin/env python3
"""Benchmark: full-state sweep of a random lattice circuit on one MI355X.

One step = the whole hot path over one synthetic circuit instance:
circuit_create (host) -> pass planning (host) -> sv_init(|+>^n, i.e. layer 0)
-> sv_apply_fused (layers 1..d, all fused passes) -> sv_norm_fp64 ->
sv_amplitudes (4096 sampled bitstrings).  Default workload: 30 qubits on a
5x6 lattice, depth 20 (full 2^30 complex64 state, 8 GiB).

value = amplitude updates per second = G * 2^n / step time, G = gates of the
circuit including layer 0.  The JSON line also carries the roofline of the
dominant kernel (the fused tile pass: 16 bytes of algorithmic HBM traffic
per amplitude per pass, timed with HIP events on the launch stream), the
unfused comparator path on the same workload, the sampled amplitude error
against stored oracle values, and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("amplitude-updates/s & HBM GB/s (% peak), batched vs plain, "
          "at ≤1e-5 amp error")
HBM_PEAK_GBPS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="5x6-d20")
    p.add_argument("--reg", type=int, default=0, help="register qubits (0 = default)")
    p.add_argument("--thr", type=int, default=0, help="thread qubits (0 = default)")
    p.add_argument("--low", type=int, default=0, help="low resident qubits (0 = default)")
    p.add_argument("--no-plain", action="store_true", help="skip the unfused comparator")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    p.add_argument("--calibrate-copy", action="store_true",
                   help="run one 1 GiB device copy first (counter calibration)")
    return p.parse_args()


def golden(name):
    path = os.path.join(ROOT, "tests", "golden", f"{name}_amplitudes.txt")
    if not os.path.exists(path):
        return None, None
    import numpy as np
    xs, amps = [], []
    for line in open(path):
        if line.startswith("#"):
            continue
        x, re, im = line.split()
        xs.append(int(x))
        amps.append(complex(float(re), float(im)))
    return np.array(xs, np.uint64), np.array(amps)


def cpu_baseline(spec, seconds):
    """The CPU oracle as it stands (complex128, gate by gate, OpenMP) on a
    bounded sample of the same workload: the first gates of the circuit on
    the full-size state, until `seconds` of work have been done."""
    import numpy as np
    from oracle import circuit as OC
    from oracle import sim
    from paper_1804_04797_amd import workloads
    lat = OC.Lattice(spec["rows"], spec["cols"], workloads.present_grid(spec))
    gates = OC.random_circuit(lat, spec["depth"], spec["seed"])
    n = lat.n
    psi = sim.zero_state(n)
    done = 0
    t0 = time.perf_counter()
    while done < len(gates) and time.perf_counter() - t0 < seconds:
        sim.run(psi, n, gates[done:done + 1])
        done += 1
    dt = time.perf_counter() - t0
    del psi
    return {"value": done * float(1 << n) / dt, "unit": "amplitude-updates/s",
            "cores": sim.threads(), "kind": "oracle",
            "sample": f"first {done} of {len(gates)} gates of {spec['name']} on the full "
                      f"2^{n} complex128 state ({dt:.1f} s)"}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1804_04797_amd import qsv, workloads

    spec = dict(workloads.WORKLOADS[a.workload])
    spec["name"] = a.workload
    n = spec["n"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    opts = None
    if a.reg or a.thr or a.low:
        opts = dict(reg_qubits=a.reg, thread_qubits=a.thr, low_qubits=a.low, plain=0)
    pres = workloads.present_mask(spec)

    if a.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    amps = torch.empty(1 << n, dtype=torch.complex64, device=dev)
    xs_np, ref = golden(a.workload)
    if xs_np is None:
        xs_np = workloads.bitstrings(n, 4096, workloads.BITSTRING_SEED_BASE + 2)
    xs = torch.from_numpy(xs_np.view(np.int64)).to(dev)
    out = torch.empty(xs_np.size, dtype=torch.complex128, device=dev)
    nrm = torch.zeros(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    ev = []

    def step(timed):
        c = qsv.circuit_create(spec["rows"], spec["cols"], pres, spec["depth"], spec["seed"])
        qsv.sv_init(amps, n, qsv.INIT_PLUS)
        if timed:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        qsv.sv_apply_fused(amps, c, layer_begin=1, opts=opts)
        if timed:
            e1.record(stream)
            ev.append((e0, e1))
        qsv.sv_norm_fp64(amps, n, nrm)
        qsv.sv_amplitudes(amps, n, xs, out, c128=True)
        return c

    c = step(False)
    n_gates = c.info()[2]
    passes = qsv.sv_plan_info(c, layer_begin=1, opts=opts)["n_passes"]
    for _ in range(a.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / a.steps
    value = n_gates * float(1 << n) / (ms * 1e-3)

    # dominant kernel: the fused pass; every launch streams 2^n amplitudes in
    # and out (16 bytes per amplitude).
    sweep_ms = sum(e0.elapsed_time(e1) for e0, e1 in ev) / len(ev)
    launch_ms = sweep_ms / passes
    bytes_per_launch = 16.0 * (1 << n)
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    traffic = None
    if a.traffic_json and os.path.exists(a.traffic_json):
        tj = json.load(open(a.traffic_json))
        t = tj.get(a.workload)
        if (t and t.get("reg") == a.reg and t.get("thr") == a.thr and t.get("low") == a.low
                and t.get("kernel_rev") == qsv.version()):
            traffic = t.get("bytes_per_launch")

    got = out.cpu().numpy()
    err = None
    if ref is not None:
        d = float(np.max(np.abs(got - ref)))
        err = {"max_abs": d, "scaled": d * 2 ** (n / 2), "vs": "complex128 oracle, 4096 sampled"}
    norm_drift = abs(nrm.item() - 1.0)

    plain = None
    if not a.no_plain:
        qsv.sv_init(amps, n, qsv.INIT_PLUS)
        qsv.sv_apply_plain(amps, c, layer_begin=1)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        qsv.sv_init(amps, n, qsv.INIT_PLUS)
        qsv.sv_apply_plain(amps, c, layer_begin=1)
        qsv.sv_norm_fp64(amps, n, nrm)
        qsv.sv_amplitudes(amps, n, xs, out, c128=True)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp0
        pd = float(np.max(np.abs(out.cpu().numpy() - ref))) if ref is not None else None
        plain = {"value": n_gates * float(1 << n) / tp, "ms_per_step": tp * 1e3,
                 "max_abs_err": pd, "speedup_fused_vs_plain": (tp * 1e3) / ms}

    del amps
    torch.cuda.empty_cache()
    cpu = None if a.no_cpu else cpu_baseline(spec, a.cpu_seconds)

    line = {
        "metric": METRIC, "value": value, "unit": "amplitude-updates/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": a.workload, "n_qubits": n, "lattice": f"{spec['rows']}x{spec['cols']}",
                   "depth": spec["depth"], "gates": n_gates, "passes": passes,
                   "sampled_bitstrings": int(xs_np.size),
                   "tile": opts or "default", "steps_include": "create+plan+init+sweep+norm+gather"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": "k_fused", "launch_ms": launch_ms,
                     "bytes_per_launch": bytes_per_launch},
        "hbm_gbps_step": passes * bytes_per_launch / (ms * 1e-3) / 1e9,
        "error": err, "norm_drift": norm_drift,
        "plain": plain,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
