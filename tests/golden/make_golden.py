"""Write oracle amplitudes for the 30-qubit workload (calls only oracle/).

Outputs: tests/golden/<workload>_amplitudes.txt for the 30-qubit depth-20
workload (4096 bitstrings) and the 30-qubit depth-16 workload used by the
split check (1024 bitstrings), and tests/golden/7x7-d16_A_branch<b>.txt for
branch states of the 28-qubit half of the 49-qubit split (branches 0, 1337
and 16 seeded random ones), one line per sampled bitstring:
"<bitstring> <re> <im>" with %.17g doubles, plus a header with the workload,
the oracle norm and the oracle's own timing.  The 4096 bitstrings are the
seeded uniform sample of paper_1804_04797_amd.workloads.bitstrings.
Needs about 17 GiB of host memory and several minutes.
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import circuit as OC  # noqa: E402
from oracle import sim  # noqa: E402
from paper_1804_04797_amd import workloads  # noqa: E402


def main(name="5x6-d20", m=4096, bitstring_seed=workloads.BITSTRING_SEED_BASE + 2):
    spec = workloads.WORKLOADS[name]
    lat = OC.Lattice(spec["rows"], spec["cols"], workloads.present_grid(spec))
    gates = OC.random_circuit(lat, spec["depth"], spec["seed"])
    xs = workloads.bitstrings(lat.n, m, bitstring_seed)
    t0 = time.time()
    psi = sim.simulate(gates, lat.n)
    dt = time.time() - t0
    nrm = sim.norm2(psi)
    out = os.path.join(HERE, f"{name}_amplitudes.txt")
    with open(out, "w") as f:
        f.write(f"# workload {name}: n={lat.n} depth={spec['depth']} seed={spec['seed']:#x} "
                f"gates={len(gates)} bitstring_seed={bitstring_seed:#x}\n")
        f.write(f"# oracle complex128 norm2={nrm:.17g} time_s={dt:.1f} threads={sim.threads()}\n")
        for x in xs.tolist():
            a = psi[x]
            f.write(f"{x} {a.real:.17g} {a.imag:.17g}\n")
    print(out, dt)




def split_branch(name="7x7-d16", after_col=3, branches=(0, 1337), m=1024):
    """Oracle amplitudes of single branch states of the side-A half of a cut
    circuit (Fig. 2 split; oracle/sim.py split_circuit), at m sampled local
    bitstrings.  Output: tests/golden/<name>_A_branch<l>.txt."""
    spec = workloads.WORKLOADS[name]
    lat = OC.Lattice(spec["rows"], spec["cols"], workloads.present_grid(spec))
    gates = OC.random_circuit(lat, spec["depth"], spec["seed"])
    mask = workloads.column_cut_mask(spec["rows"], spec["cols"], after_col)
    side_a = [q for q in range(lat.n) if (mask >> q) & 1]
    info = sim.split_circuit(gates, lat.n, side_a)
    na = len(info["qa"])
    c = len(info["cuts"])
    xs = workloads.bitstrings(na, m, workloads.BITSTRING_SEED_BASE + 40)
    for br in branches:
        l = tuple((br >> j) & 1 for j in range(c))
        ga, _ = info["half"](l)
        t0 = time.time()
        psi = sim.simulate(ga, na)
        dt = time.time() - t0
        out = os.path.join(HERE, f"{name}_A_branch{br}.txt")
        with open(out, "w") as f:
            f.write(f"# workload {name} cut after column {after_col}: side-A half n={na}, "
                    f"branch {br} of 2^{c}, bitstring_seed={workloads.BITSTRING_SEED_BASE + 40:#x}\n")
            f.write(f"# oracle complex128 time_s={dt:.1f}\n")
            for x in xs.tolist():
                a = psi[x]
                f.write(f"{x} {a.real:.17g} {a.imag:.17g}\n")
        print(out, dt)


def random_branches(count=16, c_eff=11, seed=workloads.BITSTRING_SEED_BASE + 41):
    """count distinct branch indices drawn uniformly from [0, 2^c_eff) (seeded),
    excluding 0 and 1337, which have their own files."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        b = int(rng.integers(0, 1 << c_eff))
        if b not in out and b not in (0, 1337):
            out.append(b)
    return sorted(out)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("all", "sweeps"):
        main("5x6-d20", 4096, workloads.BITSTRING_SEED_BASE + 2)
        main("5x6-d16", 1024, workloads.BITSTRING_SEED_BASE + 6)
    if what in ("all", "branches"):
        split_branch("7x7-d16", 3, (0, 1337), 1024)
    if what in ("all", "random_branches"):
        split_branch("7x7-d16", 3, tuple(random_branches()), 1024)
