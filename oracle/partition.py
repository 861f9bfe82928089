"""Three-part circuit partition, CPU oracle (TEST INFRASTRUCTURE ONLY).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this module; the GPU library has its own planner and split written in C++.

What it follows
---------------
* Section 2.1.1 (implicit decomposition, the 4-qubit example and eqs. (2)-(3)):
  two splitting lines divide the circuit into parts A, B and C.  While the lines
  coincide, a CZ joining the two sides is decomposed (one branch bit); part C
  starts from psi_in = sum over branches of phi_l (x) xi_l and applies its own
  gates, which touch only the qubits between the lines, so it acts on each block
  of fixed outside qubits independently (eq. (3)).  A cut whose projector side
  sees no further non-diagonal gate in its part needs no branch bit on that side
  (the bit equals the qubit's value).
* Section 2.1.2 (dynamic programming, Algorithm 1): f(t, i_1..i_K) is the
  smallest space exponent of part A when the upper line sits at offsets i_k at
  layer t; a position is reached from any earlier position j <= i (per column);
  a position that cuts a CZ after the lines have separated is illegal; the best
  scheme minimises S_A + S_B + S_C with S_C = 2^(sum of the offsets) (here: the
  number of qubits between the lines).

Readings (the paper is terse or garbled here)
---------------------------------------------
P1  The lines run between lattice rows.  Initially both lie between rows r0-1
    and r0: part A's qubits are the sites with row < r0, part B's the others.
    In column k the upper line sits i_k rows higher and the lower line j_k rows
    lower; at layer t a site (r, k) belongs to A if r < r0 - i_k(t), to B if
    r >= r0 + j_k(t), otherwise to C.  Offsets are capped by ``max_move``
    (Algorithm 1 uses 0..3) and by the rows available.
P2  Both lines leave the initial position at one separation layer t_s.  For
    layers 1..t_s-1 every CZ joining the two sides is cut (a branch bit of both
    parts).  From t_s on, offsets never decrease and no CZ of layer t may join
    two different parts.  (Run independently, one line could stay put while the
    other moves; a CZ cut there would put a branch-dependent gate into part C,
    which the block form of eq. (3) cannot hold.)
P3  A cut CZ on (a in A, b in B) is CZ = sum_l Z^l(a) P_l(b) (projector on B,
    as in the paper's example) or sum_l P_l(a) Z^l(b).  It is free on side B if
    no non-diagonal gate acts on b after the cut while b belongs to part B;
    then P_l(b) commutes to the end of part B and xi_l = [x_b = l] xi', so part
    B needs no branch bit for it.  Free on side A alike.  Free on both sides, it
    is the output sign (-1)^(x_a x_b) (no bit on either side).
P4  Space exponents: f = n_A + (cuts not free on side A), g = n_B + (cuts not
    free on side B), c = qubits in part C after the last layer; the scheme
    minimises 2^f + 2^g + 2^c.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import circuit as C
from . import sim

DIAGONAL = set(C.DIAGONAL)


# --- geometry -------------------------------------------------------------------

def _sites(lat):
    """qubit -> (row, col)."""
    return {q: rc for rc, q in lat.qubit.items()}


def max_offsets(lat, r0, max_move):
    """Largest upper and lower offset of each column (P1)."""
    up = [min(max_move, r0) for _ in range(lat.cols)]
    dn = [min(max_move, lat.rows - r0) for _ in range(lat.cols)]
    return up, dn


def part_of(row, col, r0, up, dn):
    """'A', 'B' or 'C' for a site under line offsets up/dn (P1)."""
    if row < r0 - up[col]:
        return "A"
    if row >= r0 + dn[col]:
        return "B"
    return "C"


def _layers(gates):
    depth = max((g[3] for g in gates), default=0)
    cz = {t: [] for t in range(depth + 1)}
    for g in gates:
        if g[0] == "CZ":
            cz[g[3]].append((g[1], g[2]))
    return depth, cz


def upper_crosses(lat, r0, pos, pairs):
    """Number of CZ pairs with exactly one qubit above the upper line."""
    site = _sites(lat)
    n = 0
    for p, q in pairs:
        (rp, cp), (rq, cq) = site[p], site[q]
        if (rp < r0 - pos[cp]) != (rq < r0 - pos[cq]):
            n += 1
    return n


def lower_crosses(lat, r0, pos, pairs):
    """Number of CZ pairs with exactly one qubit below the lower line."""
    site = _sites(lat)
    n = 0
    for p, q in pairs:
        (rp, cp), (rq, cq) = site[p], site[q]
        if (rp >= r0 + pos[cp]) != (rq >= r0 + pos[cq]):
            n += 1
    return n


# --- cuts and free cuts ---------------------------------------------------------

def cuts_before(lat, gates, r0, t_s):
    """CZs of layers 1..t_s-1 joining the two sides: [(gate index, a, b, layer)], a in A."""
    site = _sites(lat)
    out = []
    for i, (name, q0, q1, t) in enumerate(gates):
        if name != "CZ" or not (1 <= t < t_s):
            continue
        a_side0 = site[q0][0] < r0
        a_side1 = site[q1][0] < r0
        if a_side0 != a_side1:
            a, b = (q0, q1) if a_side0 else (q1, q0)
            out.append((i, a, b, t))
    return out


def free_after(gates, gi, q, enter_layer):
    """True if no non-diagonal gate acts on q after gate gi at a layer < enter_layer (P3)."""
    for name, q0, q1, t in gates[gi + 1:]:
        if t >= enter_layer:
            break
        if name not in DIAGONAL and q0 == q:
            return False
    return True


def enter_layer(lat, r0, t_s, ups, dns, q):
    """First layer at which q belongs to part C (depth+1 if never); ups/dns[t - t_s]."""
    site = _sites(lat)
    r, c = site[q]
    for k, (u, d) in enumerate(zip(ups, dns)):
        if part_of(r, c, r0, u, d) == "C":
            return t_s + k
    return t_s + len(ups)


# --- evaluation of one scheme -------------------------------------------------------

def evaluate(lat, gates, scheme):
    """Check a scheme (P1, P2) and return its cut bookkeeping and space exponents.

    scheme: dict with r0, t_s and ups / dns = offsets for layers t_s..depth.
    Raises ValueError for an illegal scheme.
    """
    depth, cz = _layers(gates)
    r0, t_s = scheme["r0"], scheme["t_s"]
    ups, dns = [list(u) for u in scheme["ups"]], [list(d) for d in scheme["dns"]]
    if not (1 <= t_s <= depth + 1) or len(ups) != depth + 1 - t_s or len(dns) != len(ups):
        raise ValueError("scheme does not cover layers t_s..depth")
    umax, dmax = max_offsets(lat, r0, 10 ** 6)
    prev_u, prev_d = [0] * lat.cols, [0] * lat.cols
    for k, t in enumerate(range(t_s, depth + 1)):
        u, d = ups[k], dns[k]
        for col in range(lat.cols):
            if not (prev_u[col] <= u[col] <= umax[col] and prev_d[col] <= d[col] <= dmax[col]):
                raise ValueError(f"offsets not monotone or out of range at layer {t}")
        if upper_crosses(lat, r0, u, cz[t]) or lower_crosses(lat, r0, d, cz[t]):
            raise ValueError(f"a CZ of layer {t} joins two parts")
        prev_u, prev_d = u, d
    site = _sites(lat)
    qa = sorted(q for q in range(lat.n) if site[q][0] < r0)
    qb = sorted(q for q in range(lat.n) if site[q][0] >= r0)
    cuts = cuts_before(lat, gates, r0, t_s)
    info = []
    for gi, a, b, t in cuts:
        fa = free_after(gates, gi, a, enter_layer(lat, r0, t_s, ups, dns, a))
        fb = free_after(gates, gi, b, enter_layer(lat, r0, t_s, ups, dns, b))
        info.append({"gate": gi, "a": a, "b": b, "layer": t, "free_a": fa, "free_b": fb})
    fin_u = ups[-1] if ups else [0] * lat.cols
    fin_d = dns[-1] if dns else [0] * lat.cols
    qc = sorted(q for q in range(lat.n) if part_of(*site[q], r0, fin_u, fin_d) == "C")
    f = len(qa) + sum(1 for x in info if not x["free_a"])
    g = len(qb) + sum(1 for x in info if not x["free_b"])
    c = len(qc)
    return {"qa": qa, "qb": qb, "qc": qc, "cuts": info, "f": f, "g": g, "c": c,
            "objective": 2 ** f + 2 ** g + 2 ** c}


# --- Algorithm 1: dynamic programming over line positions ----------------------

def _line_dp(lat, gates, r0, t_s, depth, cz, cuts, offs, upper):
    """Best gain (free cuts on this line's side) per final position.

    f(t, i) of Algorithm 1 is n + K - (gain); the DP keeps the gain.  Layer
    t_s - 1 holds the initial position 0 only, with the cuts that are free
    whatever the lines do (no later non-diagonal gate on their qubit on this
    side) already counted; a position at layer t is
    legal if it cuts no CZ of layer t and is reached from any legal position
    j <= i of layer t - 1.  Moving from j to i at layer t puts the qubits
    between the two positions into part C from layer t on; each cut whose
    qubit on this side enters then and saw no non-diagonal gate since the cut
    becomes free.  Returns {final position: (gain, [positions t_s..depth])}.
    """
    at = dict(lat.qubit)
    mycuts = [(gi, (a if upper else b)) for gi, a, b, _t in cuts]

    def entering(j, i):
        qs = []
        for col in range(lat.cols):
            for step in range(j[col], i[col]):
                r = (r0 - 1 - step) if upper else (r0 + step)
                if (r, col) in at:
                    qs.append(at[(r, col)])
        return qs

    never = len(gates) + depth + 2  # a layer after every gate

    def gain(j, i, t):
        # cuts free only because their qubit enters part C at layer t
        g = 0
        for q in entering(j, i):
            for gi, cq in mycuts:
                if cq == q and free_after(gates, gi, q, t) and not free_after(gates, gi, q, never):
                    g += 1
        return g

    cross = upper_crosses if upper else lower_crosses
    zero = tuple([0] * lat.cols)
    # a cut whose qubit sees no later non-diagonal gate at all is free anyway
    base = sum(1 for gi, q in mycuts if free_after(gates, gi, q, never))
    h = {zero: (base, [])}
    positions = list(itertools.product(*[range(m + 1) for m in offs]))
    for t in range(t_s, depth + 1):
        nh = {}
        for i in positions:
            if cross(lat, r0, i, cz[t]):
                continue  # illegal: this position cuts a CZ of layer t
            best = None
            for j in itertools.product(*[range(x + 1) for x in i]):
                if j not in h:
                    continue
                v = h[j][0] + gain(j, i, t)
                if best is None or v > best[0]:
                    best = (v, h[j][1] + [i])
            if best is not None:
                nh[i] = best
        h = nh
    return h


def plan(lat, gates, r0, max_move=3):
    """The scheme with the smallest 2^f + 2^g + 2^c over every separation layer.

    Ties keep the first scheme found in the order t_s = 1, 2, ...; upper and
    lower final positions in lexicographic order.
    """
    depth, cz = _layers(gates)
    up_max, dn_max = max_offsets(lat, r0, max_move)
    site = _sites(lat)
    nA = sum(1 for q in range(lat.n) if site[q][0] < r0)
    nB = lat.n - nA
    best = None
    for t_s in range(1, depth + 2):
        cuts = cuts_before(lat, gates, r0, t_s)
        K = len(cuts)
        fu = _line_dp(lat, gates, r0, t_s, depth, cz, cuts, up_max, True)
        fd = _line_dp(lat, gates, r0, t_s, depth, cz, cuts, dn_max, False)
        for iu in sorted(fu):
            for jd in sorted(fd):
                nC = sum(1 for q in range(lat.n) if part_of(*site[q], r0, iu, jd) == "C")
                f = nA + K - fu[iu][0]
                g = nB + K - fd[jd][0]
                obj = 2 ** f + 2 ** g + 2 ** nC
                if best is None or obj < best["objective"]:
                    best = {"r0": r0, "t_s": t_s, "ups": fu[iu][1], "dns": fd[jd][1],
                            "f": f, "g": g, "c": nC, "objective": obj}
    return best


# --- the three parts and the output state ---------------------------------------------

def parts(lat, gates, scheme):
    """Gate lists of parts A, B, C (global qubit numbers) and the cut list.

    Every gate but the cut CZs belongs to the part that holds its qubit(s) at
    its layer (the scheme's legality puts both qubits of a CZ in one part).
    """
    ev = evaluate(lat, gates, scheme)
    site = _sites(lat)
    r0, t_s = scheme["r0"], scheme["t_s"]
    depth, _ = _layers(gates)
    cut_at = {x["gate"]: x for x in ev["cuts"]}
    ga, gb, gc = [], [], []
    for i, g in enumerate(gates):
        t = g[3]
        if i in cut_at:
            ga.append(("CUT", i))
            gb.append(("CUT", i))
            continue
        r, c = site[g[1]]
        if t < t_s:
            p = "A" if r < r0 else "B"
        else:
            k = t - t_s
            p = part_of(r, c, r0, scheme["ups"][k], scheme["dns"][k])
        (ga if p == "A" else gb if p == "B" else gc).append(g)
    return ev, ga, gb, gc


def _local(gates, qubits):
    loc = {q: i for i, q in enumerate(qubits)}
    return [(g[0], loc[g[1]], loc[g[2]] if g[2] >= 0 else -1, g[3]) for g in gates]


def partition_state(lat, gates, scheme):
    """psi_out of the three-part method (eqs. (2)-(3)) in complex128.

    Every cut keeps its branch bit on both sides here (the plain form of
    eq. (2)): for each branch tuple l, phi_l gets Z^{l_c} on the cut's A qubit
    and xi_l gets P_{l_c} on its B qubit; psi_in = sum_l phi_l (x) xi_l on the
    full index space; part C's gates are then applied to psi_in.
    """
    ev, ga, gb, gc = parts(lat, gates, scheme)
    n = lat.n
    qa, qb = ev["qa"], ev["qb"]
    cut_of = {x["gate"]: (j, x) for j, x in enumerate(ev["cuts"])}
    K = len(ev["cuts"])
    xs = np.arange(1 << n, dtype=np.int64)
    ia = np.zeros(1 << n, np.int64)
    ib = np.zeros(1 << n, np.int64)
    for i, q in enumerate(qa):
        ia |= ((xs >> q) & 1) << i
    for i, q in enumerate(qb):
        ib |= ((xs >> q) & 1) << i
    psi = np.zeros(1 << n, np.complex128)
    for br in range(1 << K):
        la, lb = [], []
        for g in ga:
            if g[0] == "CUT":
                j, x = cut_of[g[1]]
                if (br >> j) & 1:
                    la.append(("Z", x["a"], -1, x["layer"]))
            else:
                la.append(g)
        for g in gb:
            if g[0] == "CUT":
                j, x = cut_of[g[1]]
                lb.append(("P1" if (br >> j) & 1 else "P0", x["b"], -1, x["layer"]))
            else:
                lb.append(g)
        phi = sim.simulate(_local(la, qa), len(qa))
        xi = sim.simulate(_local(lb, qb), len(qb))
        psi += phi[ia] * xi[ib]
    return sim.run(psi, n, gc)
