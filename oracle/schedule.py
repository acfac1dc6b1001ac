"""The paper's scheduling algorithms, written from their descriptions --
TEST INFRASTRUCTURE ONLY (the product's planner is separate C++ code).

Operators are given by their target sets T(C_i) (tuples of qubits); a tile is
``(Q_L, [operator indices in schedule order])``.

* :func:`depths`, :func:`depth_order` -- depth = critical-path length over the
  dependency relation (Section "Quantum state update"), order = ascending depth,
  ties by ascending target qubits (Section "Flat tiling").
* :func:`tile_construction` -- Alg. 2 (P1).
* :func:`qubit_mapping` -- Alg. 3 (P2), boundary fill configurable.
* :func:`flat_tiling` -- Alg. 1.
* :func:`hierarchical_tiling` -- Algs. 4 and 5.
* :func:`ad_hoc` -- the breadth-first baseline of Section "Quantum state
  update" (evaluation): remap on each wide operator without lookahead.
* :func:`tiling_pauli` -- Alg. 6 (optionally with diagonalization: T(P) is
  then the X/Y support only, eq. without_QR / eq. par_exp).
* :func:`n_qr` -- eq. n_qr with the indicator reading of eq. f_eq.

Readings where the paper is ambiguous:
* Alg. 1 increments x before removing g(x); read as "remove the operator just
  scheduled, then increment".
* eq. f_eq calls delta a Kronecker delta but returns 1 when the arguments
  differ; read as the indicator [M(g(i-1)) != M(g(i))], M(g(-1)) = {0..n_L-1}.
* Same-depth ties: key (depth, sorted targets, original index).
* Alg. 2/3 iterate a snapshot of C' in order.
* Alg. 6 enumerates Q_locals in lexicographic order of sorted qubit tuples;
  the strict '<' keeps the first maximal set.
* The ad hoc eviction rule is unspecified: evict the local qubits at the
  highest physical positions that the operator does not target; pair evicted
  and incoming qubits in ascending physical position (parity unpinned: the
  paper gives no worked example of the ad hoc mapping).
"""
from __future__ import annotations

from itertools import combinations


def depths(targets):
    last = {}
    out = []
    for t in targets:
        d = max((last[q] + 1 for q in t if q in last), default=0)
        out.append(d)
        for q in t:
            last[q] = d
    return out


def depth_order(targets):
    d = depths(targets)
    return sorted(range(len(targets)), key=lambda i: (d[i], tuple(sorted(targets[i])), i))


def tile_construction(QL, remain, targets):
    """Alg. 2: greedily take operators (depth order) whose targets are all
    still available; a rejected operator blocks its targets."""
    avail = set(QL)
    tile = []
    for i in list(remain):
        T = set(targets[i])
        if T <= avail:
            tile.append(i)
        else:
            avail -= T
        if not avail:
            break
    return tile


def qubit_mapping(Q, remain, targets, nL, fill="lowest"):
    """Alg. 3: pick the targets of the shallowest remaining operators as the
    next local set; fill up to n_L (boundary treatment)."""
    avail = set(Q)
    QL = set()
    for i in list(remain):
        T = set(targets[i])
        if T <= avail and len(QL | T) <= nL:
            QL |= T
        else:
            avail -= T
        if not avail:
            break
    if not QL:
        return set()
    rest = sorted(set(Q) - QL, reverse=(fill == "highest"))
    for q in rest:
        if len(QL) >= nL:
            break
        QL.add(q)
    return QL


def flat_tiling(n, targets, nL, fill="lowest"):
    """Alg. 1.  Returns (order, M, tiles) with M[x] the local set of the x-th
    scheduled operator and tiles = [(Q_L, [ops])]."""
    for t in targets:
        if len(set(t)) > nL:
            raise ValueError("operator wider than the local qubit count")
    Q = range(n)
    QL = set(range(nL))
    remain = depth_order(targets)
    order, M, tiles = [], [], []
    while remain:
        G = tile_construction(QL, remain, targets)
        taken = set(G)
        for i in G:
            order.append(i)
            M.append(frozenset(QL))
        remain = [i for i in remain if i not in taken]
        if G:
            tiles.append((frozenset(QL), G))
        if remain:
            QL = qubit_mapping(Q, remain, targets, nL, fill)
    return order, M, tiles


def hierarchical_qubit_mapping(Q, remain, targets, QL, Qintra, fill="lowest"):
    """Alg. 5: try an intra-only remap from Q_L u Q_intra; otherwise remap from
    all qubits (an inter QR)."""
    nL = len(QL)
    pool = set(QL) | set(Qintra)
    QLn = qubit_mapping(sorted(pool), remain, targets, nL, fill)
    # Reading: an intra-only map is "valid" only if it admits at least one
    # remaining operator; otherwise the flat loop would make no progress.
    if QLn and tile_construction(QLn, remain, targets):
        return QLn, pool - QLn
    QLn = qubit_mapping(Q, remain, targets, nL, fill)
    Qp = qubit_mapping(Q, remain, targets, nL + len(Qintra), fill)
    Qi = set(Qp) - QLn
    # Reading: keep |Q_intra| fixed when the two greedy picks diverge.
    for q in sorted(set(Q) - QLn - Qi, reverse=(fill == "highest")):
        if len(Qi) >= len(Qintra):
            break
        Qi.add(q)
    while len(Qi) > len(Qintra):
        Qi.remove(max(Qi) if fill == "lowest" else min(Qi))
    return QLn, Qi


def hierarchical_tiling(n, targets, nL, n_intra, fill="lowest"):
    """Alg. 4.  Returns (order, M, tiles, events) where events lists
    (position, 'intra'|'inter', Q_intra, Q_inter) for every remap."""
    Q = list(range(n))
    QL = set(range(nL))
    Qintra = set(range(nL, nL + n_intra))
    remain = depth_order(targets)
    order, M, tiles, events = [], [], [], []
    while remain:
        G = tile_construction(QL, remain, targets)
        taken = set(G)
        for i in G:
            order.append(i)
            M.append(frozenset(QL))
        remain = [i for i in remain if i not in taken]
        if G:
            tiles.append((frozenset(QL), G))
        if remain:
            old_inter = set(Q) - QL - Qintra
            QL, Qintra = hierarchical_qubit_mapping(Q, remain, targets, QL, Qintra, fill)
            new_inter = set(Q) - QL - Qintra
            kind = "intra" if new_inter == old_inter else "inter"
            events.append((len(order), kind, frozenset(Qintra), frozenset(new_inter)))
    return order, M, tiles, events


def qr_kinds_by_position(M, n, nL, n_intra):
    """Intra and inter reorders (fig:qr_types) of a flat or ad hoc plan's
    local-set sequence M on a cluster whose global positions nL .. nL+n_intra-1
    are intra-node PE bits and the rest inter-node ones.  Reading (the paper
    does not say where such a plan puts the qubits it evicts): a reorder swaps
    its incoming qubits with its outgoing ones pairwise in ascending order of
    position, as the ad hoc method does, and is inter when an incoming qubit
    comes from an inter position.  Returns (N_intra, N_inter)."""
    pos = list(range(n))
    prev = frozenset(range(nL))
    n_in = n_out = 0
    for m in M:
        m = frozenset(m)
        if m == prev:
            continue
        incoming = sorted(m - prev, key=lambda q: pos[q])
        outgoing = sorted(prev - m, key=lambda q: pos[q])
        vacated = [pos[q] for q in incoming]
        freed = [pos[q] for q in outgoing]
        if any(p >= nL + n_intra for p in vacated):
            n_out += 1
        else:
            n_in += 1
        for q, p in zip(outgoing, vacated):
            pos[q] = p
        for q, p in zip(incoming, freed):
            pos[q] = p
        prev = m
    return n_in, n_out


def hierarchical_kinds(events, n, nL, n_intra):
    """(N_intra, N_inter) of hierarchical tiling's remaps (Alg. 4): a remap is
    a reorder when it changes Q_intra or Q_inter (and so Q_L); it is inter when
    Q_inter changes."""
    prev = (frozenset(range(nL, nL + n_intra)), frozenset(range(nL + n_intra, n)))
    n_in = n_out = 0
    for _, kind, qi, qe in events:
        cur = (frozenset(qi), frozenset(qe))
        if cur == prev:
            continue
        if kind == "inter":
            n_out += 1
        else:
            n_in += 1
        prev = cur
    return n_in, n_out


def comm_cost(n_intra, n_inter, w_intra, w_inter):
    """eq. comm_cost: weighted count of intra and inter reorders."""
    return w_intra * n_intra + w_inter * n_inter


def n_qr(M, nL):
    """eq. n_qr: number of positions whose local set differs from the previous
    one, starting from {0..n_L-1}."""
    prev = frozenset(range(nL))
    cnt = 0
    for m in M:
        if m != prev:
            cnt += 1
        prev = m
    return cnt


def ad_hoc(n, targets, nL, order=None):
    """Breadth-first (depth) order; on a wide operator, swap the missing
    qubits in, evicting local qubits at the highest physical positions that
    the operator does not target.  Returns (order, M, transpositions) where
    transpositions[k] lists the (physical position, physical position) pairs
    swapped by the k-th reordering."""
    pos = list(range(n))                      # physical position of each qubit
    order = depth_order(targets) if order is None else list(order)
    M, qrs = [], []
    for i in order:
        T = set(targets[i])
        if len(T) > nL:
            raise ValueError("operator wider than the local qubit count")
        local = {q for q in range(n) if pos[q] < nL}
        if not T <= local:
            incoming = sorted(T - local, key=lambda q: pos[q])
            cand = sorted(local - T, key=lambda q: -pos[q])[:len(incoming)]
            evicted = sorted(cand, key=lambda q: pos[q])
            pairs = []
            for a, b in zip(evicted, incoming):
                pairs.append((pos[a], pos[b]))
                pos[a], pos[b] = pos[b], pos[a]
            qrs.append(pairs)
        M.append(frozenset(q for q in range(n) if pos[q] < nL))
    return order, M, qrs


def tiling_pauli(n, supports, nL):
    """Alg. 6 over operator supports (bit masks).  Returns [(Q_L, [term idx])]."""
    remain = list(range(len(supports)))
    tiles = []
    all_sets = [frozenset(c) for c in combinations(range(n), nL)]
    masks = [sum(1 << q for q in c) for c in all_sets]
    while remain:
        best, best_set = 0, None
        for QL, mk in zip(all_sets, masks):
            cnt = sum(1 for i in remain if supports[i] & ~mk == 0)
            if best < cnt:
                best, best_set = cnt, (QL, mk)
        if best_set is None:
            raise ValueError("a term is wider than the local qubit count")
        QL, mk = best_set
        G = [i for i in remain if supports[i] & ~mk == 0]
        tiles.append((QL, G))
        taken = set(G)
        remain = [i for i in remain if i not in taken]
    return tiles


def pauli_support(x: int, z: int, diagonalize: bool) -> int:
    """T(P) (eq. pauli_target); with diagonalization only the X/Y sites."""
    return int(x) if diagonalize else int(x) | int(z)


def tiles_n_qr(tiles, nL):
    prev = frozenset(range(nL))
    cnt = 0
    for QL, _ in tiles:
        if QL != prev:
            cnt += 1
        prev = QL
    return cnt
