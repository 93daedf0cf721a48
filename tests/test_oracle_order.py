"""Pins of the oracle's ordering against facts the paper fixes.

- hand-derived permutations of small cases (tests/golden), worked from the
  definitions of Sections 4.1-4.3 and the heuristics of Section 5.1;
- closed forms on grids (strip blocks, parity coloring);
- the greedy rules checked as properties, by brute force, on random graphs;
- the ER condition (Section 3.1, eq. "equivalence") between BMC and HBMC,
  and the block structures of eqs. "BAMC1" and "BAMC-level-2".
"""
import glob
import json
import os

import numpy as np
import pytest

from paper_1908_00741_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _matrix(spec):
    if spec["kind"] == "grid2d_5pt":
        return inputs.grid2d_5pt(spec["nx"], spec["ny"])
    if spec["kind"] == "path":
        return inputs.path_1d(spec["n"])
    raise ValueError(spec)


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLDEN, "order_*.json"))),
                         ids=os.path.basename)
def test_hand_derived(orc, path):
    g = json.load(open(path))
    A = _matrix(g["matrix"])
    o = orc.order(A, g["bs"], g["w"])
    assert o.ncolors == g["ncolors"]
    assert o.n_pad == g["n_pad"]
    assert list(o.color_start) == g["color_start"]
    assert list(o.perm) == g["perm"]


def test_c1_closed_form(orc):
    # 64x64 5-point, bs=4, w=8: 1x4 strips, parity coloring, 64 L1 blocks per color
    A = inputs.grid2d_5pt(64)
    o = orc.order(A, 4, 8)
    i = np.arange(A.n)
    x, y = i % 64, i // 64
    expect = 2048 * ((y + x // 4) % 2) + 32 * y + 8 * (x % 4) + (x // 4) // 2
    assert o.ncolors == 2 and o.n_pad == 4096
    assert np.array_equal(o.perm, expect)


@pytest.mark.parametrize("N", [16, 32])
def test_3d_closed_form(orc, N):
    # N^3 7-point, bs=8, w=64, N/8 even: 1x8 strips, parity coloring, no padding
    A = inputs.diffusion3d(N, 1.0, 2)
    o = orc.order(A, 8, 64)
    i = np.arange(A.n)
    x, y, z = i % N, (i // N) % N, i // (N * N)
    s = x // 8
    c = (z + y + s) % 2
    rank = (N * z + y) * (N // 16) + s // 2
    expect = c * (N ** 3 // 2) + (rank // 64) * 512 + (x % 8) * 64 + rank % 64
    assert o.ncolors == 2 and o.n_pad == N ** 3
    assert np.array_equal(o.perm, expect)


def test_red_black(orc):
    # bs = 1, w = 1 on a 2D grid: the textbook red-black ordering
    A = inputs.grid2d_5pt(9, 7)
    o = orc.order(A, 1, 1)
    i = np.arange(A.n)
    red = ((i % 9) + (i // 9)) % 2 == 0
    expect = np.empty(A.n, np.int64)
    expect[red] = np.arange(red.sum())
    expect[~red] = red.sum() + np.arange((~red).sum())
    assert o.ncolors == 2
    assert np.array_equal(o.perm, expect)


def _adj(A):
    return [A.col[A.rowptr[i]:A.rowptr[i + 1]] for i in range(A.n)]


def _graphs():
    yield "random", inputs.random_spd(150, 0.03, 3)
    yield "random_dense", inputs.random_spd(90, 0.12, 4)
    yield "knn", inputs.knn_laplacian(300, k=6, seed_points=1, seed_perm=2)
    yield "grid_ragged", inputs.grid2d_5pt(13, 5)


@pytest.mark.parametrize("bs", [1, 3, 4, 8])
@pytest.mark.parametrize("name,A", list(_graphs()), ids=lambda v: v if isinstance(v, str) else "")
def test_blocking_greedy_rule(orc, name, A, bs):
    """Each block starts at the smallest unassigned unknown and each later
    member is the smallest unassigned unknown adjacent to the block so far,
    or the smallest unassigned one if none is adjacent."""
    o = orc.order(A, bs, 4)
    adj = _adj(A)
    n = A.n
    assert o.nblocks == -(-n // bs)
    assigned = np.zeros(n, bool)
    for b in range(o.nblocks):
        mem = o.members[b * bs:min((b + 1) * bs, n)]
        assert mem[0] == np.flatnonzero(~assigned)[0]
        assigned[mem[0]] = True
        for t in range(1, len(mem)):
            near = set()
            for u in mem[:t]:
                near.update(int(v) for v in adj[u] if not assigned[v])
            if near:
                assert mem[t] == min(near)
            else:
                assert mem[t] == np.flatnonzero(~assigned)[0]
            assigned[mem[t]] = True
    assert assigned.all()


@pytest.mark.parametrize("name,A", list(_graphs()), ids=lambda v: v if isinstance(v, str) else "")
def test_coloring_greedy_rule(orc, name, A):
    """No two adjacent blocks share a color, and each block's color is the
    smallest one not used by an adjacent block of smaller id."""
    bs = 3
    o = orc.order(A, bs, 4)
    adj = _adj(A)
    nbrs = [set() for _ in range(o.nblocks)]
    for u in range(A.n):
        for v in adj[u]:
            bu, bv = o.block_of[u], o.block_of[v]
            if bu != bv:
                nbrs[bu].add(int(bv))
    for b in range(o.nblocks):
        assert all(o.color[b] != o.color[q] for q in nbrs[b])
        used = {int(o.color[q]) for q in nbrs[b] if q < b}
        assert o.color[b] == min(set(range(len(used) + 1)) - used)
    assert o.ncolors == o.color.max() + 1


def _check_structure(o, A):
    bs, w = o.bs, o.w
    n_pad = o.n_pad
    # bijection onto [0, n_pad) minus the dummy positions
    assert len(np.unique(o.perm)) == A.n and o.perm.min() >= 0 and o.perm.max() < n_pad
    assert np.all(np.diff(o.color_start) % (bs * w) == 0)
    color_of = np.searchsorted(o.color_start, o.perm, side="right") - 1
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    cols = A.col
    pi, pj = o.perm[rows], o.perm[cols]
    same = (color_of[rows] == color_of[cols]) & (rows != cols)
    # eq. "BAMC1": no coupling between different level-1 blocks of one color
    assert np.all(pi[same] // (bs * w) == pj[same] // (bs * w))
    # eq. "BAMC-level-2": inside a level-1 block the w x w level-2 blocks are
    # diagonal, i.e. couplings join the same lane m
    assert np.all((pi[same] - pj[same]) % w == 0)
    # the color's unknowns form its segment
    for c in range(o.ncolors):
        sel = color_of == c
        assert np.all((o.perm[sel] >= o.color_start[c]) & (o.perm[sel] < o.color_start[c + 1]))


@pytest.mark.parametrize("bs,w", [(1, 4), (2, 8), (4, 8), (8, 64), (5, 3)])
@pytest.mark.parametrize("name,A", list(_graphs()), ids=lambda v: v if isinstance(v, str) else "")
def test_structure_and_er_condition(orc, name, A, bs, w):
    o = orc.order(A, bs, w)
    _check_structure(o, A)
    # ER condition between BMC (w = 1: no secondary reordering) and HBMC
    ob = orc.order(A, bs, 1)
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    s1 = np.sign(ob.perm[rows].astype(np.int64) - ob.perm[A.col])
    s2 = np.sign(o.perm[rows].astype(np.int64) - o.perm[A.col])
    assert np.array_equal(s1, s2)


@pytest.mark.parametrize("name,A", list(_graphs()), ids=lambda v: v if isinstance(v, str) else "")
def test_w1_is_bmc_numbering(orc, name, A):
    """With w = 1 the secondary reordering is the identity: each block's
    members are consecutive, in insertion order, blocks of a color ascend."""
    bs = 4
    o = orc.order(A, bs, 1)
    for b in range(o.nblocks):
        mem = o.members[b * bs:min((b + 1) * bs, A.n)]
        p = o.perm[mem]
        assert np.array_equal(p, p[0] + np.arange(len(mem)))
    first = o.perm[o.members[::bs]]
    for c in range(o.ncolors):
        assert np.all(np.diff(first[o.color == c]) > 0)


def test_permute_is_similarity(orc):
    A = inputs.random_spd(60, 0.08, 9)
    o = orc.order(A, 4, 8)
    Ab = orc.permute(A, o.perm, o.n_pad)
    D = np.zeros((o.n_pad, o.n_pad))
    for r in range(o.n_pad):
        D[r, Ab.col[Ab.rowptr[r]:Ab.rowptr[r + 1]]] = Ab.val[Ab.rowptr[r]:Ab.rowptr[r + 1]]
    dense = A.to_scipy().toarray()
    assert np.array_equal(D[np.ix_(o.perm, o.perm)], dense)
    dummy = np.setdiff1d(np.arange(o.n_pad), o.perm)
    assert np.array_equal(D[np.ix_(dummy, dummy)], np.eye(len(dummy)))
    assert not D[np.ix_(dummy, o.perm)].any()


def test_check_rejects(orc):
    A = inputs.grid2d_5pt(4)
    assert orc.check(A) == orc.OK
    v = A.val.copy(); v[1] = -0.5                       # breaks value symmetry
    assert orc.check(inputs.CSR(A.n, A.rowptr, A.col, v)) == orc.ENOTSYM
    v = A.val.copy(); v[0] = 0.0                        # zero diagonal
    assert orc.check(inputs.CSR(A.n, A.rowptr, A.col, v)) == orc.EDIAG


# ---------------------------------------------------------------------------
# Reverse Cuthill-McKee (the locality pre-pass, outside the paper): exact
# results derived by hand, and the characterization of a Cuthill-McKee
# sequence under the stated rule on larger graphs.
# ---------------------------------------------------------------------------

def _graph(n, edges):
    rows = [i for i in range(n)] + [a for a, b in edges] + [b for a, b in edges]
    cols = [i for i in range(n)] + [b for a, b in edges] + [a for a, b in edges]
    vals = [4.0] * n + [-1.0] * (2 * len(edges))
    return inputs._from_coo(n, rows, cols, vals)


def test_rcm_path_shuffled(orc):
    """A path whose unknowns are labelled at random: degree 1 at the two
    ends, so the sweep starts at the end with the smaller label and walks to
    the other; reversed, the numbering runs from the other end back."""
    n = 50
    lab = np.random.default_rng(3).permutation(n)          # lab[t]: unknown at place t of the path
    A = _graph(n, [(int(lab[t]), int(lab[t + 1])) for t in range(n - 1)])
    walk = list(lab) if lab[0] < lab[-1] else list(lab[::-1])
    assert list(orc.rcm(A)) == walk[::-1]


def test_rcm_star_and_components(orc):
    """A star (centre 7 of degree 11, leaves of degree 1): start at leaf 0,
    then the centre, then the other leaves by index.  Components: the
    isolated unknown 3 (degree 0) starts first, then the path 0-1-2 from
    its end 0, then 4-5."""
    A = _graph(12, [(7, j) for j in range(12) if j != 7])
    cm = [0, 7] + [j for j in range(1, 12) if j != 7]
    assert list(orc.rcm(A)) == cm[::-1]
    B = _graph(6, [(0, 1), (1, 2), (4, 5)])
    assert list(orc.rcm(B)) == [3, 0, 1, 2, 4, 5][::-1]


def _cm_characterization(A, order):
    """Checks that reversed(order) is the Cuthill-McKee sequence of the
    stated rule: a permutation; each component starts at the unnumbered
    unknown of least (degree, index); every other unknown's parent (its
    earliest-numbered neighbour) comes before it; parents are non-decreasing
    along the sequence, and the children of one parent run by (degree,
    index)."""
    n = A.n
    cm = np.asarray(order)[::-1]
    assert sorted(cm.tolist()) == list(range(n))
    pos = np.empty(n, np.int64)
    pos[cm] = np.arange(n)
    rp, ci = A.rowptr, A.col
    deg = np.array([int(np.sum(ci[rp[i]:rp[i + 1]] != i)) for i in range(n)])
    numbered = np.zeros(n, bool)
    last_parent = -1
    prev_key = None
    for k in range(n):
        v = int(cm[k])
        nb = [int(c) for c in ci[rp[v]:rp[v + 1]] if c != v]
        earlier = [pos[c] for c in nb if pos[c] < k]
        if not earlier:    # a component start
            rest = np.flatnonzero(~numbered)
            best = min(rest, key=lambda u: (deg[u], u))
            assert v == best, (k, v, best)
            last_parent, prev_key = -1, None
        else:
            par = min(earlier)
            assert par >= last_parent, k
            key = (deg[v], v)
            if par == last_parent:
                assert key > prev_key, k
            last_parent, prev_key = par, key
        numbered[v] = True


@pytest.mark.parametrize("make", [lambda: inputs.random_spd(400, 0.01, 5), lambda: inputs.knn_laplacian(2000, 13, 4, 5),
                                  lambda: inputs.grid2d_5pt(23, 17)], ids=["random", "knn", "grid"])
def test_rcm_characterization(orc, make):
    A = make()
    _cm_characterization(A, orc.rcm(A))


def test_rcm_restores_grid_locality(orc):
    """A 40 x 40 grid whose numbering is shuffled: bandwidth back to at most
    the grid's width + 1 (a Cuthill-McKee sweep from a corner runs along
    anti-diagonals), from about the whole matrix."""
    G = inputs.grid2d_5pt(40)
    p = np.random.default_rng(9).permutation(G.n)
    A = orc.renumber(G, p)
    r = orc.rcm(A)
    pos = np.empty(A.n, np.int64)
    pos[r] = np.arange(A.n)
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    assert np.abs(rows - A.col).max() > 1000
    assert np.abs(pos[rows] - pos[A.col]).max() <= 41


def test_order_rcm_composition(orc):
    """order_rcm's permutation is the plain ordering of the renumbered system
    read back in the input's numbering, a bijection onto the non-dummy HBMC
    positions."""
    A = inputs.knn_laplacian(3000, 13, 4, 5)
    r = orc.rcm(A)
    o = orc.order_rcm(A, 2, 32)
    ref = orc.order(orc.renumber(A, r), 2, 32)
    assert np.array_equal(o.perm[r], ref.perm)
    assert len(set(o.perm.tolist())) == A.n and o.perm.max() < o.n_pad
