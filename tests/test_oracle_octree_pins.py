"""Pins of the oracle's octree field: Q2 node numbering, hanging-node
constraints and their resolution (Sec. 2.5, adaptively refined meshes; the
field on a refined mesh must stay continuous, so a node that lies on a
coarser leaf's boundary without being one of that leaf's nodes takes the
coarse leaf's Q2 interpolant).

CPU only.  What fixes the expected results here is geometry and polynomial
algebra, not the oracle itself:

* the hanging set and each constraining leaf against a brute-force test in
  physical coordinates (a node on a leaf's closed box that is not one of the
  leaf's 27 nodes; the coarsest such leaf, the lowest index among equals);
* every Q2 polynomial is reproduced exactly: resolving the hanging nodes of
  its nodal values changes nothing, and evaluation through the cell -> node
  map gives the polynomial back at random points of every leaf;
* a field that is not Q2 does change at the hanging nodes (and only there),
  and after resolution it is continuous across every face between leaves of
  different levels, whichever side evaluates it.

The last tests plant mistakes in copies of the oracle's octree tables (local
node order with a and b swapped, the finest instead of the coarsest
constraining leaf, fine levels resolved first, no resolution) and check
that each one fails a pin.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1612_03369_amd import inputs as I

MAX_LEVEL = 4


def _shell_tree(balanced=True):
    lv, an = I.octree_shell_leaves(base_level=1, max_level=MAX_LEVEL, r_in=0.0, r_out=0.2, width=1.0,
                                   centre=(0.3, 0.35, 0.4))
    if balanced:
        lv, an = I.balance_octree(lv, an, MAX_LEVEL)
    return lv, an


@pytest.fixture(scope="module")
def tree():
    lv, an = _shell_tree(True)
    return O.OracleMesh.octree(lv, an, MAX_LEVEL)


@pytest.fixture(scope="module")
def unbalanced_tree():
    """Level-3 leaves next to level-1 leaves: some nodes lie on the closed boxes of leaves of two
    coarser levels without being nodes of either (outside what the library accepts, but the
    oracle's constraint rule is defined for any tiling, and only such a tree tells the coarsest
    constraining leaf from a finer one)."""
    f = 1 << MAX_LEVEL
    g = np.stack(np.meshgrid(*(np.arange(2),) * 3, indexing="ij")).reshape(3, -1)[::-1] * (f // 2)
    lv, an = I.morton_sort(np.full(8, 1), g, MAX_LEVEL)
    lv, an = I.refine_leaves(lv, an, MAX_LEVEL, np.all(an == 0, axis=0))
    lv, an = I.refine_leaves(lv, an, MAX_LEVEL, np.all(an == f // 4, axis=0) & (lv == 2))
    return O.OracleMesh.octree(lv, an, MAX_LEVEL)


def _boxes(om):
    fine = 1 << om.max_level
    lo = om.anchor.astype(np.float64) / fine                      # [3][nc]
    H = 2.0 ** -om.level.astype(np.float64)                       # [nc]
    return lo, H


def _geometric_constraints(om):
    """(node, leaf) pairs from the definition, in physical coordinates only."""
    P = om.q2_node_coords()                                       # [3][nn], dyadic: exact
    lo, H = _boxes(om)
    best = {}
    for K in range(om.n_cells):
        r = (P - lo[:, K:K + 1]) * (2.0 / H[K])                   # node lattice of K: integers 0..2
        inbox = np.all((r >= 0.0) & (r <= 2.0), axis=0)
        is_node = np.all(r == np.round(r), axis=0)
        for p in np.nonzero(inbox & ~is_node)[0]:
            q = best.get(int(p))
            if q is None or H[K] > H[q] or (H[K] == H[q] and K < q):
                best[int(p)] = K
    return best


def _q2_poly(X):
    x, y, z = X
    return np.stack([x * x + 0.5 * y - z, x * y + z * z - 0.25, y * z * z - x * y * z + 2.0 * x * x * y * y * z * z])


def _rough(X):
    x, y, z = X
    return np.stack([np.sin(7.0 * x + 1.3 * y) * np.cos(5.0 * z), x ** 3 - y * z ** 3, np.exp(x * y) + z ** 4])


def _eval_points(om, U, K, T):
    return np.stack([om.eval(U, K, t) for t in T.T], axis=1)


def _reproduction_error(om, U, F, rng, per_leaf=2):
    """max |u_h - f| over random points of every leaf (f a Q2 polynomial)."""
    lo, H = _boxes(om)
    err = 0.0
    for K in range(om.n_cells):
        T = rng.random((3, per_leaf))
        X = lo[:, K:K + 1] + T * H[K]
        err = max(err, float(np.abs(_eval_points(om, U, K, T) - F(X)).max()))
    return err


def _face_pairs(om):
    """(fine leaf, coarse neighbour, axis, side) for faces between leaves of different levels."""
    fine = 1 << om.max_level
    table = om.fine.reshape(fine, fine, fine)                     # [z][y][x] -> leaf
    out = []
    for F in range(om.n_cells):
        s = 1 << (om.max_level - int(om.level[F]))
        a = om.anchor[:, F].astype(np.int64)
        for ax in range(3):
            for side in (0, 1):
                c = a + s // 2 if s > 1 else a.copy()
                c[ax] = a[ax] - 1 if side == 0 else a[ax] + s
                if c[ax] < 0 or c[ax] >= fine:
                    continue
                N = int(table[c[2], c[1], c[0]])
                if om.level[N] < om.level[F]:
                    out.append((F, N, ax, side))
    return out


def _continuity_error(om, U, pairs, rng, per_face=3):
    """max jump of u_h across the given faces, evaluated from both sides."""
    lo, H = _boxes(om)
    err = 0.0
    for F, N, ax, side in pairs:
        T = rng.random((3, per_face))
        T[ax] = float(side)
        X = lo[:, F:F + 1] + T * H[F]
        TN = (X - lo[:, N:N + 1]) / H[N]
        assert np.all((TN >= 0.0) & (TN <= 1.0))
        err = max(err, float(np.abs(_eval_points(om, U, F, T) - _eval_points(om, U, N, TN)).max()))
    return err


# ----------------------------------------------------------------------------
# pins
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["balanced", "unbalanced"])
def test_hanging_constraints_match_geometry(which, tree, unbalanced_tree):
    om = tree if which == "balanced" else unbalanced_tree
    geo = _geometric_constraints(om)
    got = om.hanging_constraints()
    assert len(got) > (100 if which == "balanced" else 20)
    assert dict(got) == geo
    # coarse levels first (so that a constraining leaf's own hanging nodes are final before use)
    lv = [int(om.level[K]) for _, K in got]
    assert lv == sorted(lv)
    if which == "unbalanced":
        # the tree is chosen so that the coarsest-leaf rule decides: some node is hanging
        # with respect to leaves of two levels
        P = om.q2_node_coords()
        lo, H = _boxes(om)
        multi = 0
        for p, K in geo.items():
            r = (P[:, p:p + 1] - lo) * (2.0 / H)
            hang = np.all((r >= 0) & (r <= 2), axis=0) & ~np.all(r == np.round(r), axis=0)
            multi += len(set(H[hang].tolist())) > 1
        assert multi > 0


def test_node_numbering_is_the_distinct_lattice_points(tree):
    """Every leaf's 27 nodes are its lattice points x0 + (a, b, c) H / 2 in local order a + 3b + 9c,
    nodes are distinct points, and they are numbered in ascending x + M (y + M z) order."""
    om = tree
    P = om.q2_node_coords()
    lo, H = _boxes(om)
    loc = np.array([[a, b, c] for c in range(3) for b in range(3) for a in range(3)], np.float64).T
    for K in range(0, om.n_cells, 7):
        want = lo[:, K:K + 1] + loc * (H[K] / 2)
        assert np.array_equal(P[:, om.cell_nodes[K]], want)
    M = (1 << (MAX_LEVEL + 1)) + 1
    lat = np.round(P * (1 << (MAX_LEVEL + 1))).astype(np.int64)
    key = lat[0] + M * (lat[1] + M * lat[2])
    assert np.all(np.diff(key) > 0)


def test_q2_polynomial_is_reproduced(tree):
    om = tree
    P = om.q2_node_coords()
    U = _q2_poly(P)
    R = om.resolve_hanging(U)
    assert np.abs(R - U).max() <= 1e-15 * np.abs(U).max()
    assert _reproduction_error(om, R, _q2_poly, np.random.default_rng(5)) <= 1e-14


def test_non_q2_field_changes_only_at_hanging_nodes_and_becomes_continuous(tree):
    om = tree
    P = om.q2_node_coords()
    U = _rough(P)
    R = om.resolve_hanging(U)
    hang = np.zeros(om.n_nodes, bool)
    hang[[p for p, _ in om.hanging_constraints()]] = True
    assert np.array_equal(R[:, ~hang], U[:, ~hang])
    assert np.abs(R[:, hang] - U[:, hang]).max() > 1e-3
    pairs = _face_pairs(om)
    assert len(pairs) > 100
    rng = np.random.default_rng(6)
    assert _continuity_error(om, U, pairs, np.random.default_rng(6)) > 1e-3   # visible before resolution
    assert _continuity_error(om, R, pairs, rng) <= 1e-14


def test_resolution_order_matters_and_is_coarse_first(unbalanced_tree):
    """Where a constraining leaf's own face nodes hang on a coarser leaf, they must be final
    before they are used: resolved coarse levels first, the field is continuous everywhere."""
    om = unbalanced_tree
    P = om.q2_node_coords()
    R = om.resolve_hanging(_rough(P))
    assert _continuity_error(om, R, _face_pairs(om), np.random.default_rng(7)) <= 1e-14
    R2 = om.resolve_hanging(_q2_poly(P))
    assert np.abs(R2 - _q2_poly(P)).max() <= 1e-15 * np.abs(R2).max()


# ----------------------------------------------------------------------------
# planted mistakes: each must fail one of the pins above
# ----------------------------------------------------------------------------
def _copy(om):
    return O.OracleMesh.octree(om.level.copy(), om.anchor.copy(), om.max_level)


def test_mutation_swapped_local_order_fails_reproduction(tree):
    om = _copy(tree)
    cn = om.cell_nodes.reshape(-1, 3, 3, 3)                       # [K][c][b][a]
    om.cell_nodes = np.ascontiguousarray(cn.transpose(0, 1, 3, 2).reshape(-1, 27))   # a <-> b
    om.c.cell_nodes = O._p(om.cell_nodes)
    U = om.resolve_hanging(_q2_poly(om.q2_node_coords()))
    assert _reproduction_error(om, U, _q2_poly, np.random.default_rng(5)) > 1e-3


def test_mutation_finest_constraining_leaf_fails_geometry(unbalanced_tree):
    om = _copy(unbalanced_tree)
    orig = O.OracleMesh.hanging_constraints

    def finest(self):
        L = self.max_level
        pairs = orig(self)
        geo_all = {}
        P = self.q2_node_coords()
        lo, H = _boxes(self)
        for p, _ in pairs:
            r = (P[:, p:p + 1] - lo) * (2.0 / H)
            hang = np.nonzero(np.all((r >= 0) & (r <= 2), axis=0) & ~np.all(r == np.round(r), axis=0))[0]
            geo_all[p] = int(hang[np.argmin(H[hang])])
        return sorted(geo_all.items(), key=lambda q: (int(self.level[q[1]]), q[0]))

    om.hanging_constraints = finest.__get__(om)
    assert dict(om.hanging_constraints()) != _geometric_constraints(om)


def test_mutation_fine_levels_first_fails_continuity(unbalanced_tree):
    # (in a vertex-balanced tree no constraining leaf's nodes that a hanging node depends on are
    # themselves hanging, so the order shows only where levels 1 and 3 meet)
    om = _copy(unbalanced_tree)
    orig = O.OracleMesh.hanging_constraints
    om.hanging_constraints = (lambda self: sorted(orig(self), key=lambda q: -int(self.level[q[1]]))).__get__(om)
    R = om.resolve_hanging(_rough(om.q2_node_coords()))
    assert _continuity_error(om, R, _face_pairs(om), np.random.default_rng(6)) > 1e-6


def test_mutation_no_resolution_fails_continuity(tree):
    om = _copy(tree)
    om.hanging_constraints = (lambda self: []).__get__(om)
    R = om.resolve_hanging(_rough(om.q2_node_coords()))
    assert _continuity_error(om, R, _face_pairs(om), np.random.default_rng(6)) > 1e-3
