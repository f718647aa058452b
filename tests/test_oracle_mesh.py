"""Pins of the oracle's mesh set-up: orientation, rest values, edges, colours.

Checked against closed-form counts of the 5-tetrahedra-per-hexahedron slab,
the slab's exact volume, a library determinant, and exhaustive properties of
a greedy colouring (no shared particle inside a colour; every colour c > 0 of
a constraint is forced by an earlier neighbour of each smaller colour).
"""
import numpy as np
import pytest

from paper_2503_18616_amd import workloads as W

GRIDS = [(1, 1, 1), (2, 1, 1), (3, 2, 2), (8, 5, 3), (16, 10, 4), (12, 8, 3)]


def closed_form_counts(nx, ny, nz):
    V = (nx + 1) * (ny + 1) * (nz + 1)
    axis = nx * (ny + 1) * (nz + 1) + (nx + 1) * ny * (nz + 1) + (nx + 1) * (ny + 1) * nz
    diag = nx * ny * (nz + 1) + nx * (ny + 1) * nz + (nx + 1) * ny * nz
    pinned_face_edges = nx * (ny + 1) + (nx + 1) * ny + nx * ny
    return V, axis + diag, axis + diag - pinned_face_edges, 5 * nx * ny * nz


@pytest.mark.parametrize("grid", GRIDS)
def test_counts_and_volumes(oracle_lib, grid):
    m = W.slab_mesh(*grid)
    om = oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
    V, E_all, E_free, T = closed_form_counts(*grid)
    assert om.num_vertices == V
    assert om.num_tets == T
    assert om.num_edges == E_free
    # orientation: every rest volume positive, they tile the slab exactly
    assert (om.rest_volume > 0).all()
    vol = np.prod(np.float64(np.float32(W.SLAB_EXTENT)))
    assert abs(om.rest_volume.sum() - np.prod([float(np.float32(e)) for e in W.SLAB_EXTENT])) < 1e-12 * vol + 1e-15
    # rest volume equals a library determinant of the oriented tetrahedra
    X = om.rest
    t = om.tets
    det = np.linalg.det(np.stack([X[t[:, 1]] - X[t[:, 0]], X[t[:, 2]] - X[t[:, 0]],
                                  X[t[:, 3]] - X[t[:, 0]]], axis=1)) / 6.0
    np.testing.assert_allclose(om.rest_volume, det, rtol=1e-12)
    # oriented tets are the input tets with at most the last two ids swapped
    same = (t == m.tets).all(axis=1)
    swapped = (t[:, :2] == m.tets[:, :2]).all(axis=1) & (t[:, 2] == m.tets[:, 3]) & (t[:, 3] == m.tets[:, 2])
    assert (same | swapped).all()


@pytest.mark.parametrize("grid", GRIDS)
def test_edges_are_unique_tet_edges(oracle_lib, grid):
    m = W.slab_mesh(*grid)
    om = oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
    e = om.edges
    assert (e[:, 0] < e[:, 1]).all()
    key = e[:, 0].astype(np.int64) * om.num_vertices + e[:, 1]
    assert (np.diff(key) > 0).all(), "edges must be sorted and unique"
    tet_pairs = set()
    for q in m.tets:
        for a in range(4):
            for b in range(a + 1, 4):
                tet_pairs.add((min(q[a], q[b]), max(q[a], q[b])))
    free = {p for p in tet_pairs if m.inv_mass[p[0]] > 0 or m.inv_mass[p[1]] > 0}
    assert set(map(tuple, e.tolist())) == free
    np.testing.assert_allclose(om.rest_length,
                               np.linalg.norm(om.rest[e[:, 0]] - om.rest[e[:, 1]], axis=1),
                               rtol=1e-15)


def _check_colouring(num_vertices, verts, colours, num_colours):
    n = len(colours)
    assert colours.min() == 0 and colours.max() == num_colours - 1
    # no particle appears twice inside one colour (exhaustive)
    for c in range(num_colours):
        members = verts[colours == c].ravel()
        assert len(np.unique(members)) == len(members), f"colour {c} shares a particle"
    # greedy-minimal: for colour c, every smaller colour is taken by an earlier neighbour
    incident = [[] for _ in range(num_vertices)]
    for j in range(n):
        for v in verts[j]:
            incident[v].append(j)
    for j in range(n):
        earlier = {colours[o] for v in verts[j] for o in incident[v] if o < j}
        assert set(range(colours[j])) <= earlier
        assert colours[j] not in earlier


@pytest.mark.parametrize("grid", [(1, 1, 1), (2, 1, 1), (8, 5, 3), (16, 10, 4)])
def test_colouring_valid_and_greedy(oracle_lib, grid):
    m = W.slab_mesh(*grid)
    om = oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
    _check_colouring(om.num_vertices, om.edges, om.edge_colour, om.num_edge_colours)
    _check_colouring(om.num_vertices, om.tets, om.tet_colour, om.num_tet_colours)
    # colour count is at least the largest number of constraints sharing a particle
    deg_e = np.bincount(om.edges.ravel(), minlength=om.num_vertices).max()
    deg_t = np.bincount(om.tets.ravel(), minlength=om.num_vertices).max()
    assert om.num_edge_colours >= deg_e
    assert om.num_tet_colours >= deg_t


def test_colour_counts_of_the_two_slabs(oracle_lib):
    """Edge colouring of both slabs is optimal (= the largest particle degree, 18)."""
    for grid, n_tc in [((8, 5, 3), 37), ((16, 10, 4), 37)]:
        m = W.slab_mesh(*grid)
        om = oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
        assert om.num_edge_colours == 18
        assert np.bincount(om.edges.ravel()).max() == 18
        assert om.num_tet_colours == n_tc


def test_schedule_groups_by_colour(oracle_lib):
    m = W.slab_mesh(8, 5, 3)
    om = oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
    for ptr, order, col, nc in [(om.edge_ptr, om.edge_order, om.edge_colour, om.num_edge_colours),
                                (om.tet_ptr, om.tet_order, om.tet_colour, om.num_tet_colours)]:
        assert ptr[0] == 0 and ptr[-1] == len(col) and len(ptr) == nc + 1
        assert sorted(order.tolist()) == list(range(len(col)))
        for c in range(nc):
            seg = order[ptr[c]:ptr[c + 1]]
            assert (col[seg] == c).all() and (np.diff(seg) > 0).all()


def test_setup_errors(oracle_lib):
    m = W.slab_mesh(1, 1, 1)
    bad = m.tets.copy()
    bad[0, 0] = 99
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, bad)
    flat = m.rest_pos.copy()
    flat[:, 2] = 0.0           # every tetrahedron degenerates to zero volume
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.prepare_mesh(flat, np.ones(len(flat), np.float32), m.tets)


def test_all_pinned_constraints_dropped(oracle_lib):
    m = W.slab_mesh(2, 1, 1)
    w = m.inv_mass.copy()
    w[:] = 0.0
    w[0] = 1000.0              # only vertex 0 free
    om = oracle_lib.prepare_mesh(m.rest_pos, w, m.tets)
    assert all((w[q] > 0).any() for q in om.tets)
    assert all((w[e] > 0).any() for e in om.edges)
    assert om.num_tets == int(sum((m.tets == 0).any(axis=1)))


# ------------------------------------------------------------------ largest-first colouring
def _chain(n):
    """n distance constraints (i, i + 1) along a chain of n + 1 particles."""
    return np.array([[i, i + 1] for i in range(n)], np.int32)


def test_largest_first_on_a_chain_by_hand(oracle_lib):
    """On a chain the conflict graph is a path.  Largest first starts with the
    lowest-index constraint of the largest conflict count (constraint 1: two
    conflicts), which rules out 0 and 2; then the candidate with the most
    ruled-out neighbours is 3, which rules out 4; then 5.  The remaining
    constraints 0, 2, 4 form the second colour.  Greedy gives the opposite
    parity."""
    lf, n_lf = oracle_lib.largest_first_colour(7, _chain(6))
    assert n_lf == 2
    assert lf.tolist() == [1, 0, 1, 0, 1, 0]
    gr, n_gr = oracle_lib.greedy_colour(7, _chain(6))
    assert n_gr == 2 and gr.tolist() == [0, 1, 0, 1, 0, 1]


def test_largest_first_star_and_ties_by_hand(oracle_lib):
    """A star of four constraints around particle 0 plus one constraint (5, 6)
    apart.  Every star constraint has three conflicts, so the first colour
    starts with the lowest index, 0, rules out 1..3 and adds the only
    candidate left, 4; the star constraints 1, 2, 3 then take one colour each
    in index order."""
    verts = np.array([[0, 1], [0, 2], [0, 3], [0, 4], [5, 6]], np.int32)
    lf, n = oracle_lib.largest_first_colour(7, verts)
    assert n == 4 and lf.tolist() == [0, 1, 2, 3, 0]


def test_largest_first_cut_keeps_the_first_64_picks(oracle_lib):
    """100 disjoint constraints form one colour of 100 members.  With the cut at
    100 that colour keeps its first 64 picks (all tied: by index, 0..63) and
    the other 36 form the next colour; with the cut at 99 it stays whole."""
    verts = np.array([[2 * i, 2 * i + 1] for i in range(100)], np.int32)
    whole, n = oracle_lib.largest_first_colour(200, verts, 99)
    assert n == 1 and not whole.any()
    cut, n = oracle_lib.largest_first_colour(200, verts, 100)
    assert n == 2
    assert (cut[:64] == 0).all() and (cut[64:] == 1).all()


def test_largest_first_cap_keeps_the_first_picks(oracle_lib):
    """300 disjoint constraints form one colour.  Capped at 256 it keeps its
    first 256 picks (all tied: by index, 0..255) and the other 44 form the
    next colour; with the cap at 300 it stays whole."""
    verts = np.array([[2 * i, 2 * i + 1] for i in range(300)], np.int32)
    whole, n = oracle_lib.largest_first_colour(600, verts, 0, 300)
    assert n == 1 and not whole.any()
    capped, n = oracle_lib.largest_first_colour(600, verts, 0, 256)
    assert n == 2
    assert (capped[:256] == 0).all() and (capped[256:] == 1).all()


@pytest.mark.parametrize("tets_in_star, capped", [(33, True), (35, False)])
def test_capped_fit_counts_each_kind_rounded_up_to_even(oracle_lib, tets_in_star, capped):
    """CAPPED_FIT keeps the cap while the edge and tetrahedron colour counts,
    each rounded up to even, sum to at most 64.  Edges: a star of 29 edges
    (29 colours) and 300 disjoint edges that join the first colour, which the
    cap splits (so the capped and uncapped edge colourings differ, with 29
    colours each); tetrahedra: a star of 33 or 35 sharing one vertex (one
    colour each).  30 + 34 = 64 keeps the cap; 30 + 36 = 66 does not, though
    29 + 35 = 64 unrounded would."""
    star = [[0, 1 + i] for i in range(29)]
    loose = [[1000 + 2 * i, 1001 + 2 * i] for i in range(300)]
    edges = np.array(star + loose, np.int32)
    tets = np.array([[0, 2000 + 3 * j, 2001 + 3 * j, 2002 + 3 * j] for j in range(tets_in_star)],
                    np.int32)
    V = 2000 + 3 * tets_in_star
    (ec, nec), (tc, ntc) = oracle_lib.mesh_colours(V, edges, tets, oracle_lib.COLOURING_CAPPED_FIT)
    cap_e, n_cap = oracle_lib.colour(V, edges, oracle_lib.COLOURING_CAPPED)
    free_e, n_free = oracle_lib.colour(V, edges, oracle_lib.COLOURING_LARGEST_FIRST)
    assert n_cap == n_free == 29 and not np.array_equal(cap_e, free_e)
    assert ntc == tets_in_star
    assert np.array_equal(ec, cap_e if capped else free_e) and nec == 29
    with pytest.raises(ValueError):
        oracle_lib.colour(V, edges, oracle_lib.COLOURING_CAPPED_FIT)


def test_capped_first_colour_is_a_prefix_of_the_uncapped_one(oracle_lib):
    """The cap changes no pick before it applies: on the 16x10x4 slab the first
    capped edge colour is 256 of the first uncapped colour's members (which
    has more), and every colour of the capped edge colouring holds at most
    256 edges."""
    m = W.slab_mesh(16, 10, 4)
    om = oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
    free, _ = oracle_lib.largest_first_colour(m.num_vertices, om.edges)
    capped, n = oracle_lib.largest_first_colour(m.num_vertices, om.edges, 0, 256)
    first_free, first_capped = set(np.flatnonzero(free == 0)), set(np.flatnonzero(capped == 0))
    assert len(first_free) > 256 and len(first_capped) == 256
    assert first_capped <= first_free
    assert np.bincount(capped).max() <= 256 and n >= 18


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("colouring", [1, 2, 3, 4])
def test_largest_first_colours_are_valid_and_maximal(oracle_lib, grid, colouring):
    """Every colour is a set of constraints sharing no particle; a colour that
    was not cut is maximal among the constraints coloured after it (each of
    them conflicts with one of its members); with the cut no colour has 65 to
    100 members, with the cap none more than 256."""
    m = W.slab_mesh(*grid)
    om = oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets, colouring=colouring)
    for verts, col, nc in ((om.edges, om.edge_colour, om.num_edge_colours),
                           (om.tets, om.tet_colour, om.num_tet_colours)):
        assert col.min() == 0 and col.max() == nc - 1
        sizes = np.bincount(col, minlength=nc)
        touched = []
        for c in range(nc):
            members = verts[col == c].ravel()
            assert len(np.unique(members)) == len(members), f"colour {c} shares a particle"
            touched.append(set(members.tolist()))
        for j in range(len(col)):
            for c in range(col[j]):
                cap = {3: oracle_lib.COLOUR_CAP, 4: oracle_lib.COLOUR_CAP_128}.get(colouring)
                cut = (colouring == 2 and sizes[c] == 64) or (cap is not None and sizes[c] == cap)
                if not cut:
                    assert touched[c] & set(verts[j].tolist()), (j, c)
        if colouring == 2:
            assert not ((sizes > 64) & (sizes <= oracle_lib.WAVE_CUT_ABOVE)).any()
        if colouring == 3:
            assert sizes.max() <= oracle_lib.COLOUR_CAP
        if colouring == 4:
            assert sizes.max() <= oracle_lib.COLOUR_CAP_128


def test_largest_first_reaches_the_degree_bound(oracle_lib):
    """On the 8x5x3 and 12x8x3 slabs largest first colours the tetrahedra with
    32 colours: the largest number of tetrahedra sharing one particle, a lower
    bound for any colouring, so the count is optimal (greedy needs 37)."""
    for grid in ((8, 5, 3), (12, 8, 3)):
        m = W.slab_mesh(*grid)
        om = oracle_lib.prepare_mesh(m.rest_pos, m.inv_mass, m.tets, colouring=1)
        degree = np.bincount(om.tets.ravel()).max()
        assert degree == 32 and om.num_tet_colours == degree
