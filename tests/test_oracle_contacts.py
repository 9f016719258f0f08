"""Pins of the oracle's incremental recolouring (Sec. "Collision Coloring")
and the brute-force proximity reference used to check contact detection."""
import numpy as np

import oracle as O
from paper_2306_09021_amd import scenarios as S

from .test_oracle_solve import check_valid_coloring


def add_contacts(sc, pairs, normals, k_n):
    """Scenario with the contacts appended as weak constraints
    C = y_a - y_b, K = k_n n n^T."""
    import copy
    out = copy.copy(sc)
    ptr = list(np.asarray(sc.wc_ptr, np.int64))
    vert = list(np.asarray(sc.wc_vert, np.int64))
    w = list(np.asarray(sc.wc_w, np.float64))
    K = [list(r) for r in np.asarray(sc.wc_K, np.float64).reshape(-1, 6)]
    for (a, b), nrm in zip(pairs, normals):
        nrm = np.asarray(nrm, np.float64) / np.linalg.norm(nrm)
        vert += [int(a), int(b)]
        w += [1.0, -1.0]
        ptr.append(len(vert))
        nn = k_n * np.outer(nrm, nrm)
        K.append([nn[0, 0], nn[0, 1], nn[0, 2], nn[1, 1], nn[1, 2], nn[2, 2]])
    out.wc_ptr = np.array(ptr, np.int32)
    out.wc_vert = np.array(vert, np.int32)
    out.wc_w = np.array(w, np.float64)
    out.wc_K = np.array(K, np.float64).reshape(-1, 6)
    return out


def components(nv, tets):
    """Connected parts of a tet mesh (union-find)."""
    parent = np.arange(nv)

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i
    for t in np.asarray(tets):
        r0 = find(t[0])
        for j in t[1:]:
            r = find(j)
            if r != r0:
                parent[r] = r0
    roots = np.array([find(i) for i in range(nv)])
    _, comp = np.unique(roots, return_inverse=True)
    return comp


def brute_contacts(x, tets, is_dir, radius):
    """All pairs a < b of surface vertices of different parts within radius
    (not both Dirichlet), sorted, with normals (x_b - x_a) / |x_b - x_a|."""
    comp = components(x.shape[0], tets)
    surf = np.sort(S.surface_vertices(np.asarray(tets)))
    pairs, normals = [], []
    for ia, a in enumerate(surf):
        d = x[surf[ia + 1:]] - x[a]
        dist = np.linalg.norm(d, axis=1)
        for jb in np.nonzero(dist <= radius)[0]:
            b = surf[ia + 1 + jb]
            if comp[a] == comp[b] or (is_dir[a] and is_dir[b]) or dist[jb] == 0.0:
                continue
            pairs.append((a, b))
            normals.append(d[jb] / dist[jb])
    order = np.lexsort((np.array([p[1] for p in pairs]), np.array([p[0] for p in pairs]))) \
        if pairs else []
    return (np.array(pairs, np.int32).reshape(-1, 2)[order],
            np.array(normals, np.float64).reshape(-1, 3)[order])


def test_recolor_by_hand():
    """Two separate tets coloured 0..3 each; a contact between vertex 0 and
    vertex 4 (both colour 0): vertex 0 (processed first) sees 1, 2, 3 from
    its tet and 0 from vertex 4, so it takes colour 4; vertex 4 then sees
    1, 2, 3 and 4 and keeps colour 0."""
    X = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1],
                  [3.0, 0, 0], [4, 0, 0], [3, 1, 0], [3, 0, 1]])
    T = np.array([[0, 1, 2, 3], [4, 5, 6, 7]], np.int32)
    sc = S.Scenario(name="hand", rest_pos=X, tets=T, model="nh", E=np.asarray(1.0),
                    nu=np.asarray(0.3), dirichlet_idx=np.zeros(0, np.int32),
                    dirichlet_x=np.zeros((0, 3)), x0=X)
    col, nc = O.color(O.make_problem(sc))
    assert list(col) == [0, 1, 2, 3, 0, 1, 2, 3]
    sc2 = add_contacts(sc, [(0, 4)], [(1.0, 0, 0)], 1.0)
    new, nc2 = O.recolor(O.make_problem(sc2), col, [0, 4])
    assert list(new) == [4, 1, 2, 3, 0, 1, 2, 3] and nc2 == 5


def test_recolor_two_blocks_is_valid_and_local():
    sc = S.two_blocks(5, gap=0.05)
    op = O.make_problem(sc)
    col, _ = O.color(op)
    x = sc.initial_iterate()
    x[sc.n_verts // 2:, 0] -= 0.04          # bring the blocks within reach
    pairs, normals = brute_contacts(x, sc.tets, op.is_dir, 0.05)
    assert pairs.shape[0] > 10
    sc2 = add_contacts(sc, pairs, normals, 1e8)
    op2 = O.make_problem(sc2)
    nodes = np.unique(pairs.reshape(-1))
    nodes = nodes[op2.is_dir[nodes] == 0]
    new, nc = O.recolor(op2, col, nodes)
    check_valid_coloring(op2, new)
    # only vertices incident to the new constraints may change
    changed = np.nonzero(new != col)[0]
    assert set(changed.tolist()) <= set(nodes.tolist())


def test_brute_contacts_symmetric_and_sorted():
    sc = S.two_blocks(4, gap=0.01)
    op = O.make_problem(sc)
    pairs, normals = brute_contacts(sc.initial_iterate(), sc.tets, op.is_dir, 0.02)
    # facing faces of two 4x4 grids at distance 0.01: each vertex pairs with its mirror
    assert pairs.shape[0] == 16
    assert np.all(pairs[:, 0] < pairs[:, 1])
    assert np.allclose(normals, [1.0, 0.0, 0.0])
