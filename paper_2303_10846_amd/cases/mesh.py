"""Seeded tetrahedral, hexahedral and mixed meshes for the synthetic workloads.

This module only builds inputs: node coordinates, cells, tagged boundary
faces and a colour-major cell order.  It holds none of the scheme's
arithmetic (no face geometry, no fluxes); the solver library and the CPU
oracle each derive their own geometry from these arrays.

Boundary tags used by the case definitions:
    1  solid wall (diffuse reflection)
    2  second wall group (cavity lid) or far field (external flows)
"""
from __future__ import annotations

import itertools
import math

import numpy as np

__all__ = [
    "folded_faces",
    "kuhn_box_mesh",
    "hex_box_mesh",
    "mixed_box_mesh",
    "color_major_cells",
    "shell_mesh",
    "sphere_body",
    "capsule_body",
    "color_major",
    "boundary_triangles",
    "tet_volumes",
]


def tet_volumes(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Signed volumes (positive for right-handed vertex order)."""
    a = xyz[tets[:, 0]]
    d1 = xyz[tets[:, 1]] - a
    d2 = xyz[tets[:, 2]] - a
    d3 = xyz[tets[:, 3]] - a
    return np.einsum("ij,ij->i", d1, np.cross(d2, d3)) / 6.0


def _orient(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    v = tet_volumes(xyz, tets)
    tets = tets.copy()
    neg = v < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    return tets


def _face_keys(tets: np.ndarray) -> np.ndarray:
    """The 4 faces of every tet as sorted vertex triples, shape [4*nt, 3]."""
    loc = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    f = tets[:, loc].reshape(-1, 3)
    return np.sort(f, axis=1)


def _match_faces(tets: np.ndarray):
    """Returns (pairs [n_int,2] of tet ids sharing a face, boundary keys [n_b,3])."""
    keys = _face_keys(tets)
    owner = np.repeat(np.arange(len(tets)), 4)
    order = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
    ks = keys[order]
    same = np.all(ks[1:] == ks[:-1], axis=1)
    if np.any(same[1:] & same[:-1]):
        raise ValueError("non-manifold mesh: a face is shared by more than two tets")
    first = np.nonzero(same)[0]
    pairs = np.stack([owner[order[first]], owner[order[first + 1]]], axis=1)
    in_pair = np.zeros(len(ks), dtype=bool)
    in_pair[first] = True
    in_pair[first + 1] = True
    bkeys = ks[~in_pair]
    return pairs, bkeys


def boundary_triangles(tets: np.ndarray) -> np.ndarray:
    return _match_faces(tets)[1]


def folded_faces(xyz: np.ndarray, tets: np.ndarray) -> int:
    """Number of interior faces whose two tets lie on the same side of the face plane (a folded mesh)."""
    keys = _face_keys(tets)
    owner = np.repeat(np.arange(len(tets)), 4)
    opp = tets[:, [0, 1, 2, 3]].reshape(-1)  # vertex opposite face slot a is tets[:, a]
    order = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
    ks = keys[order]
    same = np.nonzero(np.all(ks[1:] == ks[:-1], axis=1))[0]
    fa, fb = order[same], order[same + 1]
    k = keys[fa]
    a, b, c = xyz[k[:, 0]], xyz[k[:, 1]], xyz[k[:, 2]]
    n = np.cross(b - a, c - a)
    sa = np.einsum("ij,ij->i", xyz[opp[fa]] - a, n)
    sb = np.einsum("ij,ij->i", xyz[opp[fb]] - a, n)
    return int(np.sum(sa * sb >= 0.0))


def _kempe_free(x, nbr, color, top, max_chain=4096):
    """Give cell x (colour `top`) a colour below `top`, by a Kempe-chain interchange if none is free.

    For a neighbour y of x, of colour a, and a colour b != a below `top`: the connected set of cells coloured
    a or b that contains y (the chain) has its two colours swapped, which keeps the colouring proper.  If
    afterwards no neighbour of x is coloured a, x takes a.  Chains above max_chain cells are not tried.
    Returns True on success (color updated in place).
    """
    used = {int(color[j]) for j in nbr[x]}
    free = [c for c in range(top) if c not in used]
    if free:
        color[x] = free[0]
        return True
    for y in nbr[x]:
        a = int(color[y])
        for b in range(top):
            if b == a:
                continue
            chain, stack = {y}, [y]
            while stack and len(chain) <= max_chain:
                u = stack.pop()
                for v in nbr[u]:
                    if v not in chain and int(color[v]) in (a, b):
                        chain.add(v)
                        stack.append(v)
            if len(chain) > max_chain:
                continue
            after = [(b if int(color[j]) == a else a) if j in chain else int(color[j]) for j in nbr[x]]
            if a in after:
                continue
            for u in chain:
                color[u] = b if color[u] == a else a
            color[x] = a
            return True
    return False


def _greedy_colours(nbr, order, n):
    """First-fit colouring of the cells in `order` (colours as bit positions of a small mask)."""
    color = [-1] * n
    for i in order:
        used = 0
        for j in nbr[i]:
            cj = color[j]
            if cj >= 0:
                used |= 1 << cj
        c = 0
        while used >> c & 1:
            c += 1
        color[i] = c
    return np.array(color, dtype=np.int64)


def _sweep_cost(color):
    """Cell relaxations of two forward + backward colour pairs with the classes ordered second largest first and
    largest last: the last class is relaxed twice, the first three times, the others four times."""
    s = np.sort(np.bincount(color))[::-1]
    return 2 * s[0] + (3 * s[1] if len(s) > 1 else 0) + 4 * int(s[2:].sum())


def color_major(xyz: np.ndarray, tets: np.ndarray, search_cells: int = 150_000):
    """Colouring of the face-adjacency graph and colour-major renumbering.

    1. Cells are put in Morton order of their centroids (locality) and coloured greedily (first fit).
    2. Meshes of up to `search_cells` cells: iterated greedy recolouring (Culberson's method: recolour first fit
       with the cells taken class by class, the classes largest first or in a seeded random order), which never
       adds a colour, until three colours are reached (a face graph with odd cycles needs three); then a few
       more rounds keep the three-colouring with the fewest sweep relaxations (_sweep_cost).
    3. Otherwise, a sparse highest class (under 5% of the cells) is removed by Kempe-chain interchanges while
       that succeeds.
    4. The classes are ordered so that the largest comes last and the second largest first.  A forward +
       backward pair of colour sweeps relaxes the last class once at the turn (its second relaxation would
       repeat the first bit for bit) and, from the second pair on, the first class once at the other turn, so
       large end classes mean fewer relaxations per pair; fewer colours mean fewer sweep launches.

    Cells keep their Morton order within a class.  Returns (tets_reordered, color_offsets) with
    color_offsets[c]..color_offsets[c+1] the cells of colour c.  No two cells of one colour share a face.
    """
    morton = _morton_order(xyz[tets].mean(axis=1))
    tets = tets[morton]
    pairs, _ = _match_faces(tets)
    order, offsets = _colour_major_order(pairs, len(tets), search_cells)
    return np.ascontiguousarray(tets[order]), offsets


def _morton_order(cen: np.ndarray) -> np.ndarray:
    lo = cen.min(axis=0)
    span = np.maximum(cen.max(axis=0) - lo, 1e-300)
    q = np.minimum(((cen - lo) / span * 1023.0).astype(np.int64), 1023)
    code = np.zeros(len(cen), dtype=np.int64)
    for b in range(10):
        for ax in range(3):
            code |= ((q[:, ax] >> b) & 1) << (3 * b + ax)
    return np.argsort(code, kind="stable")


def _colour_major_order(pairs: np.ndarray, nt: int, search_cells: int):
    """Steps 1-4 of color_major on cells already in Morton order: (cell order, colour offsets)."""
    nbr = [[] for _ in range(nt)]
    for a, b in pairs.tolist():
        nbr[a].append(b)
        nbr[b].append(a)
    color = _greedy_colours(nbr, range(nt), nt)

    def reorder(col, rng, largest_first):
        classes = [np.nonzero(col == k)[0] for k in range(int(col.max()) + 1)]
        perm = (np.argsort([-len(x) for x in classes], kind="stable") if largest_first
                else rng.permutation(len(classes)))
        return _greedy_colours(nbr, np.concatenate([classes[k] for k in perm]), nt)

    if nt <= search_cells:
        rng = np.random.default_rng(0)
        for it in range(400):
            if color.max() + 1 <= 3:
                break
            new = reorder(color, rng, largest_first=(it % 2 == 0))
            if new.max() <= color.max():
                color = new
        if color.max() + 1 == 3:
            best, cur = color, color
            for it in range(30):
                new = reorder(cur, rng, largest_first=(it % 3 != 0))
                if new.max() + 1 == 3:
                    cur = new
                    if _sweep_cost(cur) < _sweep_cost(best):
                        best = cur
            color = best
    ncol = int(color.max()) + 1
    while ncol > 2:
        top = ncol - 1
        cells = np.nonzero(color == top)[0]
        if len(cells) > 0.05 * nt:
            break
        trial = color.copy()
        if not all(_kempe_free(int(x), nbr, trial, top) for x in cells):
            break
        color = trial
        ncol -= 1
    sizes = np.bincount(color, minlength=ncol)
    by_size = list(np.argsort(-sizes, kind="stable"))
    seq = by_size[1:] + by_size[:1] if ncol > 1 else by_size     # second largest first, largest last
    rank = np.empty(ncol, dtype=np.int64)
    rank[np.asarray(seq, dtype=np.int64)] = np.arange(ncol)
    color = rank[color]
    order = np.argsort(color, kind="stable")
    offsets = np.zeros(ncol + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(np.bincount(color, minlength=ncol))
    return order, offsets


# --------------------------------------------------------------------------
# Mixed-element meshes: cells [nc][8] padded with -1, kinds = node count (4 tetrahedron, 5 pyramid, 6 prism,
# 8 hexahedron), boundary faces [nb][4] padded with -1 (a triangle has -1 in the last place)
# --------------------------------------------------------------------------

LOCAL_FACES = {
    4: ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)),
    5: ((0, 1, 2, 3), (0, 1, 4), (1, 2, 4), (2, 3, 4), (3, 0, 4)),
    6: ((0, 1, 2), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5)),
    8: ((0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)),
}


def _cell_face_lists(cells: np.ndarray, kinds: np.ndarray):
    """Every face of every cell: (cyclic node lists [m][4] padded with -1, sorted keys [m][4], owner [m])."""
    cyc, own = [], []
    for i, (c, k) in enumerate(zip(cells.tolist(), kinds.tolist())):
        for lf in LOCAL_FACES[k]:
            v = [c[a] for a in lf] + [-1] * (4 - len(lf))
            cyc.append(v)
            own.append(i)
    cyc = np.array(cyc, dtype=np.int64)
    keys = cyc.copy()
    tri = keys[:, 3] < 0
    keys[tri, :3] = np.sort(keys[tri, :3], axis=1)
    keys[~tri] = np.sort(keys[~tri], axis=1)
    return cyc, keys, np.array(own, dtype=np.int64)


def match_faces_cells(cells: np.ndarray, kinds: np.ndarray):
    """(pairs [n_int][2] of cells sharing a face, boundary faces [n_b][4] as cyclic node lists)."""
    cyc, keys, own = _cell_face_lists(cells, kinds)
    order = np.lexsort(keys.T[::-1])
    ks = keys[order]
    same = np.all(ks[1:] == ks[:-1], axis=1)
    if np.any(same[1:] & same[:-1]):
        raise ValueError("non-manifold mesh: a face is shared by more than two cells")
    first = np.nonzero(same)[0]
    pairs = np.stack([own[order[first]], own[order[first + 1]]], axis=1)
    in_pair = np.zeros(len(ks), dtype=bool)
    in_pair[first] = True
    in_pair[first + 1] = True
    return pairs, cyc[order[~in_pair]]


def color_major_cells(xyz: np.ndarray, cells: np.ndarray, kinds: np.ndarray, search_cells: int = 150_000):
    """color_major for mixed cells: returns (cells, kinds) in colour-major order and the colour offsets."""
    cen = np.array([xyz[c[:k]].mean(axis=0) for c, k in zip(cells, kinds)])
    morton = _morton_order(cen)
    cells, kinds = cells[morton], kinds[morton]
    pairs, _ = match_faces_cells(cells, kinds)
    order, offsets = _colour_major_order(pairs, len(cells), search_cells)
    return np.ascontiguousarray(cells[order]), np.ascontiguousarray(kinds[order]), offsets


def _sub_tet_volumes(xyz, cells, kinds):
    """Signed volumes of the tetrahedra from each cell's node average to the triangles of its faces (quads fanned
    about their node average), each face's in the orientation of its local node order; a valid cell has all of
    one face's of one sign, and that sign the same for every face when the local orders are consistent."""
    out = []
    for c, k in zip(cells.tolist(), kinds.tolist()):
        p0 = xyz[c[:k]].mean(axis=0)
        vs = []
        for lf in LOCAL_FACES[k]:
            p = xyz[[c[a] for a in lf]]
            tris = [p] if len(lf) == 3 else [np.array([p[q], p[(q + 1) % 4], p.mean(axis=0)]) for q in range(4)]
            vs.append([float(np.cross(t[1] - t[0], t[2] - t[0]) @ (t[0] - p0)) / 6.0 for t in tris])
        out.append(vs)
    return out


def _cells_valid(xyz, cells, kinds) -> bool:
    for vs in _sub_tet_volumes(xyz, cells, kinds):
        for face in vs:
            if not (all(v > 0 for v in face) or all(v < 0 for v in face)):
                return False
    return True


def _box_grid(n, seed, jitter, length):
    h = length / n
    m = n + 1
    g = np.arange(m) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    xyz0 = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    ijk = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1).reshape(-1, 3)
    interior = np.all((ijk > 0) & (ijk < n), axis=1)
    return xyz0, interior, (lambda i, j, k: (i * m + j) * m + k), h


def _hex_nodes(nid, i, j, k):
    return [nid(i, j, k), nid(i + 1, j, k), nid(i + 1, j + 1, k), nid(i, j + 1, k),
            nid(i, j, k + 1), nid(i + 1, j, k + 1), nid(i + 1, j + 1, k + 1), nid(i, j + 1, k + 1)]


def _finish_box(xyz, cells, kinds, length, tag_of_plane):
    cells_c, kinds_c, offsets = color_major_cells(xyz, cells, kinds)
    _, bcyc = match_faces_cells(cells_c, kinds_c)
    fc = np.array([xyz[[v for v in f if v >= 0]].mean(axis=0) for f in bcyc])
    tags = np.zeros(len(bcyc), dtype=np.int64)
    for ax in range(3):
        for side in (0, 1):
            on = np.abs(fc[:, ax] - side * length) < 1e-12 * max(length, 1.0)
            tags[on] = tag_of_plane(ax, side)
    if np.any(tags == 0):
        raise RuntimeError("unclassified boundary face")
    return dict(xyz=xyz, cells=cells_c.astype(np.int64), kinds=kinds_c.astype(np.int64), bface=bcyc, btag=tags,
                color_offsets=offsets)


def hex_box_mesh(n: int = 6, seed: int = 0, jitter: float = 0.15, length: float = 1.0, tag_of_plane=None):
    """n^3 hexahedra on [0,L]^3 (the paper's cavity mesh is hexahedral, Sec. 4.1).  Interior nodes are jittered by
    U(-jitter*h, jitter*h)^3 from ``numpy.random.default_rng(seed)``, so faces are warped quadrilaterals; a draw
    that folds a cell is redrawn.  Tags as kuhn_box_mesh."""
    if tag_of_plane is None:
        def tag_of_plane(axis, side):
            return 2 if (axis == 2 and side == 1) else 1
    xyz0, interior, nid, h = _box_grid(n, seed, jitter, length)
    cells = np.array([_hex_nodes(nid, i, j, k) for i in range(n) for j in range(n) for k in range(n)],
                     dtype=np.int64)
    kinds = np.full(len(cells), 8, dtype=np.int64)
    rng = np.random.default_rng(seed)
    for _ in range(100):
        xyz = xyz0.copy()
        xyz[interior] += rng.uniform(-jitter * h, jitter * h, size=(int(interior.sum()), 3))
        if _cells_valid(xyz, cells, kinds):
            break
    else:
        raise RuntimeError("could not draw a valid jitter")
    return _finish_box(xyz, cells, kinds, length, tag_of_plane)


def mixed_box_mesh(n: int = 4, seed: int = 0, jitter: float = 0.1, length: float = 1.0, tag_of_plane=None):
    """A conforming box mesh of hexahedra, pyramids and tetrahedra on [0,L]^3.  The n^3 grid cells with
    i < n/2 are hexahedra; each other cell is cut into six pyramids on its faces with their apex at the cell's
    node average, and every pyramid whose base is not shared with a hexahedron is cut again into two
    tetrahedra along the base diagonal through the base's smallest node id (so both cells of a shared quad cut
    it alike).  Interior grid nodes are jittered as in hex_box_mesh."""
    if tag_of_plane is None:
        def tag_of_plane(axis, side):
            return 2 if (axis == 2 and side == 1) else 1
    xyz0, interior, nid, h = _box_grid(n, seed, jitter, length)
    half = n // 2
    rng = np.random.default_rng(seed)
    n_grid = len(xyz0)
    for _ in range(100):
        xyz = xyz0.copy()
        xyz[interior] += rng.uniform(-jitter * h, jitter * h, size=(int(interior.sum()), 3))
        pts = [xyz]
        cells, kinds = [], []
        napex = n_grid
        for i in range(n):
            for j in range(n):
                for k in range(n):
                    hx = _hex_nodes(nid, i, j, k)
                    if i < half:
                        cells.append(hx)
                        kinds.append(8)
                        continue
                    apex = napex
                    napex += 1
                    pts.append(xyz[hx].mean(axis=0)[None, :])
                    for a, lf in enumerate(LOCAL_FACES[8]):
                        q = [hx[x] for x in lf]
                        if a == 5 and i == half:          # the -x face, shared with a hexahedron
                            cells.append(q + [apex, -1, -1, -1])
                            kinds.append(5)
                            continue
                        lo = int(np.argmin(q))
                        if lo in (0, 2):
                            tets = [[q[0], q[1], q[2], apex], [q[0], q[2], q[3], apex]]
                        else:
                            tets = [[q[0], q[1], q[3], apex], [q[1], q[2], q[3], apex]]
                        for t in tets:
                            cells.append(t + [-1, -1, -1, -1])
                            kinds.append(4)
        allxyz = np.concatenate(pts, axis=0)
        cells = np.array([c + [-1] * (8 - len(c)) for c in cells], dtype=np.int64)
        kinds = np.array(kinds, dtype=np.int64)
        if _cells_valid(allxyz, cells, kinds):
            break
    else:
        raise RuntimeError("could not draw a valid jitter")
    return _finish_box(allxyz, cells, kinds, length, tag_of_plane)




# --------------------------------------------------------------------------
# Box meshes (Kuhn split of a structured hexahedral grid)
# --------------------------------------------------------------------------

_KUHN = [p for p in itertools.permutations(range(3))]


def kuhn_box_mesh(n: int = 6, seed: int = 0, jitter: float = 0.15, length: float = 1.0,
                  tag_of_plane=None):
    """n^3 hexahedra on [0,L]^3, each split into 6 tets along the main diagonal.

    The split follows a coordinate permutation per tet (Kuhn/Freudenthal), so
    it is conforming across hexahedra.  Interior nodes are jittered by
    U(-jitter*h, jitter*h)^3 drawn from ``numpy.random.default_rng(seed)``; a
    draw that makes any tet volume non-positive is rejected and redrawn.

    ``tag_of_plane(axis, side) -> tag`` gives each of the six box faces a tag;
    the default tags the z = L plane 2 and the five others 1.
    """
    if tag_of_plane is None:
        def tag_of_plane(axis, side):
            return 2 if (axis == 2 and side == 1) else 1
    h = length / n
    m = n + 1
    g = np.arange(m) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    xyz0 = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def nid(i, j, k):
        return (i * m + j) * m + k

    tets = []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                base = np.array([i, j, k])
                for perm in _KUHN:
                    v = [base.copy()]
                    cur = base.copy()
                    for ax in perm:
                        cur = cur.copy()
                        cur[ax] += 1
                        v.append(cur)
                    tets.append([nid(*p) for p in v])
    tets = np.array(tets, dtype=np.int64)

    ijk = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1).reshape(-1, 3)
    interior = np.all((ijk > 0) & (ijk < n), axis=1)
    rng = np.random.default_rng(seed)
    for _ in range(100):
        xyz = xyz0.copy()
        d = rng.uniform(-jitter * h, jitter * h, size=(int(interior.sum()), 3))
        xyz[interior] += d
        tets_o = _orient(xyz, tets)
        if np.all(tet_volumes(xyz, tets_o) > 0):
            break
    else:
        raise RuntimeError("could not draw a valid jitter")

    tets_c, offsets = color_major(xyz, tets_o)
    bkeys = boundary_triangles(tets_c)
    tags = np.zeros(len(bkeys), dtype=np.int64)
    fc = xyz[bkeys].mean(axis=1)
    for ax in range(3):
        for side in (0, 1):
            on = np.abs(fc[:, ax] - side * length) < 1e-12 * max(length, 1.0)
            tags[on] = tag_of_plane(ax, side)
    if np.any(tags == 0):
        raise RuntimeError("unclassified boundary triangle")
    return dict(xyz=xyz, tets=tets_c, btri=bkeys, btag=tags, color_offsets=offsets)


# --------------------------------------------------------------------------
# Shell meshes around star-shaped bodies (cubed-sphere O-grid)
# --------------------------------------------------------------------------

def sphere_body(radius: float = 0.5):
    def inside(p):
        return np.einsum("ij,ij->i", p, p) <= radius * radius
    return inside, np.zeros(3)


def capsule_body(diameter: float = 1.0, nose_radius: float = 1.2, cone_half_angle_deg: float = 33.0,
                 base_radius_frac: float = 0.4):
    """Spherical-cap forebody facing -x plus a conical aftbody, cut by a flat base.

    Convex, hence star-shaped about an interior point; returns (inside(p), centre).
    """
    rmax = 0.5 * diameter
    depth = nose_radius - math.sqrt(nose_radius ** 2 - rmax ** 2)
    x_s = depth
    t = math.tan(math.radians(cone_half_angle_deg))
    x_back = x_s + (rmax - base_radius_frac * rmax) / t
    cball = np.array([nose_radius, 0.0, 0.0])

    def inside(p):
        r = np.hypot(p[:, 1], p[:, 2])
        in_ball = np.einsum("ij,ij->i", p - cball, p - cball) <= nose_radius ** 2
        in_cone = r <= rmax - (p[:, 0] - x_s) * t
        return in_ball & in_cone & (p[:, 0] <= x_back) & (p[:, 0] >= 0.0)

    centre = np.array([0.5 * (x_s + x_back) * 0.6, 0.0, 0.0])
    return inside, centre


def _ray_hit(inside, centre, dirs, rmax=10.0, iters=60):
    lo = np.zeros(len(dirs))
    hi = np.full(len(dirs), rmax)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        ins = inside(centre + dirs * mid[:, None])
        lo = np.where(ins, mid, lo)
        hi = np.where(ins, hi, mid)
    return 0.5 * (lo + hi)


def _cubed_sphere_dirs(n: int):
    """Unique directions of an equiangular cubed sphere and the 6 patch index grids."""
    a = np.tan(0.25 * np.pi * np.linspace(-1.0, 1.0, n + 1))
    A, B = np.meshgrid(a, a, indexing="ij")
    patches = []
    for ax in range(3):
        for sgn in (1.0, -1.0):
            v = np.zeros((n + 1, n + 1, 3))
            o = [x for x in range(3) if x != ax]
            v[..., ax] = sgn
            # keep each patch right-handed when viewed from outside
            if sgn > 0:
                v[..., o[0]] = A
                v[..., o[1]] = B
            else:
                v[..., o[0]] = B
                v[..., o[1]] = A
            v /= np.linalg.norm(v, axis=-1, keepdims=True)
            patches.append(v)
    allv = np.concatenate([p.reshape(-1, 3) for p in patches])
    key = np.round(allv * 1e9).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    dirs = allv[first]
    idx = inv.reshape(6, n + 1, n + 1)
    return dirs, idx


def shell_mesh(body, n_ang: int, n_rad: int, r_far: float, first_layer: float, seed: int = 0,
               jitter: float = 0.1, smooth_passes: int = 0, cells: str = "tet"):
    """Graded tetrahedral (or, with cells="hex", hexahedral) shell between a star-shaped body and a far-field
    sphere.

    Nodes sit on rays of an equiangular cubed sphere; along each ray the layers
    grow geometrically from ``first_layer`` at the wall to the far-field radius.
    Each hexahedron is split into 6 pyramids on its centre, and every pyramid
    base is cut along the diagonal through its lowest-numbered node, so the
    12-tet split is conforming.  Interior layer nodes get an isotropic
    U(-j, j)^3 jitter scaled by the local radial spacing; a draw that folds the mesh
    (two tets on one side of their shared face) or makes a volume non-positive is redrawn.
    ``smooth_passes`` rounds sharp body edges by smoothing the wall radius over the ray grid.
    cells="hex" keeps the hexahedra of the O-grid (the paper's sphere mesh is hexahedral, Sec. 4.2), with the
    same jitter, as a mixed-cell mesh dict.
    Tags: 1 = wall, 2 = far field.
    """
    inside, centre = body
    dirs, pidx = _cubed_sphere_dirs(n_ang)
    rb = _ray_hit(inside, centre, dirs, rmax=r_far)
    if smooth_passes:
        # round sharp edges of the body: Laplacian smoothing of the wall radius over the direction grid
        edges = set()
        for p in range(6):
            P = pidx[p]
            for i in range(n_ang + 1):
                for j in range(n_ang + 1):
                    if i < n_ang:
                        edges.add((min(P[i, j], P[i + 1, j]), max(P[i, j], P[i + 1, j])))
                    if j < n_ang:
                        edges.add((min(P[i, j], P[i, j + 1]), max(P[i, j], P[i, j + 1])))
        e = np.array(sorted(edges))
        deg = np.bincount(e.ravel(), minlength=len(dirs)).astype(float)
        for _ in range(smooth_passes):
            acc = np.zeros(len(dirs))
            np.add.at(acc, e[:, 0], rb[e[:, 1]])
            np.add.at(acc, e[:, 1], rb[e[:, 0]])
            rb = 0.5 * rb + 0.5 * acc / deg
    # geometric grading on the unit interval with a first step first_layer/(r_far-mean rb)
    span = r_far - rb.mean()
    f = first_layer / span
    if f * n_rad >= 1.0:
        q = 1.0
    else:
        lo_q, hi_q = 1.0 + 1e-12, 10.0
        for _ in range(200):
            mq = 0.5 * (lo_q + hi_q)
            if f * (mq ** n_rad - 1.0) / (mq - 1.0) > 1.0:
                hi_q = mq
            else:
                lo_q = mq
        q = 0.5 * (lo_q + hi_q)
    if q == 1.0:
        xi = np.linspace(0.0, 1.0, n_rad + 1)
    else:
        xi = (q ** np.arange(n_rad + 1) - 1.0) / (q ** n_rad - 1.0)
    nd = len(dirs)
    rad = rb[:, None] + (r_far - rb)[:, None] * xi[None, :]
    xyz = (centre[None, None, :] + dirs[:, None, :] * rad[:, :, None]).reshape(-1, 3)

    def nid(d, k):
        return d * (n_rad + 1) + k

    rng = np.random.default_rng(seed)
    layer = np.tile(np.arange(n_rad + 1), nd)
    interior = (layer > 0) & (layer < n_rad)
    dr = np.zeros(len(xyz))
    rr = rad.reshape(-1)
    kk = layer
    # local radial spacing = min of adjacent layer gaps
    radm = rad
    gaps = np.diff(radm, axis=1)
    loc = np.full(rad.shape, np.inf)
    loc[:, 1:] = np.minimum(loc[:, 1:], gaps)
    loc[:, :-1] = np.minimum(loc[:, :-1], gaps)
    dr = loc.reshape(-1)
    del rr, kk

    hexes = []
    for p in range(6):
        P = pidx[p]
        for i in range(n_ang):
            for j in range(n_ang):
                d00, d10, d11, d01 = P[i, j], P[i + 1, j], P[i + 1, j + 1], P[i, j + 1]
                for k in range(n_rad):
                    hexes.append([nid(d00, k), nid(d10, k), nid(d11, k), nid(d01, k),
                                  nid(d00, k + 1), nid(d10, k + 1), nid(d11, k + 1), nid(d01, k + 1)])
    hexes = np.array(hexes, dtype=np.int64)
    quads = np.array([[0, 1, 2, 3], [4, 5, 6, 7], [0, 1, 5, 4], [1, 2, 6, 5], [2, 3, 7, 6], [3, 0, 4, 7]])

    if cells == "hex":
        kinds = np.full(len(hexes), 8, dtype=np.int64)
        for _attempt in range(50):
            xj = xyz.copy()
            xj[interior] += rng.uniform(-jitter, jitter, size=(int(interior.sum()), 3)) * dr[interior, None]
            if _cells_valid(xj, hexes, kinds):
                break
        else:
            raise RuntimeError("shell mesh: folded hexahedra after 50 jitter draws")
        cells_c, kinds_c, offsets = color_major_cells(xj, hexes, kinds)
        _, bcyc = match_faces_cells(cells_c, kinds_c)
        bl = layer[bcyc]
        tags = np.zeros(len(bcyc), dtype=np.int64)
        tags[np.all(bl == 0, axis=1)] = 1
        tags[np.all(bl == n_rad, axis=1)] = 2
        if np.any(tags == 0):
            raise RuntimeError("shell mesh: unclassified boundary face")
        return dict(xyz=xj, cells=cells_c, kinds=kinds_c, bface=bcyc, btag=tags, color_offsets=offsets,
                    wall_radius=rb, centre=centre)

    for _attempt in range(50):
        xj = xyz.copy()
        d = rng.uniform(-jitter, jitter, size=(int(interior.sum()), 3)) * dr[interior, None]
        xj[interior] += d
        nn = len(xj)
        centres = xj[hexes].mean(axis=1)
        allxyz = np.concatenate([xj, centres])
        cid = nn + np.arange(len(hexes))
        tets = []
        for qd in quads:
            v = hexes[:, qd]  # [nh,4] quad in cyclic order
            m = np.argmin(v, axis=1)
            r = (np.arange(4)[None, :] + m[:, None]) % 4
            vr = np.take_along_axis(v, r, axis=1)  # rotated so vr[:,0] is the lowest id
            tets.append(np.stack([vr[:, 0], vr[:, 1], vr[:, 2], cid], axis=1))
            tets.append(np.stack([vr[:, 0], vr[:, 2], vr[:, 3], cid], axis=1))
        tets = np.concatenate(tets)
        tets = _orient(allxyz, tets)
        vol = tet_volumes(allxyz, tets)
        if np.all(vol > 1e-14) and folded_faces(allxyz, tets) == 0:
            break
    else:
        raise RuntimeError("shell mesh: folded or degenerate tets after 50 jitter draws")

    tets_c, offsets = color_major(allxyz, tets)
    bkeys = boundary_triangles(tets_c)
    lay = np.concatenate([layer, np.full(len(hexes), -1)])
    bl = lay[bkeys]
    tags = np.zeros(len(bkeys), dtype=np.int64)
    tags[np.all(bl == 0, axis=1)] = 1
    tags[np.all(bl == n_rad, axis=1)] = 2
    if np.any(tags == 0):
        raise RuntimeError("shell mesh: unclassified boundary triangle")
    return dict(xyz=allxyz, tets=tets_c, btri=bkeys, btag=tags, color_offsets=offsets,
                wall_radius=rb, centre=centre)
