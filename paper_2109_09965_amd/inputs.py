"""Seeded synthetic inputs: hybrid meshes and flow states.

This module is shared by the HIP path, the tests and the benchmark.  It holds
mesh topology and coordinates, boundary tags and seeded initial states only:
none of the scheme's arithmetic (no volumes, normals, quadrature, fluxes or
reconstruction) lives here.

Meshes are face based, the form a finite-volume scheme on polyhedral cells
needs (paper, Sec. 2.1: the boundary of a cell is a union of N_f faces):

    dim            2 or 3
    xyz            float64 [n_vert, dim]
    n_cell         int
    face_vert_ptr  int64 [n_face + 1]   CSR into face_vert
    face_vert      int64                2 ids per edge (2-D); 3 (triangle)
                                        or 4 (bilinear quad, cyclic) in 3-D,
                                        ordered so the normal points out of
                                        the owner (counter-clockwise owner
                                        boundary in 2-D, right-hand rule in 3-D)
    face_owner     int64 [n_face]
    face_neigh     int64 [n_face]       -1 on boundary faces
    face_bc        int32 [n_face]       BC_* tag (0 on interior faces)
    face_shift     float64 [n_face, dim] translation that carries the
                                        neighbour next to the owner (nonzero
                                        only across periodic faces)

The same meshes also carry the cell-based description the library's
cgks_mesh_create takes (cells by type and vertex list, boundary faces by
vertex list and tag; periodic seams as pairs of boundary faces):

    cell_type      int32 [n_cell]       CELL_* (POLY: explicit faces)
    cell_vert_ptr  int64 [n_cell + 1]   CSR into cell_vert
    cell_vert      int64                vertex ids in the type's order, or for
                                        POLY: face count, then per face its
                                        vertex count and ids
    bface_vert_ptr int64 [n_bface + 1]  CSR into bface_vert
    bface_vert     int64
    bface_tag      int32 [n_bface]      BC_* (BC_PERIODIC for seams)
    bface_pair     int64 [n_bface]      partner of a periodic face, else -1

Cell ids follow generation order (layer by layer for the O-grids).
"""
from __future__ import annotations

import math
import numpy as np

BC_INTERIOR = 0
BC_SLIP_WALL = 1
BC_NOSLIP_ISOTHERMAL = 2
BC_NOSLIP_ADIABATIC = 3
BC_FARFIELD = 4

_BIG = np.iinfo(np.int64).max


# --------------------------------------------------------------------------
# face matching (pure topology)
# --------------------------------------------------------------------------
def _dedupe_polys(F):
    """Remove cyclically repeated consecutive vertex ids from each row of F
    ([n, m], -1 = absent).  Returns ([n, m] padded with -1, count)."""
    n, m = F.shape
    keep = F >= 0
    prev = np.roll(F, 1, axis=1)
    # for rows shorter than m the cyclic predecessor of entry 0 is the last
    # valid entry, so build it explicitly
    cnt0 = keep.sum(1)
    last = F[np.arange(n), np.maximum(cnt0 - 1, 0)]
    prev[:, 0] = last
    keep &= F != prev
    out = np.full_like(F, -1)
    cnt = keep.sum(1)
    # stable compaction
    order = np.argsort(~keep, axis=1, kind="stable")
    G = np.take_along_axis(F, order, axis=1)
    col = np.arange(m)[None, :]
    out[col < cnt[:, None]] = G[col < cnt[:, None]]
    return out, cnt


def _orient(F, cnt, cell_of_face, xyz, cell_ctr):
    """Reverse faces whose vertex order does not point out of their cell."""
    dim = xyz.shape[1]
    P = xyz[np.where(F >= 0, F, 0)]
    if dim == 2:
        t = P[:, 1] - P[:, 0]
        nrm = np.stack([t[:, 1], -t[:, 0]], 1)
        fc = 0.5 * (P[:, 0] + P[:, 1])
    else:
        is_q = cnt == 4
        a = np.where(is_q[:, None], P[:, 2] - P[:, 0], P[:, 1] - P[:, 0])
        b = np.where(is_q[:, None], P[:, 3] - P[:, 1], P[:, 2] - P[:, 0])
        nrm = np.cross(a, b)
        w = (F >= 0).astype(float)
        fc = (P * w[:, :, None]).sum(1) / cnt[:, None]
    s = np.einsum("ij,ij->i", nrm, fc - cell_ctr[cell_of_face])
    flip = s < 0
    G = F.copy()
    for c in (2, 3, 4):
        rows = flip & (cnt == c)
        G[rows, :c] = F[rows, :c][:, ::-1]
    return G


def _assemble(dim, xyz, topo_of, F, cnt, cell_of_face, n_cell, classify):
    """Match faces by their topological vertex set; build the face arrays."""
    nF, m = F.shape
    T = np.where(F >= 0, topo_of[np.where(F >= 0, F, 0)], _BIG)
    K = np.sort(T, axis=1)
    order = np.lexsort(K.T[::-1])
    Ks = K[order]
    same = np.all(Ks[1:] == Ks[:-1], axis=1)
    # a face key may appear at most twice
    if np.any(same[1:] & same[:-1]):
        raise ValueError("mesh: a face is shared by more than two cells")
    pair_first = np.nonzero(same)[0]
    a = order[pair_first]
    b = order[pair_first + 1]
    paired = np.zeros(nF, bool)
    paired[a] = True
    paired[b] = True
    ca, cb = cell_of_face[a], cell_of_face[b]
    if np.any(ca == cb):
        raise ValueError("mesh: degenerate cell matched with itself")
    swap = ca > cb
    own_face = np.where(swap, b, a)
    nb_face = np.where(swap, a, b)
    owner_i = cell_of_face[own_face]
    neigh_i = cell_of_face[nb_face]

    def centre(rows):
        # vertex average, summed in increasing vertex id (padding last)
        ids = np.sort(np.where(F[rows] >= 0, F[rows], _BIG), axis=1)
        ok = ids < _BIG
        P = xyz[np.where(ok, ids, 0)]
        s = P[:, 0].copy()
        for k in range(1, F.shape[1]):
            s = s + np.where(ok[:, k:k + 1], P[:, k], 0.0)
        return s / cnt[rows][:, None]

    shift_i = centre(own_face) - centre(nb_face)
    shift_i[np.abs(shift_i) < 1e-12] = 0.0

    bnd = np.nonzero(~paired)[0]
    owner_b = cell_of_face[bnd]
    bc_b = np.asarray(classify(centre(bnd)), dtype=np.int32) if len(bnd) else np.zeros(0, np.int32)
    if np.any(bc_b <= 0):
        raise ValueError("mesh: unclassified boundary face")

    # boundary faces of the cell-based description: the unpaired faces, and
    # both sides of every periodic pair (tagged periodic, each naming the other)
    per = np.nonzero(np.any(shift_i != 0.0, axis=1))[0]
    brows = np.concatenate([bnd, own_face[per], nb_face[per]])
    btag = np.concatenate([bc_b, np.full(2 * len(per), BC_PERIODIC, np.int32)])
    bpair = np.full(len(brows), -1, np.int64)
    n0, npr = len(bnd), len(per)
    bpair[n0:n0 + npr] = n0 + npr + np.arange(npr)
    bpair[n0 + npr:] = n0 + np.arange(npr)
    bcnt = cnt[brows]
    bptr = np.zeros(len(brows) + 1, np.int64)
    bptr[1:] = np.cumsum(bcnt)
    bfv = F[brows]
    bfv = bfv[bfv >= 0].astype(np.int64)

    rows = np.concatenate([own_face, bnd])
    owner = np.concatenate([owner_i, owner_b]).astype(np.int64)
    neigh = np.concatenate([neigh_i, -np.ones(len(bnd), np.int64)]).astype(np.int64)
    bc = np.concatenate([np.zeros(len(own_face), np.int32), bc_b])
    shift = np.concatenate([shift_i, np.zeros((len(bnd), dim))])
    # deterministic face order: by owner, then neighbour (boundary last)
    key_n = np.where(neigh >= 0, neigh, n_cell + 1)
    o = np.lexsort((key_n, owner))
    rows, owner, neigh, bc, shift = rows[o], owner[o], neigh[o], bc[o], shift[o]
    c = cnt[rows]
    ptr = np.zeros(len(rows) + 1, np.int64)
    ptr[1:] = np.cumsum(c)
    fv = F[rows]
    fv = fv[fv >= 0].astype(np.int64)
    return dict(dim=dim, xyz=np.ascontiguousarray(xyz, dtype=np.float64), n_cell=int(n_cell),
                face_vert_ptr=ptr, face_vert=fv, face_owner=owner, face_neigh=neigh,
                face_bc=bc, face_shift=np.ascontiguousarray(shift),
                bface_vert_ptr=bptr, bface_vert=bfv, bface_tag=btag.astype(np.int32), bface_pair=bpair)


# --------------------------------------------------------------------------
# 2-D: structured quads, each split into two triangles along (i,j)-(i+1,j+1)
# --------------------------------------------------------------------------
def _tri_grid(X, Y, gid, tid, classify):
    """X, Y: [ni+1, nj+1] vertex coordinates; gid/tid(i, j) -> geometric /
    topological vertex id arrays."""
    ni, nj = X.shape[0] - 1, X.shape[1] - 1
    I, J = np.meshgrid(np.arange(ni), np.arange(nj), indexing="ij")
    I, J = I.ravel(), J.ravel()
    v00, v10, v11, v01 = gid(I, J), gid(I + 1, J), gid(I + 1, J + 1), gid(I, J + 1)
    nq = len(I)
    tri = np.empty((2 * nq, 3), np.int64)
    tri[0::2] = np.stack([v00, v10, v11], 1)
    tri[1::2] = np.stack([v00, v11, v01], 1)
    n_vert = int(max(gid(np.array([ni]), np.array([nj]))[0], tri.max()) + 1)
    xyz = np.zeros((n_vert, 2))
    II, JJ = np.meshgrid(np.arange(ni + 1), np.arange(nj + 1), indexing="ij")
    g = gid(II.ravel(), JJ.ravel())
    xyz[g, 0] = X.ravel()
    xyz[g, 1] = Y.ravel()
    topo = np.zeros(n_vert, np.int64)
    topo[g] = tid(II.ravel(), JJ.ravel())
    n_cell = tri.shape[0]
    F = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    cof = np.concatenate([np.arange(n_cell)] * 3)
    cnt = np.full(len(F), 2)
    ctr = xyz[tri].mean(1)
    F = _orient(F, cnt, cof, xyz, ctr)
    m = _assemble(2, xyz, topo, F, cnt, cof, n_cell, classify)
    m["cell_type"] = np.full(n_cell, CELL_TRI, np.int32)
    m["cell_vert_ptr"] = 3 * np.arange(n_cell + 1, dtype=np.int64)
    m["cell_vert"] = tri.ravel().astype(np.int64)
    return m


def radial_stations(r0, r1, n, ratio):
    """n+1 radii from r0 to r1 with a geometric spacing ratio."""
    first = (r1 - r0) * (ratio - 1.0) / (ratio ** n - 1.0)
    j = np.arange(n + 1)
    return r0 + first * (ratio ** j - 1.0) / (ratio - 1.0)


def cylinder_mesh(n_theta=64, n_r=32, r_wall=0.5, r_far=20.0, ratio=1.1, wall=BC_SLIP_WALL,
                  first_spacing=None):
    """2-D O-mesh around a circular cylinder: n_theta x n_r quads, each split
    into two triangles.  With the defaults and first_spacing=0.09695 this is the
    64 x 32 cylinder mesh with stretching 1.1 reaching r = 20."""
    if first_spacing is not None:
        r = r_wall + first_spacing * (ratio ** np.arange(n_r + 1) - 1.0) / (ratio - 1.0)
    else:
        r = radial_stations(r_wall, r_far, n_r, ratio)
    th = 2.0 * np.pi * np.arange(n_theta + 1) / n_theta
    X = np.cos(th)[:, None] * r[None, :]
    Y = np.sin(th)[:, None] * r[None, :]

    def gid(i, j):
        return (np.asarray(i) % n_theta) * (n_r + 1) + np.asarray(j)

    rmid = 0.5 * (r[0] + r[-1])

    def classify(fc):
        rr = np.hypot(fc[:, 0], fc[:, 1])
        return np.where(rr < rmid, wall, BC_FARFIELD)

    m = _tri_grid(X, Y, gid, gid, classify)
    m["name"] = f"cylinder_{n_theta}x{n_r}"
    return m


def box2d_mesh(n=8, L=2.0, periodic=True, bc=BC_SLIP_WALL, perturb=0.0, seed=0):
    """2-D square [0,L]^2, n x n quads split into triangles.  periodic=True
    joins opposite sides; otherwise every boundary edge gets tag bc.  perturb
    moves interior vertices by a smooth periodic displacement of that relative
    amplitude (in units of the grid spacing)."""
    h = L / n
    s = np.linspace(0.0, L, n + 1)
    X, Y = np.meshgrid(s, s, indexing="ij")
    if perturb:
        rng = np.random.default_rng(seed)
        ph = rng.uniform(0, 2 * np.pi, 4)
        k = 2 * np.pi / L
        X = X + perturb * h * np.sin(k * X + ph[0]) * np.sin(k * Y + ph[1])
        Y = Y + perturb * h * np.sin(k * X + ph[2]) * np.sin(k * Y + ph[3])
        if not periodic:  # keep the outer square straight
            X[0, :], X[-1, :], Y[:, 0], Y[:, -1] = 0.0, L, 0.0, L

    def gid(i, j):
        return np.asarray(i) * (n + 1) + np.asarray(j)

    if periodic:
        def tid(i, j):
            return (np.asarray(i) % n) * (n + 1) + (np.asarray(j) % n)
    else:
        tid = gid
    m = _tri_grid(X, Y, gid, tid, lambda fc: np.full(len(fc), bc))
    m["name"] = f"box2d_{n}{'_per' if periodic else ''}"
    if periodic:
        m["period"] = np.array([L, L])
    return m


# --------------------------------------------------------------------------
# 3-D: structured hex index space with per-layer cell types
# --------------------------------------------------------------------------
# local hex vertex l = a + 2b + 4c for offsets (a, b, c) in (i, j, k)
_HEX = [(0, 2, 6, 4), (1, 3, 7, 5), (0, 1, 5, 4), (2, 3, 7, 6), (0, 1, 3, 2), (4, 5, 7, 6)]
# same hex with its k+ quad replaced by the two triangles on diagonal 4-7
_HEX7 = _HEX[:5] + [(4, 5, 7), (4, 7, 6)]
# hex with its k- quad replaced by the two triangles on diagonal 0-3
_HEX7B = _HEX[:4] + [(0, 1, 3), (0, 3, 2), _HEX[5]]
# two prisms (axis along k) from the diagonal 0-3 of the k- quad
_PRISM_A = [(0, 1, 3), (4, 5, 7), (0, 1, 5, 4), (1, 3, 7, 5), (3, 0, 4, 7)]
_PRISM_B = [(0, 3, 2), (4, 7, 6), (0, 3, 7, 4), (3, 2, 6, 7), (2, 0, 4, 6)]
# Kuhn split along the main diagonal 0-7 (consistent face diagonals)
_KUHN = [(0, 1, 3, 7), (0, 1, 5, 7), (0, 2, 3, 7), (0, 2, 6, 7), (0, 4, 5, 7), (0, 4, 6, 7)]


def _tet_faces(t):
    p, q, r, s = t
    return [(p, q, r), (p, q, s), (p, r, s), (q, r, s)]


# six pyramids per hex: each hex face (corner ids i + 2j + 4k) is the base of
# one pyramid whose apex is the hex's centre, local vertex 8
_HEX_FACES = [(0, 2, 6, 4), (1, 3, 7, 5), (0, 1, 5, 4), (2, 3, 7, 6), (0, 1, 3, 2), (4, 5, 7, 6)]
_PYRAMIDS = [[base] + [(base[e], base[(e + 1) % 4], 8) for e in range(4)] for base in _HEX_FACES]

# cell types of the cell-based description (the library's CGKS_CELL_*)
CELL_TRI, CELL_QUAD, CELL_TET, CELL_PYR, CELL_PRISM, CELL_HEX, CELL_POLY = 1, 2, 3, 4, 5, 6, 7
BC_PERIODIC = 5


def _template_key(tmpl):
    return tuple(tuple(f) for f in tmpl)


# standard cell types of the templates: (type, local corner ids in the
# type's vertex order); other templates are written as POLY cells
_CANON = {_template_key(_HEX): (CELL_HEX, [0, 1, 3, 2, 4, 5, 7, 6]),
          _template_key(_PRISM_A): (CELL_PRISM, [0, 1, 3, 4, 5, 7]),
          _template_key(_PRISM_B): (CELL_PRISM, [0, 3, 2, 4, 7, 6])}
for _t in _KUHN:
    _CANON[_template_key(_tet_faces(_t))] = (CELL_TET, list(_t))
for _p in _PYRAMIDS:
    _CANON[_template_key(_p)] = (CELL_PYR, list(_p[0]) + [8])


def _cells_csr(blocks, n_cell):
    """blocks: list of (cell ids, type, [n, k] vertex rows or list of
    per-cell POLY encodings) -> cell_type, cell_vert_ptr, cell_vert in cell
    id order."""
    ctype = np.zeros(n_cell, np.int32)
    rows = [None] * n_cell
    for ids, t, verts in blocks:
        ctype[ids] = t
        for i, v in zip(ids, verts):
            rows[i] = v
    ptr = np.zeros(n_cell + 1, np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    return ctype, ptr, np.concatenate([np.asarray(r, np.int64) for r in rows])


LAYER_TEMPLATES = {
    "hex": [_HEX],
    "hex7": [_HEX7],
    "hex7b": [_HEX7B],
    "prism": [_PRISM_A, _PRISM_B],
    "tet": [_tet_faces(t) for t in _KUHN],
    "pyr": _PYRAMIDS,   # conforming with hex layers (quad faces) only
}


def _fast_ctr(ncell, cell_vs, xyz):
    ctr = np.zeros((ncell, 3))
    for ids, V in cell_vs:
        s = np.sort(V, axis=1)
        uniq = np.ones_like(s, bool)
        uniq[:, 1:] = s[:, 1:] != s[:, :-1]
        P = xyz[s] * uniq[:, :, None]
        ctr[ids] = P.sum(1) / uniq.sum(1)[:, None]
    return ctr


def _hybrid_grid(ni, nj, layer_types, gid, tid, coords, classify, cells=None):
    """Cells from a structured (i, j, k) hex index space.  layer_types[k] in
    LAYER_TEMPLATES; gid/tid(i, j, k) give geometric/topological vertex ids;
    coords(ids) -> xyz.  Collapsed vertices (poles) are handled generically:
    repeated vertices are removed from each face, faces with < 3 vertices and
    cells with < 4 faces are dropped.  cells = (I, J) restricts the surface
    index pairs used (default: all ni x nj)."""
    if cells is None:
        I, J = np.meshgrid(np.arange(ni), np.arange(nj), indexing="ij")
        I, J = I.ravel(), J.ravel()
    else:
        I, J = (np.asarray(c, np.int64) for c in cells)
    faces, cof, cell_vs, cell_blocks = [], [], [], []
    ncell = 0
    corners = [np.stack([gid(I + (l & 1), J + ((l >> 1) & 1), np.full_like(I, k) + ((l >> 2) & 1))
                         for l in range(8)], 1) for k in range(len(layer_types))]
    # hex centres (apexes of pyramid layers) get ids after every corner id
    base_id = int(max(G.max() for G in corners)) + 1
    centre_of = []                      # [n_centre, 8] corner ids of each centre
    for k, lt in enumerate(layer_types):
        G = corners[k]
        if lt == "pyr":
            first = base_id + sum(len(c) for c in centre_of)
            G = np.concatenate([G, (first + np.arange(len(I)))[:, None]], 1)
            centre_of.append(corners[k])
        for tmpl in LAYER_TEMPLATES[lt]:
            fl = []
            for f in tmpl:
                Fa = np.full((len(I), 4), -1, np.int64)
                Fa[:, :len(f)] = G[:, list(f)]
                fl.append(_dedupe_polys(Fa))
            nvalid = sum((c >= 3).astype(int) for _, c in fl)
            ok = nvalid >= 4
            ids = np.full(len(I), -1, np.int64)
            ids[ok] = ncell + np.arange(ok.sum())
            ncell += int(ok.sum())
            used = sorted({v for f in tmpl for v in f})
            cell_vs.append((ids[ok], G[ok][:, used]))
            for Fd, c in fl:
                sel = ok & (c >= 3)
                faces.append(Fd[sel])
                cof.append(ids[sel])
            # cell-based description: the standard type where no vertex
            # collapsed, else the cell's remaining faces as a POLY cell
            collapsed = np.zeros(len(I), bool)
            for f, (_, c) in zip(tmpl, fl):
                collapsed |= c != len(f)
            canon = _CANON.get(_template_key(tmpl))
            std = ok & ~collapsed if canon else np.zeros(len(I), bool)
            if std.any():
                cell_blocks.append((ids[std], canon[0], G[std][:, canon[1]]))
            poly = ok & ~std
            if poly.any():
                enc = []
                for r in np.nonzero(poly)[0]:
                    fs = [Fd[r][:c[r]] for Fd, c in fl if c[r] >= 3]
                    enc.append([len(fs)] + [x for f in fs for x in [len(f)] + list(f)])
                cell_blocks.append((ids[poly], CELL_POLY, enc))
    F = np.concatenate(faces)
    cof = np.concatenate(cof)
    cnt = (F >= 0).sum(1)
    all_ids = np.unique(F[F >= 0])
    n_vert = int(all_ids.max() + 1)
    xyz = np.zeros((n_vert, 3))
    cid = all_ids[all_ids < base_id]
    xyz[cid] = coords(cid)
    topo = np.arange(n_vert, dtype=np.int64)
    topo[cid] = tid(cid)
    if centre_of:
        C = np.concatenate(centre_of)
        xyz[base_id:base_id + len(C)] = coords(C.ravel()).reshape(len(C), 8, 3).mean(1)
    ctr = _fast_ctr(ncell, cell_vs, xyz)
    F = _orient_fast(F, cnt, cof, xyz, ctr)
    m = _assemble(3, xyz, topo, F, cnt, cof, ncell, classify)
    m["cell_type"], m["cell_vert_ptr"], m["cell_vert"] = _cells_csr(cell_blocks, ncell)
    return m


def _orient_fast(F, cnt, cof, xyz, ctr):
    P = xyz[np.where(F >= 0, F, 0)]
    is_q = cnt == 4
    a = np.where(is_q[:, None], P[:, 2] - P[:, 0], P[:, 1] - P[:, 0])
    b = np.where(is_q[:, None], P[:, 3] - P[:, 1], P[:, 2] - P[:, 0])
    nrm = np.cross(a, b)
    w = (F >= 0).astype(float)
    fc = (P * w[:, :, None]).sum(1) / cnt[:, None]
    flip = np.einsum("ij,ij->i", nrm, fc - ctr[cof]) < 0
    G = F.copy()
    # reverse the first cnt entries of flipped rows
    for c in (3, 4):
        rows = flip & (cnt == c)
        G[rows, :c] = F[rows, :c][:, ::-1]
    return G


def sphere_layer_types(n_layers=40, n_hex=20, n_prism=10):
    """Per-layer cell types of the hybrid sphere O-grid: hexahedra, then
    2 prisms per hex, then 6 tetrahedra per hex.  The outermost hex layer
    has its outer quad split into the two triangles of the prism layer above
    (a 7-face cell), which keeps the mesh conforming."""
    lt = []
    for k in range(n_layers):
        if k < n_hex:
            lt.append("hex7" if (k == n_hex - 1 and n_layers > n_hex) else "hex")
        elif k < n_hex + n_prism:
            lt.append("prism")
        else:
            lt.append("tet")
    return lt


def sphere_mesh(n_theta=48, n_phi=96, n_layers=40, n_hex=20, n_prism=10, r_wall=0.5, r_far=15.0,
                ratio=1.08, first_spacing=None, wall=BC_NOSLIP_ADIABATIC):
    """3-D hybrid O-grid around a sphere on a latitude-longitude surface grid
    (n_theta x n_phi quads; the polar rows collapse to triangles), n_layers
    radial layers: hexahedra, prisms, tetrahedra (see sphere_layer_types)."""
    if first_spacing is not None:
        r = r_wall + first_spacing * (ratio ** np.arange(n_layers + 1) - 1.0) / (ratio - 1.0)
    else:
        r = radial_stations(r_wall, r_far, n_layers, ratio)
    per_level = 2 + (n_theta - 1) * n_phi

    def gid(i, j, k):
        i, j, k = np.broadcast_arrays(np.asarray(i), np.asarray(j), np.asarray(k))
        out = k * per_level + 2 + (i - 1) * n_phi + (j % n_phi)
        out = np.where(i == 0, k * per_level, out)
        out = np.where(i == n_theta, k * per_level + 1, out)
        return out.astype(np.int64)

    def coords(ids):
        k = ids // per_level
        rem = ids % per_level
        i = np.where(rem == 0, 0, np.where(rem == 1, n_theta, (rem - 2) // n_phi + 1))
        j = np.where(rem < 2, 0, (rem - 2) % n_phi)
        th = np.pi * i / n_theta
        ph = 2.0 * np.pi * j / n_phi
        rr = r[k]
        return np.stack([rr * np.cos(th), rr * np.sin(th) * np.cos(ph), rr * np.sin(th) * np.sin(ph)], 1)

    rmid = 0.5 * (r[0] + r[-1])

    def classify(fc):
        rr = np.linalg.norm(fc, axis=1)
        return np.where(rr < rmid, wall, BC_FARFIELD)

    lt = sphere_layer_types(n_layers, n_hex, n_prism)
    m = _hybrid_grid(n_theta, n_phi, lt, gid, lambda ids: ids, coords, classify)
    m["name"] = f"sphere_{n_theta}x{n_phi}x{n_layers}"
    m["r"] = r
    return m


def cubed_sphere_mesh(n=28, n_layers=40, n_hex=20, n_prism=10, r_wall=0.5, r_far=15.0, ratio=1.08,
                      first_spacing=None, wall=BC_NOSLIP_ADIABATIC):
    """3-D hybrid O-grid around a sphere on a cubed-sphere surface grid: the
    six faces of a cube, each n x n quads (equiangular gnomonic map), pushed
    onto the sphere, then extruded through n_layers radial layers of
    hexahedra, prisms and tetrahedra (see sphere_layer_types).  No surface
    vertex is singular (at the 8 cube corners three quads meet).  Every
    patch runs its two index directions along the positive global axes, so
    the face diagonals of the Kuhn tetrahedra agree across patch edges."""
    if first_spacing is not None:
        r = r_wall + first_spacing * (ratio ** np.arange(n_layers + 1) - 1.0) / (ratio - 1.0)
    else:
        r = radial_stations(r_wall, r_far, n_layers, ratio)
    # patch p: (normal axis, sign, i axis, j axis)
    patches = [(0, -1.0, 1, 2), (0, 1.0, 1, 2), (1, -1.0, 0, 2), (1, 1.0, 0, 2), (2, -1.0, 0, 1), (2, 1.0, 0, 1)]
    a = np.arange(n + 1)
    t = np.tan(-0.25 * np.pi + 0.5 * np.pi * a / n)
    t[0], t[-1] = -1.0, 1.0
    t[n - a[a > n // 2]] = -t[a > n // 2]          # exact antisymmetry
    pts = np.zeros((6, n + 1, n + 1, 3))
    A, B = np.meshgrid(a, a, indexing="ij")
    for p, (ax, sg, ai, aj) in enumerate(patches):
        pts[p, :, :, ax] = sg
        pts[p, :, :, ai] = t[A]
        pts[p, :, :, aj] = t[B]
    flat = pts.reshape(-1, 3)
    key = np.round(flat * (1 << 30)).astype(np.int64)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    inv = inv.reshape(6, n + 1, n + 1)
    dirs = np.zeros((len(uniq), 3))
    dirs[inv.ravel()] = flat
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    n_surf = len(uniq)
    assert n_surf == 6 * n * n + 2

    def gid(i, j, k):
        i, j, k = np.broadcast_arrays(np.asarray(i), np.asarray(j), np.asarray(k))
        return (k * n_surf + inv[i // (n + 1), i % (n + 1), j]).astype(np.int64)

    def coords(ids):
        return dirs[ids % n_surf] * r[ids // n_surf][:, None]

    rmid = 0.5 * (r[0] + r[-1])

    def classify(fc):
        return np.where(np.linalg.norm(fc, axis=1) < rmid, wall, BC_FARFIELD)

    P, Ai, Bj = np.meshgrid(np.arange(6), np.arange(n), np.arange(n), indexing="ij")
    cells = (P.ravel() * (n + 1) + Ai.ravel(), Bj.ravel())
    lt = sphere_layer_types(n_layers, n_hex, n_prism)
    m = _hybrid_grid(6 * (n + 1), n + 1, lt, gid, lambda ids: ids, coords, classify, cells=cells)
    m["name"] = f"cubed_sphere_6x{n}x{n}x{n_layers}"
    m["r"] = r
    return m


def box3d_mesh(n=(4, 4, 4), L=(1.0, 1.0, 1.0), layer_types=None, periodic=False, bc=BC_SLIP_WALL,
               perturb=0.0, seed=0):
    """3-D box of n[0] x n[1] x n[2] hex index cells, layer types along z
    (default: cycle hex, hex7, prism, tet).  periodic joins opposite sides."""
    ni, nj, nk = n
    if layer_types is None:
        # conforming through the z-seam as well: tet (k+ triangles) meets
        # hex7b (k- triangles)
        base = ["hex7b", "hex", "hex7", "prism", "tet"]
        layer_types = [base[k % 5] for k in range(nk)]
    assert len(layer_types) == nk

    def gid(i, j, k):
        return (np.asarray(i) * (nj + 1) + np.asarray(j)) * (nk + 1) + np.asarray(k)

    def split(ids):
        k = ids % (nk + 1)
        j = (ids // (nk + 1)) % (nj + 1)
        i = ids // ((nk + 1) * (nj + 1))
        return i, j, k

    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, 9)

    def coords(ids):
        i, j, k = split(ids)
        x = np.stack([i * L[0] / ni, j * L[1] / nj, k * L[2] / nk], 1)
        if perturb:
            h = np.array([L[0] / ni, L[1] / nj, L[2] / nk])
            kx = 2 * np.pi / np.asarray(L)
            base = x.copy()
            for a in range(3):
                d = (np.sin(kx[0] * base[:, 0] + ph[3 * a]) * np.sin(kx[1] * base[:, 1] + ph[3 * a + 1])
                     * np.sin(kx[2] * base[:, 2] + ph[3 * a + 2]))
                if not periodic:
                    # keep the box faces planar
                    on = np.isclose(base[:, a], 0.0) | np.isclose(base[:, a], L[a])
                    d = np.where(on, 0.0, d)
                x[:, a] += perturb * h[a] * d
        return x

    if periodic:
        def tid(ids):
            i, j, k = split(ids)
            return gid(i % ni, j % nj, k % nk)
    else:
        def tid(ids):
            return ids
    m = _hybrid_grid(ni, nj, layer_types, gid, tid, coords, lambda fc: np.full(len(fc), bc))
    m["name"] = f"box3d_{ni}x{nj}x{nk}{'_per' if periodic else ''}"
    if periodic:
        m["period"] = np.asarray(L, float)
    return m



def extrude_two_layers(mesh2d, dz=None):
    """The paper's way of running a 2-D case on a 3-D code (Sec. 4): the
    triangle mesh extruded through two layers of prisms in z, each of
    thickness dz (default: the smallest edge length of the 2-D mesh).  The
    2-D boundary edges become quads with the same tags; the two layers are
    periodic in z (the top of layer 1 is joined to the bottom of layer 0),
    so each prism meets the other layer through both of its triangles and
    a sweep that updates one layer before the other exerts no net z force
    on it.  Cell k of layer l has id k + l n; vertex v of plane z = l dz
    has id v + l n_vert."""
    assert mesh2d["dim"] == 2 and (mesh2d["cell_type"] == CELL_TRI).all()
    xy = mesh2d["xyz"]
    nv2, n2 = len(xy), mesh2d["n_cell"]
    tri = mesh2d["cell_vert"].reshape(n2, 3).copy()
    ptr, fv = mesh2d["face_vert_ptr"], mesh2d["face_vert"]
    own2, nb2, bc2 = mesh2d["face_owner"], mesh2d["face_neigh"], mesh2d["face_bc"]
    e = xy[fv[ptr[1:] - 1]] - xy[fv[ptr[:-1]]]
    if dz is None:
        dz = float(np.sqrt((e * e).sum(1)).min())
    xyz = np.concatenate([np.column_stack([xy, np.full(nv2, l * dz)]) for l in range(3)])
    # counter-clockwise triangles: their (a, b, c) normal is +z
    P = xy[tri]
    ccw = ((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1])
           - (P[:, 1, 1] - P[:, 0, 1]) * (P[:, 2, 0] - P[:, 0, 0])) > 0
    tri[~ccw] = tri[~ccw][:, ::-1]
    fvs, own, nb, bc, sh = [], [], [], [], []
    ed = np.stack([fv[ptr[:-1]], fv[ptr[:-1] + 1]], 1)     # 2-D edges, normal out of their owner
    for l in range(2):
        for f in range(len(own2)):
            p_, q_ = ed[f]
            fvs.append([p_ + l * nv2, q_ + l * nv2, q_ + (l + 1) * nv2, p_ + (l + 1) * nv2])
            own.append(own2[f] + l * n2)
            nb.append(nb2[f] + l * n2 if nb2[f] >= 0 else -1)
            bc.append(bc2[f])
            sh.append([0.0, 0.0, 0.0])
    for k in range(n2):
        a, b, c = tri[k]
        fvs.append([a + nv2, b + nv2, c + nv2])                 # mid plane, +z out of layer 0
        own.append(k)
        nb.append(k + n2)
        bc.append(BC_INTERIOR)
        sh.append([0.0, 0.0, 0.0])
    # periodic seam: layer 0's bottom (owner) and layer 1's top
    top0 = np.array([[c, b, a] for a, b, c in tri])             # -z out of layer 0
    top2 = tri + 2 * nv2

    def centre(ids):
        ids = np.sort(ids)
        s = xyz[ids[0]].copy()
        for v in ids[1:]:
            s = s + xyz[v]
        return s / len(ids)
    for k in range(n2):
        fvs.append(list(top0[k]))
        own.append(k)
        nb.append(k + n2)
        bc.append(BC_INTERIOR)
        d = centre(top0[k]) - centre(top2[k])
        d[np.abs(d) < 1e-12] = 0.0
        sh.append(list(d))
    cnt = np.array([len(x) for x in fvs])
    m = dict(dim=3, xyz=xyz, n_cell=2 * n2,
             face_vert_ptr=np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64),
             face_vert=np.concatenate(fvs).astype(np.int64), face_owner=np.array(own, np.int64),
             face_neigh=np.array(nb, np.int64), face_bc=np.array(bc, np.int32), face_shift=np.array(sh))
    # cell-based description
    cells = np.concatenate([np.concatenate([tri + l * nv2, tri + (l + 1) * nv2], 1) for l in range(2)])
    m["cell_type"] = np.full(2 * n2, CELL_PRISM, np.int32)
    m["cell_vert_ptr"] = 6 * np.arange(2 * n2 + 1, dtype=np.int64)
    m["cell_vert"] = cells.ravel().astype(np.int64)
    bnd = np.flatnonzero(nb2 < 0)
    bf = [[ed[f][0] + l * nv2, ed[f][1] + l * nv2, ed[f][1] + (l + 1) * nv2, ed[f][0] + (l + 1) * nv2]
          for l in range(2) for f in bnd]
    btag = [bc2[f] for l in range(2) for f in bnd]
    nbd = len(bf)
    bf += [list(top0[k]) for k in range(n2)] + [list(top2[k]) for k in range(n2)]
    btag += [BC_PERIODIC] * (2 * n2)
    pair = np.full(len(bf), -1, np.int64)
    pair[nbd:nbd + n2] = nbd + n2 + np.arange(n2)
    pair[nbd + n2:] = nbd + np.arange(n2)
    bcnt = np.array([len(x) for x in bf])
    m["bface_vert_ptr"] = np.concatenate([[0], np.cumsum(bcnt)]).astype(np.int64)
    m["bface_vert"] = np.concatenate(bf).astype(np.int64)
    m["bface_tag"] = np.array(btag, np.int32)
    m["bface_pair"] = pair
    m["name"] = f"two_layer_{mesh2d.get('name', '2d')}"
    m["dz"] = dz
    m["period"] = np.array([0.0, 0.0, 2 * dz])
    return m


def lift_state(W2, dW2, n_layers=2):
    """A 2-D state [4][n], [2][4][n] as the z-uniform 3-D state of an
    extruded mesh: w momentum and every z derivative zero."""
    n = W2.shape[1]
    W = np.zeros((5, n_layers * n))
    dW = np.zeros((3, 5, n_layers * n))
    for l in range(n_layers):
        s = slice(l * n, (l + 1) * n)
        W[[0, 1, 2, 4], s] = W2
        dW[:2, [0, 1, 2, 4], s] = dW2
    return W, dW

# --------------------------------------------------------------------------
# flow conditions and states
# --------------------------------------------------------------------------
def free_stream(dim, mach, aoa_deg=0.0, gamma=1.4):
    """Uniform state (rho, rho U, rho E) with rho = 1, p = 1/gamma (so c = 1)
    and |U| = mach at angle of attack aoa_deg in the x-y plane."""
    a = math.radians(aoa_deg)
    u = np.zeros(dim)
    u[0], u[1] = mach * math.cos(a), mach * math.sin(a)
    rho, p = 1.0, 1.0 / gamma
    W = np.zeros(dim + 2)
    W[0] = rho
    W[1:1 + dim] = rho * u
    W[-1] = p / (gamma - 1.0) + 0.5 * rho * float(u @ u)
    return W


def cell_centres(mesh):
    """Mean of each cell's distinct vertices (for sampling input fields only)."""
    dim, n = mesh["dim"], mesh["n_cell"]
    ptr, fv = mesh["face_vert_ptr"], mesh["face_vert"]
    nv = np.diff(ptr)
    fidx = np.repeat(np.arange(len(nv)), nv)
    acc = np.zeros((n, dim))
    cnt = np.zeros(n)
    for side in ("face_owner", "face_neigh"):
        c = mesh[side][fidx]
        ok = c >= 0
        x = mesh["xyz"][fv]
        if side == "face_neigh":
            x = x - mesh["face_shift"][fidx]
        np.add.at(acc, c[ok], x[ok])
        np.add.at(cnt, c[ok], 1.0)
    return acc / cnt[:, None]


def smooth_state(mesh, W_inf, seed=0, amp=0.05, gamma=1.4, n_modes=3):
    """Seeded smooth perturbation of a uniform state, sampled at cell centres.
    Returns (W [n_v, n_cell], dW [dim, n_v, n_cell]) where dW is the analytic
    gradient of the sampled field (an independent input, not a derived one)."""
    dim = mesh["dim"]
    x = cell_centres(mesh)
    rng = np.random.default_rng(seed)
    scale = float(np.max(np.ptp(x, axis=0)))
    nv = dim + 2
    # primitive perturbations q = (rho, u.., p)
    q0 = np.zeros(nv)
    q0[0] = W_inf[0]
    q0[1:1 + dim] = W_inf[1:1 + dim] / W_inf[0]
    q0[-1] = (gamma - 1.0) * (W_inf[-1] - 0.5 * float(W_inf[1:1 + dim] @ W_inf[1:1 + dim]) / W_inf[0])
    q = np.tile(q0[:, None], (1, len(x)))
    dq = np.zeros((dim, nv, len(x)))
    for v in range(nv):
        for _ in range(n_modes):
            kvec = rng.normal(size=dim) * (2.0 * np.pi / scale) * 2.0
            ph = rng.uniform(0, 2 * np.pi)
            a = amp * rng.uniform(0.5, 1.0) * (1.0 if v in (0, nv - 1) else 0.3)
            arg = x @ kvec + ph
            q[v] += a * np.sin(arg) * (q0[v] if v in (0, nv - 1) else 1.0)
            for d in range(dim):
                dq[d, v] += a * kvec[d] * np.cos(arg) * (q0[v] if v in (0, nv - 1) else 1.0)
    rho, u, p = q[0], q[1:1 + dim], q[-1]
    W = np.zeros((nv, len(x)))
    W[0] = rho
    W[1:1 + dim] = rho * u
    W[-1] = p / (gamma - 1.0) + 0.5 * rho * (u * u).sum(0)
    dW = np.zeros((dim, nv, len(x)))
    for d in range(dim):
        drho, du, dp = dq[d, 0], dq[d, 1:1 + dim], dq[d, -1]
        dW[d, 0] = drho
        dW[d, 1:1 + dim] = drho * u + rho * du
        dW[d, -1] = dp / (gamma - 1.0) + 0.5 * drho * (u * u).sum(0) + rho * (u * du).sum(0)
    return W, dW


def uniform_state(mesh, W_inf):
    n = mesh["n_cell"]
    W = np.tile(np.asarray(W_inf, float)[:, None], (1, n))
    dW = np.zeros((mesh["dim"], len(W_inf), n))
    return W, dW


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
def cylinder_case_mesh():
    """64 x 32 O-mesh (4096 triangles), first radial spacing 0.09695, ratio
    1.1, outer radius 20, slip wall."""
    return cylinder_mesh(64, 32, 0.5, 20.0, 1.1, BC_SLIP_WALL, first_spacing=0.09695)


def sphere_case_mesh():
    """Cubed-sphere hybrid O-grid, 6 x 28 x 28 surface quads (about the 4608
    quads of a 48 x 96 latitude-longitude grid, without its polar slivers),
    40 layers, first spacing 0.05597, ratio 1.08, outer radius 15; layers
    1-20 hex, 21-30 prisms, 31-40 tets (470,400 cells)."""
    return cubed_sphere_mesh(28, 40, 20, 10, 0.5, 15.0, 1.08, first_spacing=0.05597)


def serve_trace(n_requests=256, seed=9965, rate=20.0, frac_2d=0.7, mach=(0.1, 0.5), re_2d=(50.0, 300.0),
                re_3d=(50.0, 300.0), n_theta_2d=(32, 64, 128, 256)):
    """Seeded steady-solve request trace: exponential inter-arrival times at
    `rate` per second; frac_2d of the requests are viscous cylinders built
    like the batch cases (n_theta from n_theta_2d, n_r = n_theta/2) with a
    no-slip adiabatic wall, the rest hybrid cubed-sphere O-grids with n in
    {14..28} quads per cube edge (about the 24x48 .. 48x96 surface quads of
    latitude-longitude grids) and L in {16..40} layers (L/2 hex, L/4 prism,
    the rest tet), stretched to r = 15.  Mach ~ U[mach]; Re ~ U[re_2d] /
    U[re_3d] on the diameter.  Above Re of about 47 (cylinder) and 210
    (sphere) the physical flow sheds vortices, so some requests have no
    steady state: a server caps their cycles and reports them apart."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    out = []
    for k in range(n_requests):
        if rng.uniform() < frac_2d:
            nt = int(rng.choice(list(n_theta_2d)))
            spec = dict(dim=2, n_theta=nt, n_r=nt // 2, re=float(rng.uniform(*re_2d)))
        else:
            n = int(rng.integers(14, 29))
            L = int(rng.integers(16, 41))
            spec = dict(dim=3, n=n, layers=L, re=float(rng.uniform(*re_3d)))
        spec.update(arrival=float(t[k]), mach=float(rng.uniform(*mach)), aoa=float(rng.uniform(-5.0, 5.0)))
        out.append(spec)
    return out


def serve_mesh(spec):
    """Mesh of one trace request: the cylinder with a no-slip adiabatic
    wall, or the cubed-sphere O-grid (radial ratio 1.08^(40/L) to r = 15)."""
    if spec["dim"] == 2:
        nr = spec["n_r"]
        return cylinder_mesh(spec["n_theta"], nr, ratio=1.1 ** (32.0 / nr), wall=BC_NOSLIP_ADIABATIC)
    L = spec["layers"]
    return cubed_sphere_mesh(spec["n"], L, L // 2, L // 4, 0.5, 15.0, 1.08 ** (40.0 / L))


def batch_case_mesh(case):
    """Cylinder O-mesh of one batch case, built like the 64 x 32 cylinder:
    radius 0.5 to 20 with the same total radial stretch (ratio 1.1 per
    layer at 32 layers, 1.1^(32/n_r) at n_r layers), split triangles."""
    nr = case["n_r"]
    return cylinder_mesh(case["n_theta"], nr, ratio=1.1 ** (32.0 / nr))


def batch_cases(n_cases=64, seed=2109, mach=(0.1, 0.6)):
    """Seeded list of 2-D inviscid cylinder cases: n_theta in {32,64,128,256},
    n_r = n_theta/2, Mach ~ U[mach], AoA ~ U[-5,5] deg.  Above the
    cylinder's critical Mach number (about 0.4) supersonic pockets and
    shocks form: such cases are marked transonic (the paper runs them with
    the full gas-kinetic solution and nonlinear reconstruction weights)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_cases):
        nt = int(rng.choice([32, 64, 128, 256]))
        m = float(rng.uniform(*mach))
        out.append(dict(n_theta=nt, n_r=nt // 2, mach=m, aoa=float(rng.uniform(-5.0, 5.0)), transonic=m > 0.4))
    return out
