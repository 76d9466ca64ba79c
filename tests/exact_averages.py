"""Exact cell averages of a plane wave over the cells of a mesh description,
by the divergence theorem on the same faces the method integrates over:
segments in 2-D, planar triangles and bilinear quadrilaterals in 3-D (a
warped quad face bounds the cell by its bilinear surface).

For g = sin(k.x - phi), the fields F = -cos(k.x - phi) k / |k|^2 and
G = sin(k.x - phi) k / |k|^2 have div F = g and div G = cos(k.x - phi), so
cell integrals of the wave and of its gradient k cos(k.x - phi) become face
integrals, taken with an 8 x 8 Gauss rule on each face's parameter square
(a triangle as a quad with one collapsed edge).  The integrands are smooth,
so the rule's error is far below rounding at the sizes used.  Nothing here
is part of the method: the design-order tests take initial data and exact
solutions from it."""
import numpy as np

NQ = 8


def _face_points(mesh):
    """Points [n_face, q, d] and area-weighted normals [n_face, q, d]
    (pointing out of the owner) of every face's quadrature."""
    d = mesh["dim"]
    xyz = mesh["xyz"][:, :d]
    ptr, fv = mesh["face_vert_ptr"], mesh["face_vert"]
    x, w = np.polynomial.legendre.leggauss(NQ)
    x, w = 0.5 * (x + 1), 0.5 * w
    nf = len(ptr) - 1
    cnt = np.diff(ptr)
    if d == 2:
        P0, P1 = xyz[fv[ptr[:-1]]], xyz[fv[ptr[:-1] + 1]]
        t = P1 - P0
        pts = P0[:, None, :] + x[None, :, None] * t[:, None, :]
        nw = np.stack([t[:, 1], -t[:, 0]], -1)[:, None, :] * w[None, :, None]
        return pts, np.broadcast_to(nw, pts.shape).copy()
    assert set(np.unique(cnt)) <= {3, 4}, "faces with 3 or 4 vertices only"
    P = np.zeros((nf, 4, 3))
    for k in range(4):
        idx = ptr[:-1] + np.minimum(k, cnt - 1)             # triangles repeat their last vertex
        P[:, k] = xyz[fv[idx]]
    s, t = np.meshgrid(x, x, indexing="ij")
    s, t = s.reshape(-1), t.reshape(-1)
    ww = np.outer(w, w).reshape(-1)
    N = [((1 - s) * (1 - t)), (s * (1 - t)), (s * t), ((1 - s) * t)]
    pts = sum(N[k][None, :, None] * P[:, k][:, None, :] for k in range(4))
    xs = (1 - t)[None, :, None] * (P[:, 1] - P[:, 0])[:, None, :] + t[None, :, None] * (P[:, 2] - P[:, 3])[:, None, :]
    xt = (1 - s)[None, :, None] * (P[:, 3] - P[:, 0])[:, None, :] + s[None, :, None] * (P[:, 2] - P[:, 1])[:, None, :]
    return pts, np.cross(xs, xt) * ww[None, :, None]


def wave_averages(mesh, k, phi):
    """(<sin(k.x - phi)>, <cos(k.x - phi)>, volume) of every cell."""
    d, n = mesh["dim"], mesh["n_cell"]
    k = np.asarray(k, float)
    pts, nw = _face_points(mesh)
    own, nb, sh = mesh["face_owner"], mesh["face_neigh"], mesh["face_shift"][:, :d]
    kn = (nw @ k) / (k @ k)

    def face_integrals(X):
        ph = X @ k - phi
        return ((-np.cos(ph) * kn).sum(1), (np.sin(ph) * kn).sum(1), (X * nw).sum((1, 2)) / d)

    acc = np.zeros((3, n))
    a = face_integrals(pts)
    for j in range(3):
        np.add.at(acc[j], own, a[j])
    inner = nb >= 0
    b = face_integrals(pts[inner] - sh[inner][:, None, :])
    for j in range(3):
        np.add.at(acc[j], nb[inner], -b[j])
    vol = acc[2]
    return acc[0] / vol, acc[1] / vol, vol
