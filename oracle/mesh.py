"""Triangulation, connectivity and element geometry (Section 2, eq.
triangulation; Section 3.1 'value across the boundary'; Section 3.2
'immediate neighbors').

Conventions (also the C-ABI's, stated in include/cswdg.h):

* every triangle is made counter-clockwise by swapping its local vertices
  1 and 2 when its signed area is negative; a zero-area triangle is an error;
* local face f joins local vertices f and f+1 (mod 3);
* nbr[e, f] is the element across face f, or -1 on a transmissive boundary;
* info[e, f] (uint8): bits 0-1 the neighbour's local face f', bits 2-3 the x
  shift code, bits 4-5 the y shift code, bit 6 set on a boundary face.  A
  shift code says what to add to the neighbour's coordinates to place it
  next to e: 0 nothing, 1 +period, 2 -period.

Parity status: pinned by tests/test_oracle_mesh.py (an O(K^2) brute-force
search on tiny meshes, edge-pair symmetry, closed-form geometry).
"""
from __future__ import annotations

import numpy as np

BC_PERIODIC = 0
BC_TRANSMISSIVE = 1

INFO_FACE_MASK = 0x3
INFO_BOUNDARY = 0x40
# kind of a boundary face, kept in the face bits of its info byte
# (Section 4, Examples 4-6: outflow / non-reflecting, reflective wall, inflow)
BKIND_OUTFLOW, BKIND_WALL, BKIND_INFLOW, BKIND_SHOCK = 0, 1, 2, 3


class MeshError(ValueError):
    pass


def ccw_fix(vxy, tri):
    vxy = np.asarray(vxy, dtype=np.float64)
    tri = np.array(tri, dtype=np.int64, copy=True)
    p = vxy[tri]
    area2 = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    if np.any(area2 == 0.0):
        raise MeshError("zero-area triangle")
    flip = area2 < 0.0
    tri[flip, 1], tri[flip, 2] = tri[flip, 2].copy(), tri[flip, 1].copy()
    return tri, int(flip.sum())


def _shift_code(s, P):
    if s == 0:
        return 0
    return 1 if s > 0 else 2


def connectivity(vxy, tri, bc, period=(0.0, 0.0)):
    """Neighbour and face-info tables from integer vertex ids (interior
    edges) and exact coordinate matching up to one period (periodic edges).

    Returns (tri_ccw int64 [K,3], nbr int32 [K,3], info uint8 [K,3])."""
    vxy = np.asarray(vxy, dtype=np.float64)
    tri, _ = ccw_fix(vxy, tri)
    K = tri.shape[0]
    e = np.repeat(np.arange(K), 3)
    f = np.tile(np.arange(3), K)
    a = tri[e, f]
    b = tri[e, (f + 1) % 3]
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    nv = vxy.shape[0]
    key = lo * nv + hi
    order = np.argsort(key, kind="stable")
    ks = key[order]
    nbr = -np.ones((K, 3), dtype=np.int32)
    info = np.zeros((K, 3), dtype=np.uint8)
    # runs of equal keys: 1 = boundary edge, 2 = interior edge, >2 = error
    starts = np.flatnonzero(np.r_[True, ks[1:] != ks[:-1]])
    counts = np.diff(np.r_[starts, len(ks)])
    if np.any(counts > 2):
        raise MeshError("non-manifold edge")
    pairs = starts[counts == 2]
    h0, h1 = order[pairs], order[pairs + 1]
    if np.any(a[h0] == a[h1]):
        raise MeshError("inconsistently oriented neighbours")
    nbr[e[h0], f[h0]] = e[h1]
    nbr[e[h1], f[h1]] = e[h0]
    info[e[h0], f[h0]] = f[h1]
    info[e[h1], f[h1]] = f[h0]
    boundary = np.asarray(order[starts[counts == 1]], dtype=np.int64)
    if bc == BC_TRANSMISSIVE:
        info[e[boundary], f[boundary]] = INFO_BOUNDARY
        return tri, nbr, info
    if bc != BC_PERIODIC:
        raise MeshError("unknown boundary condition")
    Px, Py = float(period[0]), float(period[1])
    if len(boundary) == 0:
        return tri, nbr, info
    tol = 1e-9 * max(abs(Px), abs(Py), 1e-300)
    A = vxy[a[boundary]]  # start of each boundary edge
    B = vxy[b[boundary]]
    shifts = [(Px, 0.0), (-Px, 0.0), (0.0, Py), (0.0, -Py)]
    # partner q of edge p: q's start + s == p's end and q's end + s == p's start
    match = np.zeros((len(boundary), len(boundary)), dtype=np.int64)
    which = -np.ones((len(boundary), len(boundary)), dtype=np.int64)
    for si, (sx, sy) in enumerate(shifts):
        if (sx == 0.0 and sy == 0.0):
            continue
        c1 = (np.abs(A[None, :, 0] + sx - B[:, None, 0]) <= tol) & (np.abs(A[None, :, 1] + sy - B[:, None, 1]) <= tol)
        c2 = (np.abs(B[None, :, 0] + sx - A[:, None, 0]) <= tol) & (np.abs(B[None, :, 1] + sy - A[:, None, 1]) <= tol)
        m = c1 & c2
        match += m
        which = np.where(m, si, which)
    cnt = match.sum(axis=1)
    # periodic in one direction only (the other period 0, as Example 4's
    # sides): edges without a partner stay boundary faces
    one_way = (Px == 0.0) != (Py == 0.0)
    if np.any(cnt > 1) or (not one_way and np.any(cnt != 1)):
        raise MeshError("unmatched or ambiguous periodic boundary edge")
    info[e[boundary[cnt == 0]], f[boundary[cnt == 0]]] = INFO_BOUNDARY
    q = np.argmax(match, axis=1)
    for p in np.nonzero(cnt == 1)[0]:
        hp, hq = boundary[p], boundary[q[p]]
        sx, sy = shifts[which[p, q[p]]]
        ep, fp, eq_, fq = e[hp], f[hp], e[hq], f[hq]
        nbr[ep, fp] = eq_
        info[ep, fp] = fq | (_shift_code(sx, Px) << 2) | (_shift_code(sy, Py) << 4)
    return tri, nbr, info


def connectivity_bruteforce(vxy, tri, bc, period=(0.0, 0.0)):
    """O(K^2) reference for tiny meshes: compare every face with every face
    by vertex coordinates (plus one period for periodic meshes)."""
    vxy = np.asarray(vxy, dtype=np.float64)
    tri, _ = ccw_fix(vxy, tri)
    K = tri.shape[0]
    Px, Py = period
    nbr = -np.ones((K, 3), dtype=np.int32)
    info = np.zeros((K, 3), dtype=np.uint8)
    for e in range(K):
        for f in range(3):
            pa = vxy[tri[e, f]]
            pb = vxy[tri[e, (f + 1) % 3]]
            found = []
            for e2 in range(K):
                for f2 in range(3):
                    if e2 == e and f2 == f:
                        continue
                    qa = vxy[tri[e2, f2]]
                    qb = vxy[tri[e2, (f2 + 1) % 3]]
                    cands = [(0.0, 0.0)]
                    if bc == BC_PERIODIC:
                        cands += [c for c in [(Px, 0.0), (-Px, 0.0), (0.0, Py), (0.0, -Py)] if c != (0.0, 0.0)]
                    for sx, sy in cands:
                        if (np.allclose(qa + (sx, sy), pb, rtol=0, atol=1e-12)
                                and np.allclose(qb + (sx, sy), pa, rtol=0, atol=1e-12)):
                            found.append((e2, f2, sx, sy))
            if len(found) == 0:
                if bc == BC_PERIODIC and Px != 0.0 and Py != 0.0:
                    raise MeshError("unmatched")
                info[e, f] = INFO_BOUNDARY
            else:
                assert len(found) == 1, found
                e2, f2, sx, sy = found[0]
                nbr[e, f] = e2
                info[e, f] = f2 | (_shift_code(sx, Px) << 2) | (_shift_code(sy, Py) << 4)
    return tri, nbr, info


def shift_vector(info, period):
    """(sx, sy) to add to the neighbour's coordinates, from info codes."""
    info = np.asarray(info).astype(np.int64)
    cx = (info >> 2) & 3
    cy = (info >> 4) & 3
    sx = np.where(cx == 1, period[0], np.where(cx == 2, -period[0], 0.0))
    sy = np.where(cy == 1, period[1], np.where(cy == 2, -period[1], 0.0))
    return sx, sy


class Mesh:
    """Triangulation with connectivity and the geometric quantities the
    method uses (Section 2 affine map; Section 3.1 circumradius; Section 3.2
    mean side length)."""

    def __init__(self, vxy, tri, bc, period=(0.0, 0.0)):
        self.vxy = np.asarray(vxy, dtype=np.float64)
        self.bc = bc
        self.period = (float(period[0]), float(period[1]))
        self.tri, self.nbr, self.info = connectivity(self.vxy, tri, bc, self.period)
        self.K = self.tri.shape[0]
        V = self.vxy[self.tri]  # [K,3,2]
        self.V = V
        x0, y0 = V[:, 0, 0], V[:, 0, 1]
        x1, y1 = V[:, 1, 0], V[:, 1, 1]
        x2, y2 = V[:, 2, 0], V[:, 2, 1]
        # x(r,s) = v0 + (1+r)/2 (v1-v0) + (1+s)/2 (v2-v0)
        xr, xs = 0.5 * (x1 - x0), 0.5 * (x2 - x0)
        yr, ys = 0.5 * (y1 - y0), 0.5 * (y2 - y0)
        J = xr * ys - xs * yr
        self.J = J
        self.area = 2.0 * J
        self.rx, self.ry = ys / J, -xs / J
        self.sx, self.sy = -yr / J, xr / J
        d = V[:, [1, 2, 0], :] - V  # face f vector v_{f+1}-v_f  [K,3,2]
        L = np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2)
        self.L = L
        self.nx = d[..., 1] / L
        self.ny = -d[..., 0] / L
        a, b, c = L[:, 0], L[:, 1], L[:, 2]
        self.circumradius = a * b * c / (4.0 * self.area)
        self.mean_side = (a + b + c) / 3.0
        self.inradius = 2.0 * self.area / (a + b + c)
        self.centroid = V.mean(axis=1)

    def neighbour_shift(self):
        sx, sy = shift_vector(self.info, self.period)
        return sx, sy

    def boundary_mask(self):
        return (self.info & INFO_BOUNDARY) != 0

    def set_boundary_kinds(self, kinds):
        """kinds [K, 3]: for boundary faces BKIND_OUTFLOW (the default), _WALL,
        _INFLOW or _SHOCK (a moving planar shock); entries of interior faces
        are ignored."""
        kinds = np.asarray(kinds)
        if kinds.shape != self.info.shape or np.any((kinds < 0) | (kinds > 3)):
            raise ValueError("boundary kinds: [K, 3] array of 0, 1, 2, 3")
        b = self.boundary_mask()
        self.info = np.where(b, INFO_BOUNDARY | kinds.astype(np.uint8), self.info).astype(np.uint8)

    def boundary_kind(self):
        """[K, 3]: the kind of each boundary face, -1 on interior faces."""
        return np.where(self.boundary_mask(), (self.info & INFO_FACE_MASK).astype(np.int64), -1)

    def neighbour_face(self):
        return (self.info & INFO_FACE_MASK).astype(np.int64)

    def physical_points(self, r, s, elems=None):
        """x, y [K, q] for reference points (r_q, s_q)."""
        V = self.V if elems is None else self.V[np.asarray(elems)]
        lam1 = 0.5 * (1.0 + np.asarray(r))
        lam2 = 0.5 * (1.0 + np.asarray(s))
        x = V[:, 0, 0, None] + lam1 * (V[:, 1, 0, None] - V[:, 0, 0, None]) + lam2 * (V[:, 2, 0, None] - V[:, 0, 0, None])
        y = V[:, 0, 1, None] + lam1 * (V[:, 1, 1, None] - V[:, 0, 1, None]) + lam2 * (V[:, 2, 1, None] - V[:, 0, 1, None])
        return x, y

    def reference_coords(self, elems, x, y, shift=None):
        """Inverse affine map of element(s) elems for physical points x, y
        (arrays broadcastable to [len(elems), q])."""
        V = self.V[elems]
        x0 = V[:, 0, 0, None]
        y0 = V[:, 0, 1, None]
        if shift is not None:
            x0 = x0 + shift[0][:, None]
            y0 = y0 + shift[1][:, None]
        xr = 0.5 * (V[:, 1, 0] - V[:, 0, 0])[:, None]
        xs = 0.5 * (V[:, 2, 0] - V[:, 0, 0])[:, None]
        yr = 0.5 * (V[:, 1, 1] - V[:, 0, 1])[:, None]
        ys = 0.5 * (V[:, 2, 1] - V[:, 0, 1])[:, None]
        J = xr * ys - xs * yr
        dx = x - x0
        dy = y - y0
        r = -1.0 + (ys * dx - xs * dy) / J
        s = -1.0 + (-yr * dx + xr * dy) / J
        return r, s
