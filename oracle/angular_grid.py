"""Geodesic angular grid (paper Sec. 2.6, 'Angular Grids').

The paper builds the grid in three steps: the 12 vertices of a regular
icosahedron; each of the 20 faces split into N^2 equilateral triangles; the
centres of all 20 N^2 triangles projected to the sphere and joined by
geodesic arcs whenever their triangles share an edge.  The result has
N_ang = 10 N^2 + 2 polygonal cells, 12 of them pentagons.

Readings taken where the paper is not explicit:
* one icosahedron vertex at +x^3 (the grid's north pole sits on a pentagon),
  a second one in the x^1-x^3 plane with x^1 > 0;
* a polygonal cell's centre (its direction n^) is the projected triangulation
  vertex the polygon surrounds;
* solid angles are exact spherical-polygon areas;
* an edge's normal nu^ is the unit tangent at the arc's midpoint m^,
  perpendicular to the arc, pointing from the lower-indexed cell to the
  higher-indexed one;
* canonical angle order: rings of equal polar angle from the north pole
  southwards, each ring by azimuth measured from psi = -0.01 rad.

Pinned by tests/test_angular_grid.py (counts, sum of solid angles = 4 pi, the
level-1 dodecahedron in closed form, Girard's-theorem areas, isotropy of the
second moment).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.spatial import cKDTree


@dataclass
class AngularGrid:
    nlev: int
    nhat: np.ndarray     # [N, 3] cell-centre directions
    domega: np.ndarray   # [N] solid angles
    polys: list          # per cell: [k, 3] polygon vertices, counter-clockwise
    lo: np.ndarray       # [E] edge: lower cell index
    hi: np.ndarray       # [E] edge: higher cell index
    length: np.ndarray   # [E] arc length
    mid: np.ndarray      # [E, 3] arc midpoint direction
    nu: np.ndarray       # [E, 3] unit normal at the midpoint, lo -> hi
    # latitude-longitude grids only: the cells beyond lo and beyond hi along
    # the edge's coordinate line (the PLM stencil ll, lo, hi, rr)
    ll: np.ndarray = None
    rr: np.ndarray = None

    @property
    def nang(self):
        return self.nhat.shape[0]


def _icosahedron():
    """12 unit vertices: poles at +-z, two rings at z = +-1/sqrt5 offset by 36 deg;
    the first upper-ring vertex lies in the x-z plane with x > 0."""
    v = [np.array([0.0, 0.0, 1.0])]
    zr = 1.0 / math.sqrt(5.0)
    rr = 2.0 / math.sqrt(5.0)
    for k in range(5):
        ph = 2.0 * math.pi * k / 5.0
        v.append(np.array([rr * math.cos(ph), rr * math.sin(ph), zr]))
    for k in range(5):
        ph = 2.0 * math.pi * (k + 0.5) / 5.0
        v.append(np.array([rr * math.cos(ph), rr * math.sin(ph), -zr]))
    v.append(np.array([0.0, 0.0, -1.0]))
    return np.array(v)


def _faces(verts):
    """Triangles = triples of mutually nearest-neighbour vertices."""
    d = np.linalg.norm(verts[:, None, :] - verts[None, :, :], axis=-1)
    dmin = np.min(d[d > 1e-12])
    adj = np.abs(d - dmin) < 1e-9
    faces = []
    n = len(verts)
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if adj[i, k] and adj[j, k]:
                    faces.append((i, j, k))
    assert len(faces) == 20
    return faces


def _unit(x):
    return x / np.linalg.norm(x, axis=-1, keepdims=True)


def spherical_triangle_area(a, b, c):
    """Van Oosterom & Strackee (1983): tan(E/2) = |a.(b x c)| / (1 + a.b + b.c + c.a)."""
    num = np.abs(np.einsum("...i,...i->...", a, np.cross(b, c)))
    den = (1.0 + np.einsum("...i,...i->...", a, b) + np.einsum("...i,...i->...", b, c)
           + np.einsum("...i,...i->...", c, a))
    return 2.0 * np.arctan2(num, den)


def build(nlev: int) -> AngularGrid:
    """Geodesic grid of level ``nlev`` (>= 1)."""
    if nlev < 1:
        raise ValueError("nlev must be >= 1")
    N = nlev
    ico = _icosahedron()
    pts = []        # flat triangulation vertices (before projection)
    tris = []       # flat sub-triangles as index triples into pts
    for (a, b, c) in _faces(ico):
        A, B, C = ico[a], ico[b], ico[c]
        index = {}
        for i in range(N + 1):
            for j in range(N + 1 - i):
                index[(i, j)] = len(pts)
                pts.append(A + (i / N) * (B - A) + (j / N) * (C - A))
        for i in range(N):
            for j in range(N - i):
                tris.append((index[(i, j)], index[(i + 1, j)], index[(i, j + 1)]))
                if i + j <= N - 2:
                    tris.append((index[(i + 1, j)], index[(i + 1, j + 1)],
                                 index[(i, j + 1)]))
    pts = np.array(pts)
    tris = np.array(tris)
    assert len(tris) == 20 * N * N
    # polygon vertices: centres of the flat sub-triangles, projected
    corner = _unit(pts[tris].mean(axis=1))

    # merge triangulation vertices duplicated along shared icosahedron edges
    proj = _unit(pts)
    pairs = cKDTree(proj).query_pairs(r=1e-9, output_type="ndarray")
    parent = np.arange(len(pts))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for i, j in pairs:
        ri, rj = find(i), find(j)
        if ri != rj:
            parent[max(ri, rj)] = min(ri, rj)
    roots = np.array([find(i) for i in range(len(pts))])
    uniq, cell_of_pt = np.unique(roots, return_inverse=True)
    cell_dir = proj[uniq]
    ncell = len(uniq)
    assert ncell == 10 * N * N + 2

    # canonical order: rings by polar angle, then azimuth from -0.01 rad
    zeta = np.arctan2(np.hypot(cell_dir[:, 0], cell_dir[:, 1]), cell_dir[:, 2])
    psi = np.mod(np.arctan2(cell_dir[:, 1], cell_dir[:, 0]) + 0.01, 2.0 * math.pi)
    order_z = np.argsort(zeta, kind="stable")
    ring = np.zeros(ncell, dtype=np.int64)
    r = 0
    for k in range(1, ncell):
        if zeta[order_z[k]] - zeta[order_z[k - 1]] > 1e-9:
            r += 1
        ring[order_z[k]] = r
    order = np.lexsort((psi, ring))
    newidx = np.empty(ncell, dtype=np.int64)
    newidx[order] = np.arange(ncell)
    nhat = cell_dir[order]
    tri_cells = newidx[cell_of_pt[tris]]          # [T, 3] cell indices

    # polygons: incident sub-triangle centres, sorted counter-clockwise
    incident = [[] for _ in range(ncell)]
    for t in range(len(tri_cells)):
        for c in tri_cells[t]:
            incident[c].append(t)
    polys = []
    domega = np.zeros(ncell)
    for c in range(ncell):
        v = nhat[c]
        P = corner[incident[c]]
        # tangent basis at v
        ref = np.array([1.0, 0.0, 0.0]) if abs(v[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        t1 = _unit(ref - v * np.dot(ref, v))
        t2 = np.cross(v, t1)
        ang = np.arctan2(P @ t2, P @ t1)
        P = P[np.argsort(ang)]
        polys.append(P)
        Q = np.roll(P, -1, axis=0)
        domega[c] = np.sum(spherical_triangle_area(v[None, :], P, Q))

    # edges: each triangulation edge separates two cells and is crossed by
    # the arc joining the centres of the two sub-triangles that share it
    edge_tris = {}
    for t in range(len(tri_cells)):
        a, b, c = tri_cells[t]
        for (p, q) in ((a, b), (b, c), (c, a)):
            key = (min(p, q), max(p, q))
            edge_tris.setdefault(key, []).append(t)
    keys = sorted(edge_tris.keys())
    E = len(keys)
    lo = np.zeros(E, dtype=np.int64)
    hi = np.zeros(E, dtype=np.int64)
    length = np.zeros(E)
    mid = np.zeros((E, 3))
    nu = np.zeros((E, 3))
    for e, key in enumerate(keys):
        ts = edge_tris[key]
        assert len(ts) == 2, "every triangulation edge is shared by two triangles"
        p1, p2 = corner[ts[0]], corner[ts[1]]
        lo[e], hi[e] = key
        cr = np.cross(p1, p2)
        length[e] = math.atan2(np.linalg.norm(cr), np.dot(p1, p2))
        mid[e] = _unit(p1 + p2)
        nrm = cr / np.linalg.norm(cr)
        if np.dot(nrm, nhat[hi[e]] - nhat[lo[e]]) < 0.0:
            nrm = -nrm
        nu[e] = nrm
    return AngularGrid(nlev=nlev, nhat=nhat, domega=domega, polys=polys, lo=lo,
                       hi=hi, length=length, mid=mid, nu=nu)


def build_latlong(n_zeta: int, n_psi: int) -> AngularGrid:
    """Latitude-longitude grid (Sec. 2.6): n_zeta + 1 latitude lines equally
    spaced in cos(zeta) from +1 to -1 (zeta from the +x^3 tetrad axis) and
    n_psi + 1 longitudes equally spaced in psi from 0 to 2 pi (psi from +x^1
    towards +x^2), so every cell has solid angle 4 pi / (n_zeta n_psi).
    Cell n = l n_psi + m; its direction is at the middle of its cos(zeta) and
    psi ranges.  Edges: constant-zeta arcs between rows l and l+1 (length
    sin(zeta) dpsi, normal +zeta-hat) and meridian arcs between columns m and
    m+1 (length dzeta, normal +psi-hat, midpoint at the middle of the arc).
    The PLM stencil of an edge continues along its coordinate line; across a
    pole it continues in the cell at psi + pi (Sec. 2.3), hence n_psi even."""
    if n_zeta < 2 or n_psi < 2 or n_psi % 2:
        raise ValueError("n_zeta >= 2 and an even n_psi >= 2 are required")
    cz = 1.0 - 2.0 * np.arange(n_zeta + 1) / n_zeta
    cz[-1] = -1.0
    zb = np.arccos(cz)
    dpsi = 2.0 * math.pi / n_psi
    pb = dpsi * np.arange(n_psi + 1)
    zc = np.arccos(0.5 * (cz[:-1] + cz[1:]))
    pc = 0.5 * (pb[:-1] + pb[1:])

    def sph(z, p):
        return np.array([math.sin(z) * math.cos(p), math.sin(z) * math.sin(p), math.cos(z)])

    def cell(l, m):
        return l * n_psi + (m % n_psi)

    N = n_zeta * n_psi
    nhat = np.array([sph(zc[l], pc[m]) for l in range(n_zeta) for m in range(n_psi)])
    domega = np.array([(cz[l] - cz[l + 1]) * dpsi for l in range(n_zeta) for _ in range(n_psi)])
    polys = []
    for l in range(n_zeta):
        for m in range(n_psi):
            P = [sph(zb[l], pb[m]), sph(zb[l + 1], pb[m]), sph(zb[l + 1], pb[m + 1]),
                 sph(zb[l], pb[m + 1])]
            if l == 0:
                P = P[:3]                 # the north-pole corner is shared
            elif l == n_zeta - 1:
                P = [P[0], P[2], P[3]]    # the south-pole corner is shared
            polys.append(np.array(P))
    lo, hi, ll, rr, length, mid, nu = [], [], [], [], [], [], []
    for l in range(n_zeta - 1):
        z = zb[l + 1]
        for m in range(n_psi):
            lo.append(cell(l, m))
            hi.append(cell(l + 1, m))
            ll.append(cell(l - 1, m) if l > 0 else cell(0, m + n_psi // 2))
            rr.append(cell(l + 2, m) if l + 2 < n_zeta else cell(n_zeta - 1, m + n_psi // 2))
            length.append(math.sin(z) * dpsi)
            mid.append(sph(z, pc[m]))
            nu.append(np.array([math.cos(z) * math.cos(pc[m]), math.cos(z) * math.sin(pc[m]),
                                -math.sin(z)]))
    for l in range(n_zeta):
        zm = 0.5 * (zb[l] + zb[l + 1])
        for m in range(n_psi):
            p = pb[m + 1]
            lo.append(cell(l, m))
            hi.append(cell(l, m + 1))
            ll.append(cell(l, m - 1))
            rr.append(cell(l, m + 2))
            length.append(zb[l + 1] - zb[l])
            mid.append(sph(zm, p))
            nu.append(np.array([-math.sin(p), math.cos(p), 0.0]))
    return AngularGrid(nlev=0, nhat=nhat, domega=domega, polys=polys,
                       lo=np.array(lo, dtype=np.int64), hi=np.array(hi, dtype=np.int64),
                       length=np.array(length), mid=np.array(mid), nu=np.array(nu),
                       ll=np.array(ll, dtype=np.int64), rr=np.array(rr, dtype=np.int64))


def _tangent_basis(v):
    ref = np.array([1.0, 0.0, 0.0]) if abs(v[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    t1 = _unit(ref - v * np.dot(ref, v))
    return t1, np.cross(v, t1)


def _gnomonic(p, v, t1, t2):
    """Coordinates of unit vector p in the plane tangent to the sphere at v."""
    s = np.dot(p, v)
    return np.array([np.dot(p, t1) / s, np.dot(p, t2) / s])


def mapr_geometry(g: AngularGrid):
    """Geometry of minimum-angle plane reconstruction (MAPR) on a polygon grid
    (Sec. 2.6; the method of Christov & Popov as used on hexagonal geodesic
    grids by Florinski et al.).  In the plane tangent at each cell centre
    (gnomonic coordinates) the neighbours are taken in angular order; every
    pair of consecutive neighbours with the cell defines a candidate plane,
    whose gradient solves the 2x2 system of the two neighbours' offsets.
    The neighbours run counter-clockwise about the outward direction, starting
    from the one of smallest index, so that the order (which breaks ties
    between equally flat planes) does not depend on the tangent basis.
    Returns (nbr [N, 6], pair_inv [N, 6, 2, 2], valid [N, 6], d_lo [E, 2],
    d_hi [E, 2]): candidate i uses neighbours nbr[:, i] and nbr[:, i+1 mod k];
    d_lo / d_hi are the edge midpoint's offsets from the lo / hi cell."""
    N = g.nhat.shape[0]
    nb = [[] for _ in range(N)]
    for e in range(len(g.lo)):
        nb[g.lo[e]].append(int(g.hi[e]))
        nb[g.hi[e]].append(int(g.lo[e]))
    nbr = np.zeros((N, 6), dtype=np.int64)
    inv = np.zeros((N, 6, 2, 2))
    valid = np.zeros((N, 6), dtype=bool)
    basis = []
    for c in range(N):
        v = g.nhat[c]
        t1, t2 = _tangent_basis(v)
        basis.append((v, t1, t2))
        xs = np.array([_gnomonic(g.nhat[k], v, t1, t2) for k in nb[c]])
        order = list(np.argsort(np.arctan2(xs[:, 1], xs[:, 0])))
        first = int(np.argmin([nb[c][i] for i in order]))
        order = order[first:] + order[:first]
        ks = [nb[c][i] for i in order]
        xs = xs[order]
        kk = len(ks)
        nbr[c, :kk] = ks
        nbr[c, kk:] = c
        for i in range(kk):
            A = np.array([xs[i], xs[(i + 1) % kk]])
            inv[c, i] = np.linalg.inv(A)
            valid[c, i] = True
    d_lo = np.array([_gnomonic(g.mid[e], *basis[g.lo[e]]) for e in range(len(g.lo))])
    d_hi = np.array([_gnomonic(g.mid[e], *basis[g.hi[e]]) for e in range(len(g.lo))])
    return nbr, inv, valid, d_lo, d_hi
