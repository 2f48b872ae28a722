"""Surface quadrature points from the union-of-spheres level set (Section 4.1.1).

Steps, in the order the section gives them:
  1. level set phi(x) = min_p |x - x_p| - r, the union of spheres of radius r around the
     interior particles, not smoothed or shifted; r = 0.73 dx in 2D, 0.867 dx in 3D;
  2. the explicit zero isocontour, extracted on the node lattice;
  3. per-triangle Monte-Carlo samples, uniform in each triangle (Osada et al. 2002: the
     square-root barycentric map), each carrying the area-weighted outward normal
     dA_r = n_t * area_t / count_t, so that sum |dA_r| equals the mesh area.

Choices where the section is silent: phi is evaluated exactly at the grid nodes; the
isocontour is extracted by marching tetrahedra (six tets around each cube's main
diagonal) in 3D and marching triangles (two per square) in 2D, which have no ambiguous
cases; the per-triangle count is max(1, floor(rho_s * area + u)) with u uniform, and the
random numbers come from SplitMix64 (Steele, Lea and Flood 2014) used as a counter-based
generator keyed by (seed, step, triangle id), so any implementation that enumerates
triangles the same way draws the same samples.

Triangle ids: cube c = i_0 + (n-1)(i_1 + (n-1) i_2) over the (n-1)^d lattice cells whose
corners are nodes; id = (c * T + t) * 2 + j with t the tet (T=6) or triangle (T=2) of the
cube and j the triangle within it.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from . import bspline

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64(z):
    """SplitMix64 output function applied to uint64 array z (already advanced by GAMMA)."""
    z = np.asarray(z, np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def counter_uniform(key, tri, j):
    """Uniform [0,1) number j of triangle tri's stream under key: the stream state is
    s = SplitMix64(key + (tri+1) GAMMA) and draw j is SplitMix64(s + (j+1) GAMMA), top 53
    bits scaled by 2^-53."""
    tri = np.asarray(tri, np.uint64)
    j = np.asarray(j, np.uint64)
    with np.errstate(over="ignore"):
        s = splitmix64(np.uint64(key) + (tri + np.uint64(1)) * np.uint64(GAMMA))
        z = splitmix64(s + (j + np.uint64(1)) * np.uint64(GAMMA))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def stream_key(seed, step):
    return ((int(seed) << 32) + int(step)) & MASK64


def level_set(x, n, dim, r):
    """phi at every node (natural order), exact min-distance minus r.  Nodes farther than
    4 dx outside the particles' bounding box are set to +inf (they cannot be a corner of a
    cube that has a negative corner)."""
    dx = 1.0 / n
    phi = np.full(n ** dim, np.inf)
    if len(x) == 0:
        return phi
    lo = np.maximum(np.floor(x.min(0) / dx - 4).astype(int), 0)
    hi = np.minimum(np.ceil(x.max(0) / dx + 4).astype(int), n - 1)
    axes = [np.arange(lo[a], hi[a] + 1) for a in range(dim)]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")[::-1]
    nodes = np.stack([m.ravel() for m in mesh], axis=1)
    pos = (nodes + 0.5) * dx
    d, _ = cKDTree(x).query(pos, k=1)
    phi[nodes @ (n ** np.arange(dim))] = d - r
    return phi


TETS = np.array([(0, 1, 3, 7), (0, 3, 2, 7), (0, 2, 6, 7), (0, 6, 4, 7), (0, 4, 5, 7), (0, 5, 1, 7)])
TRIS2 = np.array([(0, 1, 3), (0, 3, 2)])


def _edge_point(xu, xv, pu, pv):
    """Zero crossing on the edge from the inside vertex u (phi<0) to the outside vertex v."""
    t = pu / (pu - pv)
    return xu + t[:, None] * (xv - xu)


def isocontour(phi, n, dim):
    """Triangles (3D) or segments (2D) of the zero isocontour.

    Returns ids (M,), verts (M, d, d) [vertex, coord] and orient (M, d): the mean of the
    outside vertices minus the mean of the inside vertices of the simplex that produced
    the element (it fixes which side of the element is outward)."""
    dx = 1.0 / n
    m = n - 1
    corner_bits = np.array([[(b >> a) & 1 for a in range(dim)] for b in range(2 ** dim)])
    negn = np.nonzero(phi < 0)[0]
    if len(negn) == 0:
        return np.zeros(0, np.int64), np.zeros((0, dim, dim)), np.zeros((0, dim))
    nm = bspline.node_multi_index(negn, n, dim)
    lo = np.maximum(nm.min(0) - 1, 0)
    hi = np.minimum(nm.max(0), m - 1)
    axes = [np.arange(lo[a], hi[a] + 1) for a in range(dim)]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")[::-1]
    cm = np.stack([q.ravel() for q in mesh], axis=1)
    cubes = cm @ (m ** np.arange(dim))
    mult = n ** np.arange(dim)
    corner_idx = (cm[:, None, :] + corner_bits[None]) @ mult          # (ncube, 2^d)
    cphi = phi[corner_idx]
    neg = cphi < 0
    mixed = neg.any(1) & ~neg.all(1)
    cubes, cm, corner_idx, cphi = cubes[mixed], cm[mixed], corner_idx[mixed], cphi[mixed]
    cpos = (cm[:, None, :] + corner_bits[None] + 0.5) * dx             # (C, 2^d, d)
    simplices = TETS if dim == 3 else TRIS2
    T = len(simplices)
    ids, verts, orient = [], [], []
    for t, sv in enumerate(simplices):
        sp = cphi[:, sv]                                   # (C, dim+1)
        sx = cpos[:, sv, :]                                # (C, dim+1, d)
        sneg = sp < 0
        cnt = sneg.sum(1)
        base_id = (cubes * T + t) * 2
        # orientation helper: mean(outside) - mean(inside)
        w_out = (~sneg).astype(float)
        w_in = sneg.astype(float)
        with np.errstate(invalid="ignore", divide="ignore"):
            mo = (w_out[:, :, None] * sx).sum(1) / w_out.sum(1)[:, None]
            mi = (w_in[:, :, None] * sx).sum(1) / w_in.sum(1)[:, None]
        ori = mo - mi
        if dim == 3:
            # one inside vertex, or one outside vertex: a single triangle
            for single_in in (True, False):
                sel = np.where(cnt == (1 if single_in else 3))[0]
                if len(sel) == 0:
                    continue
                lone_mask = sneg[sel] if single_in else ~sneg[sel]
                a = np.argmax(lone_mask, axis=1)
                others = np.array([[k for k in range(4) if k != ai] for ai in a])
                pts = []
                for k in range(3):
                    o = others[:, k]
                    if single_in:
                        u, v = a, o
                    else:
                        u, v = o, a
                    pts.append(_edge_point(sx[sel, u], sx[sel, v], sp[sel, u], sp[sel, v]))
                ids.append(base_id[sel])
                verts.append(np.stack(pts, 1))
                orient.append(ori[sel])
            sel = np.where(cnt == 2)[0]
            if len(sel):
                order = np.argsort(~sneg[sel], axis=1, kind="stable")   # inside first, tet order kept
                a, b, c, d = (order[:, k] for k in range(4))
                r = np.arange(len(sel))
                P = lambda u, v: _edge_point(sx[sel][r, u], sx[sel][r, v], sp[sel][r, u], sp[sel][r, v])
                p_ac, p_ad, p_bd, p_bc = P(a, c), P(a, d), P(b, d), P(b, c)
                ids.append(base_id[sel])
                verts.append(np.stack([p_ac, p_ad, p_bd], 1))
                orient.append(ori[sel])
                ids.append(base_id[sel] + 1)
                verts.append(np.stack([p_ac, p_bd, p_bc], 1))
                orient.append(ori[sel])
        else:
            for single_in in (True, False):
                sel = np.where(cnt == (1 if single_in else 2))[0]
                if len(sel) == 0:
                    continue
                lone_mask = sneg[sel] if single_in else ~sneg[sel]
                a = np.argmax(lone_mask, axis=1)
                others = np.array([[k for k in range(3) if k != ai] for ai in a])
                r = np.arange(len(sel))
                pts = []
                for k in range(2):
                    o = others[:, k]
                    u, v = (a, o) if single_in else (o, a)
                    pts.append(_edge_point(sx[sel][r, u], sx[sel][r, v], sp[sel][r, u], sp[sel][r, v]))
                ids.append(base_id[sel])
                verts.append(np.stack(pts, 1))
                orient.append(ori[sel])
    if not ids:
        return np.zeros(0, np.int64), np.zeros((0, dim, dim)), np.zeros((0, dim))
    ids = np.concatenate(ids)
    verts = np.concatenate(verts)
    orient = np.concatenate(orient)
    o = np.argsort(ids, kind="stable")
    return ids[o], verts[o], orient[o]


def element_normals(verts, orient):
    """Unit outward normal and measure (area in 3D, length in 2D) of each element."""
    dim = verts.shape[2]
    if dim == 3:
        nv = np.cross(verts[:, 1] - verts[:, 0], verts[:, 2] - verts[:, 0])
        meas = 0.5 * np.linalg.norm(nv, axis=1)
    else:
        e = verts[:, 1] - verts[:, 0]
        nv = np.stack([-e[:, 1], e[:, 0]], axis=1)
        meas = np.linalg.norm(e, axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        nhat = nv / np.linalg.norm(nv, axis=1, keepdims=True)
    flip = np.sum(nhat * orient, axis=1) < 0
    nhat[flip] *= -1.0
    return nhat, meas


def sample_surface(x, params, step=0):
    """Surface samples of the level set around particle positions x (N, d).

    Returns dict(s (S,d), dA (S,d), label (S,) int32, tri (S,) element ids, area total)."""
    dim, n = params["dim"], params["n"]
    r = params["ls_radius"]
    rho_s = params["sample_density"]
    phi = level_set(np.asarray(x, np.float64), n, dim, r)
    ids, verts, orient = isocontour(phi, n, dim)
    nhat, meas = element_normals(verts, orient)
    keep = meas > 0
    ids, verts, nhat, meas = ids[keep], verts[keep], nhat[keep], meas[keep]
    key = stream_key(params["seed"], step)
    u0 = counter_uniform(key, ids, np.zeros_like(ids))
    cnt = np.maximum(1, np.floor(rho_s * meas + u0).astype(np.int64))
    rep = np.repeat(np.arange(len(ids)), cnt)
    j = np.arange(len(rep)) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    tid = ids[rep]
    if dim == 3:
        r1 = counter_uniform(key, tid, 1 + 2 * j)
        r2 = counter_uniform(key, tid, 2 + 2 * j)
        sq = np.sqrt(r1)
        V = verts[rep]
        s = ((1 - sq)[:, None] * V[:, 0] + (sq * (1 - r2))[:, None] * V[:, 1]
             + (sq * r2)[:, None] * V[:, 2])
    else:
        r1 = counter_uniform(key, tid, 1 + j)
        V = verts[rep]
        s = V[:, 0] + r1[:, None] * (V[:, 1] - V[:, 0])
    dA = nhat[rep] * (meas[rep] / cnt[rep])[:, None]
    lo = np.asarray(params["label_lo"][:dim])
    hi = np.asarray(params["label_hi"][:dim])
    label = np.all((s >= lo) & (s < hi), axis=1).astype(np.int32)
    return dict(s=np.ascontiguousarray(s), dA=np.ascontiguousarray(dA), label=label,
                tri=tid, area=float(meas.sum()), phi=phi)
