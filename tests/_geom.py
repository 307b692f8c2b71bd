"""Exact-geometry helpers for pinning the oracle (tests only).

These are written from textbook geometry, not from the shadow-map algorithm:
a Moeller-Trumbore ray/triangle test for exact occlusion along the sun
direction, and 2D point-segment distances for the edge band.
"""
from __future__ import annotations

import numpy as np


def all_triangles(w):
    """World-space triangles drawn for a workload: scene, then two per module."""
    sc, g = w.scene, w.gen
    t = sc.xyz[sc.tri]                                   # [T,3,3]
    o, u, v = g.origin, g.edge_u, g.edge_v
    c0, c1, c2, c3 = o, o + u, (o + u) + v, o + v
    mods = np.stack([np.stack([c0, c1, c2], 1), np.stack([c0, c2, c3], 1)], 1).reshape(-1, 3, 3)
    owner = np.concatenate([np.full(t.shape[0], -1), np.repeat(np.arange(g.n_mod), 2)])
    if not g.add_as_occluders:
        return t, np.full(t.shape[0], -1)
    return np.concatenate([t, mods], 0), owner


def sample_points(g, k):
    """World positions [M, n_cv, n_cu, k, k, 3] of the k x k sub-cell centres, index order
    (module, cv, cu, b, a), a along edge_u."""
    cu = np.arange(g.n_cu)[None, :, None, None]
    cv = np.arange(g.n_cv)[:, None, None, None]
    a = np.arange(k)[None, None, None, :]
    b = np.arange(k)[None, None, :, None]
    fu = (cu + (a + 0.5) / k) / g.n_cu
    fv = (cv + (b + 0.5) / k) / g.n_cv
    fu, fv = np.broadcast_arrays(fu, fv)
    p = (g.origin[:, None, None, None, None, :]
         + fu[None, ..., None] * g.edge_u[:, None, None, None, None, :]
         + fv[None, ..., None] * g.edge_v[:, None, None, None, None, :])
    return p


def ray_hits(orig, d, tris, tmin=1e-9):
    """Distances along d to each triangle for each ray origin ([n, m], inf = miss)."""
    v0, v1, v2 = tris[:, 0], tris[:, 1], tris[:, 2]
    e1, e2 = v1 - v0, v2 - v0
    pvec = np.cross(d[None, :], e2)                       # [m,3]
    det = np.einsum("ij,ij->i", e1, pvec)
    ok = np.abs(det) > 1e-14
    inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
    tvec = orig[:, None, :] - v0[None, :, :]              # [n,m,3]
    uu = np.einsum("nmk,mk->nm", tvec, pvec) * inv[None]
    qvec = np.cross(tvec, e1[None, :, :])
    vv = np.einsum("k,nmk->nm", d, qvec) * inv[None]
    tt = np.einsum("mk,nmk->nm", e2, qvec) * inv[None]
    hit = ok[None] & (uu >= 0) & (vv >= 0) & (uu + vv <= 1) & (tt > tmin)
    return np.where(hit, tt, np.inf)


def seg_dist(p, a, b):
    """Distance from 2D points p [n,2] to segments a-b [m,2] -> [n,m]."""
    ab = b - a
    ap = p[:, None, :] - a[None]
    den = np.einsum("mk,mk->m", ab, ab)
    t = np.clip(np.einsum("nmk,mk->nm", ap, ab) / np.where(den > 0, den, 1.0)[None], 0, 1)
    q = a[None] + t[..., None] * ab[None]
    return np.linalg.norm(p[:, None, :] - q, axis=-1)


def unpack_bits(bits, k):
    """[n_cells, words] uint32 -> [n_cells, k*k] bool, sample index b*k + a."""
    n = bits.shape[0]
    by = bits.astype("<u4").view(np.uint8).reshape(n, -1)
    return np.unpackbits(by, axis=1, bitorder="little")[:, : k * k].astype(bool)
