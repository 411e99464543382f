"""Seeded synthetic scene generators.

This module is the only code shared by the CPU oracle and the HIP path.  It
holds scene *data* only: triangle soups, per-object material records and a
pinhole camera.  It contains none of the method's arithmetic (no sampling, no
MIS, no statistics, no acceleration structure).

The paper evaluates on third-party scenes (a Cornell box and ten production
interiors, Sections 4.2 and 5.2) that are not available here; these generators
are procedural stand-ins with the same structure: small area emitters, mixed
diffuse/glossy materials, and enough occlusion that the per-technique sample
counts matter.

Layout of a scene dict
----------------------
``V``        float32 [N, 9]   triangle vertices v0, v1, v2 (x, y, z each)
``tri_mat``  uint32  [N]      material index per triangle
``mats``     float32 [M, 8]   kind (0 Lambert, 1 GGX), albedo rgb, GGX alpha,
                              emitted radiance rgb (one-sided, front = the
                              side the winding normal (v1-v0)x(v2-v0) points to)
``camera``   float32 [10]     position, target, up, vertical fov in degrees
``width``, ``height``         image size in pixels
"""
from __future__ import annotations

import math

import numpy as np

LAMBERT = 0.0
GGX = 1.0


def _mat(kind, albedo, alpha=0.0, le=(0.0, 0.0, 0.0)):
    a = np.broadcast_to(np.asarray(albedo, dtype=np.float64), (3,))
    e = np.broadcast_to(np.asarray(le, dtype=np.float64), (3,))
    return [kind, a[0], a[1], a[2], alpha, e[0], e[1], e[2]]


def _quad(p, e1, e2):
    """Two triangles covering the parallelogram p, p+e1, p+e1+e2, p+e2.
    The winding normal is e1 x e2."""
    p = np.asarray(p, np.float64)
    e1 = np.asarray(e1, np.float64)
    e2 = np.asarray(e2, np.float64)
    a, b, c, d = p, p + e1, p + e1 + e2, p + e2
    return [np.concatenate([a, b, c]), np.concatenate([a, c, d])]


def _box(lo, hi, inward=False):
    """12 triangles of an axis-aligned box with outward (or inward) winding."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    dx, dy, dz = x1 - x0, y1 - y0, z1 - z0
    quads = [
        ((x0, y0, z0), (0, 0, dz), (dx, 0, 0)),   # bottom, normal -y
        ((x0, y1, z0), (dx, 0, 0), (0, 0, dz)),   # top, +y
        ((x0, y0, z0), (dx, 0, 0), (0, dy, 0)),   # front, -z
        ((x0, y0, z1), (0, dy, 0), (dx, 0, 0)),   # back, +z
        ((x0, y0, z0), (0, dy, 0), (0, 0, dz)),   # left, -x
        ((x1, y0, z0), (0, 0, dz), (0, dy, 0)),   # right, +x
    ]
    tris = []
    for p, e1, e2 in quads:
        if inward:
            e1, e2 = e2, e1
        tris += _quad(p, e1, e2)
    return tris


def _finish(tris, tri_mat, mats, camera, width, height, name, **extra):
    sc = {
        "name": name,
        "V": np.asarray(tris, dtype=np.float32).reshape(-1, 9),
        "tri_mat": np.asarray(tri_mat, dtype=np.uint32),
        "mats": np.asarray(mats, dtype=np.float32).reshape(-1, 8),
        "camera": np.asarray(camera, dtype=np.float32),
        "width": int(width),
        "height": int(height),
    }
    sc.update(extra)
    assert sc["V"].shape[0] == sc["tri_mat"].shape[0]
    return sc


# --------------------------------------------------------------------------
# Cornell box: 12 axis-aligned quads (24 triangles), one 0.2 x 0.2 emitter
# --------------------------------------------------------------------------
def make_cornell(width=64, height=64):
    mats = [
        _mat(LAMBERT, 0.7),                       # 0 white
        _mat(LAMBERT, (0.7, 0.2, 0.2)),           # 1 red (left wall)
        _mat(LAMBERT, (0.2, 0.7, 0.2)),           # 2 green (right wall)
        _mat(LAMBERT, 0.0, le=(15.0, 15.0, 15.0)),  # 3 emitter
    ]
    tris, tm = [], []

    def add(ts, m):
        tris.extend(ts)
        tm.extend([m] * len(ts))

    add(_quad((0, 0, 0), (0, 0, 1), (1, 0, 0)), 0)       # floor (normal +y)
    add(_quad((0, 1, 0), (1, 0, 0), (0, 0, 1)), 0)       # ceiling (-y)
    add(_quad((0, 0, 1), (1, 0, 0), (0, 1, 0)), 0)       # back wall (-z)
    add(_quad((0, 0, 0), (0, 1, 0), (0, 0, 1)), 1)       # left wall (+x)
    add(_quad((1, 0, 0), (0, 0, 1), (0, 1, 0)), 2)       # right wall (-x)
    add(_box((0.2, 0.0, 0.4), (0.5, 0.6, 0.7)), 0)       # tall box
    # emitter at y = 0.999, facing -y, centred, 0.2 x 0.2
    add(_quad((0.4, 0.999, 0.4), (0.2, 0, 0), (0, 0, 0.2)), 3)
    cam = [0.5, 0.5, -1.0, 0.5, 0.5, 0.0, 0.0, 1.0, 0.0, 53.13010235415598]
    return _finish(tris, tm, mats, cam, width, height, "cornell",
                   light_rect=np.array([0.4, 0.999, 0.4, 0.2, 0.2], np.float64),
                   occluder_box=np.array([0.2, 0.0, 0.4, 0.5, 0.6, 0.7], np.float64))


# --------------------------------------------------------------------------
# White furnace: closed icosphere, inward winding, Le = 1 everywhere,
# Lambert albedo 0.5.
# --------------------------------------------------------------------------
def _icosphere(subdiv):
    t = (1.0 + 5.0 ** 0.5) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
             (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(v, np.float64) / np.linalg.norm(v) for v in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
             (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
             (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts), faces


def make_furnace(width=16, height=16, subdiv=3, albedo=0.5, le=1.0):
    verts, faces = _icosphere(subdiv)
    tris = []
    for a, b, c in faces:
        # outward winding reversed -> emitting (front) side faces the centre
        tris.append(np.concatenate([verts[a], verts[c], verts[b]]))
    mats = [_mat(LAMBERT, albedo, le=(le, le, le))]
    cam = [0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 1.0, 0.0, 60.0]
    return _finish(tris, [0] * len(tris), mats, cam, width, height, "furnace",
                   furnace_albedo=albedo, furnace_le=le)


# --------------------------------------------------------------------------
# Guided-PT scene: displaced 256 x 256 heightfield + 200 random boxes,
# GGX materials, 4 quad emitters with log-uniform radiance.
# --------------------------------------------------------------------------
def make_heightfield_scene(seed=1, width=512, height=512, grid=256, n_boxes=200):
    rng = np.random.default_rng(seed)
    mats, tris, tm = [], [], []

    def ggx_mat():
        return _mat(GGX, rng.uniform(0.2, 0.9, size=3), alpha=rng.uniform(0.05, 0.5))

    # heightfield over [-1,1]^2 in x/z, height = sum of 8 Gaussian bumps
    cx = rng.uniform(-1, 1, 8)
    cz = rng.uniform(-1, 1, 8)
    sg = rng.uniform(0.1, 0.4, 8)
    amp = 0.2
    xs = np.linspace(-1.0, 1.0, grid)
    X, Z = np.meshgrid(xs, xs, indexing="ij")
    Y = np.zeros_like(X)
    for k in range(8):
        Y += amp * np.exp(-((X - cx[k]) ** 2 + (Z - cz[k]) ** 2) / (2 * sg[k] ** 2))
    P = np.stack([X, Y, Z], axis=-1)
    a = P[:-1, :-1].reshape(-1, 3)
    b = P[1:, :-1].reshape(-1, 3)
    c = P[1:, 1:].reshape(-1, 3)
    d = P[:-1, 1:].reshape(-1, 3)
    # winding normals point +y: (d - a) x (b - a) ... use a, d, c and a, c, b
    hf = np.concatenate([np.concatenate([a, d, c], 1), np.concatenate([a, c, b], 1)], 0)
    mats.append(ggx_mat())
    tris.extend(list(hf))
    tm.extend([0] * hf.shape[0])

    def height_at(x, z):
        return float(sum(amp * math.exp(-((x - cx[k]) ** 2 + (z - cz[k]) ** 2) / (2 * sg[k] ** 2))
                         for k in range(8)))

    for _ in range(n_boxes):
        s = rng.uniform(0.02, 0.15, size=3)
        px, pz = rng.uniform(-0.95, 0.95, size=2)
        yaw = rng.uniform(0, 2 * math.pi)
        base = height_at(px, pz) - 0.01
        cs, sn = math.cos(yaw), math.sin(yaw)
        box = _box((-s[0] / 2, 0.0, -s[2] / 2), (s[0] / 2, s[1], s[2] / 2))
        out = []
        for t in box:
            t = t.reshape(3, 3).copy()
            x, z = t[:, 0].copy(), t[:, 2].copy()
            t[:, 0] = cs * x - sn * z + px
            t[:, 2] = sn * x + cs * z + pz
            t[:, 1] += base
            out.append(t.reshape(9))
        mats.append(ggx_mat())
        tris.extend(out)
        tm.extend([len(mats) - 1] * len(out))

    for _ in range(4):
        sx, sz = rng.uniform(0.1, 0.3, size=2)
        px, pz = rng.uniform(-0.8, 0.8, size=2)
        h = rng.uniform(0.8, 1.5)
        le = math.exp(rng.uniform(math.log(1.0), math.log(100.0)))
        mats.append(_mat(LAMBERT, 0.0, le=(le, le, le)))
        # facing -y: e1 = +x, e2 = +z gives normal (+x)x(+z) = -y
        q = _quad((px - sx / 2, h, pz - sz / 2), (sx, 0, 0), (0, 0, sz))
        tris.extend(q)
        tm.extend([len(mats) - 1] * 2)
    cam = [0.0, 1.3, -2.4, 0.0, 0.05, 0.15, 0.0, 1.0, 0.0, 42.0]
    return _finish(tris, tm, mats, cam, width, height, f"heightfield_s{seed}")


def scaled(scene, width, height):
    """Same geometry and camera, different image size (used for the CPU
    baseline sample and the small parity cases)."""
    sc = dict(scene)
    sc["width"] = int(width)
    sc["height"] = int(height)
    return sc


# --------------------------------------------------------------------------
# Bidirectional workload: a closed 10 x 3 x 8 room filled with instanced
# furniture (unions of 3-6 boxes whose faces are tessellated into 3 x 3
# grids, ~500 triangles per piece), lit by one small 0.1 x 0.1 emitter
# (Le = 2000) hidden above an occluder panel, so that most light reaches the
# scene indirectly and connections to light subpaths matter.
# --------------------------------------------------------------------------
def _tess_box(lo, hi, n):
    """Outward-wound box with every face split into n x n quads."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    d = hi - lo
    faces = [
        (lo, np.array([0, 0, d[2]]), np.array([d[0], 0, 0])),
        (np.array([lo[0], hi[1], lo[2]]), np.array([d[0], 0, 0]), np.array([0, 0, d[2]])),
        (lo, np.array([d[0], 0, 0]), np.array([0, d[1], 0])),
        (np.array([lo[0], lo[1], hi[2]]), np.array([0, d[1], 0]), np.array([d[0], 0, 0])),
        (lo, np.array([0, d[1], 0]), np.array([0, 0, d[2]])),
        (np.array([hi[0], lo[1], lo[2]]), np.array([0, 0, d[2]]), np.array([0, d[1], 0])),
    ]
    tris = []
    for p, e1, e2 in faces:
        for i in range(n):
            for j in range(n):
                tris += _quad(p + e1 * (i / n) + e2 * (j / n), e1 / n, e2 / n)
    return np.array(tris)


def make_interior(seed=1, width=1280, height=720, n_pieces=2000, n_proto=16, tess=3):
    rng = np.random.default_rng(seed)
    mats, chunks, tm = [], [], []
    mats.append(_mat(LAMBERT, 0.6))                                   # 0 room
    room = np.array(_box((-5.0, 0.0, -4.0), (5.0, 3.0, 4.0), inward=True))
    chunks.append(room)
    tm += [0] * len(room)
    protos = []
    for _ in range(n_proto):
        boxes = []
        for _ in range(int(rng.integers(3, 7))):
            c = rng.uniform([-0.4, 0.0, -0.4], [0.4, 0.8, 0.4])
            s = rng.uniform([0.05, 0.05, 0.05], [0.5, 0.6, 0.5])
            lo = np.array([c[0] - s[0] / 2, c[1], c[2] - s[2] / 2])
            boxes.append(_tess_box(lo, lo + s, tess))
        protos.append(np.concatenate(boxes))
        if rng.random() < 0.5:
            mats.append(_mat(LAMBERT, rng.uniform(0.2, 0.8, 3)))
        else:
            mats.append(_mat(GGX, rng.uniform(0.2, 0.8, 3), alpha=rng.uniform(0.05, 0.5)))
    for _ in range(n_pieces):
        k = int(rng.integers(0, n_proto))
        scale = rng.uniform(0.4, 1.2)
        yaw = rng.uniform(0, 2 * math.pi)
        px, pz = rng.uniform([-4.5, -3.5], [4.5, 3.5])
        t = protos[k].reshape(-1, 3, 3) * scale
        cs, sn = math.cos(yaw), math.sin(yaw)
        x, z = t[..., 0].copy(), t[..., 2].copy()
        t[..., 0] = cs * x - sn * z + px
        t[..., 2] = sn * x + cs * z + pz
        chunks.append(t.reshape(-1, 9))
        tm += [1 + k] * t.shape[0]
    # hidden emitter near the ceiling, occluder panel below it
    mats.append(_mat(LAMBERT, 0.0, le=(2000.0, 2000.0, 2000.0)))
    le_id = len(mats) - 1
    mats.append(_mat(LAMBERT, 0.7))
    occ_id = len(mats) - 1
    light = np.array(_quad((3.9, 2.95, 2.9), (0.1, 0, 0), (0, 0, 0.1)))   # faces -y
    chunks.append(light)
    tm += [le_id] * len(light)
    panel = np.array(_box((3.55, 2.55, 2.55), (4.45, 2.6, 3.45)))
    chunks.append(panel)
    tm += [occ_id] * len(panel)
    cam = [-4.3, 1.6, -3.4, 1.0, 0.9, 1.5, 0.0, 1.0, 0.0, 60.0]
    return _finish(np.concatenate(chunks), tm, mats, cam, width, height, f"interior_s{seed}")


# --------------------------------------------------------------------------
# Batched workload: independent requests of uneven size.  Resolution uniform
# over {64, 128, 256, 512, 1024}^2, triangle count log-uniform in
# [tris_lo, tris_hi], half guided-PT heightfields and half BDPT interiors
# (shuffled), path depth uniform in [6, 12].  Each entry is a scene dict
# with the extra keys "mode" ("guided" or "bdpt") and "max_depth".
# --------------------------------------------------------------------------
def make_batch(seed=1, n=32, tris_lo=1000, tris_hi=500000, res=(64, 128, 256, 512, 1024),
               depth_lo=6, depth_hi=12):
    rng = np.random.default_rng(seed)
    kinds = np.array(["guided"] * (n // 2) + ["bdpt"] * (n - n // 2))
    rng.shuffle(kinds)
    out = []
    for j in range(n):
        r = int(rng.choice(res))
        target = math.exp(rng.uniform(math.log(tris_lo), math.log(tris_hi)))
        depth = int(rng.integers(depth_lo, depth_hi + 1))
        sub = int(rng.integers(1, 1 << 30))
        if kinds[j] == "guided":
            # 2 (grid - 1)^2 heightfield triangles carry ~90 % of the target
            grid = max(8, int(round(math.sqrt(0.45 * target))) + 1)
            boxes = max(2, int(0.1 * target / 12))
            sc = make_heightfield_scene(seed=sub, width=r, height=r, grid=grid, n_boxes=boxes)
        else:
            tess = 3 if target > 20000 else 1
            per_piece = 4.5 * 6 * tess * tess * 2
            pieces = max(1, int(round((target - 26) / per_piece)))
            sc = make_interior(seed=sub, width=r, height=r, n_pieces=pieces,
                               n_proto=min(16, pieces), tess=tess)
        sc["mode"] = str(kinds[j])
        sc["max_depth"] = depth
        sc["name"] = f"batch{seed}_{j}_{sc['mode']}_{r}"
        out.append(sc)
    return out
