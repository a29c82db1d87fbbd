"""Seeded synthetic scan pairs for ICP (inputs only; no registration arithmetic).

Stand-ins for the fragment pairs of the paper's reconstruction workloads
(Sec. 3.4: fragments built from RGB-D sequences, then registered pairwise with
ICP, Sec. 3.3).  Those recordings are not available, so two generators emit
clouds with the same structure: a smooth heightfield and a furnished room.

Every random draw comes from ``numpy.random.Generator(PCG64(seed))``; sub-seeds
are derived with ``numpy.random.SeedSequence`` so target and source sampling
are independent but reproducible.  Arithmetic is float64, outputs are float32
C-contiguous (N, 3) arrays.  The rigid motion G applied to the source is built
with ``scipy.spatial.transform.Rotation`` (a library routine), so nothing here
shares code with either ICP implementation.

Returned dict keys (both generators):
  src, tgt, tgt_normals, src_normals : float32 (N, 3)
  G       : float64 (4, 4), the motion applied to the source (moved = G @ orig)
  T_gt    : float64 (4, 4), inverse of G: maps the moved source back onto the target
  area    : float, sampled surface area of the target in m^2
  meta    : dict of the drawn parameters
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial.transform import Rotation


def _rng(seed, *tags) -> np.random.Generator:
    """Generator for ``seed`` and a tuple of string/int tags (stable across runs)."""
    words = [int(seed)]
    for t in tags:
        if isinstance(t, str):
            words.append(int.from_bytes(t.encode("utf-8")[:8].ljust(8, b"\0"), "little"))
        else:
            words.append(int(t))
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(words)))


def unit_vector(rng: np.random.Generator) -> np.ndarray:
    v = rng.normal(size=3)
    while np.linalg.norm(v) < 1e-12:
        v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def random_motion(rng: np.random.Generator, max_deg: float, max_trans: float,
                  centre: np.ndarray) -> np.ndarray:
    """Rigid motion: rotation about ``centre`` by U(0, max_deg) degrees around a
    uniform axis, then a translation of magnitude U(0, max_trans) in a uniform
    direction.  Returns the 4x4 float64 matrix G."""
    axis = unit_vector(rng)
    ang = math.radians(rng.uniform(0.0, max_deg))
    R = Rotation.from_rotvec(axis * ang).as_matrix()
    tdir = unit_vector(rng)
    tmag = rng.uniform(0.0, max_trans)
    G = np.eye(4)
    G[:3, :3] = R
    G[:3, 3] = centre - R @ centre + tdir * tmag
    return G


def apply(G: np.ndarray, pts: np.ndarray) -> np.ndarray:
    return pts @ G[:3, :3].T + G[:3, 3]


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


# --------------------------------------------------------------------------
# Heightfield pair: z = sum_k a_k exp(-|p - c_k|^2 / (2 s_k^2)) on [0,1]^2
# --------------------------------------------------------------------------

def heightfield_params(seed: int, n_bumps: int = 8) -> dict:
    rng = _rng(seed, "hf-surface")
    return {
        "a": rng.uniform(0.02, 0.1, n_bumps),
        "s": rng.uniform(0.05, 0.2, n_bumps),
        "c": rng.uniform(0.0, 1.0, (n_bumps, 2)),
    }


def heightfield_eval(prm: dict, xy: np.ndarray):
    """Height and unit normal (from the analytic gradient) at (M, 2) points."""
    dx = xy[:, None, 0] - prm["c"][None, :, 0]
    dy = xy[:, None, 1] - prm["c"][None, :, 1]
    s2 = prm["s"][None, :] ** 2
    e = prm["a"][None, :] * np.exp(-(dx * dx + dy * dy) / (2.0 * s2))
    z = e.sum(axis=1)
    fx = (e * (-dx / s2)).sum(axis=1)
    fy = (e * (-dy / s2)).sum(axis=1)
    n = np.stack([-fx, -fy, np.ones_like(fx)], axis=1)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return z, n


def heightfield_surface(seed: int, n: int, tag: str = "tgt"):
    """``n`` points drawn uniformly in (x, y) on the seed's heightfield."""
    prm = heightfield_params(seed)
    rng = _rng(seed, "hf-" + tag)
    xy = rng.uniform(0.0, 1.0, (n, 2))
    z, nrm = heightfield_eval(prm, xy)
    return np.column_stack([xy, z]), nrm


def heightfield_pair(seed: int = 0, n_tgt: int = 5000, n_src: int = 5000,
                     noise: float = 0.001, max_deg: float = 5.0,
                     max_trans: float = 0.02) -> dict:
    """Target: ``n_tgt`` points on the heightfield with analytic normals.
    Source: an independent ``n_src`` resample plus iid N(0, noise^2) per axis,
    moved by a rigid motion about its centroid."""
    tgt, tgt_n = heightfield_surface(seed, n_tgt, "tgt")
    src0, src_n0 = heightfield_surface(seed, n_src, "src")
    rng = _rng(seed, "hf-motion")
    src0 = src0 + rng.normal(0.0, noise, src0.shape)
    G = random_motion(rng, max_deg, max_trans, src0.mean(axis=0))
    src = apply(G, src0)
    src_n = src_n0 @ G[:3, :3].T
    return {
        "src": _f32(src), "tgt": _f32(tgt), "tgt_normals": _f32(tgt_n),
        "src_normals": _f32(src_n), "G": G, "T_gt": np.linalg.inv(G),
        "area": 1.0, "meta": {"kind": "heightfield", "seed": seed},
    }


# --------------------------------------------------------------------------
# Room pair: a box room with axis-aligned boxes and spheres, surface-sampled
# --------------------------------------------------------------------------

def room_scene(seed: int, W: float, D: float, H: float, n_box: int, n_sph: int) -> dict:
    """Scene geometry: boxes resting on the floor (sides U(0.2, 1.0) m per axis)
    and spheres (radius U(0.1, 0.4) m) lying fully inside the room."""
    rng = _rng(seed, "room-scene")
    boxes = []
    for _ in range(n_box):
        size = rng.uniform(0.2, 1.0, 3)
        lo = np.array([rng.uniform(0.0, W - size[0]), rng.uniform(0.0, D - size[1]), 0.0])
        boxes.append((lo, lo + size))
    spheres = []
    for _ in range(n_sph):
        r = rng.uniform(0.1, 0.4)
        c = np.array([rng.uniform(r, W - r), rng.uniform(r, D - r), rng.uniform(r, H - r)])
        spheres.append((c, r))
    return {"W": W, "D": D, "H": H, "boxes": boxes, "spheres": spheres}


def _lattice_rect(rng, u_len, v_len, h):
    """Points of a lattice of pitch h on [0,u_len]x[0,v_len] with a random offset."""
    ou, ov = rng.uniform(0.0, h, 2)
    u = np.arange(ou, u_len, h)
    v = np.arange(ov, v_len, h)
    uu, vv = np.meshgrid(u, v, indexing="ij")
    return uu.ravel(), vv.ravel()


def _face(rng, h, axis, value, lo, hi, normal_sign):
    """Axis-aligned rectangle {x_axis = value} x [lo, hi] on the other two axes."""
    a1, a2 = [k for k in range(3) if k != axis]
    u, v = _lattice_rect(rng, hi[a1] - lo[a1], hi[a2] - lo[a2], h)
    p = np.empty((u.size, 3))
    p[:, axis] = value
    p[:, a1] = lo[a1] + u
    p[:, a2] = lo[a2] + v
    n = np.zeros_like(p)
    n[:, axis] = normal_sign
    return p, n


def _fibonacci_sphere(rng, c, r, h):
    m = max(4, int(math.ceil(4.0 * math.pi * r * r / (h * h))))
    i = np.arange(m) + 0.5
    phi = np.arccos(1.0 - 2.0 * i / m)
    theta = math.pi * (1.0 + 5.0 ** 0.5) * i
    d = np.column_stack([np.cos(theta) * np.sin(phi), np.sin(theta) * np.sin(phi), np.cos(phi)])
    d = d @ Rotation.random(random_state=rng).as_matrix().T
    return c + r * d, d


def _inside_any(p, scene, skip_box=-1, skip_sph=-1):
    """True where p lies strictly inside a solid other than the skipped one.
    Boxes count their floor contact as inside, so floor samples hidden under a
    box are removed."""
    out = np.zeros(len(p), dtype=bool)
    for bi, (lo, hi) in enumerate(scene["boxes"]):
        if bi == skip_box:
            continue
        m = ((p[:, 0] > lo[0]) & (p[:, 0] < hi[0]) & (p[:, 1] > lo[1]) & (p[:, 1] < hi[1])
             & (p[:, 2] >= lo[2] - 1e-9) & (p[:, 2] < hi[2]))
        out |= m
    for si, (c, r) in enumerate(scene["spheres"]):
        if si == skip_sph:
            continue
        d2 = ((p - c) ** 2).sum(axis=1)
        out |= d2 < r * r
    return out


def room_surface(scene: dict, rng: np.random.Generator, h: float = 0.01):
    """All visible surface samples of the scene at lattice pitch ``h`` (exact
    normals: inward for the room shell, outward for objects)."""
    W, D, H = scene["W"], scene["D"], scene["H"]
    pts, nrm = [], []
    lo0, hi0 = np.zeros(3), np.array([W, D, H])
    for axis, (a, b) in enumerate(((0.0, W), (0.0, D), (0.0, H))):
        for value, sign in ((a, +1.0), (b, -1.0)):
            p, n = _face(rng, h, axis, value, lo0, hi0, sign)
            keep = ~_inside_any(p, scene)
            pts.append(p[keep]); nrm.append(n[keep])
    for bi, (lo, hi) in enumerate(scene["boxes"]):
        for axis in range(3):
            for value, sign in ((lo[axis], -1.0), (hi[axis], +1.0)):
                if axis == 2 and sign < 0:
                    continue  # bottom face rests on the floor
                p, n = _face(rng, h, axis, value, lo, hi, sign)
                keep = ~_inside_any(p, scene, skip_box=bi)
                pts.append(p[keep]); nrm.append(n[keep])
    for si, (c, r) in enumerate(scene["spheres"]):
        p, n = _fibonacci_sphere(rng, c, r, h)
        keep = ~_inside_any(p, scene, skip_sph=si)
        pts.append(p[keep]); nrm.append(n[keep])
    return np.concatenate(pts), np.concatenate(nrm)


def _rect_random(rng, m, axis, value, lo, hi, sign):
    a1, a2 = [k for k in range(3) if k != axis]
    p = np.empty((m, 3))
    p[:, axis] = value
    p[:, a1] = rng.uniform(lo[a1], hi[a1], m)
    p[:, a2] = rng.uniform(lo[a2], hi[a2], m)
    n = np.zeros_like(p)
    n[:, axis] = sign
    return p, n


def room_surface_random(scene: dict, rng: np.random.Generator, n: int):
    """``n`` points drawn uniformly by area on the visible surfaces of the scene
    (the limit of subsampling a fine lattice), with exact normals.  Returns the
    points, normals and the visible area (m^2)."""
    W, D, H = scene["W"], scene["D"], scene["H"]
    parts = []  # (area, sampler(m) -> (p, n), skip_box, skip_sph)
    lo0, hi0 = np.zeros(3), np.array([W, D, H])
    for axis, (a, b) in enumerate(((0.0, W), (0.0, D), (0.0, H))):
        others = [k for k in range(3) if k != axis]
        area = (hi0[others[0]] - lo0[others[0]]) * (hi0[others[1]] - lo0[others[1]])
        for value, sign in ((a, +1.0), (b, -1.0)):
            parts.append((area, (axis, value, lo0, hi0, sign), -1, -1))
    for bi, (lo, hi) in enumerate(scene["boxes"]):
        for axis in range(3):
            others = [k for k in range(3) if k != axis]
            area = (hi[others[0]] - lo[others[0]]) * (hi[others[1]] - lo[others[1]])
            for value, sign in ((lo[axis], -1.0), (hi[axis], +1.0)):
                if axis == 2 and sign < 0:
                    continue
                parts.append((area, (axis, value, lo, hi, sign), bi, -1))
    for si, (c, r) in enumerate(scene["spheres"]):
        parts.append((4.0 * math.pi * r * r, (c, r), -1, si))
    areas = np.array([p[0] for p in parts])
    total = areas.sum()
    pts, nrm, kept_area = [], [], 0.0
    want = int(n * 1.3) + 64
    counts = rng.multinomial(want, areas / total)
    for (area, prm, sb, ss), m in zip(parts, counts):
        if m == 0:
            continue
        if ss >= 0:
            c, r = prm
            d = rng.normal(size=(m, 3))
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            p, q = c + r * d, d
        else:
            p, q = _rect_random(rng, m, *prm)
        keep = ~_inside_any(p, scene, skip_box=sb, skip_sph=ss)
        kept_area += area * keep.mean()
        pts.append(p[keep]); nrm.append(q[keep])
    pts, nrm = np.concatenate(pts), np.concatenate(nrm)
    if len(pts) < n:  # rare: top up with a second round
        p2, n2, _ = room_surface_random(scene, rng, n - len(pts))
        pts, nrm = np.concatenate([pts, p2]), np.concatenate([nrm, n2])
    sel = rng.permutation(len(pts))[:n]
    return pts[sel], nrm[sel], kept_area


def room_pair_random(seed: int, n_tgt: int, n_src: int, W: float = 6.0, D: float = 4.0,
                     H: float = 3.0, n_box: int = 20, n_sph: int = 10, overlap: float = 0.7,
                     noise: float = 0.002, max_deg: float = 10.0, max_trans: float = 0.10) -> dict:
    """Same scene, crop, noise and motion recipe as ``room_pair``, with the
    surfaces sampled uniformly at random by area instead of through a 1 cm
    lattice and a subsample (equivalent in distribution, O(N) cost)."""
    scene = room_scene(seed, W, D, H, n_box, n_sph)
    rt, rs, rm = _rng(seed, "tgt"), _rng(seed, "src"), _rng(seed, "motion")
    tp, tn, area = room_surface_random(scene, rt, n_tgt)
    tp = tp + rt.normal(0.0, noise, tp.shape)
    from_low = bool(rm.integers(0, 2))
    xs = np.sort(tp[:, 0])
    k = min(len(xs) - 1, max(0, int(round(overlap * len(xs))) - 1))
    cut = xs[k] if from_low else xs[len(xs) - 1 - k]
    # draw the source from the slab: sample generously, crop, trim
    sp, sn = np.empty((0, 3)), np.empty((0, 3))
    want = n_src
    while len(sp) < n_src:
        p, q, _ = room_surface_random(scene, rs, int(want / max(overlap, 0.05) * 1.2) + 64)
        keep = p[:, 0] <= cut if from_low else p[:, 0] >= cut
        sp, sn = np.concatenate([sp, p[keep]]), np.concatenate([sn, q[keep]])
        want = n_src - len(sp) + 64
    sp, sn = sp[:n_src], sn[:n_src]
    sp = sp + rs.normal(0.0, noise, sp.shape)
    G = random_motion(rm, max_deg, max_trans, sp.mean(axis=0))
    src = apply(G, sp)
    return {
        "src": _f32(src), "tgt": _f32(tp), "tgt_normals": _f32(tn),
        "src_normals": _f32(sn @ G[:3, :3].T), "G": G, "T_gt": np.linalg.inv(G),
        "area": float(area),
        "meta": {"kind": "room-random", "seed": seed, "W": W, "D": D, "H": H, "n_box": n_box,
                 "n_sph": n_sph, "overlap": overlap, "from_low": from_low, "cut": float(cut)},
    }


def room_pair(seed: int = 0, n_tgt: int = 300_000, n_src: int = 300_000,
              W: float = 6.0, D: float = 4.0, H: float = 3.0, n_box: int = 20,
              n_sph: int = 10, overlap: float = 0.7, noise: float = 0.002,
              max_deg: float = 10.0, max_trans: float = 0.10, h: float = 0.01) -> dict:
    """Target: the whole room sampled at pitch ``h`` plus N(0, noise^2) position
    noise, subsampled to ``n_tgt``.  Source: an independent sampling cropped to an
    x-slab that starts at a random end wall and holds a fraction ``overlap`` of
    the target's samples, subsampled to ``n_src``, then moved by a rigid motion
    about its centroid.  Normals are exact (never perturbed)."""
    scene = room_scene(seed, W, D, H, n_box, n_sph)
    rt, rs, rm = _rng(seed, "tgt"), _rng(seed, "src"), _rng(seed, "motion")

    tp, tn = room_surface(scene, rt, h)
    area = tp.shape[0] * h * h
    tp = tp + rt.normal(0.0, noise, tp.shape)
    sp, sn = room_surface(scene, rs, h)
    sp = sp + rs.normal(0.0, noise, sp.shape)

    # x-slab holding a fraction `overlap` of the target's samples
    from_low = bool(rm.integers(0, 2))
    xs = np.sort(tp[:, 0])
    k = min(len(xs) - 1, max(0, int(round(overlap * len(xs))) - 1))
    if from_low:
        cut = xs[k]
        keep = sp[:, 0] <= cut
    else:
        cut = xs[len(xs) - 1 - k]
        keep = sp[:, 0] >= cut
    sp, sn = sp[keep], sn[keep]

    ti = rt.choice(len(tp), size=min(n_tgt, len(tp)), replace=False)
    si = rs.choice(len(sp), size=min(n_src, len(sp)), replace=False)
    tp, tn = tp[np.sort(ti)], tn[np.sort(ti)]
    sp, sn = sp[np.sort(si)], sn[np.sort(si)]
    # shuffle so that storage order carries no spatial structure
    tperm, sperm = rt.permutation(len(tp)), rs.permutation(len(sp))
    tp, tn, sp, sn = tp[tperm], tn[tperm], sp[sperm], sn[sperm]

    G = random_motion(rm, max_deg, max_trans, sp.mean(axis=0))
    src = apply(G, sp)
    src_n = sn @ G[:3, :3].T
    return {
        "src": _f32(src), "tgt": _f32(tp), "tgt_normals": _f32(tn),
        "src_normals": _f32(src_n), "G": G, "T_gt": np.linalg.inv(G),
        "area": float(area),
        "meta": {"kind": "room", "seed": seed, "W": W, "D": D, "H": H,
                 "n_box": n_box, "n_sph": n_sph, "overlap": overlap,
                 "from_low": from_low, "cut": float(cut)},
    }


# --------------------------------------------------------------------------
# Workload recipes (sizes and parameters of the five benchmark configurations)
# --------------------------------------------------------------------------

def c1_heightfield(seed: int = 0) -> dict:
    """5k/5k heightfield pair, point-to-plane, r = 5 cm, 30 iterations."""
    d = heightfield_pair(seed, 5000, 5000)
    d.update(max_corr_dist=0.05, max_iter=30, variant="point_to_plane")
    return d


def c2_room(seed: int = 0) -> dict:
    """300k/300k room pair (6x4x3 m, 20 boxes, 10 spheres), r = 3 cm, 50 iterations."""
    d = room_pair(seed, 300_000, 300_000, 6.0, 4.0, 3.0, 20, 10, overlap=0.7)
    d.update(max_corr_dist=0.03, max_iter=50, variant="point_to_plane")
    return d


def c3_room(seed: int = 0) -> dict:
    """2M/2M room pair (12x8x3 m, 80 boxes, 40 spheres), r = 2 cm, 50 iterations."""
    d = room_pair(seed, 2_000_000, 2_000_000, 12.0, 8.0, 3.0, 80, 40, overlap=0.7)
    d.update(max_corr_dist=0.02, max_iter=50, variant="point_to_plane")
    return d


def with_far_outliers(d: dict, seed: int = 0, frac: float = 0.01, dist: float = 100.0) -> dict:
    """The pair with ``frac`` of its target points copied ``dist`` metres away
    from the target's box centre (uniform directions, with their normals) and
    appended to the target: a box ~2 dist wide, most of it empty.  The
    original target points keep their indices; no source point comes within
    any correspondence distance of the copies."""
    rng = _rng(seed, "far_outliers")
    tgt, nrm = d["tgt"], d["tgt_normals"]
    m = max(1, int(round(frac * len(tgt))))
    pick = rng.choice(len(tgt), size=m, replace=False)
    u = rng.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    centre = 0.5 * (tgt.min(axis=0).astype(np.float64) + tgt.max(axis=0).astype(np.float64))
    far = centre + dist * u + (tgt[pick].astype(np.float64) - centre) * 0.01
    out = dict(d)
    out["tgt"] = _f32(np.concatenate([tgt, far]))
    out["tgt_normals"] = _f32(np.concatenate([nrm, nrm[pick]]))
    out["meta"] = dict(d.get("meta", {}), far_outliers=m, far_dist=dist)
    return out


def loguniform_size(rng: np.random.Generator, lo: float, hi: float) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def c4_pair(p: int, lo: float = 2e3, hi: float = 2e5) -> dict:
    """Pair ``p`` of the batched workload: seed 1000+p, size log-uniform in
    [2k, 200k], overlap U(0.5, 0.9), r = max(3 cm, 2 sqrt(A/N))."""
    seed = 1000 + p
    rng = _rng(seed, "c4-size")
    n = loguniform_size(rng, lo, hi)
    o = rng.uniform(0.5, 0.9)
    d = room_pair_random(seed, n, n, 6.0, 4.0, 3.0, 20, 10, overlap=o)
    d.update(max_corr_dist=max(0.03, 2.0 * math.sqrt(d["area"] / len(d["tgt"]))),
             max_iter=30, rel_tol=1e-6, variant="point_to_plane")
    return d


def c5_request_size(q: int, lo: float = 5e3, hi: float = 5e5):
    """Size and overlap of served request ``q`` (seed 10000+q)."""
    rng = _rng(10_000 + q, "c5-size")
    return loguniform_size(rng, lo, hi), rng.uniform(0.5, 0.9)


def c5_request(q: int, lo: float = 5e3, hi: float = 5e5) -> dict:
    n, o = c5_request_size(q, lo, hi)
    d = room_pair_random(10_000 + q, n, n, 6.0, 4.0, 3.0, 20, 10, overlap=o)
    d.update(rel_tol=1e-6, variant="point_to_plane")
    return d


def c5_scene(k: int, n_max: int = 500_000, noise: float = 0.002) -> dict:
    """Scene ``k`` of the served workload's pool (seed 20000+k): a 6x4x3 m room
    with 20 boxes and 10 spheres, its target surface sampled at the largest
    request size (``n_max`` points, exact normals, N(0, noise^2) positions) and
    an independent source surface sampling twice as dense, both in random
    order.  Requests are cut from these samplings by ``c5_request_pooled``."""
    seed = 20_000 + k
    scene = room_scene(seed, 6.0, 4.0, 3.0, 20, 10)
    rt, rs = _rng(seed, "tgt"), _rng(seed, "src")
    tp, tn, area = room_surface_random(scene, rt, n_max)
    tp = tp + rt.normal(0.0, noise, tp.shape)
    sp, _, _ = room_surface_random(scene, rs, 2 * n_max + 64)
    sp = sp + rs.normal(0.0, noise, sp.shape)
    return {"tgt": tp, "tgt_normals": tn, "src": sp, "area": float(area)}


def _c5_pool_params(q: int, scenes: list):
    """Random choices of pooled request q: size, overlap, scene, offsets, side."""
    n, o = c5_request_size(q)
    rng = _rng(10_000 + q, "c5-pool")
    k = int(rng.integers(len(scenes)))
    N = len(scenes[k]["tgt"])
    n = min(n, N)
    off = int(rng.integers(N))
    from_low = bool(rng.integers(0, 2))
    kk = min(n - 1, max(0, int(round(o * n)) - 1))
    return n, o, rng, k, off, from_low, kk


def _c5_motion(rng, lo, hi) -> np.ndarray:
    """Random motion of a pooled request: rotation <= 10 deg about the centre
    of the source's bounding box, translation <= 10 cm (the box centre is an
    exact function of the points, unlike a centroid's rounded sum)."""
    return random_motion(rng, 10.0, 0.10, (np.asarray(lo, np.float64) + np.asarray(hi, np.float64)) / 2.0)


def c5_request_pooled(q: int, scenes: list) -> dict:
    """Served request ``q`` (seed 10000+q) cut from a pool of scenes: its size
    n and overlap o come from ``c5_request_size``; the target is n points of a
    scene's target sampling taken from a random offset of its random order (a
    random subsample), the source the first n points, from a random offset of
    the scene's source sampling, inside the x-slab from a random end wall that
    holds a fraction o of those target points, moved by a random motion
    (``_c5_motion``).  Returns float32 clouds, the target spacing sqrt(A / n)
    and the motion.  ``c5_request_pooled_torch`` computes the same arrays
    with torch (e.g. on the GPU)."""
    n, o, rng, k, off, from_low, kk = _c5_pool_params(q, scenes)
    P = scenes[k]
    N = len(P["tgt"])
    idx = (off + np.arange(n)) % N
    tp, tn = P["tgt"][idx], P["tgt_normals"][idx]
    xs = np.sort(tp[:, 0])
    cut = xs[kk] if from_low else xs[n - 1 - kk]
    sx = np.ascontiguousarray(P["src"][:, 0])
    M = len(sx)
    soff = int(rng.integers(M))
    order = (soff + np.arange(M)) % M
    inside = sx[order] <= cut if from_low else sx[order] >= cut
    sp = P["src"][order[np.nonzero(inside)[0][:n]]]
    G = _c5_motion(rng, sp.min(axis=0), sp.max(axis=0))
    moved = np.empty_like(sp)
    for a in range(3):
        moved[:, a] = ((G[a, 0] * sp[:, 0] + G[a, 1] * sp[:, 1]) + G[a, 2] * sp[:, 2]) + G[a, 3]
    return {"src": _f32(moved), "tgt": _f32(tp), "tgt_normals": _f32(tn),
            "spacing": math.sqrt(P["area"] / n), "G": G, "T_gt": np.linalg.inv(G),
            "meta": {"q": q, "n": n, "overlap": o, "from_low": from_low, "scene": k}}


def c5_request_pooled_torch(q: int, scenes: list, scenes_t: list) -> dict:
    """``c5_request_pooled`` with the array work in torch: scenes_t[k] holds
    the float64 tensors "tgt", "tgt_normals", "src" (any device) of
    scenes[k].  Every step is a selection or one rounding of the same
    float64 operation, so the float32 clouds equal the numpy ones bit for bit."""
    import torch
    n, o, rng, k, off, from_low, kk = _c5_pool_params(q, scenes)
    P, T = scenes[k], scenes_t[k]
    dev = T["tgt"].device
    N = T["tgt"].shape[0]
    idx = (off + torch.arange(n, device=dev)) % N
    tp, tn = T["tgt"][idx], T["tgt_normals"][idx]
    xs = torch.sort(tp[:, 0]).values
    cut = xs[kk] if from_low else xs[n - 1 - kk]
    M = T["src"].shape[0]
    soff = int(rng.integers(M))
    order = (soff + torch.arange(M, device=dev)) % M
    sx = T["src"][order, 0]
    inside = sx <= cut if from_low else sx >= cut
    sp = T["src"][order[torch.nonzero(inside).flatten()[:n]]]
    G = _c5_motion(rng, sp.min(dim=0).values.cpu().numpy(), sp.max(dim=0).values.cpu().numpy())
    cols = []
    for a in range(3):
        cols.append(((G[a, 0] * sp[:, 0] + G[a, 1] * sp[:, 1]) + G[a, 2] * sp[:, 2]) + G[a, 3])
    moved = torch.stack(cols, dim=1)
    return {"src": moved.float().contiguous(), "tgt": tp.float().contiguous(),
            "tgt_normals": tn.float().contiguous(), "spacing": math.sqrt(P["area"] / n), "G": G,
            "T_gt": np.linalg.inv(G), "meta": {"q": q, "n": n, "overlap": o, "from_low": from_low, "scene": k}}


def poisson_arrivals(n: int, rate: float, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson process of ``rate`` requests/s."""
    rng = _rng(seed, "arrivals")
    return np.cumsum(rng.exponential(1.0 / rate, n))


def pose_graph(seed: int, n: int, closures: int, noise_deg: float = 0.5, noise_m: float = 0.02,
               init_deg: float = 5.0, init_m: float = 0.2) -> dict:
    """A pose graph like the fragment graph of a scene reconstruction: n
    fragment poses along a closed loop (radius ~ n / (2 pi) * 0.5 m), an
    odometry edge between consecutive fragments, the loop-closing edge, and
    `closures` extra edges between random pairs.  Measurements are the true
    relative poses times a random rotation (axis uniform, angle N(0, noise_deg))
    and translation (N(0, noise_m) per axis); information matrices are random
    symmetric positive definite.  Initial poses are the truth perturbed the same
    way with init_deg / init_m, node 0 exact.  Rotations come from
    scipy.spatial.transform.Rotation (rotation vectors)."""
    from scipy.spatial.transform import Rotation
    rng = _rng(seed, "pose-graph")

    def rigid(rotvec, t):
        T = np.eye(4)
        T[:3, :3] = Rotation.from_rotvec(rotvec).as_matrix()
        T[:3, 3] = t
        return T

    def noise(deg, m):
        ax = unit_vector(rng)
        return rigid(ax * math.radians(rng.normal(0.0, deg)), rng.normal(0.0, m, 3))

    gt = [np.eye(4)]
    for k in range(1, n):
        step = rigid(np.array([0.0, 0.0, 2 * math.pi / n]) + rng.normal(0.0, 0.02, 3),
                     np.array([0.5, 0.0, 0.0]) + rng.normal(0.0, 0.02, 3))
        gt.append(gt[-1] @ step)
    pairs = [(k, k + 1) for k in range(n - 1)] + [(n - 1, 0)]
    seen = set(pairs)
    while len(pairs) < n + closures:
        i, j = (int(x) for x in sorted(rng.choice(n, 2, replace=False)))
        if (i, j) not in seen:
            seen.add((i, j))
            pairs.append((i, j))
    edges = []
    for i, j in pairs:
        Z = np.linalg.inv(gt[i]) @ gt[j] @ noise(noise_deg, noise_m)
        Q, _ = np.linalg.qr(rng.normal(size=(6, 6)))
        L = Q @ np.diag(rng.uniform(0.5, 5.0, 6)) @ Q.T
        edges.append((i, j, Z, 0.5 * (L + L.T)))
    init = [gt[0]] + [noise(init_deg, init_m) @ T for T in gt[1:]]
    return {"gt": np.array(gt), "init": np.array(init), "edges": edges}


def fpfh_like_features(rng: np.random.Generator, n: int, dim: int = 33, alpha: float = 0.6) -> np.ndarray:
    """Random descriptors shaped like FPFH: dim / 11 sub-histograms of 11 bins,
    each a Dirichlet(alpha) draw scaled to sum to 100."""
    assert dim % 11 == 0
    parts = [100.0 * rng.dirichlet(np.full(11, alpha), size=n) for _ in range(dim // 11)]
    return np.concatenate(parts, axis=1) if n else np.zeros((0, dim))


def ransac_pair(seed: int = 0, n_tgt: int = 20_000, n_src: int = 20_000, dim: int = 33,
                match_frac: float = 0.3, feat_noise: float = 1.0, W: float = 4.0, D: float = 3.0,
                H: float = 2.5, n_box: int = 10, n_sph: int = 5, overlap: float = 0.7,
                max_deg: float = 60.0, max_trans: float = 1.0) -> dict:
    """Input of feature-based global registration: a downsampled room pair
    (``room_pair_random``: uniform samples by area, ~5 cm spacing at the
    default sizes) moved by a large rigid motion, with FPFH-shaped features.
    Target features are random (``fpfh_like_features``).  A source point whose
    true counterpart (the nearest target point to its true position, if within
    5 cm) exists receives that counterpart's feature plus N(0, feat_noise^2)
    noise (clipped at 0) with probability ``match_frac``, else a fresh random
    feature, so its nearest feature is a random target point.  The true
    counterparts come from ``scipy.spatial.cKDTree``.

    Keys: src, tgt, tgt_normals (float32 (N, 3)), src_feat, tgt_feat (float32
    (N, dim)), T_gt, G, true_match (int64, -1 where the feature is random),
    meta."""
    from scipy.spatial import cKDTree
    d = room_pair_random(seed, n_tgt, n_src, W, D, H, n_box, n_sph, overlap=overlap,
                         max_deg=max_deg, max_trans=max_trans)
    rf = _rng(seed, "features")
    ft = fpfh_like_features(rf, len(d["tgt"]), dim)
    home = apply(d["T_gt"], d["src"].astype(np.float64))
    dist, j = cKDTree(d["tgt"].astype(np.float64)).query(home)
    good = (dist < 0.05) & (rf.random(len(home)) < match_frac)
    fs = fpfh_like_features(rf, len(home), dim)
    noisy = ft[j] + rf.normal(0.0, feat_noise, (len(home), dim))
    fs[good] = np.maximum(noisy[good], 0.0)
    d.update(src_feat=_f32(fs), tgt_feat=_f32(ft), true_match=np.where(good, j, -1).astype(np.int64))
    d["meta"].update(kind="ransac-room", dim=dim, match_frac=match_frac, feat_noise=feat_noise)
    return d
