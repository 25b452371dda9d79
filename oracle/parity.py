"""GPU-vs-oracle parity gate (test infrastructure, used by tests and the CPU-baseline leg of bench.py).

A ray matches when both miss, or both hit the same patch with |dt| <= 1e-4 D
(D = scene diagonal) and |du|, |dv| <= 2^-L.  Otherwise it is a disagreement,
excused only when the paper's error model explains it:
  * tie   -- the GPU's leaf is, by the oracle's own FP64 arithmetic, hit and
             entered within 1e-5 max(t, 1) of the oracle's best distance (its
             own t within the 1e-4 D tolerance): two leaves or patches are then
             equally correct answers (Sec. 3.3 records the closest box);
  * seam  -- different patches meeting at a shared edge: the two hit points are
             within 1e-4 D of each other AND at least one reported (u, v) lies
             within 2^-L of its patch boundary (Sec. 3.4: neighbours share their
             boundary curves, so a ray through the seam may name either).  A hit
             near an edge on a patch farther along the ray (a ray slipping through
             a crack) is hard; a different leaf of the same patch is never a seam;
  * graze -- the ray passes within 1e-3 of the box diagonal (plus 1e-7 (t + 1)
             of rounding) of the silhouette of the leaf box one side reported (the
             box Alg. 3 tests, the leaf's half of its parent's grid with the
             parent's displacement, or the leaf's own bound), inside or outside it:
             moving the ray sideways by that much would make it miss or hit the box
             (silhouettes, box edges and corners).  Only the nearer answer can be
             excused this way: a grazed oracle leaf when the GPU missed it and
             reports a farther hit or none, a grazed GPU leaf when the oracle missed
             it and reports a farther hit or none.  The oracle confirms the first:
             on the ray moved sideways (in double precision) just out of its grazed
             box, or by twice the slack in one of eight directions across the ray,
             it must give the GPU's answer (a match by the rule above, or a miss),
             so that a GPU that skipped a leaf whose neighbour the ray would then
             meet is not excused.  For the second (a
             false positive of rounding size, which the method allows) the GPU's
             distance must be where the ray meets its box grown by the slack.
             (The margin is measured across the ray because a leaf box is often
             thin: the path along the ray through a flat box is short wherever the
             ray crosses it.)  A GPU leaf box the ray starts outside of by at most
             the slack, reported at tmin, is the same rounding-size false positive
             (a secondary ray's origin sits a leaf-sized offset from the surface, and
             at coordinates far from the origin fp32 rounds it by more);
  * tangent -- same patch, |dt| within tolerance, the ray within 1.2 degrees of
             tangent to the surface at the oracle's hit (|cos| < 0.02), and the
             surface at the GPU's (u, v) within the GPU leaf box's diagonal of the
             ray: along a nearly tangent ray every leaf the ray grazes is a hit to
             the method's error bound (Sec. 3: the leaf box bounds the error), and
             rounding moves the first one by its size over |cos|.
The gate: identical hit/miss and patch id on >= 99.99 % of the rays of a class,
and every disagreement (in hit/miss, patch, t, u or v) excused.
"""
from __future__ import annotations

import numpy as np

from . import Scene  # noqa: F401  (type of the oracle scene argument)
from . import patch_eval

NO_HIT = 0xFFFFFFFF


def ids_of(h: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(h[:, 1]).view(np.uint32)


def _path_in_box(ray, lo, hi):
    o, d = ray[:3].astype(np.float64), ray[4:7].astype(np.float64)
    near, far = float(ray[3]), np.inf
    for a in range(3):
        if d[a] == 0.0:
            if o[a] < lo[a] or o[a] > hi[a]:
                return -np.inf
            continue
        t0, t1 = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
        near, far = max(near, min(t0, t1)), min(far, max(t0, t1))
    return (far - near) * np.linalg.norm(d)  # negative when the box is missed


def _lateral_margin(ray, lo, hi):
    """Signed distance, across the ray, from the ray's line to the silhouette of the
    box [lo, hi], and the unit vector (normal to the ray) pointing from the line to
    the nearest point of that silhouette.  The box projected along the ray's
    direction onto the plane through the origin normal to it is a convex polygon;
    the distance is positive when the line passes inside it (the distance to its
    boundary), negative outside (minus the distance to it).  The ray is the 8-float
    record {o, tmin, d, tmax}."""
    o, d = np.asarray(ray[:3], np.float64), np.asarray(ray[4:7], np.float64)
    dn = d / np.linalg.norm(d)
    a = np.array([1.0, 0.0, 0.0]) if abs(dn[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(dn, a)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(dn, e1)
    corners = np.array([[(hi if (c >> k) & 1 else lo)[k] for k in range(3)] for c in range(8)]) - o
    pts = sorted(set((float(p @ e1), float(p @ e2)) for p in corners))
    cross = lambda o_, a_, b_: (a_[0] - o_[0]) * (b_[1] - o_[1]) - (a_[1] - o_[1]) * (b_[0] - o_[0])
    hull = []
    for seq in (pts, pts[::-1]):  # monotone chain: lower, then upper hull
        part = []
        for p in seq:
            while len(part) >= 2 and cross(part[-2], part[-1], p) <= 0.0:
                part.pop()
            part.append(p)
        hull += part[:-1]
    hull = np.array(hull) if hull else np.array(pts[:1])

    def nearest(a_, b_):  # point of segment a_ b_ nearest to the origin
        ab = b_ - a_
        den = ab @ ab
        s_ = 0.0 if den == 0.0 else min(max(-(a_ @ ab) / den, 0.0), 1.0)
        return a_ + s_ * ab

    m = len(hull)
    q = min((nearest(hull[k], hull[(k + 1) % m]) for k in range(m)), key=lambda x: float(x @ x))
    dist = float(np.linalg.norm(q))
    w = (q[0] * e1 + q[1] * e2) / dist if dist > 0.0 else e1
    # a box projecting to a segment or a point has no inside
    inside = m >= 3 and all(cross(hull[k], hull[(k + 1) % m], (0.0, 0.0)) >= 0.0 for k in range(m))
    return (dist if inside else -dist), w


def _moved_ray(ray, shift):
    """The ray (8 values {o, tmin, d, tmax}) moved sideways by `shift` (world), in
    double precision."""
    out = np.array(ray, dtype=np.float64)
    out[:3] += shift
    return out


def _entry(ray, lo, hi):
    """FP64 entry distance of the ray into the box [lo, hi] (inf if missed)."""
    o, d = np.asarray(ray[:3], np.float64), np.asarray(ray[4:7], np.float64)
    near, far = float(ray[3]), float(ray[7])
    for a in range(3):
        if d[a] == 0.0:
            if o[a] < lo[a] or o[a] > hi[a]:
                return np.inf
            continue
        t0, t1 = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
        near, far = max(near, min(t0, t1)), min(far, max(t0, t1))
    return near if near <= far else np.inf


def _in_frame(osc, pid, ray):
    """The ray with origin and direction mapped by patch pid's frame rows (the
    identity in world coordinates), as the oracle's boxes of that patch are."""
    R = osc.patch_frame(int(pid))
    out = np.array(ray, dtype=np.float64)
    out[:3] = R @ out[:3]
    out[4:7] = R @ out[4:7]
    return out


def gate(gpu: np.ndarray, ora: dict, rays: np.ndarray, osc: "Scene", diameter: float, leaf_depth: int,
         min_match: float = 0.9999, label: str = "") -> dict:
    """Compares GPU hits (N, 4) float32 with oracle hits; returns a report dict."""
    n = len(rays)
    gid = ids_of(gpu)
    oid = ora["id"]
    tol_t = 1e-4 * diameter
    tol_uv = 2.0 ** -leaf_depth * (1 + 1e-6)
    g_hit, o_hit = gid != NO_HIT, oid != NO_HIT
    gt = gpu[:, 0].astype(np.float64)
    both_miss = ~g_hit & ~o_hit
    same = g_hit & o_hit & (gid == oid)
    with np.errstate(invalid="ignore"):  # inf - inf on rays both sides miss
        dt_ok = np.abs(gt - ora["t"]) <= tol_t
    close = same & dt_ok & (np.abs(gpu[:, 2] - ora["u"]) <= tol_uv) & \
        (np.abs(gpu[:, 3] - ora["v"]) <= tol_uv)
    match = both_miss | close
    kinds = {"tie": 0, "seam": 0, "graze": 0, "tangent": 0, "hard": 0}
    hard = []
    for k in np.where(~match)[0]:
        ray = rays[k]
        kind = "hard"
        if g_hit[k] and o_hit[k]:
            e = osc.leaf_entry(gid[k], ray, gpu[k, 2], gpu[k, 3])
            tol_tie = 1e-5 * max(ora["t"][k], 1.0)
            if np.isfinite(e) and abs(e - gt[k]) <= tol_t and e <= ora["t"][k] + tol_tie:
                kind = "tie"
        if kind == "hard" and g_hit[k] and o_hit[k] and gid[k] != oid[k]:
            o64, d64 = ray[:3].astype(np.float64), ray[4:7].astype(np.float64)
            xg, xo = o64 + gt[k] * d64, o64 + ora["t"][k] * d64
            m = 2.0 ** -leaf_depth
            near_edge = lambda u, v: min(u, v, 1 - u, 1 - v) <= m * (1 + 1e-6)
            if np.linalg.norm(xg - xo) <= tol_t and (near_edge(gpu[k, 2], gpu[k, 3]) or
                                                      near_edge(ora["u"][k], ora["v"][k])):
                kind = "seam"
        if kind == "hard" and g_hit[k] and o_hit[k] and gid[k] == oid[k] and dt_ok[k]:
            pid = int(gid[k])
            cp, greg = osc.cp[pid], bool(osc.types[pid])
            o64, d64 = ray[:3].astype(np.float64), ray[4:7].astype(np.float64)
            dn = d64 / np.linalg.norm(d64)
            _, fu, fv = patch_eval(cp, greg, float(ora["u"][k]), float(ora["v"][k]))
            nrm = np.cross(fu, fv)
            cosv = abs(np.dot(nrm, dn)) / max(np.linalg.norm(nrm), 1e-300)
            if cosv < 0.02:
                fg = patch_eval(cp, greg, float(gpu[k, 2]), float(gpu[k, 3]))[0]
                dist = np.linalg.norm(np.cross(fg - o64, dn))
                lo, hi = osc.leaf_box(pid, gpu[k, 2], gpu[k, 3])
                if dist <= np.linalg.norm(hi - lo) + 1e-6 * (abs(gt[k]) + 1.0):
                    kind = "tangent"
        if kind == "hard":
            # the nearer side's leaf: does the ray pass within rounding of its box's
            # silhouette, the box Alg. 3 tests (the half of the parent's grid grown by
            # the parent's displacement) or the leaf's own bound?  (Boxes are in the
            # patch's frame, where the ray is taken too.)  The oracle's grazed leaf
            # excuses a GPU that missed it only if the GPU's answer is not nearer, and
            # the GPU's grazed leaf a oracle that missed it only if the oracle's
            # answer is not nearer.
            tol_ord = 1e-5 * max(abs(ora["t"][k]) if o_hit[k] else abs(gt[k]), 1.0)
            o_first = o_hit[k] and (not g_hit[k] or gt[k] >= ora["t"][k] - tol_ord)
            g_first = g_hit[k] and (not o_hit[k] or gt[k] <= ora["t"][k] + tol_ord)
            for side, side_ok, pid, u, v, t in (("oracle", o_first, oid[k], ora["u"][k], ora["v"][k], ora["t"][k]),
                                                ("gpu", g_first, gid[k], gpu[k, 2], gpu[k, 3], gt[k])):
                if side_ok and kind == "hard":
                    R = osc.patch_frame(int(pid))
                    rf = _in_frame(osc, pid, ray)
                    for lo, hi in (osc.leaf_box_alg3(pid, u, v), osc.leaf_box(pid, u, v)):
                        diag = float(np.linalg.norm(hi - lo))
                        slack = 1e-3 * diag + 1e-7 * (abs(t) + 1.0)
                        mgn, w = _lateral_margin(rf, lo, hi)
                        if abs(mgn) > slack:
                            # the GPU's leaf box may also be one the ray starts just outside
                            # of: then it enters it at tmin by rounding alone, whatever the
                            # ray's path across it
                            p0 = rf[:3] + rf[3] * rf[4:7]
                            gap = float(np.linalg.norm(np.maximum(lo - p0, 0.0) + np.maximum(p0 - hi, 0.0)))
                            if not (side == "gpu" and 0.0 < gap <= slack and abs(t - rf[3]) <= tol_t):
                                continue
                        if side == "oracle":
                            # the GPU missed a leaf the ray grazes: the oracle itself must give
                            # the GPU's answer for the ray moved sideways (in double precision)
                            # just out of that box, or by twice the slack in one of eight
                            # directions across the ray (a ray through a corner that boxes
                            # share leaves all of them only in some directions)
                            dn = rf[4:7] / np.linalg.norm(rf[4:7])
                            a1 = np.cross(dn, w)
                            a1 /= np.linalg.norm(a1)
                            moves = [((mgn + slack) if mgn >= 0.0 else -slack) * w]
                            moves += [2.0 * slack * (np.cos(th) * w + np.sin(th) * a1)
                                      for th in np.arange(8) * (np.pi / 4)]
                            o2r = osc.intersect_f64(np.array([_moved_ray(ray, R.T @ mv) for mv in moves]))
                            if not g_hit[k]:
                                agree = bool(np.any(o2r["id"] == NO_HIT))
                            else:  # a match by the gate's own rule
                                agree = bool(np.any((o2r["id"] == gid[k]) & (np.abs(o2r["t"] - gt[k]) <= tol_t) &
                                                    (np.abs(o2r["u"] - gpu[k, 2]) <= tol_uv) &
                                                    (np.abs(o2r["v"] - gpu[k, 3]) <= tol_uv)))
                        else:
                            # the GPU hit a leaf box the ray grazes (a false positive of
                            # rounding size, which the method allows): its distance must be
                            # where the ray meets that box grown by the slack
                            e2 = _entry(rf, lo - slack, hi + slack)
                            agree = np.isfinite(e2) and abs(e2 - gt[k]) <= tol_t
                        if agree:
                            kind = "graze"
                            break
        kinds[kind] += 1
        if kind == "hard" and len(hard) < 10:
            hard.append(dict(ray=int(k), gpu=(float(gt[k]), int(gid[k]), float(gpu[k, 2]), float(gpu[k, 3])),
                             oracle=(float(ora["t"][k]), int(oid[k]), float(ora["u"][k]), float(ora["v"][k]))))
    rate = float(match.mean()) if n else 1.0
    id_rate = float((both_miss | same).mean()) if n else 1.0
    return dict(label=label, n=n, match=int(match.sum()), match_rate=rate, id_rate=id_rate,
                hits=int(g_hit.sum()), oracle_hits=int(o_hit.sum()), excused=kinds, hard=hard,
                ok=(kinds["hard"] == 0 and id_rate >= min_match))


def assert_gate(rep: dict, min_match: float = 0.9999):
    msg = (f"{rep['label']}: strict match {rep['match']}/{rep['n']} ({rep['match_rate']:.6f}), "
           f"same hit/miss+patch {rep['id_rate']:.6f}, hits gpu/oracle {rep['hits']}/{rep['oracle_hits']}, "
           f"excused {rep['excused']}, hard examples {rep['hard']}")
    print(msg, flush=True)
    assert rep["excused"]["hard"] == 0, msg
    assert rep["id_rate"] >= min_match, msg
