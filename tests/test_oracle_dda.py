"""Pins of the oracle's allocation geometry, section "Allocation" (stage one): the
band segment of a pixel and the voxel blocks it crosses.

The crossed-block rule is checked against exact rational arithmetic: a block b is
crossed when the segment meets the half-open box [b, b+1)^3.  The binary32 walk can
differ from the exact set only when two boundary crossings coincide (or nearly so);
such segments are identified exactly and checked for validity instead."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest


def exact_blocks(P0, P1):
    p0 = [Fr(float(v)) for v in P0]
    p1 = [Fr(float(v)) for v in P1]
    D = [b - a for a, b in zip(p0, p1)]
    lo = [min(math.floor(a), math.floor(b)) for a, b in zip(p0, p1)]
    hi = [max(math.floor(a), math.floor(b)) for a, b in zip(p0, p1)]
    out = set()
    for bx in range(lo[0], hi[0] + 1):
        for by in range(lo[1], hi[1] + 1):
            for bz in range(lo[2], hi[2] + 1):
                b = (bx, by, bz)
                tl, tl_c, th, th_c = Fr(0), True, Fr(1), True
                ok = True
                for a in range(3):
                    if D[a] == 0:
                        ok &= b[a] <= p0[a] < b[a] + 1
                        continue
                    te, tx = (b[a] - p0[a]) / D[a], (b[a] + 1 - p0[a]) / D[a]
                    if D[a] > 0:   # [te, tx)
                        lo_t, lo_c, hi_t, hi_c = te, True, tx, False
                    else:          # (tx, te]
                        lo_t, lo_c, hi_t, hi_c = tx, False, te, True
                    if lo_t > tl or (lo_t == tl and not lo_c):
                        tl, tl_c = lo_t, lo_c
                    if hi_t < th or (hi_t == th and not hi_c):
                        th, th_c = hi_t, hi_c
                ok &= tl < th or (tl == th and tl_c and th_c)
                if ok:
                    out.add(b)
    return out


def crossing_params(P0, P1):
    p0 = [Fr(float(v)) for v in P0]
    p1 = [Fr(float(v)) for v in P1]
    ts = []
    for a in range(3):
        d = p1[a] - p0[a]
        b0, b1 = math.floor(p0[a]), math.floor(p1[a])
        for k in range(min(b0, b1) + 1, max(b0, b1) + 1):
            ts.append((k - p0[a]) / d)
    return sorted(ts)


def near_tie(P0, P1, eps=Fr(1, 10 ** 5)):
    ts = crossing_params(P0, P1)
    return any(b - a <= eps for a, b in zip(ts[:-1], ts[1:]))


def touches_closed(P0, P1, b):
    """Segment meets the closed box [b, b+1]^3 (exact)."""
    p0 = [Fr(float(v)) for v in P0]
    p1 = [Fr(float(v)) for v in P1]
    tl, th = Fr(0), Fr(1)
    for a in range(3):
        d = p1[a] - p0[a]
        if d == 0:
            if not (b[a] <= p0[a] <= b[a] + 1):
                return False
            continue
        t1, t2 = (b[a] - p0[a]) / d, (b[a] + 1 - p0[a]) / d
        tl, th = max(tl, min(t1, t2)), min(th, max(t1, t2))
    return tl <= th


def check_walk(orc, P0, P1):
    blocks = orc.dda_blocks(P0, P1)
    f0 = [math.floor(float(v)) for v in P0]
    f1 = [math.floor(float(v)) for v in P1]
    assert tuple(blocks[0]) == tuple(f0)
    assert tuple(blocks[-1]) == tuple(f1)
    assert len(blocks) == sum(abs(a - b) for a, b in zip(f0, f1)) + 1
    steps = np.abs(np.diff(blocks, axis=0)).sum(axis=1)
    assert np.all(steps == 1), "consecutive blocks must share a face"
    got = {tuple(int(v) for v in b) for b in blocks}
    want = exact_blocks(P0, P1)
    return got, want


def test_dda_matches_exact_rational_sets(orc):
    rng = np.random.default_rng(123)
    n_tie = 0
    for i in range(3000):
        P0 = rng.uniform(-40, 40, 3).astype(np.float32)
        L = rng.uniform(0.05, 3.5)
        d = rng.standard_normal(3)
        P1 = (P0 + L * d / np.linalg.norm(d)).astype(np.float32)
        got, want = check_walk(orc, P0, P1)
        if got != want:
            assert near_tie(P0, P1), (P0, P1, got ^ want)
            n_tie += 1
            assert all(touches_closed(P0, P1, b) for b in got)
    assert n_tie <= 3


def test_dda_exact_ties_are_valid(orc):
    # segments through block edges and corners: the walk must stay valid and every
    # visited block must touch the segment
    cases = [((0.5, 0.5, 0.5), (2.5, 2.5, 0.5)), ((0.25, 0.25, 0.25), (1.75, 1.75, 1.75)),
             ((-1.5, 0.5, 0.5), (1.5, -2.5, 0.5)), ((0.0, 0.0, 0.0), (2.0, 1.0, 0.0)),
             ((3.0, 3.0, 3.0), (1.0, 1.0, 1.0))]
    for P0, P1 in cases:
        P0 = np.array(P0, np.float32)
        P1 = np.array(P1, np.float32)
        got, want = check_walk(orc, P0, P1)
        assert want <= got or near_tie(P0, P1)
        assert all(touches_closed(P0, P1, b) for b in got)


def test_dda_degenerate(orc):
    P = np.array([1.25, -3.5, 7.0], np.float32)
    b = orc.dda_blocks(P, P)
    assert b.tolist() == [[1, -4, 7]]
    # axis-aligned segment crossing three planes
    b = orc.dda_blocks(np.array([0.5, 0.5, 0.5], np.float32), np.array([0.5, 0.5, 3.5], np.float32))
    assert b.tolist() == [[0, 0, 0], [0, 0, 1], [0, 0, 2], [0, 0, 3]]


def test_band_segment_lies_on_pixel_ray(orc):
    """The two end points, scaled back to metres and moved into the camera frame,
    sit on the pixel's ray at camera depths max(d - mu, 0) and d + mu."""
    from synth import pose_look_at
    rng = np.random.default_rng(7)
    s, mu = 0.005, 0.02
    sc = orc.Scene(s, mu, 100, 2 ** 10, 2 ** 8)
    K = (525.0, 525.0, 319.5, 239.5)
    for _ in range(200):
        T = pose_look_at(rng.uniform(-3, 3, 3), rng.uniform(-3, 3, 3) + [0, 0, 5], (0, -1, 0))
        u, v = int(rng.integers(0, 640)), int(rng.integers(0, 480))
        d = np.float32(rng.uniform(0.01, 4.0))
        P0, P1 = sc.segment(d, u, v, 640, 480, K, T)
        for P, z in ((P0, max(float(d) - float(np.float32(mu)), 0.0)), (P1, float(d) + float(np.float32(mu)))):
            w = P.astype(np.float64) * 8 * float(np.float32(s))
            c = T[:3, :3].T @ (w - T[:3, 3])
            expect = z * np.array([(u - K[2]) / K[0], (v - K[3]) / K[1], 1.0])
            # binary32 rounding of block-unit coordinates up to ~60: <= 2^-18 blocks
            assert np.allclose(c, expect, atol=8 * s * 2.0 ** -17), (c, expect)
    # invalid depths give no segment
    T = np.eye(4)
    for bad in (0.0, -1.0, np.nan, np.inf):
        assert sc.segment(np.float32(bad), 10, 10, 640, 480, K, T) is None
