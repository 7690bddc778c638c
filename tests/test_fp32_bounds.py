"""The exactness argument of the FP32 fast path, checked on the CPU.

The kernels decide most assignments and every pruning step in FP32 and must
still return the FP64 oracle's assignment (lowest-index argmin of the
canonical FP64 squared distance).  That rests on a handful of conservative
decision functions (csrc/ekm_internal.hpp): the FP32 squared distance and box
distances (fused multiply-adds), the norm-based bound e on |c - fl32(c)|,
dist_hi / dist_lo, margin_safe, lo_inverse and prune_threshold.  This module
re-evaluates each of them in emulated IEEE float32 (numpy float32 for single
operations, an exactly rounded fused multiply-add, and square roots that are
also perturbed by one unit in the last place either way) and checks the
properties the kernels rely on against canonical FP64 distances:

  * margin_safe(s1, s2) => the FP32 winner is strictly nearer in FP64 than the
    runner-up (so no FP64 recheck is needed);
  * a centroid pruned for a box (box min-distance above prune_threshold(U))
    is strictly farther in FP64 than the centroid that gave U, from every
    point of the box;
  * dist_lo(s) <= h implies s <= lo_inverse(h) (the FP64 recheck visits every
    candidate that can still win);
  * inter_keep (the inter bound of Eq. (4) and (5)): a point, or every point
    of a box, kept with its centroid c_a because it lies within half of the
    FP32 distance from c_a to another centroid c_b is strictly nearer to c_a
    than to c_b in FP64.

Samples cover random, near-bisector, large-offset (|c| ~ 1e3) and tiny-scale
data, a million cases per property.
"""

import numpy as np
import pytest

F = np.float32
MARGIN_UP = F(1.0) + F(2.0 ** -16)
MARGIN_DN = F(1.0) - F(2.0 ** -16)
TAU = F(2.0 ** -120)
N = 1_000_000


# ------------------------------------------------------------ float32 helpers
def fma32(a, b, c):
    """Correctly rounded float32 fma(a, b, c) for float32 arrays.

    a*b is exact in float64; the float64 sum is corrected with TwoSum and the
    float32 rounding of s + err is taken; only exact float32 midpoints can
    round differently from s alone, and those are resolved by err's sign.
    """
    a, b, c = (np.asarray(v, np.float32).astype(np.float64) for v in (a, b, c))
    p = a * b
    s = p + c
    bb = s - p
    err = (p - (s - bb)) + (c - bb)
    r = s.astype(np.float32)
    r64 = r.astype(np.float64)
    up = np.nextafter(r, np.float32(np.inf)).astype(np.float64)
    dn = np.nextafter(r, np.float32(-np.inf)).astype(np.float64)
    # s exactly halfway between r and a neighbour: err decides the direction
    mid_up = (s - r64) * 2 == (up - r64)
    mid_dn = (r64 - s) * 2 == (r64 - dn)
    out = r.copy()
    fix_up = mid_up & (err > 0)
    fix_dn = mid_dn & (err < 0)
    out[fix_up] = np.nextafter(r[fix_up], np.float32(np.inf))
    out[fix_dn] = np.nextafter(r[fix_dn], np.float32(-np.inf))
    # s halfway and err pulling back toward r keeps r; ties (err == 0) keep numpy's even rounding
    back_up = mid_up & (err < 0) & (r64 < s)
    back_dn = mid_dn & (err > 0) & (r64 > s)
    out[back_up] = r[back_up]
    out[back_dn] = r[back_dn]
    return out


def sqrt32(v, bias=0):
    r = np.sqrt(np.asarray(v, np.float32))
    if bias > 0:
        r = np.nextafter(r, np.float32(np.inf))
    elif bias < 0:
        r = np.nextafter(r, np.float32(0)).astype(np.float32)
    return r.astype(np.float32)


# ---------------------------------------- the kernels' decision functions
def sqdist32(x, c):
    t = (x[0] - c[0]).astype(F)
    s = (t * t).astype(F)
    for i in range(1, len(x)):
        t = (x[i] - c[i]).astype(F)
        s = fma32(t, t, s)
    return s


def box_mind(lo, hi, c):
    s = np.zeros_like(c[0], dtype=F)
    for i in range(len(c)):
        g = np.maximum(np.maximum(lo[i] - c[i], c[i] - hi[i]), F(0)).astype(F)
        s = fma32(g, g, s)
    return s


def box_maxd(lo, hi, c):
    s = np.zeros_like(c[0], dtype=F)
    for i in range(len(c)):
        g = np.maximum(np.abs(c[i] - lo[i]), np.abs(hi[i] - c[i])).astype(F)
        s = fma32(g, g, s)
    return s


def err_bound(cmax):
    return (cmax * F(2.0 ** -24) * (F(1.0) + F(2.0 ** -20)) + F(2.0 ** -100)).astype(F)


def dist_hi(s, e, bias=0):
    return (sqrt32(s + TAU, bias) * MARGIN_UP + e).astype(F)


def dist_lo(s, e, bias=0):
    return (sqrt32(np.maximum(s - TAU, F(0)), bias) * MARGIN_DN - e).astype(F)


def lo_inverse(h, e):
    r = ((h + e) * MARGIN_UP * MARGIN_UP).astype(F)
    return (r * r * MARGIN_UP + TAU).astype(F)


def margin_safe(s1, s2, e, bias=0):
    return dist_lo(s2, e, -bias) > dist_hi(s1, e, bias)


def prune_threshold(U, e, bias=0):
    r = ((sqrt32(U + TAU, bias) * MARGIN_UP + F(2.0) * e) * MARGIN_UP * MARGIN_UP).astype(F)
    return (r * r * MARGIN_UP + TAU).astype(F)


def inter_keep(cb_s, s, e, bias=0):
    lhs = dist_lo(cb_s, F(2.0) * e, -bias)
    rhs = ((F(2.0) * dist_hi(s, e, bias)).astype(F) * (F(1.0) + F(2.0 ** -14))).astype(F)
    return lhs > rhs


def d64(x, c):
    """Canonical FP64 squared distance (rounded differences, squares, left-to-right sum)."""
    t = x[0].astype(np.float64) - c[0]
    s = t * t
    for i in range(1, len(x)):
        t = x[i].astype(np.float64) - c[i]
        s = s + t * t
    return s


def cmax_bound(*cs):
    """The FP32 upper bound on max ||c|| the tree kernel computes (norm in FP64,
    inflated by 2^-40, rounded up to FP32)."""
    nrm = np.sqrt(max(np.max(np.sum(np.asarray(c) ** 2, axis=0)) for c in cs)) * (1 + 2.0 ** -40)
    b = np.float32(nrm)
    if float(b) < nrm:
        b = np.nextafter(b, np.float32(np.inf))
    return F(b)


# -------------------------------------------------------------- samples
def _scenario(rng, kind, d, n):
    """x (float32, [d][n]) and two FP64 centroids a, b ([d][n])."""
    if kind == "uniform":
        x = rng.uniform(0, 1, (d, n))
        a = rng.uniform(0, 1, (d, n))
        b = rng.uniform(0, 1, (d, n))
    elif kind == "bisector":
        # x on (or within a few ulps of) the bisector of a and b
        a = rng.uniform(0, 1, (d, n))
        b = a + rng.uniform(-1e-2, 1e-2, (d, n))
        m = 0.5 * (a + b)
        u = rng.standard_normal((d, n))
        nrm = b - a
        u -= nrm * (np.sum(u * nrm, 0) / np.sum(nrm * nrm, 0))
        # signed offsets from the bisector, log-uniform over 1e-10..1e-2 of |b - a|:
        # the margin test's decision boundary lies inside this range
        off = np.exp(rng.uniform(np.log(1e-10), np.log(1e-2), n)) * rng.choice([-1.0, 1.0], n)
        x = m + u * rng.uniform(0, 0.05, n) + nrm * off
    elif kind == "offset":
        base = 1e3 + rng.uniform(0, 1, (d, 1))
        x = base + rng.uniform(0, 1e-2, (d, n))
        a = base + rng.uniform(0, 1e-2, (d, n))
        b = a + rng.uniform(-1e-3, 1e-3, (d, n))
        x = 0.5 * (a + b) + (x - base) * 1e-2
    else:  # tiny
        x = rng.uniform(0, 1e-6, (d, n))
        a = rng.uniform(0, 1e-6, (d, n))
        b = a + rng.uniform(-1e-8, 1e-8, (d, n))
    return x.astype(np.float32), a, b


KINDS = ["uniform", "bisector", "offset", "tiny"]


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("kind", KINDS)
def test_margin_safe_implies_fp64_order(kind, d):
    rng = np.random.default_rng(100 + 7 * d + KINDS.index(kind))
    x, a, b = _scenario(rng, kind, d, N // 4)
    e = err_bound(cmax_bound(a, b))
    ca, cb = a.astype(F), b.astype(F)
    sa, sb = sqdist32(x, ca), sqdist32(x, cb)
    Da, Db = d64(x, a), d64(x, b)
    # the FP32 winner (lowest index on equal values: a is index 0)
    a_wins = sa <= sb
    s1 = np.where(a_wins, sa, sb)
    s2 = np.where(a_wins, sb, sa)
    D1 = np.where(a_wins, Da, Db)
    D2 = np.where(a_wins, Db, Da)
    checked = 0
    for bias in (-1, 0, 1):
        safe = margin_safe(s1, s2, e, bias)
        assert not np.any(safe & (s1 == s2)), "an FP32 tie was declared safe"
        bad = safe & ~(D1 < D2)
        assert not bad.any(), f"{bad.sum()} safe decisions disagree with FP64 ({kind}, d={d})"
        checked += int(safe.sum())
    # the test is only meaningful if many decisions are made both ways
    assert checked > 0
    if kind in ("uniform", "bisector"):
        assert (~margin_safe(s1, s2, e)).sum() > 0


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("kind", KINDS)
def test_pruned_centroid_is_strictly_farther_from_every_box_point(kind, d):
    rng = np.random.default_rng(200 + 7 * d + KINDS.index(kind))
    n = N // 8
    x0, a, b = _scenario(rng, kind, d, n)
    scale = {"uniform": 1e-2, "bisector": 1e-3, "offset": 1e-4, "tiny": 1e-8}[kind]
    ext = rng.uniform(0, scale, (d, n))
    lo = x0.astype(np.float64)
    hi = (lo + ext).astype(np.float32)
    lo = x0
    e = err_bound(cmax_bound(a, b))
    ca, cb = a.astype(F), b.astype(F)
    for bias in (-1, 0, 1):
        U = box_maxd(lo, hi, ca)
        thr = prune_threshold(U, e, bias)
        pruned = box_mind(lo, hi, cb) > thr
        # corners and random interior points of each box
        for trial in range(2 ** d + 4):
            if trial < 2 ** d:
                pick = [(trial >> i) & 1 for i in range(d)]
                xs = np.stack([np.where(pick[i], hi[i], lo[i]) for i in range(d)])
            else:
                w = rng.uniform(0, 1, (d, n))
                xs = (lo + w * (hi.astype(np.float64) - lo)).astype(np.float32)
                xs = np.minimum(np.maximum(xs, lo), hi)
            bad = pruned & ~(d64(xs, b) > d64(xs, a))
            assert not bad.any(), f"{bad.sum()} pruned centroids not strictly farther ({kind}, d={d})"
    assert pruned.sum() > 0 or kind == "tiny"


@pytest.mark.parametrize("kind", KINDS)
def test_recheck_visits_every_possible_winner(kind):
    """The FP64 recheck scans only candidates with s <= lo_inverse(dist_hi(s1));
    any other candidate must be strictly farther in FP64 than the FP32 best."""
    d = 3
    rng = np.random.default_rng(300 + KINDS.index(kind))
    x, a, b = _scenario(rng, kind, d, N // 4)
    e = err_bound(cmax_bound(a, b))
    sa, sb = sqdist32(x, a.astype(F)), sqdist32(x, b.astype(F))
    for bias in (-1, 0, 1):
        cap = lo_inverse(dist_hi(sa, e, bias), e)
        skipped = sb > cap
        bad = skipped & ~(d64(x, b) > d64(x, a))
        assert not bad.any()
        # lo_inverse is a true inverse bound of dist_lo
        h = dist_hi(sa, e, bias)
        assert not np.any((dist_lo(sb, e, -bias) <= h) & (sb > cap))


def test_err_bound_covers_rounding_of_centroids():
    rng = np.random.default_rng(400)
    for scale in (1e-6, 1.0, 1e3, 1e6):
        c = rng.uniform(-scale, scale, (3, N // 4))
        e = err_bound(cmax_bound(c))
        delta = np.sqrt(np.sum((c - c.astype(F).astype(np.float64)) ** 2, 0))
        assert delta.max() <= float(e)


def test_fma32_emulation_is_exact():
    """The emulated fma agrees with exact rational arithmetic."""
    from fractions import Fraction
    rng = np.random.default_rng(500)
    a = rng.standard_normal(3000).astype(F)
    b = rng.standard_normal(3000).astype(F)
    c = (rng.standard_normal(3000) * 10.0 ** rng.integers(-8, 8, 3000)).astype(F)
    # plant exact float32 midpoints: a*b + c lands halfway between two float32
    a[:50] = F(1.0) + F(2.0 ** -12)
    b[:50] = F(1.0) + F(2.0 ** -12)
    c[:50] = F(0.0)
    got = fma32(a, b, c)
    for i in range(3000):
        want = Fraction(float(a[i])) * Fraction(float(b[i])) + Fraction(float(c[i]))
        w32 = np.float32(float(want))  # float(Fraction) is correctly rounded to double
        # double -> float32 can double-round at midpoints: resolve exactly
        cand = [np.nextafter(w32, F(-np.inf)), w32, np.nextafter(w32, F(np.inf))]
        best = min(cand, key=lambda v: (abs(Fraction(float(v)) - want), int(np.float32(v).view(np.uint32)) & 1))
        assert got[i] == best, i


def _near_half(rng, d, n, kind):
    """Owner a, other centroid b, and points x at distance ~ (0.4 .. 0.6) |a - b|
    from a (the keep test's boundary is at one half)."""
    scale = {"uniform": 1.0, "offset": 1.0, "tiny": 1e-6}[kind]
    base = 1e3 if kind == "offset" else 0.0
    a = base + rng.uniform(0, scale, (d, n))
    b = a + rng.uniform(-0.05, 0.05, (d, n)) * scale
    u = rng.standard_normal((d, n))
    u /= np.sqrt(np.sum(u * u, 0))
    r = np.sqrt(np.sum((b - a) ** 2, 0)) * rng.uniform(0.4, 0.6, n)
    x = (a + u * r).astype(np.float32)
    return x, a, b


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("kind", ["uniform", "offset", "tiny"])
def test_inter_keep_point_implies_fp64_order(kind, d):
    rng = np.random.default_rng(600 + 7 * d + ["uniform", "offset", "tiny"].index(kind))
    x, a, b = _near_half(rng, d, N // 4, kind)
    e = err_bound(cmax_bound(a, b))
    ca, cb = a.astype(F), b.astype(F)
    cb_s = sqdist32(ca, cb)
    kept = 0
    for bias in (-1, 0, 1):
        keep = inter_keep(cb_s, sqdist32(x, ca), e, bias)
        bad = keep & ~(d64(x, a) < d64(x, b))
        assert not bad.any(), f"{bad.sum()} kept points not strictly nearer in FP64 ({kind}, d={d})"
        kept += int(keep.sum())
    assert kept > 0 and kept < 3 * x.shape[1]  # both outcomes occur near the boundary


@pytest.mark.parametrize("d", [2, 3])
def test_inter_keep_box_implies_fp64_order(d):
    rng = np.random.default_rng(700 + d)
    n = N // 8
    x0, a, b = _near_half(rng, d, n, "uniform")
    ext = rng.uniform(0, 2e-3, (d, n))
    lo = x0
    hi = (x0.astype(np.float64) + ext).astype(np.float32)
    e = err_bound(cmax_bound(a, b))
    ca, cb = a.astype(F), b.astype(F)
    keep = inter_keep(sqdist32(ca, cb), box_maxd(lo, hi, ca), e)
    assert keep.sum() > 0
    for trial in range(2 ** d + 4):
        if trial < 2 ** d:
            pick = [(trial >> i) & 1 for i in range(d)]
            xs = np.stack([np.where(pick[i], hi[i], lo[i]) for i in range(d)])
        else:
            w = rng.uniform(0, 1, (d, n))
            xs = (lo + w * (hi.astype(np.float64) - lo)).astype(np.float32)
            xs = np.minimum(np.maximum(xs, lo), hi)
        bad = keep & ~(d64(xs, a) < d64(xs, b))
        assert not bad.any(), f"{bad.sum()} kept boxes with a point not strictly nearer to the owner"
