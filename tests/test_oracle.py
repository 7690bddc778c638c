"""Pins for the FP64 oracle: each test checks it against something the paper
or the mathematics fixes, not against a retyped copy of its own formulas.

* exact summation      -> math.fsum (a correctly rounded library sum) and
                          hand cases with known rounding
* assignment           -> brute force on tiny inputs, hand-built ties,
                          duplicate / far centroids (empty-cluster rule)
* centroid update      -> k=1 global mean, dyadic cluster means, fsum/count
* whole trajectory     -> a hand-worked example (tests/golden), closed forms
                          (k=n, well separated clusters), Lloyd invariants
                          (non-increasing objective, fixed point), and
                          scikit-learn / scipy Lloyd on well separated data
* distortion gradient  -> FP64 central differences and torch autograd
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from synth import gaussian_mixture_2d, init_centroids

GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


# ----------------------------------------------------------------- exact sum
def test_exact_sum_matches_fsum_random():
    rng = np.random.default_rng(1)
    for _ in range(300):
        m = int(rng.integers(1, 200))
        v = rng.standard_normal(m) * 10.0 ** rng.integers(-300, 300, size=m).astype(np.float64)
        if m > 3:
            v[: m // 3] = -v[m // 3: 2 * (m // 3)] * (1 + 2.0 ** -52)  # heavy cancellation
        assert oracle.exact_sum(v) == math.fsum(v)


def test_exact_sum_hand_cases():
    # naive left-to-right summation gives 0 here; the exact answer is 1
    assert oracle.exact_sum([1e16, 1.0, -1e16]) == 1.0
    # 2^53 + 1 is a tie -> even (2^53); a tiny extra term breaks the tie upwards
    assert oracle.exact_sum([2.0 ** 53, 1.0]) == 2.0 ** 53
    assert oracle.exact_sum([2.0 ** 53, 1.0, 2.0 ** -60]) == 2.0 ** 53 + 2
    assert oracle.exact_sum([2.0 ** 53, 3.0]) == 2.0 ** 53 + 4  # 3 -> tie at ...+3 -> even +4
    # subnormals and the largest doubles
    tiny = 5e-324
    assert oracle.exact_sum([tiny] * 7) == 7 * tiny
    assert oracle.exact_sum([1.7e308, 1.7e308, -1.7e308]) == 1.7e308
    assert oracle.exact_sum([]) == 0.0
    assert oracle.exact_sum([-3.0, 1.0]) == -2.0


def test_exact_sum_float32_inputs_order_independent():
    rng = np.random.default_rng(2)
    v = rng.uniform(0, 1, 100_000).astype(np.float32).astype(np.float64)
    s = oracle.exact_sum(v)
    assert s == math.fsum(v)
    assert oracle.exact_sum(v[::-1]) == s
    assert oracle.exact_sum(rng.permutation(v)) == s


# ---------------------------------------------------------------- assignment
def _brute_argmin(x, c):
    """Tiny-input brute force: every distance by hand, first minimum wins."""
    a = []
    for p in x:
        best, bj = None, None
        for j, q in enumerate(c):
            D = 0.0
            for i in range(len(p)):
                t = float(p[i]) - float(q[i])
                D = D + t * t
            if best is None or D < best:
                best, bj = D, j
        a.append(bj)
    return np.array(a)


def test_assign_matches_brute_force_tiny():
    rng = np.random.default_rng(3)
    for d in (2, 3):
        for _ in range(20):
            n, k = int(rng.integers(1, 40)), int(rng.integers(1, 12))
            x = rng.uniform(-1, 1, (n, d))
            c = rng.uniform(-1, 1, (k, d))
            # plant exact ties: some centroids duplicated, some points on a bisector
            if k > 2:
                c[k - 1] = c[0]
            a, dm = oracle.assign(x, c)
            np.testing.assert_array_equal(a, _brute_argmin(x, c))
            # the distance reported is the one to the chosen centroid (3D: all dims used)
            def canon(p, q):
                s = 0.0
                for t in range(d):
                    u = float(p[t]) - float(q[t])
                    s = s + u * u  # each operation rounded once, left to right
                return s
            ref = np.array([canon(x[i], c[a[i]]) for i in range(n)])
            np.testing.assert_array_equal(dm, ref)  # bitwise: the canonical rounding, no FMA


def _fma(a, b, c):
    """fl(a*b + c) with one rounding (exact rational arithmetic)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def test_distance_is_not_contracted_into_fma():
    """Hand cases where fl(fl(dx^2) + fl(dy^2)) and fma(dx, dx, fl(dy^2))
    order two centroids differently: the oracle must take the canonical one."""
    rows = [line.split() for line in open(f"{GOLDEN}/fma_flip_2d.txt")
            if line.strip() and not line.startswith("#")]
    assert len(rows) >= 3
    for r in rows:
        v = [float.fromhex(t) for t in r[:6]]
        x, c1, c2, want = np.array([v[0:2]]), v[2:4], v[4:6], int(r[6])

        def canon(c):
            dx, dy = v[0] - c[0], v[1] - c[1]
            return dx * dx + dy * dy  # Python rounds each operation once

        def fused(c):
            dx, dy = v[0] - c[0], v[1] - c[1]
            return _fma(dx, dx, dy * dy)

        d1, d2 = canon(c1), canon(c2)
        assert want == (0 if d1 <= d2 else 1)                      # the fixture's answer is the canonical one
        assert (0 if fused(c1) <= fused(c2) else 1) != want        # and a contracted distance disagrees
        a, dm = oracle.assign(x, np.array([c1, c2]))
        assert a.tolist() == [want]
        assert dm[0] == (d1 if want == 0 else d2)


def test_assign_tie_goes_to_lowest_index():
    x = np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.0]])
    c = np.array([[0.5, 0.0], [1.5, 0.0]])
    a, _ = oracle.assign(x, c)
    assert a.tolist() == [0, 0, 1]  # point 1 is equidistant -> lower index
    # reversed centroid order: the tie still goes to index 0, now the (1.5,0) centroid
    a, _ = oracle.assign(x, c[::-1])
    assert a.tolist() == [1, 0, 0]


def test_duplicate_and_far_centroids_keep_position():
    x = np.array([[0.0, 0.0], [0.25, 0.0], [0.0, 0.5], [0.75, 0.25]])
    c = np.array([[0.5, 0.5], [9.0, 9.0], [0.5, 0.5]])
    a, _ = oracle.assign(x, c)
    assert a.tolist() == [0, 0, 0, 0]
    cn, cnt = oracle.update(x, a, c)
    assert cnt.tolist() == [4, 0, 0]
    # dyadic mean by hand: (1/4, 3/16)
    assert cn[0].tolist() == [0.25, 0.1875]
    assert cn[1].tolist() == [9.0, 9.0] and cn[2].tolist() == [0.5, 0.5]


def test_assign_3d_uses_every_coordinate():
    # differing only in z: a mistake that drops the last dimension ties them
    x = np.array([[0.0, 0.0, 1.0]])
    c = np.array([[0.0, 0.0, -1.0], [0.0, 0.0, 0.9]])
    assert oracle.assign(x, c)[0].tolist() == [1]


# ------------------------------------------------------------------- update
def test_update_k1_is_global_mean():
    rng = np.random.default_rng(4)
    for d in (2, 3):
        x = rng.standard_normal((1001, d))
        c, cnt = oracle.update(x, np.zeros(1001, np.int32), np.zeros((1, d)))
        assert cnt.tolist() == [1001]
        for t in range(d):
            assert c[0, t] == math.fsum(x[:, t]) / 1001


def test_update_matches_fsum_per_cluster():
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, (5000, 3)).astype(np.float32).astype(np.float64)
    a = rng.integers(0, 37, 5000).astype(np.int32)
    c_prev = rng.standard_normal((40, 3))
    c, cnt = oracle.update(x, a, c_prev)
    for j in range(40):
        sel = x[a == j]
        assert cnt[j] == sel.shape[0]
        if sel.shape[0] == 0:
            assert (c[j] == c_prev[j]).all()
        else:
            for t in range(3):
                assert c[j, t] == math.fsum(sel[:, t]) / sel.shape[0]


# --------------------------------------------------------------- trajectory
def _read_golden(name):
    sec, out = None, {}
    for line in open(f"{GOLDEN}/{name}"):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if ":" not in line and not line[0].isdigit():
            sec = line
            out[sec] = []
            continue
        out[sec].append(line.split(":", 1)[-1].split())
    return out


def test_hand_worked_trajectory():
    g = _read_golden("lloyd_worked_2d.txt")
    x = np.array([[float(v) for v in r] for r in g["points"]])
    c0 = np.array([[float(v) for v in r] for r in g["c0"]])
    res = oracle.lloyd(x, c0, max_iter=20, stop_when_stable=True)
    assert res["iters"] == int(g["iters_until_stable"][0][0])
    for t, row in enumerate(g["assign"]):
        assert res["a_hist"][t].tolist() == [int(v) for v in row]
    for t, row in enumerate(g["centroids"]):
        want = [float(Fraction(v)) for v in row]  # exact rational, rounded once
        assert res["c_hist"][t].ravel().tolist() == want
    for t, row in enumerate(g["sse"]):
        assert res["sse"][t] == pytest.approx(float(Fraction(row[0])), rel=1e-15)


def test_k_equals_n_identity():
    rng = np.random.default_rng(6)
    x = rng.uniform(0, 1, (64, 2))
    perm = rng.permutation(64)
    c0 = x[perm]
    res = oracle.lloyd(x, c0, max_iter=5, stop_when_stable=True)
    inv = np.empty(64, np.int64)
    inv[perm] = np.arange(64)
    assert res["a_hist"][0].tolist() == inv.tolist()
    assert res["sse"][0] == 0.0
    assert res["iters"] == 2  # iteration 2 repeats iteration 1's assignment
    np.testing.assert_array_equal(res["c"], c0)


def test_well_separated_clusters_converge_to_cluster_means():
    rng = np.random.default_rng(7)
    centers = np.array([[0.0, 0.0], [10.0, 0.0], [0.0, 10.0]])
    lab = rng.integers(0, 3, 3000)
    x = centers[lab] + rng.uniform(-1, 1, (3000, 2))
    c0 = x[[int(np.flatnonzero(lab == j)[0]) for j in range(3)]]
    res = oracle.lloyd(x, c0, max_iter=10, stop_when_stable=True)
    assert res["iters"] == 2
    assert (res["a"] == lab).all()
    for j in range(3):
        sel = x[lab == j]
        assert res["c"][j].tolist() == [math.fsum(sel[:, 0]) / len(sel), math.fsum(sel[:, 1]) / len(sel)]


def test_lloyd_invariants_monotone_and_fixed_point():
    x = gaussian_mixture_2d(3000, seed=1000)
    c0 = init_centroids(x, 40, 2000)
    res = oracle.lloyd(x, c0, max_iter=200, stop_when_stable=True)
    sse = res["sse"]
    assert (np.diff(sse) <= 1e-12 * sse[:-1]).all()
    assert res["iters"] < 200
    a_star, _ = oracle.assign(x, res["c"])
    np.testing.assert_array_equal(a_star, res["a"])
    c_star, _ = oracle.update(x, a_star, res["c"])
    np.testing.assert_array_equal(c_star, res["c"])
    # the history ends where the run ends
    np.testing.assert_array_equal(res["a_hist"][-1], res["a"])
    np.testing.assert_array_equal(res["c_hist"][-1], res["c"])


def test_stop_flag_runs_fixed_iterations_otherwise():
    x = gaussian_mixture_2d(500, seed=11)
    c0 = init_centroids(x, 5, 12)
    assert oracle.lloyd(x, c0, max_iter=30, stop_when_stable=False)["iters"] == 30


def test_matches_sklearn_and_scipy_on_separated_data():
    sklearn = pytest.importorskip("sklearn.cluster")
    vq = pytest.importorskip("scipy.cluster.vq")
    rng = np.random.default_rng(8)
    centers = rng.uniform(0, 100, (8, 2))
    lab = rng.integers(0, 8, 4000)
    x = centers[lab] + rng.standard_normal((4000, 2))
    c0 = init_centroids(x, 8, 9)
    res = oracle.lloyd(x, c0, max_iter=50, stop_when_stable=True)
    km = sklearn.KMeans(n_clusters=8, init=c0, n_init=1, algorithm="lloyd", tol=0.0, max_iter=50).fit(x)
    assert (km.labels_ == res["a"]).all()
    np.testing.assert_allclose(km.cluster_centers_, res["c"], rtol=1e-12, atol=1e-12)
    cent, lab2 = vq.kmeans2(x, c0.copy(), iter=50, minit="matrix")
    assert (lab2 == res["a"]).all()
    np.testing.assert_allclose(cent, res["c"], rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- distortion
def _distortion_case(seed=10, B=2, n=300, k=7, d=3):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (B, n, d))
    c = rng.uniform(0, 1, (B, k, d))
    return x, c


def test_distortion_fwd_hand_case():
    x = np.array([[[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [3.0, 0.0, 4.0]]])
    c = np.array([[[0.0, 0.0, 1.0], [3.0, 0.0, 3.0]]])
    a, loss = oracle.distortion_fwd(x, c)
    assert a.tolist() == [[0, 0, 1]]
    assert loss.tolist() == [1.0 + 2.0 + 1.0]


def test_distortion_grad_vs_autograd():
    torch = pytest.importorskip("torch")
    x, c = _distortion_case()
    a, loss = oracle.distortion_fwd(x, c)
    g = np.array([0.7, -1.3])
    gx, gc = oracle.distortion_bwd(x, c, a, g)
    xt = torch.tensor(x, requires_grad=True)
    ct = torch.tensor(c, requires_grad=True)
    at = torch.tensor(a, dtype=torch.long)
    sel = torch.gather(ct, 1, at[..., None].expand(-1, -1, 3))
    L = ((xt - sel) ** 2).sum(dim=(1, 2))
    np.testing.assert_allclose(L.detach().numpy(), loss, rtol=1e-14)
    (L * torch.tensor(g)).sum().backward()
    np.testing.assert_allclose(gx, xt.grad.numpy(), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(gc, ct.grad.numpy(), rtol=1e-12, atol=1e-13)


def test_distortion_grad_central_differences():
    x, c = _distortion_case(seed=12, B=1, n=200, k=6)
    a, loss = oracle.distortion_fwd(x, c)
    gx, gc = oracle.distortion_bwd(x, c, a, np.array([1.0]))
    h = 1e-6
    rng = np.random.default_rng(13)
    checked = 0
    for _ in range(60):
        which = rng.integers(2)
        arr = x if which == 0 else c
        idx = tuple(int(rng.integers(s)) for s in arr.shape)
        p, m = arr.copy(), arr.copy()
        p[idx] += h
        m[idx] -= h
        xp, cp = (p, c) if which == 0 else (x, p)
        xm, cm = (m, c) if which == 0 else (x, m)
        ap, lp = oracle.distortion_fwd(xp, cp)
        am, lm = oracle.distortion_fwd(xm, cm)
        if (ap != a).any() or (am != a).any():
            continue  # crossed a Voronoi boundary: the loss is not one quadratic there
        fd = (lp[0] - lm[0]) / (2 * h)
        an = (gx if which == 0 else gc)[idx]
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))
        checked += 1
    assert checked > 40
