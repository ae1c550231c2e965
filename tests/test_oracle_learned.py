"""Pins for the learned-rule oracle (oracle.learned).

* moments: polygon Legendre moments by the fan rule against the divergence
  theorem (tests.polyexact), on convex and star-shaped training polygons;
* the unit square: moments are 4 delta_{a0} delta_{b0} (orthogonality of the
  Legendre polynomials) and the 4 x 4 Gauss tensor rule matches them exactly;
* network: hand-written backward pass against central finite differences;
* refinement: Jacobian against finite differences; Gauss-Newton from the
  untrained template reaches the 1e-10 acceptance threshold, and from a
  perturbed Gauss rule on the square returns to a zero-residual rule;
* Philox: the generic block function against numpy's independent Philox-4x64
  (same round structure, other word width and constants), and the training
  polygons' recipe (vertex counts, box normalisation, orientation, simplicity).
"""

import numpy as np
import pytest
from numpy.polynomial import legendre as NL

from oracle import learned as L
from tests import polyexact as PE

SEED = 2007048815


def _exact_moments(v):
    out = []
    for a, b in L.EXPS:
        c = np.outer(NL.leg2poly([0] * a + [1]), NL.leg2poly([0] * b + [1]))
        out.append(PE.polygon_integral(v, c))
    return np.array(out)


def test_moment_order_and_count():
    assert L.NMOM == 28
    assert L.EXPS[:6] == [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]


@pytest.mark.parametrize("index", range(12))
def test_polygon_moments_divergence_theorem(index):
    v = L.random_polygon(index, SEED)
    M = L.polygon_moments(v)
    ref = _exact_moments(v)
    assert np.abs(M - ref).max() <= 1e-14 * abs(ref[0])
    assert abs(M[0] - L.polygon_area(v)) <= 1e-14 * abs(M[0])


def test_square_moments_and_gauss_tensor_rule():
    sq = np.array([[-1.0, -1.0], [1.0, -1.0], [1.0, 1.0], [-1.0, 1.0]])
    M = L.polygon_moments(sq)
    ref = np.zeros(L.NMOM)
    ref[0] = 4.0
    assert np.abs(M - ref).max() <= 1e-14
    n, w = L.template_rule(L.polygon_area(sq))
    assert L.residual(n, w, M, 4.0) <= 1e-15
    # a 3 x 3 Gauss rule is exact only to degree 5 per variable: P_6 is missed
    t, wt = np.polynomial.legendre.leggauss(3)
    X, Y = np.meshgrid(t, t, indexing="ij")
    r3 = L.residual(np.stack([X.ravel(), Y.ravel()], 1), np.outer(wt, wt).ravel(), M, 4.0)
    assert r3 > 1e-3


def test_rule_moments_against_direct_sums():
    rng = np.random.default_rng(2)
    n = rng.uniform(-1, 1, (16, 2))
    w = rng.uniform(0, 1, 16)
    Q = L.rule_moments(n, w)
    for m, (a, b) in enumerate(L.EXPS):
        pa = NL.legval(n[:, 0], [0] * a + [1])
        pb = NL.legval(n[:, 1], [0] * b + [1])
        assert abs(Q[m] - np.sum(w * pa * pb)) <= 1e-14 * np.sum(np.abs(w))


def _batch(k):
    polys = [L.random_polygon(i, SEED) for i in range(k)]
    X = np.stack([L.features(v) for v in polys])
    A = np.array([L.polygon_area(v) for v in polys])
    M = np.stack([L.polygon_moments(v) for v in polys])
    return X, M, A


def test_features_layout():
    v = L.random_polygon(5, SEED)
    x = L.features(v)
    m = v.shape[0]
    assert x.shape == (36,)
    assert np.array_equal(x[:2 * m].reshape(m, 2), v)
    assert np.all(x[2 * m:24] == 0.0)
    assert np.array_equal(x[24:], (np.arange(12) < m).astype(float))


def test_backward_matches_finite_differences():
    X, M, A = _batch(6)
    params = L.init_params(1)
    grads = L.backward(params, X, M, A)
    rng = np.random.default_rng(0)
    h = 1e-6
    # central differences: O(h^2) truncation plus a rounding floor of a few ulps of the loss over h
    floor = 1e-15 * L.loss(params, X, M, A) / h
    for k in range(8):
        P = params[k]
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in P.shape)
            old = P[idx]
            P[idx] = old + h
            lp = L.loss(params, X, M, A)
            P[idx] = old - h
            lm = L.loss(params, X, M, A)
            P[idx] = old
            fd = (lp - lm) / (2 * h)
            g = grads[k][idx]
            assert abs(g - fd) <= 1e-7 * abs(fd) + floor, (k, idx, g, fd)


def test_jacobian_matches_finite_differences():
    rng = np.random.default_rng(3)
    n = rng.uniform(-0.9, 0.9, (16, 2))
    w = rng.uniform(0.05, 0.3, 16)
    J = L.jacobian(n, w)
    u = np.concatenate([n.ravel(), w])
    h = 1e-6
    for k in range(48):
        up, um = u.copy(), u.copy()
        up[k] += h
        um[k] -= h
        qp = L.rule_moments(up[:32].reshape(16, 2), up[32:])
        qm = L.rule_moments(um[:32].reshape(16, 2), um[32:])
        assert np.abs(J[:, k] - (qp - qm) / (2 * h)).max() <= 1e-7 * max(1.0, np.abs(J).max())


def test_gauss_newton_recovers_square_rule():
    sq = np.array([[-1.0, -1.0], [1.0, -1.0], [1.0, 1.0], [-1.0, 1.0]])
    M = L.polygon_moments(sq)
    n, w = L.template_rule(4.0)
    rng = np.random.default_rng(5)
    n = n + 0.02 * rng.standard_normal(n.shape)
    w = w * (1 + 0.02 * rng.standard_normal(w.shape))
    assert L.residual(n, w, M, 4.0) > 1e-3
    n, w = L.gauss_newton(n, w, M, iters=6)
    assert L.residual(n, w, M, 4.0) <= 1e-13


@pytest.mark.parametrize("index", [0, 3, 6, 9, 21])
def test_gauss_newton_from_template_is_accepted(index):
    v = L.random_polygon(index, SEED)
    A = L.polygon_area(v)
    M = L.polygon_moments(v)
    n, w = L.template_rule(A)
    n, w = L.gauss_newton(n, w, M, iters=8)
    assert L.residual(n, w, M, A) <= 1e-10
    # an accepted rule integrates every polynomial of degree <= 6 over the polygon
    c = np.zeros((5, 3))
    c[4, 2] = 1.0  # xi^4 eta^2
    c[1, 0] = -2.0
    exact = PE.polygon_integral(v, c)
    got = np.sum(w * (n[:, 0] ** 4 * n[:, 1] ** 2 - 2.0 * n[:, 0]))
    assert abs(got - exact) <= 1e-9 * A


def test_philox_generic_matches_numpy_4x64():
    key = (0x0123456789ABCDEF, 0xFEDCBA9876543210)
    bg = np.random.Philox(counter=np.zeros(4, np.uint64), key=np.array(key, dtype=np.uint64))
    raw = bg.random_raw(12)
    # numpy advances the counter before each block: blocks for counters 1, 2, 3
    for b in range(3):
        got = L.philox((b + 1, 0, 0, 0), key, width=64)
        assert [int(x) for x in raw[4 * b:4 * b + 4]] == list(got)


def test_philox4x32_counter_sensitivity():
    a = L.philox4x32((1, 2, 3, 4), (5, 6))
    assert all(0 <= x < 2 ** 32 for x in a)
    assert L.philox4x32((1, 2, 3, 4), (5, 6)) == a
    for k in range(4):
        ctr = [1, 2, 3, 4]
        ctr[k] ^= 1
        b = L.philox4x32(ctr, (5, 6))
        flips = sum(bin(x ^ y).count("1") for x, y in zip(a, b))
        assert 40 <= flips <= 88  # avalanche: about half of 128 bits change


def _simple(v):
    n = v.shape[0]
    segs = [(v[i], v[(i + 1) % n]) for i in range(n)]

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    for i in range(n):
        for j in range(i + 1, n):
            if j == i + 1 or (i == 0 and j == n - 1):
                continue
            p1, p2 = segs[i]
            q1, q2 = segs[j]
            if (cross(p1, p2, q1) * cross(p1, p2, q2) < 0) and (cross(q1, q2, p1) * cross(q1, q2, p2) < 0):
                return False
    return True


def test_training_polygons_recipe():
    counts = np.zeros(13, int)
    for i in range(300):
        v = L.random_polygon(i, SEED)
        m = v.shape[0]
        counts[m] += 1
        assert 3 <= m <= 12
        assert v.min(0).tolist() == [-1.0, -1.0] and v.max(0).tolist() == [1.0, 1.0]
        assert L.polygon_area(v) > 0.0
        assert v[0, 0] == -1.0
        assert _simple(v)
    assert counts[:3].sum() == 0 and np.all(counts[3:] > 10)
    # reproducible per index, independent of the order of generation
    assert np.array_equal(L.random_polygon(77, SEED), L.random_polygon(77, SEED))


def test_adam_first_step_is_signed_learning_rate():
    """With zero moments, the bias-corrected first step is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(9)
    g = rng.standard_normal(50)
    p0 = rng.standard_normal(50)
    p1, m, v = L.adam_step(p0, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=0.0)
    assert np.allclose(p0 - p1, 0.01 * np.sign(g), rtol=1e-12, atol=0)
    # a constant gradient keeps the step at lr (the corrections cancel the moment decay)
    for t in range(2, 6):
        p1, m, v = L.adam_step(p1, g, m, v, t, lr=0.01, eps=0.0)
    assert np.allclose(p0 - p1, 0.05 * np.sign(g), rtol=1e-10, atol=0)


def test_blob_round_trip():
    params = L.init_params(4)
    blob = L.flatten(params)
    assert blob.size == 43952
    back = L.unflatten(blob)
    assert all(np.array_equal(a, b) for a, b in zip(params, back))


def test_levenberg_marquardt_accepts_from_template_and_perturbed_square():
    for index in (1, 4, 13):
        v = L.random_polygon(index, SEED)
        A = L.polygon_area(v)
        M = L.polygon_moments(v)
        n, w = L.template_rule(A)
        n, w, it, ok = L.levenberg_marquardt(n, w, M, A, max_it=10)
        assert ok and 1 <= it <= 10
        assert L.residual(n, w, M, A) <= 1e-10
    sq = np.array([[-1.0, -1.0], [1.0, -1.0], [1.0, 1.0], [-1.0, 1.0]])
    M = L.polygon_moments(sq)
    n, w = L.template_rule(4.0)
    _, _, it, ok = L.levenberg_marquardt(n, w, M, 4.0)
    assert ok and it == 0  # the Gauss tensor rule is already exact
    rng = np.random.default_rng(11)
    n2 = n + 0.3 * rng.standard_normal(n.shape)  # far from any rule: plain steps overshoot
    n2, w2, it, ok = L.levenberg_marquardt(n2, w * 1.5, M, 4.0, max_it=40)
    assert ok and L.residual(n2, w2, M, 4.0) <= 1e-10
