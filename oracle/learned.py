"""Oracle for the learned quadrature rule -- TEST INFRASTRUCTURE (plain numpy, FP64).

What is checked here is the reduced-quadrature part of the path: a small
network maps a polygon, normalised to [-1, 1]^2 by its bounding box (the box of
the element's basis, Section 3.1), to a 16-node rule; Gauss-Newton steps fit the
rule to the polygon's Legendre moments of total degree <= 6; the rule is
accepted if the moment residual is <= 1e-10, otherwise the element keeps the
sub-triangulation rule (Section 3).  The paper itself has no such component;
these readings are documented beside the code:

* moments M_ab = int_P P_a(xi) P_b(eta), a + b <= 6 (28, total degree order,
  a descending), computed by the degree-6 triangle rule on the fan from the
  first vertex (signed triangle areas, so star-shaped polygons are exact);
* rule moments Q_ab = sum_k w_k P_a(xi_k) P_b(eta_k); residual
  r = max_ab |Q_ab - M_ab| / |P|;
* network: inputs 24 vertex coordinates (zero padded) and a 12-entry validity
  mask; three hidden layers of 128 with SiLU; 48 outputs: nodes = tanh(z_0..31)
  as 16 (xi, eta) pairs, weights = |P| softmax(z_32..47);
* training loss (unsupervised): mean over polygons of sum_ab (Q_ab - M_ab)^2 / |P|^2;
* refinement: u = (nodes, weights), J = dQ/du (28 x 48), minimum-norm damped
  step du = -J^T (J J^T + lam I)^-1 (Q - M);
* training polygons: counter-based Philox4x32-10 draws (Salmon, Moraes, Dror,
  Shaw, SC'11), a rejection-free recipe (see random_polygon).
"""

import numpy as np

from . import rules as _rules

NNODE = 16
MAXV = 12
NIN = 2 * MAXV + MAXV
NHID = 128
NOUT = 3 * NNODE
DEG = 6
EXPS = [(a, k - a) for k in range(DEG + 1) for a in range(k, -1, -1)]  # 28 moments
NMOM = len(EXPS)


# ------------------------------------------------------------ Legendre moments
def legendre_table(x, n=DEG):
    """P_0..P_n at x (any shape) by the explicit power-form coefficients."""
    out = []
    for k in range(n + 1):
        c = np.polynomial.legendre.leg2poly([0] * k + [1])
        out.append(np.polynomial.polynomial.polyval(x, c))
    return np.stack(out, -1)


def rule_moments(nodes, w):
    """Q_ab = sum_k w_k P_a(xi_k) P_b(eta_k); nodes [..., K, 2], w [..., K]."""
    Lx = legendre_table(nodes[..., 0])
    Ly = legendre_table(nodes[..., 1])
    return np.stack([np.sum(w * Lx[..., a] * Ly[..., b], -1) for a, b in EXPS], -1)


def polygon_area(v):
    x, y = v[:, 0], v[:, 1]
    return 0.5 * np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y)


def polygon_moments(v):
    """M_ab over the polygon v [m, 2] by the degree-6 rule on the fan from v[0]."""
    bary, wr = _rules.triangle_rule(6)
    M = np.zeros(NMOM)
    for t in range(1, v.shape[0] - 1):
        T = np.stack([v[0], v[t], v[t + 1]])
        area = 0.5 * ((T[1, 0] - T[0, 0]) * (T[2, 1] - T[0, 1]) - (T[2, 0] - T[0, 0]) * (T[1, 1] - T[0, 1]))
        M += rule_moments(bary @ T, wr * area)
    return M


def normalise(xy):
    """Bounding-box map to [-1, 1]^2, counter-clockwise, starting at min x (then min y)."""
    lo, hi = xy.min(0), xy.max(0)
    # ((x - lo) - (hi - x)) / (hi - lo): the extreme vertices land on -1 and 1 exactly
    out = np.clip(((xy - lo) - (hi - xy)) / (hi - lo), -1.0, 1.0)
    if polygon_area(out) < 0:
        out = out[::-1]
    k = np.lexsort((out[:, 1], out[:, 0]))[0]
    return np.roll(out, -k, axis=0)


def features(v):
    """Network input: 24 zero-padded coordinates and a 12-entry mask."""
    m = v.shape[0]
    x = np.zeros(NIN)
    x[:2 * m] = v.reshape(-1)
    x[2 * MAXV:2 * MAXV + m] = 1.0
    return x


def residual(nodes, w, M, area):
    return np.max(np.abs(rule_moments(nodes, w) - M)) / abs(area)


# -------------------------------------------------------------------- network
def init_params(seed):
    rng = np.random.default_rng(seed)
    dims = [NIN, NHID, NHID, NHID, NOUT]
    params = []
    for i in range(4):
        fan_in = dims[i]
        W = rng.normal(0.0, np.sqrt(1.0 / fan_in), size=(dims[i], dims[i + 1]))
        b = np.zeros(dims[i + 1])
        params += [W, b]
    return params


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, X, area):
    """X [B, 36], area [B] -> nodes [B, 16, 2], w [B, 16], cache."""
    h = X
    zs, hs = [], [X]
    for l in range(3):
        z = h @ params[2 * l] + params[2 * l + 1]
        zs.append(z)
        h = silu(z)
        hs.append(h)
    out = h @ params[6] + params[7]
    nodes = np.tanh(out[:, :2 * NNODE]).reshape(-1, NNODE, 2)
    s = out[:, 2 * NNODE:]
    e = np.exp(s - s.max(1, keepdims=True))
    sm = e / e.sum(1, keepdims=True)
    w = area[:, None] * sm
    return nodes, w, (zs, hs, out, sm)


def loss(params, X, M, area):
    nodes, w, _ = forward(params, X, area)
    Q = rule_moments(nodes, w)
    return np.mean(np.sum((Q - M) ** 2, 1) / area ** 2)


def backward(params, X, M, area):
    """Gradients of loss() with respect to every parameter (manual chain rule)."""
    B = X.shape[0]
    nodes, w, (zs, hs, out, sm) = forward(params, X, area)
    Lx = legendre_table(nodes[..., 0])
    Ly = legendre_table(nodes[..., 1])
    dLx = np.stack([np.polynomial.polynomial.polyval(nodes[..., 0],
                                                     np.polynomial.polynomial.polyder(
                                                         np.polynomial.legendre.leg2poly([0] * k + [1])))
                    if k > 0 else np.zeros_like(nodes[..., 0]) for k in range(DEG + 1)], -1)
    dLy = np.stack([np.polynomial.polynomial.polyval(nodes[..., 1],
                                                     np.polynomial.polynomial.polyder(
                                                         np.polynomial.legendre.leg2poly([0] * k + [1])))
                    if k > 0 else np.zeros_like(nodes[..., 1]) for k in range(DEG + 1)], -1)
    Q = np.stack([np.sum(w * Lx[..., a] * Ly[..., b], -1) for a, b in EXPS], -1)
    g = 2.0 * (Q - M) / (area[:, None] ** 2) / B  # dL/dQ [B, 28]
    dw = np.zeros_like(w)
    dx = np.zeros_like(w)
    dy = np.zeros_like(w)
    for m, (a, b) in enumerate(EXPS):
        gm = g[:, m:m + 1]
        dw += gm * Lx[..., a] * Ly[..., b]
        dx += gm * w * dLx[..., a] * Ly[..., b]
        dy += gm * w * Lx[..., a] * dLy[..., b]
    # through w = area * softmax(s)
    dsm = dw * area[:, None]
    ds = sm * (dsm - np.sum(dsm * sm, 1, keepdims=True))
    # through nodes = tanh(t)
    dn = np.stack([dx, dy], -1).reshape(B, 2 * NNODE)
    dt = dn * (1.0 - np.tanh(out[:, :2 * NNODE]) ** 2)
    dout = np.concatenate([dt, ds], 1)
    grads = [None] * 8
    grads[6] = hs[3].T @ dout
    grads[7] = dout.sum(0)
    dh = dout @ params[6].T
    for l in (2, 1, 0):
        dz = dh * dsilu(zs[l])
        grads[2 * l] = hs[l].T @ dz
        grads[2 * l + 1] = dz.sum(0)
        dh = dz @ params[2 * l].T
    return grads


def flatten(params):
    """Parameter blob: W1, b1, W2, b2, W3, b3, W4, b4, each row-major ([in][out] for weights)."""
    return np.concatenate([p.ravel() for p in params])


def unflatten(blob):
    dims = [NIN, NHID, NHID, NHID, NOUT]
    out, o = [], 0
    for i in range(4):
        n = dims[i] * dims[i + 1]
        out.append(np.asarray(blob[o:o + n], dtype=np.float64).reshape(dims[i], dims[i + 1]))
        o += n
        out.append(np.asarray(blob[o:o + dims[i + 1]], dtype=np.float64))
        o += dims[i + 1]
    return out


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, ICLR 2015) with bias correction; returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- refinement
def jacobian(nodes, w):
    """J [28, 48] of Q with respect to (xi_1, eta_1, ..., xi_16, eta_16, w_1..w_16)."""
    K = nodes.shape[0]
    Lx, Ly = legendre_table(nodes[:, 0]), legendre_table(nodes[:, 1])
    der = lambda x, k: (np.polynomial.polynomial.polyval(
        x, np.polynomial.polynomial.polyder(np.polynomial.legendre.leg2poly([0] * k + [1]))) if k > 0 else 0.0 * x)
    J = np.zeros((NMOM, 3 * K))
    for m, (a, b) in enumerate(EXPS):
        J[m, 0:2 * K:2] = w * der(nodes[:, 0], a) * Ly[:, b]
        J[m, 1:2 * K:2] = w * Lx[:, a] * der(nodes[:, 1], b)
        J[m, 2 * K:] = Lx[:, a] * Ly[:, b]
    return J


def gauss_newton(nodes, w, M, iters=4, lam=1e-12):
    """Minimum-norm damped Gauss-Newton on the 28 moment equations."""
    nodes, w = nodes.copy(), w.copy()
    for _ in range(iters):
        r = rule_moments(nodes, w) - M
        J = jacobian(nodes, w)
        du = -J.T @ np.linalg.solve(J @ J.T + lam * np.eye(NMOM), r)
        nodes = nodes + du[:2 * NNODE].reshape(NNODE, 2)
        w = w + du[2 * NNODE:]
    return nodes, w


def levenberg_marquardt(nodes, w, M, area, max_it=8, tol=1e-10, mu0=1e-6):
    """Damped minimum-norm Gauss-Newton (Levenberg-Marquardt) on the moment equations.

    Step du = -J^T (J J^T + mu g I)^{-1} r with g = max diag(J J^T); a step is
    taken only if it lowers ||r||_2 (then mu /= 10, floor 1e-15), otherwise mu
    is multiplied by 10 and the step recomputed (giving up above mu = 1e6).
    Stops when max|r| / area <= tol (accepted) or after max_it steps.
    Returns nodes, weights, steps taken, accepted."""
    u = np.concatenate([nodes.ravel(), w])
    res = lambda u: rule_moments(u[:2 * NNODE].reshape(NNODE, 2), u[2 * NNODE:]) - M
    r = res(u)
    mu = mu0
    it = 0
    while True:
        if np.max(np.abs(r)) / abs(area) <= tol:
            return u[:2 * NNODE].reshape(NNODE, 2), u[2 * NNODE:], it, True
        if it >= max_it:
            break
        J = jacobian(u[:2 * NNODE].reshape(NNODE, 2), u[2 * NNODE:])
        G = J @ J.T
        g = np.max(np.diag(G))
        taken = False
        while mu <= 1e6:
            du = -J.T @ np.linalg.solve(G + mu * g * np.eye(NMOM), r)
            rt = res(u + du)
            if rt @ rt < r @ r:
                u, r = u + du, rt
                mu = max(mu / 10.0, 1e-15)
                taken = True
                break
            mu *= 10.0
        if not taken:
            break
        it += 1
    return u[:2 * NNODE].reshape(NNODE, 2), u[2 * NNODE:], it, False


def template_rule(area):
    """Untrained initial guess: the 4 x 4 Gauss tensor rule on [-1, 1]^2, weights scaled to the area."""
    t, wt = np.polynomial.legendre.leggauss(4)
    X, Y = np.meshgrid(t, t, indexing="ij")
    W = np.outer(wt, wt)
    return np.stack([X.ravel(), Y.ravel()], 1), W.ravel() * area / 4.0


# ------------------------------------------------------------ Philox
# Philox-4xW-R (Salmon et al., SC'11): each round multiplies words 0 and 2 by
# the round multipliers, takes the high and low halves of the products, and
# mixes the high halves with words 1 and 3 and the round key; the key is bumped
# by the Weyl constants after every round.
PHILOX_CONST = {
    32: dict(mul=(0xD2511F53, 0xCD9E8D57), weyl=(0x9E3779B9, 0xBB67AE85)),
    64: dict(mul=(0xD2E7470EE14C6C93, 0xCA5A826395121157), weyl=(0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)),
}


def philox(ctr, key, width=32, rounds=10):
    """Philox-4x`width`-`rounds` block function (pure-Python integers)."""
    mask = (1 << width) - 1
    m0, m1 = PHILOX_CONST[width]["mul"]
    w0, w1 = PHILOX_CONST[width]["weyl"]
    c0, c1, c2, c3 = [int(x) & mask for x in ctr]
    k0, k1 = int(key[0]) & mask, int(key[1]) & mask
    for _ in range(rounds):
        p0, p1 = m0 * c0, m1 * c2
        c0, c1, c2, c3 = ((p1 >> width) ^ c1 ^ k0) & mask, p1 & mask, ((p0 >> width) ^ c3 ^ k1) & mask, p0 & mask
        k0, k1 = (k0 + w0) & mask, (k1 + w1) & mask
    return c0, c1, c2, c3


def philox4x32(ctr, key):
    return philox(ctr, key, 32, 10)


def uniform24(u):
    """[0, 1) with 24 random bits, exact in every floating-point format used."""
    return (u >> 8) * (1.0 / 16777216.0)


def random_polygon(index, seed):
    """Training polygon `index`: Philox4x32-10 with key (seed low, seed high),
    counter (index, j, 0, 0) for draw j.  Draw 0 gives the vertex count m in
    3..12, the kind (convex or star), the ellipse aspect and a rotation; draw
    j >= 1 gives the angle and radius of vertex j-1.  Angles are stratified,
    theta_k = 2 pi (k + 0.1 + 0.8 u_k) / m + rotation, so the vertex list is
    already sorted and no draw is rejected."""
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    u = philox4x32((index, 0, 0, 0), key)
    m = 3 + int(uniform24(u[0]) * 10)
    convex = uniform24(u[1]) < 0.5
    aspect = 0.3 + 0.7 * uniform24(u[2])
    rot = 2.0 * np.pi * uniform24(u[3])
    pts = np.zeros((m, 2))
    for k in range(m):
        d = philox4x32((index, k + 1, 0, 0), key)
        th = 2.0 * np.pi * (k + 0.1 + 0.8 * uniform24(d[0])) / m + rot
        if convex:
            pts[k] = (np.cos(th), aspect * np.sin(th))
        else:
            r = 0.35 + 0.65 * uniform24(d[1])
            pts[k] = (r * np.cos(th), r * np.sin(th))
    return normalise(pts)
