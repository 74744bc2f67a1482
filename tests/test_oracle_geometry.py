"""Pins of the oracle's hierarchy: classification, ordering and ghost geometry.

Every check compares the oracle with something the paper or the mathematics
fixes independently of the oracle's code: invariants of the ghost definition
(section 3.3, eq. ghostdef), exactness of the biquadratic interpolation of
eq. (JssD) on polynomials, the boxed diagonal coefficient of eq. (JssD), the
zero of the interpolated level set at B, the analytic circle, SIGN(0) = +1 and
the CFL condition of eq. (CFLcond).
"""
import itertools

import numpy as np
import pytest

import lsmg_inputs as I


def _idx(g, n, dim):
    out = []
    for _ in range(dim):
        out.append(g % n)
        g //= n
    return tuple(out)


def _types(H, l):
    info = H.level_info(l)
    nn = info["n"] ** H.dim
    t = np.zeros(nn, dtype=int)
    c2g = H.compact_to_grid(l)
    t[c2g[:info["ni"]]] = 1
    t[c2g[info["ni"]:]] = 2
    return t


@pytest.mark.parametrize("kind,n,coarsest", [("disk", 65, 5), ("star", 129, 9)])
def test_classification_invariants(oracle_mod, kind, n, coarsest):
    phi = I.disk(n) if kind == "disk" else I.star(n)
    H = oracle_mod.Hierarchy(phi, 2, n, coarsest_n=coarsest)
    for l in range(H.nlev):
        info = H.level_info(l)
        nl = info["n"]
        t = _types(H, l).reshape(nl, nl)          # [j, i]
        stride = 2 ** l
        phil = phi.reshape(n, n)[::stride, ::stride]
        assert np.array_equal(t == 1, phil < 0), "inside must be exactly phi < 0"
        pad = np.zeros((nl + 2, nl + 2), dtype=bool)
        pad[1:-1, 1:-1] = (t == 1)
        nb_inside = pad[:-2, 1:-1] | pad[2:, 1:-1] | pad[1:-1, :-2] | pad[1:-1, 2:]
        assert np.array_equal(t == 2, (t != 1) & nb_inside), "ghost definition"
        # compact order: inside first, then ghosts, each strictly increasing (lexicographic)
        c2g = H.compact_to_grid(l)
        assert np.all(np.diff(c2g[:info["ni"]]) > 0) and np.all(np.diff(c2g[info["ni"]:]) > 0)


def test_level_counts_disk(oracle_mod):
    # number of lattice points strictly inside the circle of radius 0.4 on each level,
    # counted directly from the coordinates
    H = oracle_mod.Hierarchy(I.disk(65), 2, 65, coarsest_n=5)
    for l in range(H.nlev):
        info = H.level_info(l)
        ax = np.linspace(-1, 1, info["n"])
        X, Y = np.meshgrid(ax, ax)
        assert info["ni"] == int(np.sum(X * X + Y * Y < 0.16))


def _ghost_checks(H, l, polys_exact):
    info = H.level_info(l)
    gt = H.ghost_table(l)
    c2g = H.compact_to_grid(l)
    n, h, dim = info["n"], info["h"], H.dim
    coords = np.stack(I.grid_points(n, dim), axis=1)  # node coordinates
    for q in range(info["ng"]):
        order = gt["order"][q]
        st = gt["st"][q]
        w = gt["w"][q]
        B = gt["B"][q]
        assert abs(w.sum() - 1.0) < 1e-13
        if order == 0:
            continue
        pts = []
        # ST node coordinates: for nonzero weights the node is active (compact index >= 0)
        G = coords[c2g[info["ni"] + q]]
        m = np.where(gt["normal"][q] >= 0, 1, -1)
        for k in range(3 ** dim):
            kk = [(k // 3 ** a) % 3 for a in range(dim)]
            pts.append(G - h * m * np.array(kk))
            if w[k] != 0:
                assert st[k] >= 0, "nonzero weight on an inactive node"
        pts = np.array(pts)
        for p in polys_exact[order]:
            lhs = np.dot(w, p(pts))
            assert abs(lhs - p(B[None, :])[0]) < 1e-11 * (1 + abs(lhs))


def _polys(dim):
    quad = []
    lin = []
    for e in itertools.product(range(3), repeat=dim):
        f = (lambda ee: (lambda P: np.prod([P[:, a] ** ee[a] for a in range(len(ee))], axis=0)))(e)
        quad.append(f)
        if max(e) <= 1:
            lin.append(f)
    return {2: quad, 1: lin}


@pytest.mark.parametrize("kind,n,coarsest", [("disk", 65, 5), ("star", 129, 9)])
def test_ghost_weights_exact_on_polynomials(oracle_mod, kind, n, coarsest):
    phi = I.disk(n) if kind == "disk" else I.star(n)
    H = oracle_mod.Hierarchy(phi, 2, n, coarsest_n=coarsest)
    for l in range(H.nlev):
        _ghost_checks(H, l, _polys(2))


def test_ghost_weights_exact_on_polynomials_3d(oracle_mod):
    H = oracle_mod.Hierarchy(I.torus(33), 3, 33, coarsest_n=9)
    for l in range(H.nlev):
        _ghost_checks(H, l, _polys(3))


def test_ghost_diagonal_coefficient_and_cfl(oracle_mod):
    # boxed coefficient of eq. (JssD): theta_x (1 + theta_x) theta_y (1 + theta_y) / 4 with
    # theta measured from the first inner stencil node; |1 - tau w00| < 1 for tau = 0.9 (eq. CFLcond)
    H = oracle_mod.Hierarchy(I.star(257), 2, 257, coarsest_n=9)
    info = H.level_info(0)
    gt = H.ghost_table(0)
    c2g = H.compact_to_grid(0)
    x, y = I.grid_points(257, 2)
    h = info["h"]
    for q in range(info["ng"]):
        g = c2g[info["ni"] + q]
        m = np.where(gt["normal"][q] >= 0, 1, -1)
        G = np.array([x[g], y[g]])
        th = m * (gt["B"][q] - (G - m * h)) / h
        assert gt["order"][q] == 2
        w00 = th[0] * (1 + th[0]) * th[1] * (1 + th[1]) / 4
        assert abs(gt["w"][q][0] - w00) < 1e-14
        assert 0.0 < w00 <= 1.0 and abs(1 - 0.9 * w00) < 1


def test_boundary_point_on_circle(oracle_mod):
    # B lies on the zero set of the biquadratic interpolant; on the circle of radius 0.4
    # its distance to the true circle is an interpolation error that shrinks at least as h^3
    errs = []
    for n in (65, 129, 257):
        H = oracle_mod.Hierarchy(I.disk(n), 2, n, coarsest_n=5)
        B = H.ghost_table(0)["B"]
        errs.append(np.max(np.abs(np.hypot(B[:, 0], B[:, 1]) - 0.4)))
    assert errs[0] < 1e-4
    assert errs[1] < errs[0] / 6 and errs[2] < errs[1] / 6


def test_normals_and_sign_zero(oracle_mod):
    n = 65
    H = oracle_mod.Hierarchy(I.disk(n), 2, n, coarsest_n=5)
    info = H.level_info(0)
    gt = H.ghost_table(0)
    c2g = H.compact_to_grid(0)
    x, y = I.grid_points(n, 2)
    G = np.stack([x[c2g[info["ni"]:]], y[c2g[info["ni"]:]]], axis=1)
    exact = G / np.linalg.norm(G, axis=1)[:, None]
    assert np.max(np.abs(gt["normal"] - exact)) < 5e-3
    # ghosts on the y axis have n_x = 0 exactly: SIGN(0) = +1 puts the stencil at x_i, x_i - h, x_i - 2h
    on_axis = np.where(G[:, 0] == 0.0)[0]
    assert len(on_axis) == 2
    for q in on_axis:
        assert gt["normal"][q][0] == 0.0
        cg = H.compact_to_grid(0)
        gi = [_idx(cg[s], n, 2) if s >= 0 else None for s in gt["st"][q]]
        g0 = _idx(c2g[info["ni"] + q], n, 2)
        for k in range(9):
            if gt["w"][q][k] != 0:
                assert gi[k][0] == g0[0] - (k % 3)


def test_coarse_levels_use_order_fallback_only_where_needed(oracle_mod):
    H = oracle_mod.Hierarchy(I.star(1025), 2, 1025, coarsest_n=9)
    counts = [np.bincount(H.ghost_table(l)["order"], minlength=3) for l in range(H.nlev)]
    # the finest levels are fully biquadratic
    for l in range(4):
        assert counts[l][2] == H.level_info(l)["ng"]
    assert sum(c[0] + c[1] for c in counts) > 0


def _lag2(k, t):
    # 1-D quadratic Lagrange weight of stencil node k at local coordinate t (nodes k = 0, 1, 2 at
    # t = 1, 0, -1: the ghost, its inner neighbour, the next one)
    return {0: t * (1 + t) / 2, 1: (1 - t) * (1 + t), 2: t * (t - 1) / 2}[k]


def test_negative_ghost_weight_takes_axis_row(oracle_mod):
    # Reading of eq. (CFLcond) outside theta in [0, 1]: where the biquadratic weight of the ghost
    # itself would be negative (possible only if theta leaves [0, 1] on an axis), the 2-D row is
    # taken on a grid line to an inside axis neighbour: B is the zero of the 1-D quadratic
    # interpolant of phi through G and its next two nodes on that line, and the row is that 1-D
    # interpolation, checked here from the level set and B alone.  Everywhere else the biquadratic
    # weights stand.  The domain is a star of the 64-domain batch (seed 0, member 36) whose concave
    # corners produce such ghosts on the 129^2 grid.
    d = I.batch_domains(64, 0)[36]
    n = d["n"]
    phi = I.star(n, **d["shape"])
    H = oracle_mod.Hierarchy(phi, 2, n, coarsest_n=9)
    info = H.level_info(0)
    gt = H.ghost_table(0)
    c2g = H.compact_to_grid(0)
    x, y = I.grid_points(n, 2)
    h = info["h"]
    P = np.stack([x, y], axis=1)
    flipped = 0
    for q in range(info["ng"]):
        g = c2g[info["ni"] + q]
        m = np.where(gt["normal"][q] >= 0, 1, -1)
        G = P[g]
        th = m * (gt["B"][q] - (G - m * h)) / h
        wq = np.array([_lag2(k % 3, th[0]) * _lag2(k // 3, th[1]) for k in range(9)])
        if gt["bfallback"][q] == 2:
            flipped += 1
            assert gt["order"][q] == 2
            # B on a grid line through G: one coordinate moved, by at most h, towards an inside node
            dB = gt["B"][q] - G
            a = int(np.argmax(np.abs(dB)))
            assert dB[1 - a] == 0.0 and 0 < abs(dB[a]) <= h
            step = int(np.sign(dB[a]))
            gi = np.array([g % n, g // n])
            line = [gi.copy() for _ in range(3)]
            for k in range(3):
                line[k][a] += k * step
            f = [phi[v[0] + n * v[1]] for v in line]
            assert f[1] < 0.0
            t = 1.0 - abs(dB[a]) / h
            assert abs(_lag2(0, t) * f[0] + _lag2(1, t) * f[1] + _lag2(2, t) * f[2]) < 1e-12
            # the row: 1-D quadratic weights at t on G, its inside neighbour and the next node
            nodes = c2g[gt["st"][q]]
            expect = {line[k][0] + n * line[k][1]: _lag2(k, t) for k in range(3)}
            got = {}
            for node, wk in zip(nodes, gt["w"][q]):
                if wk != 0.0:
                    got[node] = got.get(node, 0.0) + wk
            assert set(got) <= set(expect)
            for node, wk in expect.items():
                assert abs(got.get(node, 0.0) - wk) < 1e-14
            assert 0.0 < gt["w"][q][0] <= 1.0
        elif gt["order"][q] == 2:
            assert wq[0] >= 0.0
            assert np.max(np.abs(gt["w"][q] - wq)) < 1e-13
    assert flipped == 4
    for l in range(H.nlev):
        g2 = H.ghost_table(l)
        li = H.level_info(l)
        for q in range(li["ng"]):
            own = g2["w"][q][g2["st"][q] == li["ni"] + q].sum()
            assert own >= 0.0 and abs(1 - 0.9 * own) < 1


def test_boundary_point_outside_stencil_takes_constant_rule(oracle_mod):
    # Reading of the case the paper assumes away (no sign change on PG, B from the projection
    # along the gradient landing outside the stencil, theta outside [-1, 2]): the constant rule,
    # on the finest level as on coarse ones.  The domain is request 12 of the seeded serving
    # stream taken as the plain (creased) union of its ellipsoids, whose crease produces such a
    # ghost on the 129^3 grid.
    r = I.serving_requests(24, 1.0, 0)[12]
    n = r["n"]
    H = oracle_mod.Hierarchy(I.ellipsoids(n, r["centres"], r["semi"], smooth=0.0), 3, n, coarsest_n=9)
    info = H.level_info(0)
    gt = H.ghost_table(0)
    c2g = H.compact_to_grid(0)
    x, y, z = I.grid_points(n, 3)
    h = info["h"]
    far = 0
    for q in range(info["ng"]):
        g = c2g[info["ni"] + q]
        m = np.where(gt["normal"][q] >= 0, 1, -1)
        G = np.array([x[g], y[g], z[g]])
        th = m * (gt["B"][q] - (G - m * h)) / h
        if np.any(th < -1.0) or np.any(th > 2.0):
            far += 1
            assert gt["bfallback"][q] == 1
            assert gt["order"][q] == 0
            assert np.array_equal(gt["w"][q], np.eye(27)[0])
    assert far >= 1
