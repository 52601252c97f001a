"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(brute force, closed forms, invariants, special cases), never against itself."""
import json
import os

import numpy as np
import pytest

from oracle import Oracle, OracleParams
from paper_2509_20012_amd import metrics
from paper_2509_20012_amd import phantom as ph
from tests.helpers import dense, from_dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

SHAPES = [(1, 1, 1.0), (7, 3, 0.5), (48, 12, 0.3), (64, 16, 0.2), (33, 5, 0.6)]


def _x(C, seed, lo=0.2, hi=2.0):
    return np.random.default_rng(seed).uniform(lo, hi, C)


# --- products against dense brute force (Section 2.2: additive numerator and
# denominator of Eq. 1, so d = D x and l = L x) ----------------------------------

@pytest.mark.parametrize("R,C,dens", SHAPES)
def test_forward_and_transposed_dense(R, C, dens):
    p = ph.tiny_problem(R, C, dens, seed=R * 31 + C)
    o = Oracle(p)
    D, L = dense(p)
    x = _x(C, 1)
    d, l = o.forward(x)
    np.testing.assert_allclose(d, D @ x, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(l, L @ x, rtol=1e-14, atol=1e-15)
    u1 = np.random.default_rng(2).normal(size=R)
    u2 = np.random.default_rng(3).normal(size=R)
    t = o.transposed(u1, u2)
    np.testing.assert_allclose(t, D.T @ u1 + L.T @ u2, rtol=1e-12, atol=1e-13)
    rows = np.arange(R)[::2]
    dr, lr = o.forward_rows(x, rows)
    np.testing.assert_array_equal(dr, d[rows])
    np.testing.assert_array_equal(lr, l[rows])


def test_empty_rows_and_columns():
    p = ph.tiny_problem(20, 6, 0.4, seed=5, empty_rows=[0, 7, 19], empty_cols=[2])
    o = Oracle(p)
    D, L = dense(p)
    x = _x(6, 4)
    d, l, letd, cdl = o.dose_let(x)
    for i in (0, 7, 19):
        assert d[i] == 0.0 and l[i] == 0.0 and letd[i] == 0.0
    t = o.transposed(np.ones(20), np.ones(20))
    assert t[2] == 0.0
    np.testing.assert_allclose(t, D.sum(0) + L.sum(0), rtol=1e-13)


def test_scipy_crosscheck():
    sp = pytest.importorskip("scipy.sparse")
    p = ph.tiny_problem(64, 16, 0.25, seed=9)
    A = sp.csr_matrix((p.d_val.astype(np.float64), p.col_idx, p.row_ptr), shape=(64, 16))
    x = _x(16, 5)
    d, _ = Oracle(p).forward(x)
    np.testing.assert_allclose(d, A @ x, rtol=1e-14)


def test_linearity():
    p = ph.tiny_problem(48, 12, 0.3, seed=11)
    o = Oracle(p)
    x1, x2 = _x(12, 1), _x(12, 2)
    a, b = 0.75, -1.5
    d12, l12 = o.forward(a * x1 + b * x2)
    d1, l1 = o.forward(x1)
    d2, l2 = o.forward(x2)
    np.testing.assert_allclose(d12, a * d1 + b * d2, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(l12, a * l1 + b * l2, rtol=1e-13, atol=1e-13)


def test_letd_convex_combination_bound():
    """LETd_i is a dose-weighted mean of LET_ij = L_ij / D_ij over contributing
    beamlets, so it lies between their min and max (Eq. 1)."""
    p = ph.tiny_problem(64, 16, 0.3, seed=13)
    o = Oracle(p)
    x = _x(16, 6)
    x[::3] = 0.0
    d, l, letd, cdl = o.dose_let(x)
    for i in range(p.n_rows):
        sl = slice(p.row_ptr[i], p.row_ptr[i + 1])
        cols = p.col_idx[sl]
        act = x[cols] > 0
        if not act.any():
            assert letd[i] == 0.0
            continue
        let = (p.l_val[sl].astype(np.float64) / p.d_val[sl].astype(np.float64))[act]
        assert let.min() * (1 - 1e-15) <= letd[i] <= let.max() * (1 + 1e-15)
    np.testing.assert_array_equal(cdl, p.c * l)


def test_constant_let_special_case():
    """L = LET0 * D gives LETd = LET0 wherever dose > 0; a LETd row with bound T is
    violated exactly when LET0 > T."""
    p = ph.tiny_problem(40, 10, 0.3, seed=17, let_range=(3.0, 3.0))
    o = Oracle(p)
    d, l, letd, _ = o.dose_let(_x(10, 7))
    np.testing.assert_allclose(letd[d > 0], 3.0, rtol=2e-7)  # FP32 storage of L = 3 D
    for T, expect in ((2.5, True), (3.5, False)):
        prob = p.problem_arrays()
        prob = {k: v.copy() for k, v in prob.items()}
        prob["kind"][:] = ph.LETD_HI
        prob["letd_max"][:] = T
        _, nv = Oracle(p, problem=prob).proximity(_x(10, 7))
        assert (nv == p.n_rows) if expect else (nv == 0)


# --- projections (Fig. 2) -----------------------------------------------------------

def _single_row_problem(kind, bound, let=(1.0, 4.0), T=None):
    """Three beamlets, two rows; only row 0 carries constraint `kind`."""
    D = np.array([[0.5, 1.0, 0.25], [0.3, 0.0, 0.6]], np.float32)
    L = D * np.array([[let[0], let[1], 2.0], [1.0, 1.0, 1.0]], np.float32)
    prob = dict(kind=[kind, 0], dose_lo=[0, 0], dose_hi=[0, 0], cdl_lo=[0, 0], cdl_hi=[0, 0],
                letd_max=[0, 0], w_feas=[1, 1])
    key = {ph.DOSE_LO: "dose_lo", ph.DOSE_HI: "dose_hi", ph.CDL_LO: "cdl_lo",
           ph.CDL_HI: "cdl_hi", ph.LETD_HI: "letd_max"}[kind]
    prob[key] = [bound if T is None else T, 0]
    return from_dense(D, L, **prob)


@pytest.mark.parametrize("kind,bound,T", [
    (ph.DOSE_HI, 2.0, None), (ph.DOSE_LO, 8.0, None),
    (ph.CDL_HI, 0.2, None), (ph.CDL_LO, 0.9, None), (ph.LETD_HI, None, 2.0)])
def test_projection_lands_on_hyperplane(kind, bound, T):
    """With lambda = w = 1 a single violated half-space is projected onto exactly:
    the new point satisfies <a, x+> = b and x+ - x is parallel to a.  This also pins
    the sign of the lower-bound step (garbled in Fig. 2): it must move toward the
    half-space."""
    p = _single_row_problem(kind, bound, T=T)
    o = Oracle(p)
    D, L = dense(p)
    c = p.c
    a = {ph.DOSE_HI: D[0], ph.DOSE_LO: D[0], ph.CDL_HI: c * L[0], ph.CDL_LO: c * L[0],
         ph.LETD_HI: L[0] - (T or 0.0) * D[0]}[kind]
    b = 0.0 if kind == ph.LETD_HI else float(np.float32(bound))
    x = np.array([3.0, 2.0, 4.0])
    assert (a @ x > b) if kind in (ph.DOSE_HI, ph.CDL_HI, ph.LETD_HI) else (a @ x < b)
    for norm in (1, 2):  # convex over violated (single row) and raw: same weight 1
        xn, prox, nv = o.ams_simultaneous(x, lam=1.0, weight_scale=1.0, normalization=norm)
        assert nv == 1 and np.all(xn > 0)
        assert a @ xn == pytest.approx(b, rel=1e-14, abs=1e-14)
        step = xn - x
        cosang = abs(step @ a) / (np.linalg.norm(step) * np.linalg.norm(a))
        assert cosang == pytest.approx(1.0, abs=1e-13)
        xs = o.ams_sequential(x, [0, 1], [0, 1], lam=1.0, weight_scale=1.0)
        np.testing.assert_allclose(xs, xn, rtol=1e-14, atol=1e-15)
    # relaxation lambda moves lambda times as far
    xh, _, _ = o.ams_simultaneous(x, lam=0.5, weight_scale=1.0, normalization=2)
    np.testing.assert_allclose(xh - x, 0.5 * (xn - x), rtol=1e-12, atol=1e-15)


def test_orthogonal_rows_simultaneous_equals_sequential():
    """Rows with disjoint beamlet supports do not interact: with raw weights the
    simultaneous and sequential sweeps coincide and every violated row lands on its
    hyperplane."""
    rng = np.random.default_rng(21)
    R, per = 6, 3
    C = R * per
    D = np.zeros((R, C), np.float32)
    for i in range(R):
        D[i, i * per:(i + 1) * per] = rng.uniform(0.2, 1.0, per)
    L = (D * 2.0).astype(np.float32)
    x = rng.uniform(1.0, 2.0, C)
    d0 = D.astype(np.float64) @ x
    kind = [ph.DOSE_HI, ph.DOSE_LO, ph.DOSE_HI | ph.DOSE_LO, ph.CDL_HI, ph.CDL_LO, ph.DOSE_HI]
    dose_hi = [0.8 * d0[0], 0, 1.1 * d0[2], 0, 0, 1.2 * d0[5]]
    dose_lo = [0, 1.2 * d0[1], 0.5 * d0[2], 0, 0, 0]
    cdl_hi = [0, 0, 0, 0.9 * ph.C_DL * 2 * d0[3], 0, 0]
    cdl_lo = [0, 0, 0, 0, 1.1 * ph.C_DL * 2 * d0[4], 0]
    p = from_dense(D, L, kind=kind, dose_hi=dose_hi, dose_lo=dose_lo, cdl_hi=cdl_hi,
                   cdl_lo=cdl_lo, w_feas=np.ones(R))
    o = Oracle(p)
    xs = o.ams_sequential(x, range(R), range(R), lam=1.0, weight_scale=1.0)
    xn, _, nv = o.ams_simultaneous(x, lam=1.0, weight_scale=1.0, normalization=2)
    assert nv == 4
    np.testing.assert_allclose(xn, xs, rtol=1e-14, atol=1e-15)
    Dd, Ld = dense(p)
    assert Dd[0] @ xn == pytest.approx(float(p.dose_hi[0]), rel=1e-14)
    assert Dd[1] @ xn == pytest.approx(float(p.dose_lo[1]), rel=1e-14)
    assert p.c * Ld[3] @ xn == pytest.approx(float(p.cdl_hi[3]), rel=1e-14)
    assert p.c * Ld[4] @ xn == pytest.approx(float(p.cdl_lo[4]), rel=1e-14)
    np.testing.assert_array_equal(xn[2 * per:3 * per], x[2 * per:3 * per])  # satisfied row


def test_sequential_hand_worked_example():
    """Fig. 2 on a 2 x 2 case worked by hand (tests/golden/ams_sequential_2x2.json)."""
    with open(os.path.join(GOLDEN, "ams_sequential_2x2.json")) as f:
        g = json.load(f)
    p = from_dense(g["D"], g["L"], c=g["c"], **g["problem"])
    o = Oracle(p)
    xs = o.ams_sequential(g["x"], g["dose_order"], g["cdl_order"], lam=g["lambda"],
                          weight_scale=1.0)
    np.testing.assert_allclose(xs, g["expected_sequential"], rtol=1e-12)
    xn, _, _ = o.ams_simultaneous(g["x"], lam=g["lambda"], weight_scale=1.0, normalization=2)
    np.testing.assert_allclose(xn, g["expected_simultaneous_raw"], rtol=1e-12)


NORMS = {"convex_all": 0, "convex_violated": 1, "raw": 2}


def _golden_simultaneous():
    with open(os.path.join(GOLDEN, "ams_simultaneous_2x2.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("case", [0, 1])
def test_simultaneous_hand_worked_weights(case):
    """The simultaneous sweep's weight totals and its proximity on 2 x 2 cases worked
    by hand (tests/golden/ams_simultaneous_2x2.json): the total over every enabled
    (row, kind) pair for the default normalisation, over the violated pairs for the
    alternative, and the factor 1/2 of the proximity.  The second case has a
    satisfied row, so the two totals differ."""
    g = _golden_simultaneous()
    c = g["cases"][case]
    p = from_dense(g["D"], g["L"], c=g["c"], w_feas=c["w_feas"], **g["problem"])
    o = Oracle(p)
    for name, norm in NORMS.items():
        xn, prox, nv = o.ams_simultaneous(c["x"], lam=c["lambda"],
                                          weight_scale=c["weight_scale"], normalization=norm)
        np.testing.assert_allclose(xn, c["expected"][name], rtol=1e-14, atol=1e-15)
        assert nv == c["n_violated"]
        assert prox == pytest.approx(c["proximity"], rel=1e-14)
    prox, nv = o.proximity(c["x"])
    assert prox == pytest.approx(c["proximity"], rel=1e-14) and nv == c["n_violated"]


def test_clamp_is_applied():
    D = np.array([[1.0, 1.0]], np.float32)
    p = from_dense(D, D, kind=[ph.DOSE_HI], dose_hi=[0.0], w_feas=[1.0])
    xn, _, _ = Oracle(p).ams_simultaneous(np.array([2.0, 0.1]), normalization=2)
    # unclamped projection onto d <= 0 would be [0.95, -0.95]
    np.testing.assert_allclose(xn, [0.95, 0.0], rtol=1e-14)


def test_feasible_point_is_fixed():
    p = ph.tiny_problem(48, 12, 0.3, seed=23)
    prob = {k: v.copy() for k, v in p.problem_arrays().items()}
    prob["dose_lo"][:] = 0.0
    prob["dose_hi"][:] = 1e6
    prob["cdl_lo"][:] = 0.0
    prob["cdl_hi"][:] = 1e6
    prob["letd_max"][:] = 1e6
    o = Oracle(p, problem=prob)
    x = _x(12, 8)
    for norm in (0, 1, 2):
        xn, prox, nv = o.ams_simultaneous(x, normalization=norm)
        assert nv == 0 and prox == 0.0
        np.testing.assert_array_equal(xn, x)


@pytest.mark.parametrize("lam", [0.5, 1.0, 1.9])
def test_proximity_monotone_convex_weights(lam):
    """Convex-weight simultaneous projection with lambda in (0, 2) is a projected
    gradient step on the proximity function, which therefore never increases."""
    p = ph.tiny_problem(64, 16, 0.3, seed=29)
    o = Oracle(p)
    x = p.x0.astype(np.float64)
    prev, _ = o.proximity(x)
    assert prev > 0
    for _ in range(30):
        x, prox_in, _ = o.ams_simultaneous(x, lam=lam, weight_scale=1.0, normalization=0)
        cur, _ = o.proximity(x)
        assert prox_in == pytest.approx(prev, rel=1e-12)
        assert cur <= prev * (1 + 1e-12)
        prev = cur


def test_convergence_feasible_by_construction():
    """Bounds [0.95, 1.05] * D x* around a non-negative x* make the set non-empty;
    the sweeps drive the proximity to zero."""
    rng = np.random.default_rng(31)
    p = ph.tiny_problem(40, 10, 0.4, seed=31, kinds="dose")
    D, _ = dense(p)
    xs = rng.uniform(0.5, 1.5, 10)
    ds = D @ xs
    prob = {k: v.copy() for k, v in p.problem_arrays().items()}
    prob["kind"][:] = ph.DOSE_LO | ph.DOSE_HI
    prob["dose_lo"][:] = 0.95 * ds
    prob["dose_hi"][:] = 1.05 * ds
    o = Oracle(p, problem=prob)
    x = np.full(10, 3.0)
    p0, _ = o.proximity(x)
    for _ in range(400):
        x, _, _ = o.ams_simultaneous(x, lam=1.5, normalization=1)
    p1, _ = o.proximity(x)
    assert p1 < 1e-10 * p0


# --- objective and superiorization (Eq. 2, Fig. 3) ----------------------------------

def test_cost_and_gradient_dense():
    p = ph.tiny_problem(48, 12, 0.3, seed=37)
    o = Oracle(p)
    D, L = dense(p)
    x = _x(12, 9)
    d, l = D @ x, L @ x
    k = p.kind
    ptv = (k & ph.OBJ_DOSE) > 0
    oar = (k & ph.OBJ_CDL) > 0
    w = p.w_obj.astype(np.float64)
    chi = np.sum(w[ptv] * (p.dose_target[ptv] - d[ptv]) ** 2) + \
        np.sum(w[oar] * (p.cdl_target[oar] - p.c * l[oar]) ** 2)
    assert o.cost(x) == pytest.approx(chi, rel=1e-13)
    # central finite differences of the brute-force cost
    g = o.gradient(x)
    h = 1e-6
    for j in range(12):
        e = np.zeros(12)
        e[j] = h
        fd = (o.cost(x + e) - o.cost(x - e)) / (2 * h)
        assert g[j] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_quadratic_line_identity():
    """chi^2(y - beta g) - chi^2(y) = -beta ||g||^2 + beta^2 Q for g = grad chi^2(y)."""
    p = ph.tiny_problem(48, 12, 0.3, seed=41)
    o = Oracle(p)
    D, L = dense(p)
    y = _x(12, 10)
    g = o.gradient(y)
    G = g @ g
    w = p.w_obj.astype(np.float64)
    ptv = (p.kind & ph.OBJ_DOSE) > 0
    oar = (p.kind & ph.OBJ_CDL) > 0
    Q = np.sum(w[ptv] * (D @ g)[ptv] ** 2) + np.sum(w[oar] * p.c ** 2 * (L @ g)[oar] ** 2)
    for beta in (1e-3, 1e-2, 0.1):
        lhs = o.cost(y - beta * g) - o.cost(y)
        assert lhs == pytest.approx(-beta * G + beta * beta * Q, rel=1e-7, abs=1e-12)


@pytest.mark.parametrize("seed", [43, 44, 45])
@pytest.mark.parametrize("r", [1, 2])
def test_literal_and_closed_form_pick_same_step(seed, r):
    p = ph.tiny_problem(48, 12, 0.3, seed=seed)
    o = Oracle(p)
    x = p.x0.astype(np.float64)
    k, s = 0, -1
    for _ in range(5):
        xa, ka, sa, ia = o.sa_iteration(x, k, s, OracleParams(reductions_n=r, line_search=0,
                                                               alpha=0.9))
        xb, kb, sb, ib = o.sa_iteration(x, k, s, OracleParams(reductions_n=r, line_search=1,
                                                               alpha=0.9))
        assert (ka, sa) == (kb, sb)
        np.testing.assert_allclose(xa, xb, rtol=1e-9, atol=1e-12)
        assert ia["n_accepted"] == ib["n_accepted"] == r
        x, k, s = xb, kb, sb


def test_perturbation_strictly_lowers_cost():
    p = ph.tiny_problem(64, 16, 0.3, seed=47)
    o = Oracle(p)
    x = p.x0.astype(np.float64)
    k, s = 0, -1
    for _ in range(10):
        x, k, s, info = o.sa_iteration(x, k, s, OracleParams(reductions_n=2))
        assert info["n_accepted"] >= 1
        assert info["cost_after_perturb"] < info["cost_before"]
    assert k == 10 and s >= 10


def test_zero_reductions_is_ams():
    """reductions_n = 0 leaves only the feasibility-seeking step with weights
    eta^k w (Fig. 3)."""
    p = ph.tiny_problem(48, 12, 0.3, seed=53)
    o = Oracle(p)
    x = p.x0.astype(np.float64)
    q = OracleParams(reductions_n=0, eta=0.9, normalization=0)
    xa = x.copy()
    k, s = 0, -1
    for it in range(4):
        xa, k, s, _ = o.sa_iteration(xa, k, s, q)
        x, _, _ = o.ams_simultaneous(x, lam=q.lam, weight_scale=0.9 ** it, normalization=0)
        np.testing.assert_array_equal(xa, x)
    assert s == -1


def test_power_of_two_scale_invariance():
    """Scaling D, L, bounds and targets by 2^m and the objective weights by 2^-2m
    leaves the iterates unchanged bit for bit (every operation is homogeneous and
    power-of-two scaling is exact)."""
    p = ph.tiny_problem(48, 12, 0.3, seed=59)
    m = 3
    s2 = 2.0 ** m
    q = ph.tiny_problem(48, 12, 0.3, seed=59)
    q.d_val = (p.d_val * s2).astype(np.float32)
    q.l_val = (p.l_val * s2).astype(np.float32)
    for k in ("dose_lo", "dose_hi", "cdl_lo", "cdl_hi", "dose_target", "cdl_target"):
        setattr(q, k, (getattr(p, k) * s2).astype(np.float32))
    q.w_obj = (p.w_obj / s2 ** 2).astype(np.float32)
    o1, o2 = Oracle(p), Oracle(q)
    x1 = x2 = p.x0.astype(np.float64)
    k1 = k2 = 0
    s1 = s2_ = -1
    prm = OracleParams(reductions_n=1, alpha=0.9)
    for _ in range(5):
        x1, k1, s1, _ = o1.sa_iteration(x1, k1, s1, prm)
        x2, k2, s2_, _ = o2.sa_iteration(x2, k2, s2_, prm)
        np.testing.assert_array_equal(x1, x2)
        assert s1 == s2_


def test_column_permutation_equivariance():
    p = ph.tiny_problem(48, 12, 0.3, seed=61)
    perm = np.random.default_rng(61).permutation(12)
    inv = np.argsort(perm)
    D, L = dense(p)
    q = from_dense(D[:, perm], L[:, perm], **{k: v for k, v in p.problem_arrays().items()})
    o1, o2 = Oracle(p), Oracle(q)
    prm = OracleParams(reductions_n=1, alpha=0.9)
    x1 = p.x0.astype(np.float64)
    x2 = x1[perm]
    k1 = k2 = 0
    s1 = s2 = -1
    for _ in range(5):
        x1, k1, s1, _ = o1.sa_iteration(x1, k1, s1, prm)
        x2, k2, s2, _ = o2.sa_iteration(x2, k2, s2, prm)
    assert s1 == s2
    np.testing.assert_allclose(x2[inv], x1, rtol=1e-10, atol=1e-13)


# --- evaluation helpers ----------------------------------------------------------

def test_metrics_helpers():
    v = np.arange(1, 101, dtype=np.float64)  # 1..100
    assert metrics.d_percent(v, 0.95) == 5.0     # rank ceil(0.05 * 100) = 5
    assert metrics.d_percent(v, 0.98) == 2.0
    assert metrics.d_percent(np.array([3.0, 1.0, 2.0]), 0.95) == 1.0
    assert metrics.d_percent(np.array([7.0]), 0.95) == 7.0
    assert metrics.mean_letd(np.array([1.0, 0.0, 2.0]), np.array([2.0, 9.0, 4.0])) == 3.0
    assert ph.percentile_nearest_rank(np.arange(1, 11), 0.7) == 7.0


# --- the one-sided OAR term (reading Q15 of Eq. 2) and the unit perturbation
# direction (reading Q11 of Fig. 3) ----------------------------------------------

def test_one_sided_objective_hand_worked():
    """2 rows x 2 beamlets, worked by hand from Eq. (2).  D = diag(1, 2),
    L = diag(1, 3), c = 0.5, x = (1, 1): d = (1, 2), l = (1, 3), c l_1 = 1.5.
    Row 0 is PTV (target 2, weight 1): (2 - 1)^2 = 1, gradient -2 (2 - 1) D_0 = (-2, 0).
    Row 1 is OAR (weight 2).  Target 1: c l_1 is above it, f = 1 - 1.5 = -0.5 counts in
    both readings: 2 * 0.25 = 0.5, gradient -2 c w f L_1 = -2 * 0.5 * 2 * (-0.5) * (0, 3)
    = (0, 3).  Target 2: c l_1 is below it, f = 0.5: as printed 0.5 and (0, -3); one-sided
    0 and (0, 0)."""
    D = np.array([[1.0, 0.0], [0.0, 2.0]])
    L = np.array([[1.0, 0.0], [0.0, 3.0]])
    x = np.array([1.0, 1.0])
    for cdl_t, two, one, g_two, g_one in (
            (1.0, 1.5, 1.5, (-2.0, 3.0), (-2.0, 3.0)),
            (2.0, 1.5, 1.0, (-2.0, -3.0), (-2.0, 0.0))):
        p = from_dense(D, L, c=0.5, kind=[ph.OBJ_DOSE, ph.OBJ_CDL], w_obj=[1.0, 2.0],
                       dose_target=[2.0, 0.0], cdl_target=[0.0, cdl_t])
        o2, o1 = Oracle(p, objective=0), Oracle(p, objective=1)
        assert o2.cost(x) == two and o1.cost(x) == one
        np.testing.assert_array_equal(o2.gradient(x), g_two)
        np.testing.assert_array_equal(o1.gradient(x), g_one)


@pytest.mark.parametrize("seed", [61, 62, 63])
def test_one_sided_cost_and_gradient_dense(seed):
    """Against dense brute force with the OAR hinge, at points where some OAR rows
    are above their target and some below; gradient against central differences."""
    p = ph.tiny_problem(64, 12, 0.3, seed=seed)
    D, L = dense(p)
    w = p.w_obj.astype(np.float64)
    ptv = (p.kind & ph.OBJ_DOSE) > 0
    oar = (p.kind & ph.OBJ_CDL) > 0
    x = _x(12, seed)
    d, l = D @ x, L @ x
    # OAR targets at the median of c l: about half the rows above, half below
    p.cdl_target[oar] = np.float32(np.median(p.c * l[oar]))
    o = Oracle(p, objective=1)
    f = p.cdl_target - p.c * l
    above = oar & (f < 0)
    assert above.any() and (oar & (f > 0)).any()
    chi = np.sum(w[ptv] * (p.dose_target[ptv] - d[ptv]) ** 2) + np.sum(w[above] * f[above] ** 2)
    assert o.cost(x) == pytest.approx(chi, rel=1e-13)
    g = o.gradient(x)
    h = 1e-6
    for j in range(12):
        e = np.zeros(12)
        e[j] = h
        fd = (o.cost(x + e) - o.cost(x - e)) / (2 * h)
        assert g[j] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    # every OAR row above its target: the one-sided cost is the printed one
    p_all = ph.tiny_problem(64, 12, 0.3, seed=seed)
    p_all.cdl_target[:] = -1.0
    assert Oracle(p_all, objective=1).cost(x) == Oracle(p_all, objective=0).cost(x)


def _objective_only(seed, R=48, C=12):
    p = ph.tiny_problem(R, C, 0.3, seed=seed)
    p.kind = (p.kind & (ph.OBJ_DOSE | ph.OBJ_CDL)).astype(p.kind.dtype)
    return p


@pytest.mark.parametrize("seed", [71, 72])
def test_unit_direction_moves_by_beta(seed):
    """With the perturbation along g / ||g|| and no constraint rows (the sweep is then
    the identity on a non-negative point), one outer iteration moves x by exactly the
    accepted beta in Euclidean norm; literal and closed-form searches pick the same s."""
    p = _objective_only(seed)
    o = Oracle(p)
    x = p.x0.astype(np.float64) + 5.0
    k, s = 0, -1
    for _ in range(4):
        xa, ka, sa, ia = o.sa_iteration(x, k, s, OracleParams(reductions_n=1, line_search=0,
                                                               unit_direction=1, alpha=0.9))
        xb, kb, sb, ib = o.sa_iteration(x, k, s, OracleParams(reductions_n=1, line_search=1,
                                                               unit_direction=1, alpha=0.9))
        assert (ka, sa) == (kb, sb) and ib["n_accepted"] == 1
        assert np.all(xb > 0)
        assert np.linalg.norm(xb - x) == pytest.approx(ib["beta_last"], rel=1e-12)
        g = o.gradient(x)
        np.testing.assert_allclose(xb, x - ib["beta_last"] * g / np.linalg.norm(g),
                                   rtol=1e-13, atol=1e-15)
        x, k, s = xb, kb, sb


@pytest.mark.parametrize("unit", [0, 1])
@pytest.mark.parametrize("seed", [81, 82])
def test_one_sided_step_is_the_first_decrease(seed, unit):
    """Fig. 3's search with the one-sided objective: the accepted s is the first
    exponent above the previous one whose step strictly lowers the cost, checked by
    evaluating the (dense-pinned) cost at every exponent in between."""
    p = _objective_only(seed, R=64)
    o = Oracle(p, objective=1)
    x = p.x0.astype(np.float64) + 1.0
    k, s = 0, -1
    for _ in range(5):
        g = o.gradient(x)
        v = g / np.linalg.norm(g) if unit else g
        c0 = o.cost(x)
        xn, kn, sn, info = o.sa_iteration(x, k, s, OracleParams(reductions_n=1, alpha=0.8,
                                                                 unit_direction=unit))
        assert info["n_accepted"] == 1 and sn > s
        for t in range(s + 1, sn):
            assert o.cost(x - 0.8 ** t * v) >= c0
        assert o.cost(x - 0.8 ** sn * v) < c0
        assert info["cost_after_perturb"] < info["cost_before"]
        x, k, s = xn, kn, sn


# --- block-sequential sweeps (Fig. 2's order over blocks of rows) ------------------

@pytest.mark.parametrize("norm", [0, 1, 2])
def test_one_block_is_the_simultaneous_sweep(norm):
    p = ph.tiny_problem(48, 12, 0.3, seed=91)
    o = Oracle(p)
    x = _x(12, 91)
    xs, _, _ = o.ams_simultaneous(x, lam=1.3, weight_scale=0.8, normalization=norm)
    for block in (48, 1000):
        xb = o.ams_blocks(x, block, lam=1.3, weight_scale=0.8, normalization=norm)
        np.testing.assert_array_equal(xb, xs)


def test_blocks_of_one_row_are_the_sequential_sweep():
    """Rows of one dose constraint each, on overlapping beamlets, raw weights and
    lambda = 1: blocks of one row project onto one half-space after the other, which
    is Fig. 2's sequential sweep (its dose block, voxels in ascending order).  The
    sweep with every row in one block differs (the rows interact)."""
    rng = np.random.default_rng(93)
    R, C = 8, 5
    D = rng.uniform(0.2, 1.0, (R, C)).astype(np.float32)
    L = (D * 3.0).astype(np.float32)
    x = rng.uniform(0.5, 1.5, C)
    d0 = D.astype(np.float64) @ x
    kind = [ph.DOSE_HI if i % 2 == 0 else ph.DOSE_LO for i in range(R)]
    dose_hi = [0.8 * d0[i] if i % 2 == 0 else 0.0 for i in range(R)]
    dose_lo = [1.2 * d0[i] if i % 2 == 1 else 0.0 for i in range(R)]
    p = from_dense(D, L, kind=kind, dose_hi=dose_hi, dose_lo=dose_lo, w_feas=np.ones(R))
    o = Oracle(p)
    xq = o.ams_sequential(x, range(R), [], lam=1.0, weight_scale=1.0)
    x1 = o.ams_blocks(x, 1, lam=1.0, weight_scale=1.0, normalization=2)
    np.testing.assert_allclose(x1, xq, rtol=1e-13, atol=1e-15)
    xall = o.ams_blocks(x, R, lam=1.0, weight_scale=1.0, normalization=2)
    assert np.max(np.abs(xall - xq)) > 1e-3


def test_block_sweep_fixed_point_and_blocks():
    """A feasible non-negative point is fixed for every block size; two blocks equal
    two simultaneous sweeps of the halves' sub-problems taken one after the other."""
    p = ph.tiny_problem(40, 10, 0.3, seed=95)
    o = Oracle(p)
    D, L = dense(p)
    x = _x(10, 95)
    for block in (1, 7, 20, 40):
        pa = ph.tiny_problem(40, 10, 0.3, seed=95)
        pa.kind[:] = 0  # no constraints: every point is feasible
        np.testing.assert_array_equal(Oracle(pa).ams_blocks(x, block), x)
    # two blocks of 20 rows: the first half's sweep, then the second half's, each with
    # weights normalised over its own half, the clamp at the end only
    half = [ph.tiny_problem(40, 10, 0.3, seed=95), ph.tiny_problem(40, 10, 0.3, seed=95)]
    half[0].kind[20:] = 0
    half[1].kind[:20] = 0
    y = x.copy()
    for h in half:
        oh = Oracle(h)
        # the half sweep without its clamp: raw move of the simultaneous form
        t = oh.ams_simultaneous(y, lam=1.2, weight_scale=0.9, normalization=0)[0]
        assert np.all(t > 0)   # no clamp in play at this point
        y = t
    xb = o.ams_blocks(x, 20, lam=1.2, weight_scale=0.9, normalization=0)
    np.testing.assert_allclose(xb, y, rtol=1e-13, atol=1e-15)
