"""Pins of the oracle's learned-tagging pieces (features, network, Adam,
tag rule) to facts fixed outside the oracle: bfloat16 rounding as torch
performs it, central finite differences of the FP64 loss, the normal
distribution function of scipy, closed forms of a zero network, invariants
of Adam, and the exact statistics of linear data."""
import numpy as np
import pytest
from scipy.stats import norm as normal

from oracle import oracle as O
from paper_1308_1472_amd import inputs as I

NI, NH, NO = O.MLP_IN, O.MLP_HID, O.MLP_OUT
OW1, OB1 = 0, NI * NH
OW2, OB2 = OB1 + NH, OB1 + NH + NH * NH
OW3, OB3 = OB2 + NH, OB2 + NH + NH * NO


def _random_net(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    P = np.empty(O.MLP_PARAMS)
    P[OW1:OB1] = rng.normal(0, scale / np.sqrt(NI), NI * NH)
    P[OB1:OW2] = rng.normal(0, 0.1, NH)
    P[OW2:OB2] = rng.normal(0, scale / np.sqrt(NH), NH * NH)
    P[OB2:OW3] = rng.normal(0, 0.1, NH)
    P[OW3:OB3] = rng.normal(0, scale / np.sqrt(NH), NH * NO)
    P[OB3:] = rng.normal(0, 0.1, NO)
    norm = np.concatenate([rng.normal(0, 1, NI), rng.uniform(0.5, 2, NI)])
    x = rng.normal(norm[:NI], norm[NI:], (7, NI))
    y = np.array([0, 1, 2, 2, 1, 0, 1], np.int32)
    return P, norm, x, y


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.normal(0, 1, 4000), rng.normal(0, 1e-30, 200),
                        rng.normal(0, 1e30, 200)]).astype(np.float32)
    # exact ties: 8 significant bits plus one half
    ties = (np.arange(1, 200) * 2 + 1).astype(np.float32) * np.float32(2.0 ** -9) + 1
    v = np.concatenate([v, ties, -ties]).astype(np.float32)
    want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(O.bf16(v.astype(np.float64)), want)


def test_gradient_is_the_derivative_of_the_fp64_loss():
    """Central finite differences on every parameter (plain FP64 network)."""
    P, norm, x, y = _random_net(1)
    cw = np.array([2.0, 0.5, 1.5])
    loss, _, g = O.mlp(P, norm, x, y, cw, scale=0.3, round_bf16=False)
    h = 1e-6
    fd = np.empty_like(P)
    for t in range(P.size):
        Pp, Pm = P.copy(), P.copy()
        Pp[t] += h
        Pm[t] -= h
        lp = O.mlp(Pp, norm, x, y, cw, 0.3, False, want_grad=False)[0]
        lm = O.mlp(Pm, norm, x, y, cw, 0.3, False, want_grad=False)[0]
        fd[t] = (lp - lm) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-6 * np.max(np.abs(g))
    # every block of the parameter vector carries gradient
    for a, b in ((OW1, OB1), (OB1, OW2), (OW2, OB2), (OB2, OW3), (OW3, OB3), (OB3, None)):
        assert np.max(np.abs(g[a:b])) > 1e-4


def test_single_path_network_is_nested_gelu():
    """Input 3 -> hidden-1 unit 5 -> hidden-2 unit 7 -> class 2: the logit
    is c * GELU(b * GELU(a * x3)) + bias, GELU(z) = z Phi(z)."""
    P = np.zeros(O.MLP_PARAMS)
    a, b, c = 1.3, -0.7, 2.1
    P[OW1 + 3 * NH + 5] = a
    P[OW2 + 5 * NH + 7] = b
    P[OW3 + 7 * NO + 2] = c
    P[OB3:] = [0.25, -0.5, 0.125]
    norm = np.concatenate([np.zeros(NI), np.ones(NI)])
    x = np.zeros((5, NI))
    x[:, 3] = [-2.0, -0.5, 0.0, 0.75, 3.0]
    gelu = lambda z: z * normal.cdf(z)
    _, z, _ = O.mlp(P, norm, x, round_bf16=False)
    want = c * gelu(b * gelu(a * x[:, 3])) + 0.125
    np.testing.assert_allclose(z[:, 2], want, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(z[:, 0], 0.25, rtol=0, atol=0)
    np.testing.assert_allclose(z[:, 1], -0.5, rtol=0, atol=0)


def test_zero_network_loss_and_output_gradient():
    P = np.zeros(O.MLP_PARAMS)
    norm = np.concatenate([np.zeros(NI), np.ones(NI)])
    rng = np.random.default_rng(3)
    x = rng.normal(size=(11, NI))
    y = rng.integers(0, 3, 11).astype(np.int32)
    cw = np.array([3.0, 1.0, 0.5])
    loss, z, g = O.mlp(P, norm, x, y, cw, scale=0.25, round_bf16=True)
    assert np.all(z == 0)
    wsum = 0.25 * cw[y].sum()
    assert loss == pytest.approx(wsum * np.log(3.0), rel=1e-15)
    # dL/db3[c] = sum_r w_r (1/3 - [y_r == c])
    g0 = O.mlp(P, norm, x, y, cw, scale=0.25, round_bf16=False)[2]
    for c in range(3):
        terms = [0.25 * cw[k] * (1 / 3 - (k == c)) for k in y]
        assert g0[OB3 + c] == pytest.approx(sum(terms), rel=1e-14)
        # rounded: each row's term carries at most half a bfloat16 step
        assert abs(g[OB3 + c] - sum(terms)) <= 2.0 ** -8 * sum(abs(t) for t in terms)


def test_rounded_network_rounds_weights_and_inputs():
    """Weights and inputs already on the bfloat16 grid: nudging them by far
    less than half a bfloat16 step leaves the rounded network bit-identical,
    while the plain FP64 network moves."""
    P, norm, x, y = _random_net(4)
    norm = np.concatenate([np.zeros(NI), np.ones(NI)])
    P = O.bf16(P)
    x = O.bf16(x)
    base = O.mlp(P, norm, x, y)
    Pn = P.copy()
    Pn[:OB1] *= 1 + 2.0 ** -12
    Pn[OW2:OB2] *= 1 - 2.0 ** -12
    Pn[OW3:OB3] *= 1 + 2.0 ** -12
    nudged = O.mlp(Pn, norm, x * (1 + 2.0 ** -12), y)
    assert nudged[0] == base[0]
    assert np.array_equal(nudged[1], base[1]) and np.array_equal(nudged[2], base[2])
    plain = O.mlp(Pn, norm, x * (1 + 2.0 ** -12), y, round_bf16=False)
    assert not np.array_equal(plain[1], O.mlp(P, norm, x, y, round_bf16=False)[1])
    # and the rounded network stays within bfloat16 error of the plain one
    ref = O.mlp(P, norm, x, y, round_bf16=False)
    assert abs(base[0] - ref[0]) <= 0.05 * abs(ref[0])
    assert np.max(np.abs(base[1] - ref[1])) <= 0.05 * np.max(np.abs(ref[1]))
    assert np.linalg.norm(base[2] - ref[2]) <= 0.05 * np.linalg.norm(ref[2])


def test_adam_invariants():
    rng = np.random.default_rng(5)
    n = 50
    g = rng.normal(size=n)
    # first step with eps = 0 moves every parameter by lr * sign(g)
    P = rng.normal(size=n)
    m1, m2 = np.zeros(n), np.zeros(n)
    P0 = P.copy()
    O.adam(P, g, m1, m2, 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(P, P0 - 0.01 * np.sign(g), rtol=0, atol=1e-15)
    # a constant gradient keeps the bias-corrected moments at g and g^2
    for t in range(2, 30):
        Pb = P.copy()
        O.adam(P, g, m1, m2, t, lr=0.01, eps=0.0)
        np.testing.assert_allclose(P, Pb - 0.01 * np.sign(g), rtol=0, atol=1e-13)
    # scaling every gradient scales nothing (eps = 0)
    Pa, Pb = P0.copy(), P0.copy()
    ma, va, mb, vb = (np.zeros(n) for _ in range(4))
    for t in range(1, 6):
        gt = rng.normal(size=n)
        O.adam(Pa, gt, ma, va, t, eps=0.0)
        O.adam(Pb, 1000.0 * gt, mb, vb, t, eps=0.0)
    np.testing.assert_allclose(Pa, Pb, rtol=1e-13, atol=1e-15)


def test_learned_tags_rule():
    z = np.array([[5.0, 0.0, 0.0],      # sure refine
                  [0.0, 5.0, 0.0],      # sure keep
                  [0.0, 0.0, 5.0],      # sure coarsen
                  [0.1, 0.0, 0.05],     # unsure -> plain
                  [0.0, 0.0, 5.0],      # plain says refine -> refine
                  [0.0, 5.0, 0.0]])
    plain = np.array([0, 0, 0, -1, 1, -1], np.int8)
    assert O.learned_tags(z, plain, 0.6).tolist() == [1, 0, -1, -1, 1, 0]
    # the threshold sits on the largest softmax probability
    p = np.exp(z[3]) / np.exp(z[3]).sum()
    assert O.learned_tags(z[3:4], plain[3:4], p.max() - 1e-9).tolist() == [1]


def test_features_of_linear_data_are_exact():
    """h, hu, hv linear in x and y on an adaptive walled forest: on every
    patch away from the walls the min / max sit at the corner cell centres,
    the mean at the patch centre, and max |grad| is the slope norm (the
    feature is its log1p), because
    copies, 2x2 means and limited interpolation all reproduce linear data."""
    trees, pl = I.walled_square()
    m = 8
    lv = O.balance(trees, I.random_leaves(9, 1, 2, 5, 20))
    mesh = O.Mesh(trees, lv, m)
    par = O.params(m, O.SHALLOW)
    coef = np.array([[2.0, 0.3, -0.2], [0.1, -0.5, 0.25], [-0.3, 0.2, 0.4]])
    q = I.state_from(lv, m, lambda x, y: np.stack(
        [c[0] + c[1] * x + c[2] * y for c in coef], axis=1))
    f = O.framed(q, m)
    O.ghost_fill(mesh, par, f)
    F = O.features(mesh, par, f)
    assert F.shape == (len(lv), 16)
    inner = 0
    for p, a in enumerate(lv):
        n = 1 << int(a["level"])
        if a["ix"] == 0 or a["iy"] == 0 or a["ix"] == n - 1 or a["iy"] == n - 1:
            continue
        inner += 1
        h = 1.0 / n
        x0, y0 = a["ix"] * h, a["iy"] * h
        lo_x, hi_x = x0 + 0.5 * h / m, x0 + h - 0.5 * h / m
        lo_y, hi_y = y0 + 0.5 * h / m, y0 + h - 0.5 * h / m
        for k, c in enumerate(coef):
            corners = [c[0] + c[1] * xx + c[2] * yy for xx in (lo_x, hi_x) for yy in (lo_y, hi_y)]
            mid = c[0] + c[1] * (x0 + h / 2) + c[2] * (y0 + h / 2)
            want = [min(corners), max(corners), mid, np.log1p(np.hypot(c[1], c[2]))]
            np.testing.assert_allclose(F[p, 4 * k:4 * k + 4], want, rtol=1e-11, atol=1e-12)
        assert F[p, 12] == a["level"]
        assert np.all(F[p, 13:] == 0)
    assert inner >= 10


@pytest.mark.parametrize("domain", ["walled", "periodic", "sphere"])
def test_dilation_is_the_touching_neighbourhood(domain):
    """A leaf below lmax becomes +1 exactly when a leaf it touches (closed
    boxes intersect, found by brute force) is +1."""
    from tests.helpers import leaf_boxes_cube, leaf_boxes_plane, touching_pairs
    if domain == "sphere":
        trees = I.cubed_sphere(); nt = 6
    elif domain == "periodic":
        trees, pl = I.periodic_square(); nt = 1
    else:
        trees, pl = I.walled_square(); nt = 1
    lv = O.balance(trees, I.random_leaves(31, nt, 1, 5, 30))
    mesh = O.Mesh(trees, lv, 8)
    if domain == "sphere":
        lo, hi = leaf_boxes_cube(lv)
        pairs = touching_pairs(lo, hi)
    else:
        lo, hi = leaf_boxes_plane(lv, pl)
        pairs = touching_pairs(lo, hi, (1.0, 1.0) if domain == "periodic" else None)
    rng = np.random.default_rng(4)
    tg = rng.choice(np.array([-1, 0, 0, 0, 0, 1], np.int8), len(lv))
    lmax = 4
    out = O.dilate_tags(mesh, tg, lmax)
    want = tg.copy()
    for a, b in pairs:
        if tg[b] == 1 and lv[a]["level"] < lmax:
            want[a] = 1
        if tg[a] == 1 and lv[b]["level"] < lmax:
            want[b] = 1
    assert np.array_equal(out, want)
    assert np.sum(out == 1) > np.sum(tg == 1)
