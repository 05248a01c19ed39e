"""Pins of the oracle's learned-closure routines (network, inputs, box filter,
closure right-hand side) against closed forms, invariants and finite
differences.  Each test states what fixes the expected value.

The closure is not part of the paper's method (the paper names surrogate
models only as future work, Sec. 6); the network shape, inputs, fallback rule
and training recipe are this library's readings.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2412_04395_amd import workloads as W

NP = 9609


def _zero_params():
    return np.zeros(NP)


# parameter layout: W1[10][64], b1, W2[64][64], b2, W3[64][64], b3, W4[64][9], b4
OFF = {"W1": 0, "b1": 640, "W2": 704, "b2": 4800, "W3": 4864, "b3": 8960, "W4": 9024, "b4": 9600}


def _view(p):
    return {"W1": p[0:640].reshape(10, 64), "b1": p[640:704], "W2": p[704:4800].reshape(64, 64),
            "b2": p[4800:4864], "W3": p[4864:8960].reshape(64, 64), "b3": p[8960:9024],
            "W4": p[9024:9600].reshape(64, 9), "b4": p[9600:9609]}


def _norm_identity():
    return np.concatenate([np.zeros(10), np.ones(10), np.zeros(9), np.ones(9)])


def test_param_count():
    assert oracle.mlp_nparams() == NP == 10 * 64 + 64 + 2 * (64 * 64 + 64) + 64 * 9 + 9


# -- bfloat16 rounding -----------------------------------------------------------
def test_bf16_rounding_closed_forms():
    """bfloat16 keeps 8 significant bits; ties go to the even significand."""
    b = oracle.bf16
    assert b(1.0) == 1.0 and b(-2.5) == -2.5 and b(0.0) == 0.0
    assert b(1 + 2 ** -8) == 1.0                      # tie, 1.0000000b is even
    assert b(1 + 3 * 2 ** -8) == 1 + 2 ** -6          # tie, rounds up to even
    assert b(1 + 2 ** -8 + 2 ** -20) == 1 + 2 ** -7   # above the tie
    assert b(-(1 + 2 ** -8 + 2 ** -20)) == -(1 + 2 ** -7)
    assert b(257.0) == 256.0 and b(387.0) == 388.0 and b(129.0) == 129.0
    assert math.isinf(b(3.4028e38))                   # above the largest bfloat16
    assert math.isnan(b(float("nan")))


# -- forward pass ----------------------------------------------------------------
def _linear_net(A, c):
    """Parameters that make the network compute y = x A + c exactly: every input
    passes as relu(x) and relu(-x), the middle layers copy, the last recombines."""
    p = _zero_params()
    v = _view(p)
    for i in range(10):
        v["W1"][i, 2 * i] = 1.0
        v["W1"][i, 2 * i + 1] = -1.0
    for h in range(20):
        v["W2"][h, h] = 1.0
        v["W3"][h, h] = 1.0
    for i in range(10):
        v["W4"][2 * i] = A[i]
        v["W4"][2 * i + 1] = -A[i]
    v["b4"][:] = c
    return p


def test_forward_linear_network_exact():
    rng = np.random.default_rng(1)
    A = rng.integers(-4, 5, size=(10, 9)).astype(float)
    c = rng.integers(-3, 4, size=9).astype(float)
    x = rng.integers(-20, 21, size=(13, 10)).astype(float)
    p = _linear_net(A, c)
    for bf in (False, True):   # small integers are exact in bfloat16 as well
        y = oracle.mlp_forward(p, x, bf16=bf)
        assert np.array_equal(y, x @ A + c)


def test_forward_bf16_rounds_inputs_and_activations():
    A = np.zeros((10, 9))
    A[0, 0] = 1.0
    p = _linear_net(A, np.zeros(9))
    x = np.zeros((1, 10))
    x[0, 0] = 257.0           # input: 257 -> 256 (tie to even)
    assert oracle.mlp_forward(p, x)[0, 0] == 257.0
    assert oracle.mlp_forward(p, x, bf16=True)[0, 0] == 256.0
    _view(p)["W1"][0, 0], _view(p)["W1"][0, 1] = 3.0, -3.0
    x[0, 0] = 129.0           # hidden activation 387 -> 388 (tie to even)
    assert oracle.mlp_forward(p, x)[0, 0] == 387.0
    assert oracle.mlp_forward(p, x, bf16=True)[0, 0] == 388.0


def _rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = np.zeros(NP)
    v = _view(p)
    for (w, b), fan in zip((("W1", "b1"), ("W2", "b2"), ("W3", "b3"), ("W4", "b4")), (10, 64, 64, 64)):
        v[w][:] = rng.normal(0, scale * math.sqrt(2.0 / fan), v[w].shape)
        v[b][:] = rng.normal(0, 0.1, v[b].shape)
    return p


def test_relu_hidden_linear_output():
    """Scaling every input by s > 0 scales a bias-free network's output by s
    (positive homogeneity of ReLU layers and a linear output layer)."""
    p = _rand_params(3)
    for b in ("b1", "b2", "b3", "b4"):
        _view(p)[b][:] = 0.0
    x = np.random.default_rng(4).normal(size=(9, 10))
    y = oracle.mlp_forward(p, x)
    assert np.allclose(oracle.mlp_forward(p, 4.0 * x), 4.0 * y, rtol=1e-14, atol=0)
    assert np.all(oracle.mlp_forward(p, 0.0 * x) == 0.0)


# -- loss and gradient ------------------------------------------------------------
def test_loss_is_mean_squared_error():
    p = _rand_params(5)
    rng = np.random.default_rng(6)
    x, t = rng.normal(size=(17, 10)), rng.normal(size=(17, 9))
    loss, _ = oracle.mlp_loss_grad(p, x, t)
    y = oracle.mlp_forward(p, x)
    assert abs(loss - np.mean((y - t) ** 2)) <= 1e-15 * loss


def test_gradient_matches_central_differences():
    """Backpropagation against central differences of the loss, every parameter
    (FP64 mode): truncation O(h^2) and rounding O(eps/h) are both < 1e-9."""
    p = _rand_params(7)
    rng = np.random.default_rng(8)
    x, t = rng.normal(size=(7, 10)), rng.normal(size=(7, 9))
    _, g = oracle.mlp_loss_grad(p, x, t)
    h = 1e-6
    fd = np.zeros(NP)
    for i in range(NP):
        q = p.copy()
        q[i] += h
        lp = np.mean((oracle.mlp_forward(q, x) - t) ** 2)
        q[i] -= 2 * h
        lm = np.mean((oracle.mlp_forward(q, x) - t) ** 2)
        fd[i] = (lp - lm) / (2 * h)
    err = np.abs(fd - g).max() / np.abs(g).max()
    assert err <= 1e-6, err
    assert np.count_nonzero(g) > NP // 2      # most parameters take part


def test_bf16_gradient_close_to_fp64():
    """Operand rounding to bfloat16 (relative 2^-9) changes the gradient by
    about that much, and no more than a few percent in norm."""
    p = _rand_params(9)
    rng = np.random.default_rng(10)
    x, t = rng.normal(size=(64, 10)), rng.normal(size=(64, 9))
    l64, g64 = oracle.mlp_loss_grad(p, x, t)
    l16, g16 = oracle.mlp_loss_grad(p, x, t, bf16=True)
    rel = np.linalg.norm(g16 - g64) / np.linalg.norm(g64)
    assert 1e-5 < rel < 3e-2, rel
    assert abs(l16 - l64) < 2e-2 * l64


@pytest.mark.parametrize("bf16", [False, True])
def test_gradient_magnitude_scale(bf16):
    """The per-parameter scale sum |terms| bounds |gradient| (triangle
    inequality), and equals it where no term can cancel: with non-negative
    weights, biases and inputs every activation is positive, and with every
    output above its target every backpropagated term is non-negative."""
    p = np.abs(_rand_params(12))
    rng = np.random.default_rng(13)
    x = np.abs(rng.normal(size=(40, 10)))
    y = oracle.mlp_forward(p, x, bf16=bf16)
    t = y - 0.5 - rng.random(y.shape)               # every output above its target
    _, g = oracle.mlp_loss_grad(p, x, t, bf16=bf16)
    ga = oracle.mlp_grad_abs(p, x, t, bf16=bf16)
    assert np.all(g >= 0.0)
    assert np.allclose(ga, g, rtol=1e-12, atol=0.0)
    # mixed signs: the scale bounds the gradient and exceeds it somewhere
    p2, x2 = _rand_params(14), rng.normal(size=(40, 10))
    t2 = rng.normal(size=(40, 9))
    _, g2 = oracle.mlp_loss_grad(p2, x2, t2, bf16=bf16)
    ga2 = oracle.mlp_grad_abs(p2, x2, t2, bf16=bf16)
    assert np.all(np.abs(g2) <= ga2 * (1 + 1e-12))
    assert np.any(np.abs(g2) < 0.5 * ga2)


def test_forward_margin_closed_forms():
    """One hidden unit per layer wired through (weight 1, every other weight
    and bias zero, so the other units have no terms and report nothing), input
    x0 = 1.  The bfloat16 values around 1 are 1 - 2^-8, 1 and 1 + 2^-7.
      * bias 2^-8: the first unit's value 1 + 2^-8 is a rounding midpoint, margin 0;
      * bias 2^-9: 2^-9 from the midpoint 1 + 2^-8, over |b| + |x W| = 1 + 2^-9
        (the later units see 1, 2^-9 from the midpoint 1 - 2^-9 below, over 1);
      * bias -1 - 2^-20: the value -2^-20 is 2^-20 from the ReLU switch at zero,
        over 2 + 2^-20 (the later units see 0 and have no terms)."""
    p = np.zeros(NP)
    v = _view(p)
    v["W1"][0, 0] = v["W2"][0, 0] = v["W3"][0, 0] = 1.0
    x = np.zeros((1, 10))
    x[0, 0] = 1.0
    out = []
    for b in (2.0 ** -8, 2.0 ** -9, -1.0 - 2.0 ** -20):
        v["b1"][0] = b
        out.append(oracle.mlp_forward_margin(p, x)[0])
    assert out[0] == 0.0
    assert out[1] == 2.0 ** -9 / (1 + 2.0 ** -9)
    assert out[2] == 2.0 ** -20 / (2 + 2.0 ** -20)
    # the counterfactual pass: 1 + 2^-9 rounds to 1 in the next layer; flipped,
    # it is handed 1 + 2^-7, which the pass-through carries to output 0
    v["b1"][0] = 2.0 ** -9
    v["W4"][0, 0] = 1.0
    y0 = oracle.mlp_forward_flipped(p, x, [-1])
    assert np.array_equal(y0, oracle.mlp_forward(p, x, bf16=True))
    assert y0[0, 0] == 1.0
    assert oracle.mlp_forward_flipped(p, x, [0])[0, 0] == 1.0 + 2.0 ** -7
    # a unit of the second layer (index 64 + 0) sees 1 and flips to 1 - 2^-8
    assert oracle.mlp_forward_flipped(p, x, [64])[0, 0] in (1.0 - 2.0 ** -8, 1.0 + 2.0 ** -7)


# -- Adam ---------------------------------------------------------------------------
def test_adam_constant_gradient_step_is_lr():
    """With a constant gradient g the bias-corrected moments equal g and g^2,
    so every step moves each parameter by lr g / (|g| + eps)."""
    rng = np.random.default_rng(11)
    g = rng.normal(size=50)
    p0 = rng.normal(size=50)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    lr, eps = 1e-3, 1e-8
    for k in range(1, 6):
        before = p.copy()
        oracle.adam(p, g, m, v, k, lr)
        step = before - p
        assert np.allclose(step, lr * g / (np.abs(g) + eps), rtol=1e-9, atol=0)


def test_training_reduces_loss():
    """Adam on a smooth target: the loss falls by more than 10x in 400 steps."""
    rng = np.random.default_rng(12)
    x = rng.normal(size=(256, 10))
    A = rng.normal(size=(10, 9)) / 3
    t = np.tanh(x @ A)
    p = _rand_params(13)
    m, v = np.zeros(NP), np.zeros(NP)
    l0, _ = oracle.mlp_loss_grad(p, x, t)
    for k in range(1, 401):
        _, g = oracle.mlp_loss_grad(p, x, t)
        oracle.adam(p, g, m, v, k, 3e-3)
    l1, _ = oracle.mlp_loss_grad(p, x, t)
    assert l1 < 0.1 * l0, (l0, l1)


# -- closure inputs ------------------------------------------------------------------
def _grid(nx=16, ny=12, nz=10, dx=30.0, dy=20.0, dzv=10.0):
    cfg = W.small(name="rest", nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=W.uniform_dz(nz, dzv),
                  sgs=2, Cs=0.17, Pr_t=1.0 / 3.0, adv_order_h=2, adv_order_v=2)
    return cfg, oracle.Oracle(cfg)


def _unit_rho_state(cfg, u=None, v=None, w=None, th=None):
    nz, ny, nx = cfg.nz, cfg.ny, cfg.nx
    S = {"rho": np.ones((nz, ny, nx)), "rt": np.full((nz, ny, nx), 300.0),
         "ru": np.zeros((nz, ny, nx)), "rv": np.zeros((nz, ny, nx)), "rw": np.zeros((nz + 1, ny, nx)),
         "rq": np.zeros((0, nz, ny, nx))}
    if u is not None:
        S["ru"] = np.broadcast_to(u, S["ru"].shape).copy()
    if v is not None:
        S["rv"] = np.broadcast_to(v, S["rv"].shape).copy()
    if w is not None:
        S["rw"] = np.broadcast_to(w, S["rw"].shape).copy()
    if th is not None:
        S["rt"] = np.broadcast_to(th, S["rt"].shape).copy()
    return S


def _feat(o, cfg, S):
    return o.sgs_features(S).reshape(cfg.nz, cfg.ny, cfg.nx, 10)


def test_features_diagonal_and_dtheta_dz():
    """Diagonal gradients are the face differences across the cell; dtheta/dz
    of a linear profile is exact inside and half its value next to a lid."""
    cfg, o = _grid()
    nx, ny, nz, dx, dy, dz = cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, cfg.dz[0]
    a, b = 2 * np.pi * 3 / nx, 2 * np.pi * 2 / ny
    i, j, k = np.arange(nx), np.arange(ny), np.arange(nz)
    u = np.sin(a * i)[None, None, :]
    v = np.cos(b * j)[None, :, None]
    kw = np.arange(nz + 1)
    w = np.sin(np.pi * kw / nz)[:, None, None] * np.ones((1, ny, nx))
    th = 300.0 + 0.01 * (k + 0.5)[:, None, None] * dz
    f = _feat(o, cfg, _unit_rho_state(cfg, u, v, w, th))
    e0 = 2 * np.cos(a * (i + 0.5)) * np.sin(a / 2) / dx
    e4 = -2 * np.sin(b * (j + 0.5)) * np.sin(b / 2) / dy
    e8 = (np.sin(np.pi * (k + 1) / nz) - np.sin(np.pi * k / nz)) / dz
    assert np.allclose(f[..., 0], e0[None, None, :], atol=1e-14)
    assert np.allclose(f[..., 4], e4[None, :, None], atol=1e-14)
    assert np.allclose(f[..., 8], e8[:, None, None] * np.ones((1, ny, nx)), atol=1e-14)
    e9 = np.full(nz, 0.01)
    e9[0] = e9[-1] = 0.005
    assert np.allclose(f[..., 9], e9[:, None, None] * np.ones((1, ny, nx)), atol=1e-13)
    for c in (1, 2, 3, 5, 6, 7):   # these fields have no cross derivatives
        assert np.abs(f[..., c]).max() <= 1e-14, c


def test_features_cross_derivatives():
    """Off-diagonal gradients are means of the four edge differences around the
    centre: for a sinusoid of wavenumber a that is sin(a) / spacing times the
    cosine at the centre (a centred difference over two cells); the lid edges
    contribute zero for du/dz, dv/dz, dw/dx, dw/dy."""
    cfg, o = _grid()
    nx, ny, nz, dx, dy, dz = cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, cfg.dz[0]
    a, b, c = 2 * np.pi * 2 / nx, 2 * np.pi * 3 / ny, np.pi * 1.5 / nz
    i, j, k = np.arange(nx), np.arange(ny), np.arange(nz)
    ci = (i + 0.5)[None, None, :]
    cj = (j + 0.5)[None, :, None]
    ck = (k + 0.5)[:, None, None]
    ones = np.ones((nz, ny, nx))
    # du/dy, dv/dx, du/dz, dv/dz
    S = _unit_rho_state(cfg, u=np.sin(b * cj) + np.sin(c * ck), v=np.sin(a * ci) + np.cos(c * ck))
    f = _feat(o, cfg, S)
    assert np.allclose(f[..., 1], np.sin(b) / dy * np.cos(b * cj) * ones, atol=1e-14)
    assert np.allclose(f[..., 3], np.sin(a) / dx * np.cos(a * ci) * ones, atol=1e-14)
    kk = np.arange(nz)
    dudz = np.sin(c) / dz * np.cos(c * (kk + 0.5))
    dudz[0] = (np.sin(c * 1.5) - np.sin(c * 0.5)) / dz / 4 * 2
    dudz[-1] = (np.sin(c * (nz - 0.5)) - np.sin(c * (nz - 1.5))) / dz / 4 * 2
    dvdz = -np.sin(c) / dz * np.sin(c * (kk + 0.5))
    dvdz[0] = (np.cos(c * 1.5) - np.cos(c * 0.5)) / dz / 2
    dvdz[-1] = (np.cos(c * (nz - 0.5)) - np.cos(c * (nz - 1.5))) / dz / 2
    assert np.allclose(f[..., 2], dudz[:, None, None] * ones, atol=1e-14)
    assert np.allclose(f[..., 5], dvdz[:, None, None] * ones, atol=1e-14)
    # dw/dx, dw/dy
    kw = np.arange(nz + 1)
    s = np.sin(np.pi * kw / nz)
    w = s[:, None, None] * (np.sin(a * (i + 0.5))[None, None, :] + np.cos(b * (j + 0.5))[None, :, None])
    f = _feat(o, cfg, _unit_rho_state(cfg, w=w))
    sm = 0.5 * (s[:-1] + s[1:])
    assert np.allclose(f[..., 6], sm[:, None, None] * np.sin(a) / dx * np.cos(a * ci) * ones, atol=1e-14)
    assert np.allclose(f[..., 7], -sm[:, None, None] * np.sin(b) / dy * np.sin(b * cj) * ones, atol=1e-14)


# -- box filter ------------------------------------------------------------------------
def test_box_filter_block_constant_gives_zero_targets():
    """Velocities and theta constant on every 4^3 block have no subfilter
    fluctuation: every target vanishes."""
    cfg, o = _grid(nx=16, ny=16, nz=8)
    rng = np.random.default_rng(14)
    r = 4
    blk = lambda a: np.repeat(np.repeat(np.repeat(a, r, 0), r, 1), r, 2)
    # centre-constant per block: u constant along x, v along y, w zero
    u = blk(rng.normal(size=(2, 4, 1)))[:, :, :1] * np.ones((1, 1, 16))
    v = blk(rng.normal(size=(2, 1, 4)))[:, :1, :] * np.ones((1, 16, 1))
    th = 300.0 + blk(rng.normal(size=(2, 4, 4)))
    S = _unit_rho_state(cfg, u=u, v=v, th=th)
    _, tg = o.box_filter(S, r)
    # rounding of a 64-term mean of products: 64 eps max|u_i u_j| (max|u theta|)
    eps = np.finfo(float).eps
    umax = max(np.abs(u).max(), np.abs(v).max())
    assert np.abs(tg[:, :6]).max() <= 64 * eps * umax ** 2
    assert np.abs(tg[:, 6:]).max() <= 64 * eps * umax * np.abs(th).max()


def test_box_filter_closed_form_variance_and_flux():
    """Centre velocity a(1,1,-1,-1) along x and theta' b(1,1,-1,-1): a 4-block
    holds one period, so tau_11 = a^2 and q_1 = a b; the rest vanish."""
    cfg, o = _grid(nx=16, ny=8, nz=8)
    a, bb = 1.5, 0.25
    face = np.tile(np.array([0.0, 2 * a, 0.0, -2 * a]), 4)   # centre = mean of two faces
    pat = np.tile(np.array([1.0, 1.0, -1.0, -1.0]), 4)
    S = _unit_rho_state(cfg, u=face[None, None, :], th=300.0 + bb * pat[None, None, :])
    _, tg = o.box_filter(S, 4)
    assert np.allclose(tg[:, 0], a * a, rtol=1e-13)
    assert np.allclose(tg[:, 6], a * bb, rtol=1e-12)
    for c in (1, 2, 3, 4, 5, 7, 8):
        assert np.abs(tg[:, c]).max() <= 1e-12


def test_box_filter_galilean_invariance_and_psd():
    cfg, o = _grid(nx=16, ny=8, nz=8)
    rng = np.random.default_rng(15)
    sh = (cfg.nz, cfg.ny, cfg.nx)
    rw = rng.normal(size=(cfg.nz + 1,) + sh[1:])
    rw[0] = rw[-1] = 0
    S = _unit_rho_state(cfg, u=rng.normal(size=sh), v=rng.normal(size=sh), w=rw,
                        th=300 + rng.normal(size=sh))
    _, t1 = o.box_filter(S, 2)
    S2 = dict(S)
    S2["ru"] = S["ru"] + 7.0
    S2["rv"] = S["rv"] - 3.0
    _, t2 = o.box_filter(S2, 2)
    assert np.abs(t1 - t2).max() <= 1e-12
    for row in t1:
        m = np.array([[row[0], row[3], row[4]], [row[3], row[1], row[5]], [row[4], row[5], row[2]]])
        assert np.linalg.eigvalsh(m).min() >= -1e-12


def test_box_filter_face_restriction_conserves_mass_flux():
    """Coarse face momenta are means over the fine faces they cover, so the
    coarse continuity tendency equals the block mean of the fine one
    (divergence theorem: interior fine faces cancel)."""
    nx, ny, nz, r = 16, 8, 8, 2
    cfg = W.small(name="rest", nx=nx, ny=ny, nz=nz, dx=30.0, dy=20.0, dz=W.uniform_dz(nz, 10.0))
    o = oracle.Oracle(cfg)
    th0 = W.theta_sounding(cfg)
    b = o.init_base_state(th0, cfg.p_surface)
    rng = np.random.default_rng(16)
    S = W.initial_state(cfg, b["rho0"], th0)
    sh = S["rho"].shape
    S["ru"] = rng.normal(size=sh)
    S["rv"] = rng.normal(size=sh)
    rw = rng.normal(size=S["rw"].shape)
    rw[0] = rw[-1] = 0
    S["rw"] = rw
    S = {k: np.ascontiguousarray(v) for k, v in S.items()}
    Cst, _ = o.box_filter(S, r)
    cc = W.small(name="rest", nx=nx // r, ny=ny // r, nz=nz // r, dx=60.0, dy=40.0, dz=W.uniform_dz(nz // r, 20.0))
    oc = oracle.Oracle(cc)
    oc.init_base_state(th0.reshape(-1, r).mean(1), cfg.p_surface)
    Cst["rq"] = np.zeros((0,) + Cst["rho"].shape)
    Rf = o.slow_rhs(S)["rho"]
    Rc = oc.slow_rhs(Cst)["rho"]
    Rf_mean = Rf.reshape(nz // r, r, ny // r, r, nx // r, r).mean(axis=(1, 3, 5))
    assert np.abs(Rc - Rf_mean).max() <= 1e-13 * np.abs(Rf).max()


def test_box_filter_adds_fine_smagorinsky_stress():
    """Uniform shear u = gamma z: the resolved part of tau_11 is the variance of
    u over the block, gamma^2 dz^2 (r^2 - 1) / 12; the fine Smagorinsky stress
    adds tau_13 = -(Cs Delta)^2 gamma |gamma| away from the lids."""
    nx, ny, nz, r = 8, 8, 16, 4
    dx, dz, Cs, gam = 10.0, 10.0, 0.17, 0.02
    cfg, o = _grid(nx=nx, ny=ny, nz=nz, dx=dx, dy=dx, dzv=dz)
    k = np.arange(nz)
    u = (gam * (k + 0.5) * dz)[:, None, None]
    S = _unit_rho_state(cfg, u=u)
    _, t0 = o.box_filter(S, r)
    _, t1 = o.box_filter(S, r, Cs=Cs)
    t0 = t0.reshape(nz // r, ny // r, nx // r, 9)
    t1 = t1.reshape(nz // r, ny // r, nx // r, 9)
    assert np.allclose(t0[..., 0], gam ** 2 * dz ** 2 * (r * r - 1) / 12, rtol=1e-12)
    assert np.abs(t0[..., 4]).max() <= 1e-15
    inner = t1[1:-1, ..., 4]
    assert np.allclose(inner, -(Cs * dx) ** 2 * gam * abs(gam), rtol=1e-12)
    assert np.allclose(t1[..., 0], t0[..., 0], rtol=1e-12)   # deviatoric S11 = 0


# -- closure right-hand side --------------------------------------------------------------
def _rest_setup(nx=12, ny=10, nz=8):
    cfg = W.small(name="rest", nx=nx, ny=ny, nz=nz, dx=30.0, dy=20.0, dz=W.uniform_dz(nz, 10.0),
                  sgs=2, Cs=0.17, adv_order_h=3, adv_order_v=3, dt=0.05)
    o = oracle.Oracle(cfg)
    th0 = W.theta_sounding(cfg)
    b = o.init_base_state(th0, cfg.p_surface)
    o0 = oracle.Oracle(cfg.replace(sgs=0))
    o0.init_base_state(th0, cfg.p_surface)
    return cfg, o, o0, b, th0


def test_zero_network_equals_no_closure():
    """A network with all parameters zero and zero output mean gives zero
    stresses: the right-hand side and a full RK3 step are bitwise those
    without any closure."""
    cfg, o, o0, b, th0 = _rest_setup()
    S = W.initial_state(cfg.replace(name="bubble"), b["rho0"], th0)
    rng = np.random.default_rng(17)
    S["ru"] = S["ru"] + rng.normal(size=S["ru"].shape)
    S = {k: np.ascontiguousarray(v) for k, v in S.items()}
    R, nfb = o.slow_rhs_mlp(S, _zero_params(), _norm_identity())
    R0 = o0.slow_rhs(S)
    assert nfb == 0
    for f in ("rho", "rt", "ru", "rv", "rw"):
        assert np.array_equal(R[f], R0[f]), f
    o.set_mlp(_zero_params(), _norm_identity())
    S1 = {k: v.copy() for k, v in S.items()}
    S2 = {k: v.copy() for k, v in S.items()}
    o.rk3_step(S1)
    o0.rk3_step(S2)
    for f in ("rho", "rt", "ru", "rv", "rw"):
        assert np.all(np.isfinite(S1[f])) and np.array_equal(S1[f], S2[f]), f


def test_constant_closure_output_divergence_closed_form():
    """Constant network output t and rest state with rho varying along x only:
    the stresses rho t act through rho differences alone.  Face and edge values
    are 2- and 4-cell means, so R_U gains -t11 (rho_i - rho_{i-1}) / dx, R_V and
    R_W gain -t12 and -t13 times the centred difference (rho_{i+1} - rho_{i-1}) /
    (2 dx), R_Theta gains -q1 times it; next to the lids the zero edge values of
    tau_13, tau_23 and the zero heat flux leave -(mean rho) t / dz."""
    nx, ny, nz = 12, 10, 8
    cfg, o, o0, b, th0 = _rest_setup(nx, ny, nz)
    rng = np.random.default_rng(18)
    rho1 = 1.0 + 0.1 * rng.normal(size=nx)
    S = {"rho": np.ascontiguousarray(np.broadcast_to(rho1[None, None, :], (nz, ny, nx))),
         "rt": np.ascontiguousarray(np.broadcast_to(300.0 * rho1[None, None, :], (nz, ny, nx))),
         "ru": np.zeros((nz, ny, nx)), "rv": np.zeros((nz, ny, nx)), "rw": np.zeros((nz + 1, ny, nx)),
         "rq": np.zeros((0, nz, ny, nx))}
    t = np.array([0.3, -0.2, 0.5, 0.7, -0.4, 0.6, 0.25, -0.15, 0.35])
    p = _zero_params()
    _view(p)["b4"][:] = t
    R, nfb = o.slow_rhs_mlp(S, p, _norm_identity())
    R0 = o0.slow_rhs(S)
    assert nfb == 0
    d = {f: R[f] - R0[f] for f in ("rho", "rt", "ru", "rv", "rw")}
    dx, dz = cfg.dx, cfg.dz[0]
    back = rho1 - np.roll(rho1, 1)
    cen = (np.roll(rho1, -1) - np.roll(rho1, 1)) / 2
    rbx = 0.5 * (rho1 + np.roll(rho1, 1))     # rho at x-faces
    eu = np.broadcast_to(-t[0] * back / dx, (nz, ny, nx)).copy()
    eu[0] -= t[4] * rbx / dz
    eu[-1] += t[4] * rbx / dz
    ev = np.broadcast_to(-t[3] * cen / dx, (nz, ny, nx)).copy()
    ev[0] -= t[5] * rho1 / dz
    ev[-1] += t[5] * rho1 / dz
    ew = np.zeros((nz + 1, ny, nx))
    ew[1:-1] = -t[4] * cen / dx
    et = np.broadcast_to(-t[6] * cen / dx, (nz, ny, nx)).copy()
    et[0] -= t[8] * rho1 / dz
    et[-1] += t[8] * rho1 / dz
    for f, e in (("ru", eu), ("rv", ev), ("rw", ew), ("rt", et)):
        # the difference R - R0 carries the rounding of R0's own terms
        tol = 16 * np.finfo(float).eps * (np.abs(R0[f]).max() + np.abs(e).max())
        assert np.abs(d[f] - e).max() <= tol, f
    assert np.all(d["rho"] == 0)


def test_fallback_on_nonfinite_and_backscatter_threshold():
    """Shear flow u = gamma z with output tau_13 = c constant: the energy
    transfer -tau:S is -c gamma, the Smagorinsky dissipation
    (Cs Delta)^2 |gamma|^3 inside the domain; next to a lid the edge mean holds
    half the shear, so the transfer halves and the dissipation falls 8x.
    A cell falls back when -c gamma < -2 (Cs Delta)^2 |gamma|^3, and always on a
    non-finite output."""
    nx, ny, nz = 8, 6, 10
    cfg, o, o0, b, th0 = _rest_setup(nx, ny, nz)
    gam, dz = 0.05, cfg.dz[0]
    k = np.arange(nz)
    u = np.broadcast_to((gam * (k + 0.5) * dz)[:, None, None], (nz, ny, nx))
    S = {"rho": np.ones((nz, ny, nx)), "rt": np.full((nz, ny, nx), 300.0), "ru": np.ascontiguousarray(u),
         "rv": np.zeros((nz, ny, nx)), "rw": np.zeros((nz + 1, ny, nx)), "rq": np.zeros((0, nz, ny, nx))}
    delta = (cfg.dx * cfg.dy * dz) ** (1 / 3)
    thr_in = 2 * (cfg.Cs * delta) ** 2 * abs(gam) ** 3 / gam
    thr_lid = thr_in / 4   # next to a lid: S_13 and the transfer halve, |S|^3 falls 8x
    ncol = nx * ny
    for c, expect in ((0.99 * thr_lid, 0), (1.01 * thr_lid, 2 * ncol), (0.99 * thr_in, 2 * ncol),
                      (1.01 * thr_in, nz * ncol)):
        p = _zero_params()
        _view(p)["b4"][4] = c
        _, nfb = o.slow_rhs_mlp(S, p, _norm_identity())
        assert nfb == expect, (c, nfb, expect)
    p = _zero_params()
    _view(p)["b4"][2] = np.nan
    R, nfb = o.slow_rhs_mlp(S, p, _norm_identity())
    assert nfb == nz * ncol
    assert np.all(np.isfinite(R["ru"]))
