"""Pins for the detector oracle (oracle/detector.py), each fixed by something other
than the oracle itself: torch's bfloat16 conversion, brute-force pooling,
scipy's 2-D correlation, adjoint identities and finite differences of the
exact network, closed forms of the loss and of Adam, and a hand-evaluated
"delta network" whose every rounding point is written out in the test.
The slow finite-difference pin runs last."""
import math

import numpy as np
import pytest
import torch
from scipy.signal import correlate2d

import oracle

cnn = oracle.cnn()


def t_bf16(x):
    """bfloat16 rounding by torch (an independent implementation)."""
    return torch.tensor(np.asarray(x, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def test_bf16_rounding():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -3.14159, 1e-3, 65504.0,
                     0.0, -0.0, 2 ** -130, 3.0e38], np.float64)
    got = cnn.bf16(vals)
    assert got[1] == 1.0 and got[2] == 1 + 2 ** -6 and got[3] == 1 + 2 ** -7
    rng = np.random.Generator(np.random.PCG64(1))
    r = np.concatenate([vals, rng.normal(0, 10, 5000), rng.normal(0, 1e-5, 1000)])
    assert np.array_equal(cnn.bf16(r), t_bf16(r))
    bits = cnn.bf16_bits(cnn.bf16(r))
    assert np.array_equal(cnn.from_bf16_bits(bits), cnn.bf16(r))


def test_pool_tiles_brute_force():
    rng = np.random.Generator(np.random.PCG64(2))
    snr = rng.normal(0, 3, (11, 77)).astype(np.float32)
    scale = 0.125
    got = cnn.pool_tiles(snr, scale)
    assert got.shape == (5, 9)
    for i in range(5):
        for j in range(9):
            m = max(float(snr[a, b]) for a in range(2 * i, 2 * i + 2) for b in range(8 * j, 8 * j + 8))
            assert got[i, j] == t_bf16(np.float32(m) * np.float32(scale))


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_against_scipy(stride):
    rng = np.random.Generator(np.random.PCG64(3 + stride))
    x = rng.normal(size=(2, 3, 7, 10))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    got = cnn.conv3x3(x, w, b, stride)
    assert got.shape == (2, 4, cnn.out_size(7, stride), cnn.out_size(10, stride))
    for n in range(2):
        for o in range(4):
            ref = sum(correlate2d(x[n, c], w[o, c], mode="same") for c in range(3))[::stride, ::stride]
            assert np.allclose(got[n, o], ref + b[o], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_backward_adjoint(stride):
    # conv is linear in x and in w: <conv(x, w), g> = <x, dx> = <w, dw>; db = sum g
    rng = np.random.Generator(np.random.PCG64(7 + stride))
    x = rng.normal(size=(3, 5, 9, 8))
    w = rng.normal(size=(6, 5, 3, 3))
    y = cnn.conv3x3(x, w, np.zeros(6), stride)
    g = rng.normal(size=y.shape)
    dx, dw, db = cnn.conv3x3_backward(x, w, g, stride)
    lhs = float((y * g).sum())
    assert math.isclose(lhs, float((x * dx).sum()), rel_tol=1e-10)
    assert math.isclose(lhs, float((w * dw).sum()), rel_tol=1e-10)
    assert np.allclose(db, g.sum(axis=(0, 2, 3)))
    # and entry by entry against brute force on one gradient component
    e = np.zeros_like(g)
    e[1, 2, 3, 1] = 1.0
    dx1, dw1, _ = cnn.conv3x3_backward(x, w, e, stride)
    for c in range(5):
        for ky in range(3):
            for kx in range(3):
                yy, xx = stride * 3 + ky - 1, stride * 1 + kx - 1
                want = x[1, c, yy, xx] if 0 <= yy < 9 and 0 <= xx < 8 else 0.0
                assert math.isclose(dw1[2, c, ky, kx], want, abs_tol=1e-15)


def _batch(n, seed, positive=(0,)):
    rng = np.random.Generator(np.random.PCG64(seed))
    tiles = np.abs(rng.normal(0, 0.3, (n, cnn.TILE_DM, cnn.TILE_T)))
    pulses = [None] * n
    for i in positive:
        r, c = rng.uniform(0, cnn.TILE_DM), rng.uniform(0, cnn.TILE_T)
        pulses[i] = (r, c)
        tiles[i, int(r), max(0, int(c) - 2):int(c) + 3] += 3.0
    return tiles, cnn.labels_for(n, pulses)


def test_loss_closed_forms():
    n = 3
    head = np.zeros((n, 3, cnn.GRID_DM, cnn.GRID_T))
    y = np.zeros_like(head)
    assert math.isclose(cnn.loss(head, y), math.log(2), rel_tol=1e-14)
    y[1, 0, 2, 5], y[1, 1, 2, 5], y[1, 2, 2, 5] = 1.0, 0.25, 0.75
    ncell = cnn.GRID_DM * cnn.GRID_T
    want_1 = math.log(2) * (ncell - 1 + cnn.POS_WEIGHT) / ncell + cnn.LAMBDA_BOX * (0.25 ** 2 + 0.75 ** 2)
    assert math.isclose(cnn.loss(head, y), (2 * math.log(2) + want_1) / n, rel_tol=1e-14)
    # large logits: BCE -> |o| on the wrong side, 0 on the right side
    head[:, 0] = -50.0
    head[1, 0, 2, 5] = 50.0
    head[1, 1, 2, 5], head[1, 2, 2, 5] = 0.25, 0.75
    assert cnn.loss(head, y) < 1e-20
    g = cnn.loss_grad_head(np.zeros_like(head), y)
    assert math.isclose(g[0, 0, 0, 0], 0.5 / ncell / n)
    assert math.isclose(g[1, 0, 2, 5], -0.5 * cnn.POS_WEIGHT / ncell / n)
    assert math.isclose(g[1, 1, 2, 5], -2 * 0.25 / n)


def test_labels():
    y = cnn.labels_for(2, [(40.0, 100.0), None])
    assert y[0, 0].sum() == 1 and y[0, 0, 1, 3] == 1.0
    assert math.isclose(y[0, 1, 1, 3], 40 / 32 - 1) and math.isclose(y[0, 2, 1, 3], 100 / 32 - 3)
    assert not y[1].any()


def test_adam_closed_forms():
    rng = np.random.Generator(np.random.PCG64(9))
    p = {"a": rng.normal(size=50)}
    g = {"a": rng.normal(size=50) * 10.0 ** rng.integers(-6, 2, 50)}
    st = {}
    lr, eps = 1e-3, 1e-8
    out = cnn.adam(p, g, st, lr, eps=eps)
    # step 1: m_hat = g, v_hat = g^2
    assert np.allclose(out["a"], p["a"] - lr * g["a"] / (np.abs(g["a"]) + eps), rtol=1e-12, atol=0)
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    cur = out
    for _ in range(9):
        cur = cnn.adam(cur, g, st, lr, eps=eps)
    assert st["t"] == 10
    assert np.allclose(cur["a"], p["a"] - 10 * lr * g["a"] / (np.abs(g["a"]) + eps),
                       rtol=1e-10, atol=1e-16)


def _delta_params(c, wh0, bh):
    p = {}
    for i, (ci, co, _) in enumerate(cnn.LAYERS):
        w = np.zeros((co, ci, 3, 3))
        w[0, 0, 1, 1] = c[i]
        p[f"w{i}"], p[f"b{i}"] = w, np.zeros(co)
    p["wh"] = np.zeros((3, cnn.LAYERS[-1][1]))
    p["wh"][:, 0] = wh0
    p["bh"] = np.asarray(bh, np.float64)
    return p


def test_delta_network_forward_and_backward_by_hand():
    # every 3x3 layer passes channel 0 through its centre tap times c_i, so
    # cell (gy, gx) sees input sample (32 gy, 32 gx) through a chain whose
    # roundings are evaluated here one by one (torch's bfloat16)
    c = [1 + 2 ** -8 + 2 ** -10, 1.5, 0.7, 1.1, 1.3, 0.9]   # c0 is not a bfloat16 value
    wh0, bh = [0.8, 0.3, -0.6], [-1.0, 0.1, 0.2]
    p = _delta_params(c, wh0, bh)
    rng = np.random.Generator(np.random.PCG64(10))
    tiles = t_bf16(rng.uniform(-1, 3, (1, cnn.TILE_DM, cnn.TILE_T)))
    pr = (40.0, 100.0)  # positive cell (1, 3)
    y = cnn.labels_for(1, [pr])
    head, acts = cnn.forward(p, tiles)
    cb = [float(t_bf16(v)) for v in c]
    assert cb[0] != c[0]
    assert np.count_nonzero(head[0, 0] != bh[0]) > 60  # most chains carry signal
    chain = np.zeros((cnn.GRID_DM, cnn.GRID_T, 7))
    for gy in range(cnn.GRID_DM):
        for gx in range(cnn.GRID_T):
            v = tiles[0, 32 * gy, 32 * gx]
            chain[gy, gx, 0] = v
            for i in range(6):
                v = float(t_bf16(max(cb[i] * v, 0.0)))
                chain[gy, gx, i + 1] = v
            for k in range(3):
                assert math.isclose(head[0, k, gy, gx], wh0[k] * v + bh[k], rel_tol=1e-15,
                                    abs_tol=1e-15)
    # backward: the signal reaching layer 6 is wh[:,0] . dL/dhead at each cell
    L, g = cnn.backward(p, tiles, y)
    ncell = cnn.GRID_DM * cnn.GRID_T
    gw = np.zeros(6)
    for gy in range(cnn.GRID_DM):
        for gx in range(cnn.GRID_T):
            pos = y[0, 0, gy, gx]
            o = head[0, 0, gy, gx]
            gh = [(cnn.POS_WEIGHT if pos else 1.0) * (1 / (1 + math.exp(-o)) - pos) / ncell,
                  2 * (head[0, 1, gy, gx] - y[0, 1, gy, gx]) * pos,
                  2 * (head[0, 2, gy, gx] - y[0, 2, gy, gx]) * pos]
            d = sum(wh0[k] * gh[k] for k in range(3))
            for i in range(5, -1, -1):
                dz = float(t_bf16(d * (chain[gy, gx, i + 1] > 0)))
                gw[i] += dz * chain[gy, gx, i]
                d = cb[i] * dz
    for i in range(6):
        assert gw[i] != 0.0
        assert math.isclose(g[f"w{i}"][0, 0, 1, 1], gw[i], rel_tol=1e-12, abs_tol=1e-18), i
    assert math.isclose(g["bh"][0], sum(
        (cnn.POS_WEIGHT if y[0, 0, a, b] else 1.0) * (1 / (1 + math.exp(-head[0, 0, a, b])) -
                                                      y[0, 0, a, b]) / ncell
        for a in range(cnn.GRID_DM) for b in range(cnn.GRID_T)), rel_tol=1e-12)


def test_gradient_finite_differences():
    params = {k: v.astype(np.float64) for k, v in cnn.init_params(5).items()}
    params["bh"] = np.array([0.3, 0.1, -0.2])
    tiles, y = _batch(1, 6)
    L, g = cnn.backward(params, tiles, y, exact=True)
    assert math.isclose(L, cnn.loss(cnn.forward(params, tiles, exact=True)[0], y), rel_tol=1e-14)
    rng = np.random.Generator(np.random.PCG64(8))
    h = 1e-6  # small enough that no ReLU kink is crossed in practice
    for name in cnn.param_names():
        # the largest gradient entry and two random non-zero ones
        nz = np.flatnonzero(g[name])
        assert nz.size > 0, name
        flat = [int(np.argmax(np.abs(g[name])))] + [int(x) for x in rng.choice(nz, 1)]
        for f in flat:
            idx = np.unravel_index(f, params[name].shape)
            p2 = {k: v.copy() for k, v in params.items()}
            p2[name][idx] += h
            lp = cnn.loss(cnn.forward(p2, tiles, exact=True)[0], y)
            p2[name][idx] -= 2 * h
            lm = cnn.loss(cnn.forward(p2, tiles, exact=True)[0], y)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-5 * abs(fd) + 2e-9, (name, idx, fd, g[name][idx])
