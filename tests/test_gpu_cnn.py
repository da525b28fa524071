"""GPU parity of the learned detector (BF16 MFMA kernels through the C ABI)
against the detector oracle: pooling bit-exact; activations, head outputs,
loss and gradients within the bounds that FP32-versus-exact accumulation
before each bfloat16 rounding allows; Adam to FP32 rounding."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402

pytestmark = pytest.mark.gpu

cnn = oracle.cnn()


@pytest.fixture(scope="module")
def sps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_02328_amd import sps as mod
    mod.library()
    return mod


def _flat(params):
    return np.concatenate([np.asarray(params[k], np.float32).ravel() for k in cnn.param_names()])


def _unflat(vec, like):
    out, o = {}, 0
    for k in cnn.param_names():
        n = like[k].size
        out[k] = vec[o:o + n].reshape(like[k].shape)
        o += n
    return out


def _tiles(n, seed, positive=()):
    rng = np.random.Generator(np.random.PCG64(seed))
    t = rng.normal(0.2, 0.6, (n, cnn.TILE_DM, cnn.TILE_T))
    pulses = [None] * n
    for i in positive:
        r, c = rng.uniform(8, cnn.TILE_DM - 8), rng.uniform(8, cnn.TILE_T - 8)
        pulses[i] = (r, c)
        t[i, int(r) - 2:int(r) + 3, int(c) - 3:int(c) + 4] += 4.0
    tb = cnn.bf16(t)
    return tb, cnn.labels_for(n, pulses)


def _to_dev_tiles(tb):
    bits = cnn.bf16_bits(tb).view(np.int16)
    return torch.from_numpy(np.ascontiguousarray(bits)).cuda()


def _bf_ulp_diff(g_bits, o_vals):
    """|g - o| in units of the oracle value's bfloat16 spacing."""
    g = cnn.from_bf16_bits(g_bits)
    o = np.asarray(o_vals, np.float64)
    e = np.floor(np.log2(np.maximum(np.abs(o), 2.0 ** -126)))
    return np.abs(g - o) / 2.0 ** (e - 7), g


def test_pool_tiles_bitexact(sps):
    rng = np.random.Generator(np.random.PCG64(1))
    for nd, nt, pitch in ((512, 4096, 4096), (37, 101, 128), (2, 8, 8)):
        snr = rng.normal(0, 3, (nd, pitch)).astype(np.float32)
        snr[rng.random((nd, pitch)) < 0.01] = 0.0
        want = cnn.pool_tiles(snr[:, :nt], 0.125)
        s = torch.from_numpy(snr).cuda()
        out = torch.zeros((nd // 2, nt // 8), dtype=torch.int16, device="cuda")
        sps.sps_cnn_pool_tiles(s, nt, 0.125, out)
        torch.cuda.synchronize()
        got = cnn.from_bf16_bits(out.cpu().numpy().view(np.uint16))
        assert np.array_equal(got, want), (nd, nt)


@pytest.fixture(scope="module")
def case(sps):
    params = cnn.init_params(11)
    params["bh"] = np.array([-1.0, 0.3, 0.6], np.float32)
    for i in range(len(cnn.LAYERS)):
        params[f"b{i}"] = np.linspace(-0.05, 0.05, cnn.LAYERS[i][1]).astype(np.float32)
    tb, y = _tiles(3, 12, positive=(0, 2))
    return params, tb, y


def test_forward_layers_and_head(sps, case):
    params, tb, y = case
    n = tb.shape[0]
    head_o, acts_o = cnn.forward(params, tb)
    with sps.sps_cnn_create(4) as net:
        sps.sps_cnn_set_params(net, _flat(params))
        T = _to_dev_tiles(tb)
        head = torch.zeros((n, 3, 8, 16), dtype=torch.float32, device="cuda")
        sps.sps_cnn_forward(net, T, n, head)
        torch.cuda.synchronize()
        for li in range(len(cnn.LAYERS)):
            g = sps.sps_cnn_activations(net, li, n)
            o = np.transpose(acts_o[li + 1], (0, 2, 3, 1))  # NCHW -> NHWC
            ulps, gv = _bf_ulp_diff(g, o)
            same = np.mean(gv == o)
            # a rounding decision can differ only where the FP32 sum lies within
            # its accumulation error of a bfloat16 rounding boundary
            assert same >= 0.99, (li, same)
            assert np.all((ulps <= 2.0) | (np.abs(gv - o) <= 1e-2 * np.abs(o).max())), li
        h = head.cpu().numpy().astype(np.float64)
        err = np.abs(h - head_o)
        assert err.max() <= 1e-2 * np.abs(head_o).max() + 1e-4, err.max()


def test_loss_and_gradients(sps, case):
    params, tb, y = case
    n = tb.shape[0]
    L_o, g_o = cnn.backward(params, tb, y)
    with sps.sps_cnn_create(4) as net:
        sps.sps_cnn_set_params(net, _flat(params))
        T = _to_dev_tiles(tb)
        Y = torch.from_numpy(y.astype(np.float32)).cuda()
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        sps.sps_cnn_loss_grad(net, T, Y, n, loss)
        torch.cuda.synchronize()
        L_g = float(loss.cpu()[0])
        g_g = _unflat(sps.sps_cnn_get_grads(net), g_o)
    assert abs(L_g - L_o) <= 1e-4 * abs(L_o), (L_g, L_o)
    for k in cnn.param_names():
        a, b = g_g[k].astype(np.float64), g_o[k]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert rel <= 2e-2, (k, rel)
        # the sign pattern of the large entries agrees
        big = np.abs(b) > 0.1 * np.abs(b).max()
        assert np.mean(np.sign(a[big]) == np.sign(b[big])) >= 0.99, k


def test_adam_matches_oracle(sps):
    rng = np.random.Generator(np.random.PCG64(21))
    params = cnn.init_params(21)
    flat = _flat(params)
    with sps.sps_cnn_create(1) as net:
        sps.sps_cnn_set_params(net, flat)
        st = {}
        cur = {k: v.astype(np.float64) for k, v in params.items()}
        for step, lr in enumerate((1e-3, 3e-4, 1e-3)):
            g = {k: (rng.normal(size=v.shape) * 10.0 ** rng.integers(-7, 0, v.shape)) for k, v in
                 params.items()}
            sps.sps_cnn_set_grads(net, _flat(g))
            sps.sps_cnn_adam(net, lr)
            cur = cnn.adam(cur, g, st, lr)
            got = _unflat(sps.sps_cnn_get_params(net), params)
            for k in cnn.param_names():
                d = np.abs(got[k] - cur[k])
                assert np.all(d <= 2e-6 * np.abs(cur[k]) + 2e-3 * lr), (step, k, d.max())


def test_training_reduces_loss_and_detect(sps):
    params = cnn.init_params(31)
    tb, y = _tiles(8, 32, positive=(0, 1, 2, 3))
    with sps.sps_cnn_create(8) as net:
        sps.sps_cnn_set_params(net, _flat(params))
        T = _to_dev_tiles(tb)
        Y = torch.from_numpy(y.astype(np.float32)).cuda()
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        hist = []
        for _ in range(60):
            sps.sps_cnn_train_step(net, T, Y, 8, 2e-3, loss)
            hist.append(float(loss.cpu()[0]))
        assert np.isfinite(hist).all() and hist[-1] < 0.5 * hist[0], hist[::10]
        head = torch.zeros((8, 3, 8, 16), dtype=torch.float32, device="cuda")
        sps.sps_cnn_forward(net, T, 8, head)
        h = head.cpu().numpy()
        cands, nf = sps.sps_cnn_detect(net, T, 8, 0.5)
        want = np.argwhere(h[:, 0] >= 0.0)
        assert nf == len(want) == len(cands)
        assert [tuple(x) for x in want] == list(zip(cands["tile"], cands["cell_dm"], cands["cell_t"]))
        for c in cands:
            assert abs(c["prob"] - 1 / (1 + np.exp(-h[c["tile"], 0, c["cell_dm"], c["cell_t"]]))) < 1e-6
        # the trained net finds the labelled cells of the positive tiles
        lab = np.argwhere(y[:, 0] > 0)
        found = {(int(a), int(b), int(c)) for a, b, c in want}
        assert sum((int(a), int(b), int(c)) in found for a, b, c in lab) >= 3


def test_argument_errors(sps):
    with sps.sps_cnn_create(2) as net:
        T = torch.zeros((3, 256, 512), dtype=torch.int16, device="cuda")
        with pytest.raises(sps.SpsError):
            sps.sps_cnn_forward(net, T, 3)  # above max_batch
        with pytest.raises(sps.SpsError):
            sps.sps_cnn_adam(net, -1.0)
        with pytest.raises(ValueError):
            sps.sps_cnn_set_params(net, np.zeros(10, np.float32))
    with pytest.raises(sps.SpsError):
        sps.sps_cnn_create(0)
