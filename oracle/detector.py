"""Plain CPU oracle of the learned candidate detector.

TEST INFRASTRUCTURE, NOT PRODUCT CODE: only the tests, the smoke check and
the benchmark's CPU-baseline leg may import this module.  It shares nothing
with the GPU library.

What it computes (numpy, float64 arithmetic, with the rounding points of the
mixed-precision method made explicit):

* ``pool_tiles``: the boxcar S/N plane max-pooled over windows of
  POOL_DM trials x POOL_T samples, multiplied by a scale in binary32 and
  rounded to bfloat16 (round to nearest, ties to even).  Only full windows.
* ``forward``: six 3x3 convolutions (zero padding 1; strides 2,2,2,2,2,1;
  channels 1->16->32->64->128->128->128), each followed by ReLU, then a
  1x1 head with 3 outputs per cell of the final 8 x 16 grid: objectness
  logit, DM offset and time offset inside the cell.  Weights of the 3x3
  layers are used rounded to bfloat16 and each layer's ReLU output is
  rounded to bfloat16 (the precision activations are stored in); sums are
  exact here (float64).  The head runs on float values.
* ``loss``: per cell, binary cross-entropy of the objectness logit against
  the cell's label, positives weighted by POS_WEIGHT, averaged over the
  cells; plus, at positive cells, the squared error of the two offsets
  times LAMBDA_BOX; averaged over the batch.
* ``backward``: the gradient of that loss, with the back-propagated signal
  rounded to bfloat16 at the input of every 3x3 layer (where it is stored
  for the matrix-core products) and the ReLU derivative taken from the
  stored activations (a > 0).
* ``adam``: Adam with bias correction (Kingma and Ba, 2015).

``exact=True`` removes every bfloat16 rounding: forward and backward are
then the exact function and its exact gradient (pinned by finite
differences).
"""
from __future__ import annotations

import numpy as np

TILE_DM, TILE_T = 256, 512          # pooled tile: 256 trial rows x 512 samples
POOL_DM, POOL_T = 2, 8              # pooling window over the S/N plane
LAYERS = ((1, 16, 2), (16, 32, 2), (32, 64, 2), (64, 128, 2), (128, 128, 2), (128, 128, 1))
GRID_DM, GRID_T = 8, 16             # output cells
CELL_DM, CELL_T = TILE_DM // GRID_DM, TILE_T // GRID_T
NHEAD = 3
POS_WEIGHT = 32.0
LAMBDA_BOX = 1.0


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) via binary32; float64 result."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x) -> np.ndarray:
    """The bfloat16 encodings (uint16) of values already representable in bfloat16."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32)
    assert np.all(u & 0xFFFF == 0), "value not representable in bfloat16"
    return (u >> 16).astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def pool_tiles(snr: np.ndarray, scale: float) -> np.ndarray:
    """[ndm][nout] binary32 S/N -> bfloat16 values [ndm/POOL_DM][nout/POOL_T] (float64)."""
    snr = np.asarray(snr, dtype=np.float32)
    nd, nt = snr.shape[0] // POOL_DM, snr.shape[1] // POOL_T
    out = np.empty((nd, nt), dtype=np.float32)
    for i in range(nd):
        blk = snr[i * POOL_DM:(i + 1) * POOL_DM, :nt * POOL_T]
        out[i] = blk.reshape(POOL_DM, nt, POOL_T).max(axis=(0, 2))
    return bf16(out * np.float32(scale))


def out_size(n: int, stride: int) -> int:
    return (n + 2 - 3) // stride + 1


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int) -> np.ndarray:
    """x [n][ci][h][w], w [co][ci][3][3], zero padding 1 -> [n][co][ho][wo]."""
    n, ci, h, wd = x.shape
    ho, wo = out_size(h, stride), out_size(wd, stride)
    xp = np.zeros((n, ci, h + 2, wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    out = np.zeros((n, w.shape[0], ho, wo)) + np.asarray(b, dtype=np.float64)[None, :, None, None]
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + stride * (ho - 1) + 1:stride, kx:kx + stride * (wo - 1) + 1:stride]
            out += np.einsum("oc,nchw->nohw", w[:, :, ky, kx], patch)
    return out


def conv3x3_backward(x: np.ndarray, w: np.ndarray, dout: np.ndarray, stride: int):
    """Gradients of conv3x3 w.r.t. x, w and b for the upstream gradient dout."""
    n, ci, h, wd = x.shape
    ho, wo = dout.shape[2], dout.shape[3]
    xp = np.zeros((n, ci, h + 2, wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros(w.shape)
    for ky in range(3):
        for kx in range(3):
            sy = slice(ky, ky + stride * (ho - 1) + 1, stride)
            sx = slice(kx, kx + stride * (wo - 1) + 1, stride)
            dw[:, :, ky, kx] = np.einsum("nohw,nchw->oc", dout, xp[:, :, sy, sx])
            dxp[:, :, sy, sx] += np.einsum("oc,nohw->nchw", w[:, :, ky, kx], dout)
    db = dout.sum(axis=(0, 2, 3))
    return dxp[:, :, 1:-1, 1:-1], dw, db


def init_params(seed: int) -> dict:
    """He-normal 3x3 weights, zero biases, head weights N(0, 1/128), head
    biases (-4, 0.5, 0.5), drawn by the shared seeded input generator."""
    from sps_inputs.synth import seeded_weights
    specs = []
    for i, (ci, co, _) in enumerate(LAYERS):
        specs += [(f"w{i}", (co, ci, 3, 3), np.sqrt(2.0 / (9 * ci))), (f"b{i}", (co,), 0.0)]
    specs += [("wh", (NHEAD, LAYERS[-1][1]), np.sqrt(1.0 / LAYERS[-1][1])), ("bh", (NHEAD,), 0.0)]
    p = seeded_weights(seed, specs)
    p["bh"] = np.array([-4.0, 0.5, 0.5], np.float32)
    return p


def param_names() -> list:
    return [f"{k}{i}" for i in range(len(LAYERS)) for k in ("w", "b")] + ["wh", "bh"]


def forward(params: dict, tiles: np.ndarray, exact: bool = False):
    """tiles [n][TILE_DM][TILE_T] -> (head [n][3][GRID_DM][GRID_T], activations)."""
    r = (lambda v: v) if exact else bf16
    a = np.asarray(tiles, dtype=np.float64)[:, None]
    acts = [a]
    for i, (_, _, s) in enumerate(LAYERS):
        z = conv3x3(a, r(params[f"w{i}"]), params[f"b{i}"], s)
        a = r(np.maximum(z, 0.0))
        acts.append(a)
    wh = np.asarray(params["wh"], dtype=np.float64)
    head = np.einsum("kc,nchw->nkhw", wh, a) + np.asarray(params["bh"], np.float64)[None, :, None, None]
    return head, acts


def labels_for(n: int, pulses) -> np.ndarray:
    """Targets [n][3][GRID_DM][GRID_T] from pulse positions in pooled-tile
    coordinates: pulses[i] = (row, col) or None.  The cell holding the pulse
    gets objectness 1 and the pulse's fractional position inside the cell."""
    y = np.zeros((n, NHEAD, GRID_DM, GRID_T))
    for i, p in enumerate(pulses):
        if p is None:
            continue
        row, col = p
        gy, gx = int(row // CELL_DM), int(col // CELL_T)
        if 0 <= gy < GRID_DM and 0 <= gx < GRID_T:
            y[i, 0, gy, gx] = 1.0
            y[i, 1, gy, gx] = row / CELL_DM - gy
            y[i, 2, gy, gx] = col / CELL_T - gx
    return y


def loss(head: np.ndarray, y: np.ndarray, pos_weight: float = POS_WEIGHT,
         lambda_box: float = LAMBDA_BOX) -> float:
    o = head[:, 0]
    pos = y[:, 0]
    wgt = np.where(pos > 0, pos_weight, 1.0)
    bce = np.maximum(o, 0.0) - pos * o + np.log1p(np.exp(-np.abs(o)))
    ncell = GRID_DM * GRID_T
    box = ((head[:, 1] - y[:, 1]) ** 2 + (head[:, 2] - y[:, 2]) ** 2) * pos
    per_tile = (wgt * bce).sum(axis=(1, 2)) / ncell + lambda_box * box.sum(axis=(1, 2))
    return float(per_tile.mean())


def loss_grad_head(head: np.ndarray, y: np.ndarray, pos_weight: float = POS_WEIGHT,
                   lambda_box: float = LAMBDA_BOX) -> np.ndarray:
    n = head.shape[0]
    o = head[:, 0]
    pos = y[:, 0]
    wgt = np.where(pos > 0, pos_weight, 1.0)
    g = np.zeros_like(head)
    g[:, 0] = wgt * (1.0 / (1.0 + np.exp(-o)) - pos) / (GRID_DM * GRID_T) / n
    g[:, 1] = 2.0 * lambda_box * (head[:, 1] - y[:, 1]) * pos / n
    g[:, 2] = 2.0 * lambda_box * (head[:, 2] - y[:, 2]) * pos / n
    return g


def backward(params: dict, tiles: np.ndarray, y: np.ndarray, exact: bool = False):
    """(loss, gradients dict) of the mean loss over the batch."""
    r = (lambda v: v) if exact else bf16
    head, acts = forward(params, tiles, exact)
    L = loss(head, y)
    gh = loss_grad_head(head, y)
    a6 = acts[-1]
    grads = {"wh": np.einsum("nkhw,nchw->kc", gh, a6), "bh": gh.sum(axis=(0, 2, 3))}
    da = np.einsum("kc,nkhw->nchw", np.asarray(params["wh"], np.float64), gh)
    for i in range(len(LAYERS) - 1, -1, -1):
        dz = r(da * (acts[i + 1] > 0))
        dx, dw, db = conv3x3_backward(acts[i], r(params[f"w{i}"]), dz, LAYERS[i][2])
        grads[f"w{i}"], grads[f"b{i}"] = dw, db
        da = dx
    return L, grads


def adam(params: dict, grads: dict, state: dict, lr: float, b1: float = 0.9,
         b2: float = 0.999, eps: float = 1e-8) -> dict:
    """One Adam step on float64 copies; state holds m, v (per name) and t."""
    t = state.get("t", 0) + 1
    out = {}
    for k, g in grads.items():
        m = b1 * state.get("m_" + k, 0.0) + (1.0 - b1) * g
        v = b2 * state.get("v_" + k, 0.0) + (1.0 - b2) * g * g
        state["m_" + k], state["v_" + k] = m, v
        mhat = m / (1.0 - b1 ** t)
        vhat = v / (1.0 - b2 ** t)
        out[k] = np.asarray(params[k], np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    state["t"] = t
    return out
