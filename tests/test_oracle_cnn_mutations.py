"""The detector oracle's pins are sensitive: each plausible mistake planted in
a copy of oracle/detector.py must make at least one pin in
test_oracle_cnn.py fail.  The real oracle is never modified."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "detector.py")

MUTATIONS = {
    "no_weight_rounding": ('z = conv3x3(a, r(params[f"w{i}"]), params[f"b{i}"], s)',
                           'z = conv3x3(a, params[f"w{i}"], params[f"b{i}"], s)'),
    "no_activation_rounding": ("a = r(np.maximum(z, 0.0))", "a = np.maximum(z, 0.0)"),
    "no_gradient_rounding": ("dz = r(da * (acts[i + 1] > 0))", "dz = da * (acts[i + 1] > 0)"),
    "relu_mask_from_layer_input": ("dz = r(da * (acts[i + 1] > 0))", "dz = r(da * (acts[i + 1] >= 0))"),
    "kernel_flipped": ('out += np.einsum("oc,nchw->nohw", w[:, :, ky, kx], patch)',
                       'out += np.einsum("oc,nchw->nohw", w[:, :, 2 - ky, 2 - kx], patch)'),
    "backward_kernel_flipped": ('dxp[:, :, sy, sx] += np.einsum("oc,nohw->nchw", w[:, :, ky, kx], dout)',
                                'dxp[:, :, sy, sx] += np.einsum("oc,nohw->nchw", w[:, :, 2 - ky, 2 - kx], dout)'),
    "bce_sign": ("bce = np.maximum(o, 0.0) - pos * o", "bce = np.maximum(o, 0.0) + pos * o"),
    "grad_drops_pos_weight": ("g[:, 0] = wgt * (1.0 / (1.0 + np.exp(-o)) - pos)",
                              "g[:, 0] = (1.0 / (1.0 + np.exp(-o)) - pos)"),
    "adam_no_bias_correction": ("mhat = m / (1.0 - b1 ** t)", "mhat = m"),
    "adam_eps_inside_sqrt": ("(np.sqrt(vhat) + eps)", "np.sqrt(vhat + eps)"),
    "pool_mean": (".max(axis=(0, 2))", ".mean(axis=(0, 2))"),
    "label_axes_swapped": ("gy, gx = int(row // CELL_DM), int(col // CELL_T)",
                           "gy, gx = int(col // CELL_DM), int(row // CELL_T)"),
    "head_bias_dropped": ('head = np.einsum("kc,nchw->nkhw", wh, a) + np.asarray(params["bh"], np.float64)[None, :, None, None]',
                          'head = np.einsum("kc,nchw->nkhw", wh, a)'),
    "bf16_truncates": ("r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16", "r = (u >> 16) << 16"),
    "padding_shift": ("patch = xp[:, :, ky:ky + stride * (ho - 1) + 1:stride, kx:kx + stride * (wo - 1) + 1:stride]",
                      "patch = xp[:, :, ky:ky + stride * (ho - 1) + 1:stride, 2 - kx:2 - kx + stride * (wo - 1) + 1:stride]"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert old in src, "mutation site vanished: update the mutation list"
    m = tmp_path / "detector_mutant.py"
    m.write_text(src.replace(old, new, 1))
    env = dict(os.environ, SPS_CNN_ORACLE_SRC=str(m))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_oracle_cnn.py")],
                       env=env, capture_output=True, text=True, cwd=os.path.dirname(HERE))
    assert r.returncode == 1, f"mutation {name} not caught:\n{r.stdout[-2000:]}"
