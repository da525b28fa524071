"""The oracle's pins are sensitive: each plausible mistake planted in a copy
of the oracle source (built to a temporary library, on the CPU) must make at
least one pin test fail.  The real oracle is never modified."""
import os
import subprocess
import sys

import pytest

from oracle.build import SRC, build

HERE = os.path.dirname(os.path.abspath(__file__))
PIN_FILES = ["test_oracle_delays.py", "test_oracle_dedisperse.py",
             "test_oracle_stats_boxcar.py", "test_oracle_detect.py", "test_oracle_subband.py"]

MUTATIONS = {
    "truncate_instead_of_round": ("floor(x + 0.5)", "floor(x)"),
    "one_over_f_not_f_squared": ("1.0 / (f * f)", "1.0 / f"),
    "ms_reading_of_K": ("ORACLE_K_DM = 4.148808e3", "ORACLE_K_DM = 4.148808"),
    "reads_past_nsamp_in": ("if (idx < nsamp_in) acc[t]", "if (idx <= nsamp_in) acc[t]"),
    "transposed_delay_index": ("D[(int64_t)d * nchan + c];\n      for (int64_t t = 0; t < nout; ++t) {",
                               "D[(int64_t)c * ndm + d];\n      for (int64_t t = 0; t < nout; ++t) {"),
    "upper_median": ("int64_t k = (nout - 1) / 2;", "int64_t k = nout / 2;"),
    "no_mad_scale": ("ORACLE_MAD_TO_SIGMA = 1.4826", "ORACLE_MAD_TO_SIGMA = 1.0"),
    "w_not_sqrt_w": ("(sigma * sqrt((double)w))", "(sigma * (double)w)"),
    "largest_width_on_tie": ("best_i == 0xFF || f > best_f", "best_i == 0xFF || f >= best_f"),
    "partial_window": ("if (t + w > nout) break;", "if (t + w > nout + 1) break;"),
    "tile_tie_last": ("best_p.t < 0 || v > best_p.snr", "best_p.t < 0 || v >= best_p.snr"),
    "strict_nms_radius": ("if (dd <= nms_dm && dt <= nms_t)", "if (dd < nms_dm && dt <= nms_t)"),
    "order_ignores_t": ("if (p->t != q->t) return p->t < q->t ? -1 : 1;", ""),
    "checksum_no_clamp": ("if (hi > nsamp_in) hi = nsamp_in;", ""),
    "residual_full_dm": ("(ORACLE_K_DM * (dm_m - dm_j) / tsamp_s)", "(ORACLE_K_DM * dm_m / tsamp_s)"),
    "subband_top_channel_centre": ("double inv_f2 = acc / (double)(sub[s + 1] - sub[s]);",
                                   "double inv_f2 = 1.0 / (freq_mhz[sub[s]] * freq_mhz[sub[s]]);"),
    "stage2_wrong_subband": ("t + R[(int64_t)m * nsub + s]]", "t + R[(int64_t)m * nsub + (nsub - 1 - s)]]"),
    "stage1_no_bounds": ("if (u + shift < nsamp_in) row[u]", "if (u + shift <= nsamp_in) row[u]"),
    "zero_dm_truncating_mean": ("(sum + nchan / 2) / nchan", "sum / nchan"),
    "downsample_ties_down": ("while (r > 0 && (2 * r - 1) * (2 * r - 1) * (int64_t)factor > 4 * V * S) --r;",
                             "while (r > 0 && (2 * r - 1) * (2 * r - 1) * (int64_t)factor >= 4 * V * S) --r;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert old in src, "mutation site vanished: update the mutation list"
    msrc = tmp_path / "mutant.c"
    msrc.write_text(src.replace(old, new, 1))
    lib = build(str(msrc), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, SPS_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *[os.path.join(HERE, f) for f in PIN_FILES]],
                       env=env, capture_output=True, text=True, cwd=os.path.dirname(HERE))
    assert r.returncode == 1, f"mutation {name} not caught:\n{r.stdout[-2000:]}"
