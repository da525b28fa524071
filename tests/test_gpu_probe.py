"""The device probes behind the bench's measured peaks: every rate lands
below and near the figures derived from MI355X's unit counts and clock
(256 CUs x 64 lanes x 2 lane-ops per clock x 2.4 GHz of 32-bit ops; 256
B/clk/CU of LDS reads), and bad arguments are refused."""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DERIVED_OPS = 256 * 64 * 2 * 2.4e9
DERIVED_LDS = 256 * 256 * 2.4e9


@pytest.fixture(scope="module")
def sps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_02328_amd import sps as mod
    mod.library()
    return mod


def test_probe_rates_plausible(sps):
    p = sps.sps_probe_peaks(0)
    print(" ".join(f"{k} {v:.4e}" for k, v in p.items()))
    # two-operand adds come close to the full rate; three-operand ops issue
    # at half of it
    assert 0.6 * DERIVED_OPS < p["valu_add_ops_per_s"] < 1.05 * DERIVED_OPS
    for k in ("valu_add3_ops_per_s", "valu_perm_ops_per_s"):
        assert 0.3 * DERIVED_OPS < p[k] < 0.55 * DERIVED_OPS, k
    assert 0.5 * DERIVED_LDS < p["lds_read_bytes_per_s"] < 1.05 * DERIVED_LDS
    # 4-byte reads move at most as much per clock as 16-byte ones
    assert 0.2 * DERIVED_LDS < p["lds_read32_bytes_per_s"] <= 1.05 * p["lds_read_bytes_per_s"]


def test_probe_rejects_missing_device(sps):
    with pytest.raises(sps.SpsError) as ei:
        sps.sps_probe_peaks(torch.cuda.device_count() + 3)
    assert ei.value.name == "SPS_ERR_INVALID_ARG"
