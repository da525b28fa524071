"""GPU checks of the detector's training-set factory: the tiles are the
oracle's pooling of the library's own S/N planes, the labels sit where the
injected pulses are, and pulses the boxcar search reports are strong in the
tiles."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402

pytestmark = pytest.mark.gpu

cnn = oracle.cnn()


@pytest.fixture(scope="module")
def factory():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_02328_amd import detector
    fac = detector.TileFactory(batch=8)
    yield fac
    fac.close()


def test_tiles_labels_and_search(factory):
    from paper_2511_02328_amd import detector
    tiles, labels, meta = factory.make(12, seed=5)   # one full and one ragged batch
    tb = cnn.from_bf16_bits(tiles.cpu().numpy().view(np.uint16))
    # the last batch's planes are still in the factory: pooling is the oracle's
    snr = factory.snr[:4].cpu().numpy()
    for i in range(4):
        assert np.array_equal(tb[8 + i], cnn.pool_tiles(snr[i], detector.TILE_SCALE))
    lab = labels.cpu().numpy()
    pos = meta["positive"]
    assert 0 < pos.sum() < 12
    assert np.array_equal(lab[:, 0].sum(axis=(1, 2)) > 0, pos)
    for j in np.flatnonzero(pos):
        gy, gx = np.argwhere(lab[j, 0] > 0)[0]
        assert int(meta["row"][j] // 32) == gy and int(meta["col"][j] // 32) == gx
        assert 0 <= lab[j, 1, gy, gx] < 1 and 0 <= lab[j, 2, gy, gx] < 1
        r, c = int(meta["row"][j]), int(meta["col"][j])
        assert abs(meta["d_star"][j] - 2 * meta["row"][j]) < 1e-9
        if meta["pulse_snr"][j] >= 15:
            # the tile is bright near the pulse (S/N / 8 after pooling)
            win = tb[j, max(0, r - 4):r + 5, max(0, c - 12):c + 5]
            assert win.max() >= 0.8 * meta["pulse_snr"][j] / 8, (j, win.max(), meta["pulse_snr"][j])
            assert meta["boxcar_hit"][j]
    assert np.all(meta["plane_max_snr"] >= np.nan_to_num(meta["pulse_snr"]) - 1e-3)
