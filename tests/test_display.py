"""The display pyramid's oracle (pinned by hand-worked cases) and the
library's pyramidal tiled TIFF writer (host code), read back by an
independent parser.  CPU only."""
import numpy as np
import pytest

from oracle import display
from tests import tiff_read


def test_quantise_by_hand():
    v = np.array([0.0, 1.0, 0.5, -3.0, 2.0, np.nan, np.inf, -np.inf, 1.0 / 255.0, 0.25], np.float32)
    # 0.5 * 255 + 1/2 = 128 exactly; 0.25 * 255 + 1/2 = 64.25 -> 64; an FP32
    # 1/255 times 255 lies within 2^-24 of 1, so + 1/2 floors to 1
    assert display.quantise(v).tolist() == [0, 255, 128, 0, 255, 0, 255, 0, 1, 64]


def test_halve_by_hand():
    # 2x2 checkerboard of 0 / 255: (510 + 2) // 4 = 128 in every channel
    cb = np.zeros((2, 2, 4), np.uint8)
    cb[0, 0] = cb[1, 1] = 255
    assert display.halve(cb).tolist() == [[[128] * 4]]
    # 3 x 3: the last column and row average 2 pixels (round half up), the
    # corner copies its single pixel
    lv = np.arange(9 * 4, dtype=np.uint8).reshape(3, 3, 4)
    out = display.halve(lv)
    assert out.shape == (2, 2, 4)
    for c in range(4):
        a = [lv[0, 0, c], lv[0, 1, c], lv[1, 0, c], lv[1, 1, c]]
        assert out[0, 0, c] == (sum(int(x) for x in a) + 2) // 4
        assert out[0, 1, c] == (int(lv[0, 2, c]) + int(lv[1, 2, c]) + 1) // 2
        assert out[1, 0, c] == (int(lv[2, 0, c]) + int(lv[2, 1, c]) + 1) // 2
        assert out[1, 1, c] == lv[2, 2, c]


def test_pyramid_levels_and_constant_image():
    img = np.full((600, 1000, 4), 0.5, np.float32)
    lv = display.pyramid(img, tile=128)
    assert [x.shape[:2] for x in lv] == [(600, 1000), (300, 500), (150, 250), (75, 125)]
    for x in lv:
        assert (x == 128).all()
    assert len(display.pyramid(np.zeros((100, 128, 4), np.float32), tile=128)) == 1


def test_pixel_matches_whole_levels():
    rng = np.random.default_rng(3)
    img = rng.uniform(-0.2, 1.2, (37, 53, 4)).astype(np.float32)
    lv = display.pyramid(img, tile=16)
    for level in range(len(lv)):
        h, w = lv[level].shape[:2]
        for (y, x) in [(0, 0), (h - 1, w - 1), (h // 2, w // 3)]:
            assert np.array_equal(display.pixel(img, level, x, y), lv[level][y, x])


@pytest.mark.parametrize("bigtiff", [False, True])
@pytest.mark.parametrize("w,h,tile", [(700, 300, 128), (16, 16, 16), (513, 1, 64)])
def test_tiff_writer_round_trip(tmp_path, w, h, tile, bigtiff):
    from paper_1012_2909_amd import vr
    rng = np.random.default_rng(w + h)
    img = rng.uniform(0, 1, (h, w, 4)).astype(np.float32)
    lv = display.pyramid(img, tile=tile)
    buf = np.concatenate([x.reshape(-1) for x in lv])
    assert buf.size == vr.lib().vr_pyramid_bytes(w, h, tile, None)
    path = tmp_path / "p.tif"
    vr.write_pyramid_tiff(str(path), buf, w, h, tile, bigtiff=bigtiff)
    got = tiff_read.read(str(path))
    assert got["bigtiff"] == bigtiff
    assert len(got["levels"]) == len(lv)
    for k, (g, ref) in enumerate(zip(got["levels"], lv)):
        t = g["tags"]
        assert t[254] == [0 if k == 0 else 1]
        assert (t[256][0], t[257][0]) == (ref.shape[1], ref.shape[0])
        assert t[258] == [8, 8, 8, 8] and t[259] == [1] and t[262] == [2] and t[277] == [4]
        assert t[284] == [1] and t[322] == [tile] and t[323] == [tile] and t[338] == [1]
        assert np.array_equal(g["image"], ref)


def test_tiff_writer_rejects_bad_arguments(tmp_path):
    from paper_1012_2909_amd import vr
    buf = np.zeros(16 * 16 * 4, np.uint8)
    for args in ((0, 16, 16), (16, 16, 24), (16, 16, 8)):
        with pytest.raises(vr.VRError):
            vr.write_pyramid_tiff(str(tmp_path / "x.tif"), buf, *args)
    with pytest.raises(vr.VRError):
        vr.write_pyramid_tiff(str(tmp_path / "no_such_dir" / "x.tif"), buf, 16, 16, 16)
