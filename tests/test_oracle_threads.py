"""The oracle's threaded raster and resolve give the sequential results bit for
bit: the raster takes each pixel's minimum by compare-and-swap, so the buffer
(a minimum over covering segments) cannot depend on the order in which threads
meet a pixel, and the resolve's pixels are independent.  The whole-frame GPU
parity tests and the all-cores CPU baseline rely on this."""
import numpy as np
import pytest

from paper_2607_04230_amd import scenes


def _cases():
    tiny = scenes.config_tiny()
    small = scenes.config_head(width=320, height=180)
    batched = scenes.config_batched(n_scenes=3, res=96, n_max=4e3)
    return [("tiny", tiny), ("head_320x180", small), ("batched_3", batched)]


@pytest.mark.parametrize("name,sc", _cases(), ids=lambda x: x if isinstance(x, str) else "")
def test_threaded_oracle_equals_sequential(O, name, sc):
    one = O.render(sc)
    many = O.render(sc, n_threads=8)
    assert np.array_equal(one["vis"], many["vis"])
    assert np.array_equal(one["out"], many["out"])


def test_threaded_raster_with_windows_and_occluder(O):
    sc = scenes.config_head(width=256, height=144)
    table, soff, (ns, ncp) = O.lod_select(sc)
    pos, rgb, fl = O.generate(sc, table, ncp)
    for win in (None, (40, 30, 150, 100)):
        ref = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z,
                       window=win)
        with O.threads(6):
            got = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z,
                           window=win)
        assert np.array_equal(ref, got)
    assert O.lib().orc_get_threads() == 1
