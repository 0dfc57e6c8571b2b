"""Host checks of the synthetic input generators (no GPU)."""
import numpy as np

from paper_2405_13409_amd import scenes


def test_tiled_points_are_a_permutation_in_pixel_tiles():
    """The 16 x 16 tile order holds the same points as the row-major grid, and
    every 256 consecutive points form one 16 x 16 pixel tile (the cull's tile
    test relies on consecutive points being close)."""
    n, tile = 64, 16
    rows = scenes.points_grid(n, -1.0, 1.0, 2.0)
    tiled = scenes.points_grid(n, -1.0, 1.0, 2.0, tile)
    assert tiled.shape == rows.shape
    key = lambda P: np.lexsort((P[:, 0], P[:, 1]))  # noqa: E731
    assert np.array_equal(rows[key(rows)], tiled[key(tiled)])
    step = 2.0 / n
    for b in range(0, n * n, tile * tile):
        blk = tiled[b: b + tile * tile]
        assert np.isclose(np.ptp(blk[:, 0]), (tile - 1) * step)
        assert np.isclose(np.ptp(blk[:, 1]), (tile - 1) * step)
        assert len(np.unique(blk[:, :2], axis=0)) == tile * tile
    # the first tile is the lower-left corner, row-major inside
    assert np.allclose(tiled[1] - tiled[0], [step, 0.0, 0.0])
    assert np.allclose(tiled[tile] - tiled[0], [0.0, step, 0.0])


def test_glints_points_default_to_tiles():
    P = scenes.glints_large_points("R")
    assert P.shape == (65536, 3)
    assert np.all(P[:, 2] == 2.0)
    assert np.isclose(np.ptp(P[:256, 0]), 15 * 2.0 / 256) and np.isclose(np.ptp(P[:256, 1]), 15 * 2.0 / 256)
