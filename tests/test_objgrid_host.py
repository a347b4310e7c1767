"""The offset-grid guarantee the resting-object grids rely on (Appendix G:
four regular grids, cells at least 4x the largest sphere radius, offset so
that any query sphere lies wholly inside one cell of one of them), for the
library's cell (0.5 m), offsets (0 or half a cell on each axis) and the
paper's largest radius (12 cm) up to a quarter cell."""
import numpy as np

CELL = 0.5


def inside_some_grid(x, y, r):
    for g in range(4):
        ox, oy = (g & 1) * CELL / 2, (g >> 1) * CELL / 2
        lx = (x - ox) % CELL
        ly = (y - oy) % CELL
        if lx >= r and CELL - lx >= r and ly >= r and CELL - ly >= r:
            return True
    return False


def test_every_sphere_fits_one_cell():
    rng = np.random.default_rng(0)
    for r in (0.015, 0.05, 0.12, CELL / 4):
        pts = rng.uniform(-20, 20, size=(20000, 2))
        # and the hardest places: cell corners and edge midpoints of every grid
        k = np.arange(-4, 5) * (CELL / 2)
        grid = np.stack(np.meshgrid(k, k), -1).reshape(-1, 2)
        for x, y in np.concatenate([pts, grid, grid + 1e-7]):
            assert inside_some_grid(x, y, r), (x, y, r)


def test_a_wider_sphere_can_fit_none():
    """Past a quarter cell the guarantee ends (the kernel then tests every
    object): a sphere at a point a quarter cell from all borders."""
    assert not inside_some_grid(CELL / 4, CELL / 4, CELL / 4 + 1e-3)
