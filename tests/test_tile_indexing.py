"""CPU replay of the index arithmetic of the tiled radiation kernels
(paper_1306_0010_amd/csrc/rhd_tile.hpp) for every thread, block and plane: every
global read and write stays inside its buffer, and every output cell is written
exactly once. The replay mirrors the kernels' integer expressions line by line."""
import numpy as np
import pytest

BX = 64


def map_index(q, n, lo, hi):
    """Boundary mapping of the kernels (vectorised): returns the source index."""
    q = np.asarray(q)
    out = q.copy()
    low = q < 0
    high = q >= n
    if lo == 0:
        out = np.where(low, np.mod(q, n), out)
    elif lo == 1:
        out = np.where(low, 0, out)
    else:
        out = np.where(low, -1 - q, out)
    if hi == 0:
        out = np.where(high, np.mod(q, n), out)
    elif hi == 1:
        out = np.where(high, n - 1, out)
    else:
        out = np.where(high, 2 * n - 1 - q, out)
    return out


def replay(n, bc, BY, zc):
    n0, n1, n2 = n
    TX, TY = BX - 2, BY - 2
    N = n0 * n1 * n2
    ps = (n0 + 4, n1 + 4, n2 + 4)
    NP = ps[0] * ps[1] * ps[2]
    padded = lambda x, y, z: (x + 2) + ps[0] * ((y + 2) + ps[1] * (z + 2))
    mapped = lambda x, y, z: (map_index(x, n0, bc[0], bc[1])
                              + n0 * (map_index(y, n1, bc[2], bc[3]) + n1 * map_index(z, n2, bc[4], bc[5])))
    ty, tx = np.meshgrid(np.arange(BY), np.arange(BX), indexing="ij")
    tx, ty = tx.ravel(), ty.ravel()

    # predictor
    writes = np.zeros(NP, dtype=np.int64)
    grid = ((n0 + 4 + TX - 1) // TX, (n1 + 4 + TY - 1) // TY, (n2 + 4 + zc - 1) // zc)
    for bz in range(grid[2]):
        for by in range(grid[1]):
            for bx in range(grid[0]):
                x = -2 + bx * TX + tx - 1
                y = -2 + by * TY + ty - 1
                xl = np.minimum(x, n0 + 2)
                yl = np.minimum(y, n1 + 2)
                out_xy = (tx >= 1) & (tx <= TX) & (ty >= 1) & (ty <= TY) & (x < n0 + 2) & (y < n1 + 2)
                z0 = -2 + bz * zc
                z1 = min(z0 + zc, n2 + 2)
                for t in range(z0 - 1, z1 + 1):
                    a = mapped(xl, yl, t)
                    assert a.min() >= 0 and a.max() < N
                    if t > z0:
                        a2 = mapped(xl, yl, t - 1)
                        assert a2.min() >= 0 and a2.max() < N
                        p = padded(x[out_xy], y[out_xy], t - 1)
                        assert p.min() >= 0 and p.max() < NP
                        np.add.at(writes, p, 1)
    region = np.zeros(ps[::-1], dtype=np.int64)
    region[...] = 1
    assert np.array_equal(writes.reshape(ps[::-1]), region), "predictor writes each padded cell once"

    # corrector
    writes = np.zeros(N, dtype=np.int64)
    grid = ((n0 + TX - 1) // TX, (n1 + TY - 1) // TY, (n2 + zc - 1) // zc)
    RX, RY = BX + 2, BY + 2
    for bz in range(grid[2]):
        for by in range(grid[1]):
            for bx in range(grid[0]):
                x0, y0 = bx * TX, by * TY
                x = x0 + tx - 1
                y = y0 + ty - 1
                out_xy = (tx >= 1) & (tx <= TX) & (ty >= 1) & (ty <= TY) & (x < n0) & (y < n1)
                z0 = bz * zc
                z1 = min(z0 + zc, n2)
                xl = np.clip(x, -2, n0 + 1)
                yl = np.clip(y, -2, n1 + 1)
                for t in [z0 - 2, z0 - 1] + list(range(z0, z1 + 2)):
                    p = padded(xl, yl, t)
                    assert p.min() >= 0 and p.max() < NP, (t, z0, z1)
                for t in range(z0 - 1, z1 + 1):
                    idx = np.arange(RX * RY)
                    gx = np.clip(x0 - 2 + idx % RX, -2, n0 + 1)
                    gy = np.clip(y0 - 2 + idx // RX, -2, n1 + 1)
                    p = padded(gx, gy, t)
                    assert p.min() >= 0 and p.max() < NP
                    if t > z0:
                        a = x[out_xy] + n0 * (y[out_xy] + n1 * (t - 1))
                        if a.size:
                            assert a.min() >= 0 and a.max() < N
                        np.add.at(writes, a, 1)
    assert np.all(writes == 1), "corrector writes each interior cell once"


@pytest.mark.parametrize("n,bc", [
    ((37, 29, 21), (0, 0, 0, 0, 0, 0)),
    ((70, 9, 10), (1, 1, 1, 1, 1, 1)),
    ((24, 20, 18), (1, 1, 0, 0, 2, 2)),
    ((3, 3, 3), (2, 2, 2, 2, 2, 2)),
    ((2, 5, 2), (0, 0, 1, 1, 0, 0)),
    ((128, 17, 33), (0, 0, 2, 2, 1, 1)),
])
@pytest.mark.parametrize("BY,zc", [(4, 16), (8, 16), (16, 5), (8, 1)])
def test_tiled_kernel_indexing(n, bc, BY, zc):
    replay(n, bc, BY, zc)
