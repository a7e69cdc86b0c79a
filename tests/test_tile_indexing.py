"""CPU replay of the index arithmetic of the tiled radiation kernels
(paper_1306_0010_amd/csrc/rhd_tile.hpp) for every thread, block and plane: every
global read and write stays inside its buffer, and every output cell is written
exactly once. The replay mirrors the kernels' integer expressions line by line. The
tiled gas kernels (rhd_gas_tile.hpp) use the same grid, tile, ring, halo and z-chunk
expressions with five fields per cell, so the replay covers their indexing too."""
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


def balanced_chunk(L, zc):
    chunks = (L + zc - 1) // zc
    return (L + chunks - 1) // chunks


def ring_rc(e, BY):
    """LDS (row, column) of ring cell e of the corrector's plane buffer."""
    W = BX + 4
    if e < 4 * W:
        q, c = divmod(e, W)
        return (q if q < 2 else BY + q), c
    k = e - 4 * W
    s = k & 3
    return 2 + (k >> 2), (s if s < 2 else BX + s)


def replay(n, bc, BY, zc):
    n0, n1, n2 = n
    N = n0 * n1 * n2
    ps = (n0 + 4, n1 + 4, n2 + 4)
    NP = ps[0] * ps[1] * ps[2]
    padded = lambda x, y, z: (x + 2) + ps[0] * ((y + 2) + ps[1] * (z + 2))
    mapped = lambda x, y, z: (map_index(x, n0, bc[0], bc[1])
                              + n0 * (map_index(y, n1, bc[2], bc[3]) + n1 * map_index(z, n2, bc[4], bc[5])))

    def check_mapped(x, y, z):
        for q, lim in ((x, n0), (y, n1), (z, n2)):
            q = np.asarray(q)
            assert q.min() >= -3 and q.max() <= lim + 2, "boundary mapping defined on [-3, n + 2]"
        a = mapped(x, y, z)
        assert a.min() >= 0 and a.max() < N

    ty, tx = np.meshgrid(np.arange(BY), np.arange(BX), indexing="ij")
    tx, ty = tx.ravel(), ty.ravel()
    ntx = (n0 + BX - 1) // BX
    zcp, zcc = balanced_chunk(n2 + 4, zc), balanced_chunk(n2, zc)
    assert zcp <= zc and zcc <= zc

    # predictor: main tiles and the ghost-column blocks
    writes = np.zeros(NP, dtype=np.int64)
    grid = (ntx + 1, (n1 + 4 + BY - 1) // BY, (n2 + 4 + zcp - 1) // zcp)
    for bz in range(grid[2]):
        for by in range(grid[1]):
            y0 = -2 + by * BY
            z0 = -2 + bz * zcp
            z1 = min(z0 + zcp, n2 + 2)
            for bx in range(grid[0]):
                if bx >= ntx:
                    ylim = min(y0 + BY, n1 + 2)
                    e = np.arange(4 * BY * (z1 - z0))
                    g, r, pl = e & 3, (e >> 2) % BY, (e >> 2) // BY
                    x = np.where(g < 2, g - 2, n0 + g - 2)
                    keep = y0 + r < ylim
                    x, yy, zz = x[keep], (y0 + r)[keep], (z0 + pl)[keep]
                    if x.size:
                        for dx, dy, dz in ((0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0),
                                           (0, 0, -1), (0, 0, 1)):
                            check_mapped(x + dx, yy + dy, zz + dz)
                        np.add.at(writes, padded(x, yy, zz), 1)
                    continue
                x0 = bx * BX
                x, y = x0 + tx, y0 + ty
                xl, yl = np.minimum(x, n0 + 2), np.minimum(y, n1 + 2)
                out_xy = (x < n0) & (y < n1 + 2)
                # a closure that feeds a face of an output cell is never clamped
                need = (x <= n0) & (y <= n1 + 2)
                assert np.array_equal(xl[need], x[need]) and np.array_equal(yl[need], y[need])
                # extra items: wave 0 brings the y data of row y0 - 1, wave 1 that of row
                # y0 + BY, lanes < 2 BY of wave 2 the x data of cells x0 - 1 and x0 + 64;
                # lanes 0 and 63 of every row store their own x data
                hrole = np.where(ty == 0, 1, np.where(ty == 1, 2, np.where((ty == 2) & (tx < 2 * BY), 3, 0)))
                hrow = tx % BY
                hx = np.where(hrole == 3, np.where(tx < BY, x0 - 1, np.minimum(x0 + BX, n0 + 2)), xl)
                hy = np.where(hrole == 1, y0 - 1,
                              np.where(hrole == 2, min(y0 + BY, n1 + 2), np.minimum(y0 + hrow, n1 + 2)))
                slots = sorted([("sy", 0, int(c)) for c in tx[hrole == 1]]
                               + [("sy", BY + 1, int(c)) for c in tx[hrole == 2]]
                               + [("sxe", int(r), 0 if t < BY else 3)
                                  for r, t in zip(hrow[hrole == 3], tx[hrole == 3])]
                               + [("sxe", int(r), 1 if t == 0 else 2)
                                  for r, t in zip(ty, tx) if t == 0 or t == BX - 1])
                # every LDS slot of the halo and row-end data is written once per plane
                assert slots == sorted([("sxe", r, k) for r in range(BY) for k in range(4)]
                                       + [("sy", 0, c) for c in range(BX)] + [("sy", BY + 1, c) for c in range(BX)])
                # the row-end x faces: lanes < 2 BY of wave 0, face k of row lane mod BY
                ends = sorted((int(t % BY), 0 if t < BY else 1) for t in tx[(ty == 0) & (tx < 2 * BY)])
                assert ends == sorted((r, k) for r in range(BY) for k in range(2))
                live = hrole > 0
                for t in range(z0 - 1, z1 + 1):
                    check_mapped(xl, yl, t)
                    if t > z0:
                        check_mapped(x[out_xy], y[out_xy], t - 1)
                        p = padded(x[out_xy], y[out_xy], t - 1)
                        np.add.at(writes, p, 1)
                    if z0 <= t < z1:
                        check_mapped(hx[live], hy[live], t)
    assert np.all(writes == 1), "predictor writes each padded cell once"

    # corrector
    writes = np.zeros(N, dtype=np.int64)
    grid = (ntx, (n1 + BY - 1) // BY, (n2 + zcc - 1) // zcc)
    W = BX + 4
    ring_cells = 4 * W + 4 * BY
    slots = np.zeros((BY + 4) * W, dtype=np.int64)
    for e in range(ring_cells):
        r, c = ring_rc(e, BY)
        slots[r * W + c] += 1
    slots[((ty + 2) * W + tx + 2)] += 1
    assert np.all(slots == 1), "ring and interior fill every LDS slot of a plane once"
    for bz in range(grid[2]):
        for by in range(grid[1]):
            for bx in range(grid[0]):
                x0, y0 = bx * BX, by * BY
                x, y = x0 + tx, y0 + ty
                out_xy = (x < n0) & (y < n1)
                z0 = bz * zcc
                z1 = min(z0 + zcc, n2)
                xl, yl = np.clip(x, -2, n0 + 1), np.clip(y, -2, n1 + 1)
                need = (x <= n0) & (y <= n1)
                assert np.array_equal(xl[need], x[need]) and np.array_equal(yl[need], y[need])
                ring = [ring_rc(e, BY) for e in range(ring_cells)]
                gx = np.clip(np.array([x0 - 2 + c for r, c in ring]), -2, n0 + 1)
                gy = np.clip(np.array([y0 - 2 + r for r, c in ring]), -2, n1 + 1)
                for t in range(z0 - 2, z1 + 2):
                    p = padded(xl, yl, t)
                    assert p.min() >= 0 and p.max() < NP, (t, z0, z1)
                for t in range(z0, z1):
                    p = padded(gx, gy, t)
                    assert p.min() >= 0 and p.max() < NP
                for t in range(z0 + 1, z1 + 1):
                    a = x[out_xy] + n0 * (y[out_xy] + n1 * (t - 1))
                    np.add.at(writes, a, 1)
    assert np.all(writes == 1), "corrector writes each interior cell once"


@pytest.mark.parametrize("n,bc", [
    ((37, 29, 21), (0, 0, 0, 0, 0, 0)),
    ((70, 9, 10), (1, 1, 1, 1, 1, 1)),
    ((24, 20, 18), (1, 1, 0, 0, 2, 2)),
    ((3, 3, 3), (2, 2, 2, 2, 2, 2)),
    ((2, 5, 2), (0, 0, 1, 1, 0, 0)),
    ((128, 17, 33), (0, 0, 2, 2, 1, 1)),
    ((64, 16, 9), (2, 2, 1, 1, 0, 0)),
    ((130, 4, 3), (1, 1, 0, 0, 2, 2)),
])
@pytest.mark.parametrize("BY,zc", [(4, 16), (8, 16), (16, 5), (8, 1), (4, 7), (4, 11), (16, 64)])
def test_tiled_kernel_indexing(n, bc, BY, zc):
    replay(n, bc, BY, zc)


def xcd_tile(L, N):
    """The kernels' XCD-aware renumbering of block L of a launch of N blocks."""
    j, k, q, r = L & 7, L >> 3, N >> 3, N & 7
    return j * q + min(j, r) + k


@pytest.mark.parametrize("N", [1, 2, 7, 8, 9, 15, 16, 17, 63, 64, 65, 867, 2805, 4096, 10007])
def test_xcd_tile_order_is_a_permutation(N):
    T = [xcd_tile(L, N) for L in range(N)]
    assert sorted(T) == list(range(N))
    # every XCD (L mod 8) gets one contiguous range of tiles, in order
    for j in range(8):
        mine = T[j::8]
        assert mine == list(range(mine[0], mine[0] + len(mine))) if mine else True
