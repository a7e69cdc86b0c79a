"""CPU replay of the index arithmetic of the face-split radiation kernels
(k_rad_predict_fs, k_rad_correct_fs in paper_1306_0010_amd/csrc/rhd_device.hpp) and of
the host launch that sizes them, for every block, lane and role: the roles cover the low
and the high face of each active dimension in the order x, y, z, every padded (predictor)
or interior (corrector) cell is handled by exactly one lane of one block, every read of
the padded half-step arrays stays inside them, and the LDS slots a role writes are the
ones the divergence reads. The replay mirrors the kernels' integer expressions."""
import itertools

import numpy as np
import pytest

FS_LANES = 64
FS_MAX_ROLES = 6


def geometry(n):
    act = [1 if m > 1 else 0 for m in n]
    g = [2 * a for a in act]
    ps = [m + 2 * gg for m, gg in zip(n, g)]
    return act, g, ps


def active_dim(act, s):
    """The kernels' active_dim: the s-th active dimension (2 when none remains)."""
    d = 0
    while d < 2:
        if act[d]:
            if s == 0:
                break
            s -= 1
        d += 1
    return d


def launch(n):
    """Host side: block (64, roles) and the two grid sizes, as enqueue_subcycles sets them."""
    act, g, ps = geometry(n)
    roles = 2 * sum(act)
    NP = ps[0] * ps[1] * ps[2]
    N = n[0] * n[1] * n[2]
    return roles, (NP + FS_LANES - 1) // FS_LANES, (N + FS_LANES - 1) // FS_LANES, NP, N


SHAPES = [(1, 1, 1), (7, 1, 1), (64, 1, 1), (65, 1, 1), (1, 9, 1), (1, 1, 13), (5, 3, 1),
          (64, 2, 1), (3, 1, 70), (1, 17, 19), (9, 5, 4), (64, 3, 3), (31, 33, 2)]


@pytest.mark.parametrize("n", SHAPES)
def test_roles_cover_each_active_face_once_in_order(n):
    act, _, _ = geometry(n)
    roles = 2 * sum(act)
    assert roles <= FS_MAX_ROLES
    seen = [(active_dim(act, r >> 1), r & 1) for r in range(roles)]
    want = [(d, side) for d in range(3) if act[d] for side in (0, 1)]
    assert seen == want
    # face_divergence walks the active dimensions in order and reads slots r, r + 1
    r = 0
    for d in range(3):
        if not act[d]:
            continue
        assert seen[r] == (d, 0) and seen[r + 1] == (d, 1)
        r += 2
    assert r == roles


@pytest.mark.parametrize("n", SHAPES)
def test_predictor_lanes_cover_the_padded_region_once(n):
    act, g, ps = geometry(n)
    roles, gp, _, NP, _ = launch(n)
    if roles == 0:
        pytest.skip("a single cell runs the per-cell kernels")
    hits = np.zeros(NP, dtype=np.int64)
    for b in range(gp):
        for lane in range(FS_LANES):
            pu = b * FS_LANES + lane
            if pu >= NP:
                continue
            q = pu // ps[0]
            i = pu - q * ps[0] - g[0]
            j = q % ps[1] - g[1]
            k = q // ps[1] - g[2]
            assert -g[0] <= i < n[0] + g[0] and -g[1] <= j < n[1] + g[1] and -g[2] <= k < n[2] + g[2]
            # the store goes to padded_cell(i, j, k), which must be the lane's own index
            p = (i + g[0]) + ps[0] * ((j + g[1]) + ps[1] * (k + g[2]))
            assert p == pu
            hits[p] += 1
    assert (hits == 1).all()
    assert gp * FS_LANES < 2 ** 32  # the unsigned lane index cannot wrap


@pytest.mark.parametrize("n", SHAPES)
def test_corrector_lanes_cover_the_interior_once_and_read_inside(n):
    act, g, ps = geometry(n)
    roles, _, gc, NP, N = launch(n)
    if roles == 0:
        pytest.skip("a single cell runs the per-cell kernels")
    hits = np.zeros(N, dtype=np.int64)
    for b in range(gc):
        for lane in range(FS_LANES):
            a = b * FS_LANES + lane
            if a >= N:
                continue
            q = a // n[0]
            i = a - q * n[0]
            j = q % n[1]
            k = q // n[1]
            assert 0 <= i < n[0] and 0 <= j < n[1] and 0 <= k < n[2]
            assert i + n[0] * (j + n[1] * k) == a
            hits[a] += 1
            pc = (i + g[0]) + ps[0] * ((j + g[1]) + ps[1] * (k + g[2]))
            for role in range(roles):
                d = active_dim(act, role >> 1)
                stride = 1 if d == 0 else (ps[0] if d == 1 else ps[0] * ps[1])
                offs = (-1, 1, 2) if role & 1 else (-2, -1, 1)
                for o in (0,) + offs:
                    assert 0 <= pc + o * stride < NP, (n, a, role, o)
                # and the cell read is the neighbour along d, inside the ghost layers
                idx = [i, j, k]
                for o in offs:
                    nb = list(idx)
                    nb[d] += o
                    assert -g[d] <= nb[d] < n[d] + g[d]
    assert (hits == 1).all()


def test_lds_footprint_fits():
    # FaceFluxes<double>: 4 components x 6 roles x 64 lanes x 8 bytes
    assert 4 * FS_MAX_ROLES * FS_LANES * 8 <= 64 * 1024
    for n in SHAPES:
        roles = launch(n)[0]
        assert FS_LANES * roles <= FS_LANES * FS_MAX_ROLES  # within the launch bound


def test_default_switch_keeps_one_d_grids_on_the_per_cell_kernels():
    """The host's default for grids that do not take the tiled kernels: 2D and 3D grids
    (roles >= 4) up to 2^17 cells run the face-split kernels, 1D grids the per-cell ones."""
    limit = 1 << 17

    def default_face_split(n):
        roles, _, _, _, N = launch(n)
        return roles >= 4 and N <= limit

    assert not default_face_split((2048, 1, 1))
    assert default_face_split((280, 80, 1))
    assert default_face_split((32, 32, 32))
    assert not default_face_split((64, 64, 64))
    for nx, ny in itertools.product((1, 2, 300), (1, 437)):
        roles = launch((nx, ny, 1))[0]
        assert default_face_split((nx, ny, 1)) == (roles >= 4 and nx * ny <= limit)
