"""CPU check of the two-steps-per-launch schedule of the 2D channel kernel
(k_pair2d): the mapping of workgroups to tiles, the LDS ring of step-t rows
and the LDS wall partials, emulated with the kernel's own index arithmetic.

For every tile the emulation replays the sweep: the rows that the first phase
writes into the ring, then every ring read of the second phase (each velocity's
pull source, rows clamped into the channel as in the kernel) must find exactly
the row it wants in the slot it reads, every LDS index must stay inside its
array, every wall row of the second phase must find the partials of all the
wall rows of its face, and the tiles' second phases must cover every node of
the channel exactly once."""
import itertools

import pytest

LDS_BUDGET = 156 * 1024


def tile_shape(V, H, HN, elem):
    def nbytes(bx, rr):
        return (rr + 2 * HN) * (bx + 2 * H) * V * elem + 2 * HN * bx * 8

    bx = 64 if nbytes(64, 8) <= LDS_BUDGET else 32
    if nbytes(bx, 16) <= LDS_BUDGET and 16 * (bx + 2 * H) <= 1024:
        rr = 16
    elif nbytes(bx, 8) <= LDS_BUDGET:
        rr = 8
    elif nbytes(bx, 4) <= LDS_BUDGET:
        rr = 4
    else:
        rr = 2
    return bx, rr


def grid_of(nx, ny, bx, rr, band_rows, cus=256):
    nstrips = (nx + bx - 1) // bx
    if band_rows <= 0:
        bands = max(1, min(ny, (cus + nstrips - 1) // nstrips))
        band_rows = (ny + bands - 1) // bands
        band_rows = (band_rows + rr - 1) // rr * rr
    bands = (ny + band_rows - 1) // band_rows
    return nstrips, bands, band_rows


def emulate(nx, ny, V, H, HN, elem, band_rows):
    bx, rr = tile_shape(V, H, HN, elem)
    ew, ring_rows = bx + 2 * H, rr + 2 * HN
    nstrips, bands, band_rows = grid_of(nx, ny, bx, rr, band_rows)
    total = nstrips * bands
    seen_tiles = set()
    owned = {}
    for wg in range(total):
        xcd, q = wg & 7, wg >> 3
        lin = xcd * (total >> 3) + min(xcd, total & 7) + q
        assert 0 <= lin < total
        seen_tiles.add(lin)
        strip, band = lin % nstrips, lin // nstrips
        x0 = strip * bx
        ncols = min(bx, nx - x0)
        y0 = band * band_rows
        y1 = min(y0 + band_rows, ny)
        a = max(y0 - HN, 0)
        slot_row = [None] * ring_rows
        partial_rows = set()
        ready = a
        lo = y0
        while lo < y1:
            hi = min(lo + rr, y1)
            need = min(hi + HN, ny)
            # first phase: rows [ready, need), columns 0 .. ncols + 2H - 1
            assert need - ready <= ring_rows
            for j in range(ready, need):
                assert 0 <= j < ny
                slot = (j - a) % ring_rows
                slot_row[slot] = j
                top = (slot * V + (V - 1)) * ew + (ncols + 2 * H - 1)
                assert top < ring_rows * V * ew
                if j < HN:
                    partial_rows.add((0, j))
                if j >= ny - HN:
                    partial_rows.add((1, ny - 1 - j))
            ready = need
            # second phase: rows [lo, hi), own columns
            for j in range(lo, hi):
                for ey in range(-HN, HN + 1):
                    jr = min(max(j - ey, 0), ny - 1)
                    slot = (jr - a) % ring_rows
                    assert slot_row[slot] == jr, (nx, ny, wg, j, ey)
                for il in range(ncols):
                    for ex in range(-H, H + 1):
                        col = il + H - ex
                        assert 0 <= col < ncols + 2 * H <= ew
                    key = (j, x0 + il)
                    assert key not in owned
                    owned[key] = wg
                if j < HN or j >= ny - HN:
                    if j < HN:
                        assert all((0, r) in partial_rows for r in range(HN))
                    if j >= ny - HN:
                        assert all((1, r) in partial_rows for r in range(HN))
            lo += rr
    assert seen_tiles == set(range(total))
    assert len(owned) == nx * ny


# (V, H, HN, bytes per stored population) of the compiled 2D sets that take
# the two-step kernel: D2V17, D2V37, D2V16, D2V33 in FP64, FP32 and FP16
SETS = [(17, 3, 3), (37, 3, 3), (16, 4, 4), (33, 4, 4)]


@pytest.mark.parametrize("V,H,HN", SETS)
@pytest.mark.parametrize("elem", [8, 4, 2])
def test_tile_fits_lds(V, H, HN, elem):
    bx, rr = tile_shape(V, H, HN, elem)
    assert (rr + 2 * HN) * (bx + 2 * H) * V * elem + 2 * HN * bx * 8 <= LDS_BUDGET


@pytest.mark.parametrize("V,H,HN", SETS)
@pytest.mark.parametrize("elem", [8, 4, 2])
@pytest.mark.parametrize("nx,ny,band_rows", [
    (70, 13, 0), (128, 20, 0), (2, 5, 0), (1, 21, 0), (64, 4, 0), (192, 11, 3),
    (130, 24, 5), (64, 64, 1), (96, 17, 7), (5, 9, 2), (128, 7, 0), (3, 40, 6),
])
def test_pair_schedule_small(V, H, HN, elem, nx, ny, band_rows):
    if ny < HN:
        pytest.skip("ny below the wall-normal reach is rejected by the library")
    emulate(nx, ny, V, H, HN, elem, band_rows)


def test_pair_schedule_benchmark_sizes():
    # the throughput channel and the above-cache channel, D2V37 FP32
    emulate(2048, 512, 37, 3, 3, 4, 0)
    emulate(4096, 64, 37, 3, 3, 4, 0)
    grid = grid_of(4096, 2048, *tile_shape(37, 3, 3, 4), 0)
    assert grid[0] * grid[1] >= 256


def test_every_band_height_at_one_shape():
    for band_rows, elem in itertools.product(range(1, 30), (4, 2)):
        emulate(100, 29, 37, 3, 3, elem, band_rows)
