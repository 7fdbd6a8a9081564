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

import numpy as np
import pytest

LDS_BUDGET = 156 * 1024
ALTERNATE, SPLIT, TWIN = 1, 2, 3     # the kernel's three schedules


def ring_rows(kind, rr, HN):
    return (1 if kind == ALTERNATE else 2) * rr + 2 * HN


def nbytes(V, H, HN, elem, bx, rr, kind):
    return ring_rows(kind, rr, HN) * (bx + 2 * H) * V * elem + 2 * HN * bx * 8


def _up64(x):
    return (x + 63) // 64 * 64


def _threads(H, bx, rr, kind):
    """(producer threads, all groups; consumer threads)"""
    groups = 2 if kind == TWIN else 1
    return groups * _up64(rr * (bx + 2 * H)), (0 if kind == ALTERNATE else _up64(rr * bx))


def max_threads(kind):
    # two producer groups: at most three waves per SIMD, for the register budget
    return 768 if kind == TWIN else 1024


def tile_shape(V, H, HN, elem, kind=ALTERNATE):
    def fits(bx, rr):
        return (nbytes(V, H, HN, elem, bx, rr, kind) <= LDS_BUDGET
                and sum(_threads(H, bx, rr, kind)) <= max_threads(kind))

    bx = 64 if fits(64, {ALTERNATE: 8, SPLIT: 4, TWIN: 3}[kind]) else 32
    for rr in (16, 8, 6, 4):
        if fits(bx, rr):
            return bx, rr
    return bx, (3 if kind == TWIN and fits(bx, 3) else 2)


def threads(V, H, HN, elem, kind):
    bx, rr = tile_shape(V, H, HN, elem, kind)
    return _threads(H, bx, rr, kind)


def grid_of(nx, ny, bx, rr, band_rows, cus=256):
    nstrips = (nx + bx - 1) // bx
    if band_rows <= 0:
        bands = max(1, min(ny, (cus + nstrips - 1) // nstrips))
        band_rows = (ny + bands - 1) // bands
        band_rows = (band_rows + rr - 1) // rr * rr
    bands = (ny + band_rows - 1) // band_rows
    return nstrips, bands, band_rows


def slot_from(sl0, r0, row, ring_rows):
    """The kernel's ring slot of `row` from the slot sl0 of row r0: one
    conditional add and one conditional subtract, valid for
    |row - r0| < ring_rows."""
    assert abs(row - r0) < ring_rows
    x = sl0 + (row - r0)
    x = x + ring_rows if x < 0 else x
    return x - ring_rows if x >= ring_rows else x


def emulate(nx, ny, V, H, HN, elem, band_rows, kind=ALTERNATE):
    """Replays every tile. The split schedule is replayed with the producer as
    far ahead as its waits allow: chunk k + 1 of step t is written before the
    consumer reads chunk k."""
    bx, rr = tile_shape(V, H, HN, elem, kind)
    if (nbytes(V, H, HN, elem, bx, rr, kind) > LDS_BUDGET or H > 4
            or sum(_threads(H, bx, rr, kind)) > max_threads(kind)):
        return False     # not compiled (the library reports LBM_E_UNSUPPORTED)
    pt, ct = threads(V, H, HN, elem, kind)
    assert pt + ct <= max_threads(kind)
    ew, nring = bx + 2 * H, ring_rows(kind, rr, HN)
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
        chunks = (y1 - y0 + rr - 1) // rr
        need = [min(y0 + (k + 1) * rr + HN, y1 + HN, ny) for k in range(chunks)]
        slot_row = [None] * nring
        partial_rows = set()

        def produce(k):
            lo = a if k == 0 else need[k - 1]
            hi = need[k]
            assert hi - lo <= nring
            sl = (lo - a) % nring
            for j in range(lo, hi):
                assert 0 <= j < ny
                slot = slot_from(sl, lo, j, nring)
                assert slot == (j - a) % nring
                slot_row[slot] = j
                top = (slot * V + (V - 1)) * ew + (ncols + 2 * H - 1)
                assert top < nring * V * ew
                if j < HN:
                    partial_rows.add((0, j))
                if j >= ny - HN:
                    partial_rows.add((1, ny - 1 - j))

        def consume(k):
            lo, hi = y0 + k * rr, min(y0 + (k + 1) * rr, y1)
            sl = (lo - a) % nring
            for j in range(lo, hi):
                for ey in range(-HN, HN + 1):
                    jr = min(max(j - ey, 0), ny - 1)
                    slot = slot_from(sl, lo, jr, nring)
                    assert slot_row[slot] == jr, (nx, ny, wg, j, ey)
                for il in range(ncols):
                    for ex in range(-H, H + 1):
                        assert 0 <= il + H - ex < ncols + 2 * H <= ew
                    key = (j, x0 + il)
                    assert key not in owned
                    owned[key] = wg
                if j < HN:
                    assert all((0, r) in partial_rows for r in range(HN))
                if j >= ny - HN:
                    assert all((1, r) in partial_rows for r in range(HN))

        if kind in (SPLIT, TWIN):
            # (TWIN: the other producer group may write chunk k + 1 while
            # chunk k is read, never chunk k + 2: its ring-write wait)
            if chunks:
                produce(0)
            for k in range(chunks):
                if k + 1 < chunks:
                    produce(k + 1)      # allowed once chunk k - 1 is consumed
                consume(k)
        else:
            for k in range(chunks):
                produce(k)
                consume(k)
    assert seen_tiles == set(range(total))
    assert len(owned) == nx * ny
    return True


# (V, H, HN, bytes per stored population) of the compiled 2D sets that take
# the two-step kernel: D2V17, D2V37, D2V16, D2V33 in FP64, FP32 and FP16
SETS = [(17, 3, 3), (37, 3, 3), (16, 4, 4), (33, 4, 4)]


@pytest.mark.parametrize("V,H,HN", SETS)
@pytest.mark.parametrize("elem", [8, 4, 2])
def test_alternate_tile_fits_lds(V, H, HN, elem):
    bx, rr = tile_shape(V, H, HN, elem)
    assert nbytes(V, H, HN, elem, bx, rr, ALTERNATE) <= LDS_BUDGET


@pytest.mark.parametrize("kind", [ALTERNATE, SPLIT, TWIN])
@pytest.mark.parametrize("V,H,HN", SETS)
@pytest.mark.parametrize("elem", [8, 4, 2])
@pytest.mark.parametrize("nx,ny,band_rows", [
    (70, 13, 0), (128, 20, 0), (2, 5, 0), (1, 21, 0), (64, 4, 0), (192, 11, 3),
    (130, 24, 5), (64, 64, 1), (96, 17, 7), (5, 9, 2), (128, 7, 0), (3, 40, 6),
])
def test_pair_schedule_small(V, H, HN, elem, nx, ny, band_rows, kind):
    if ny < HN:
        pytest.skip("ny below the wall-normal reach is rejected by the library")
    emulate(nx, ny, V, H, HN, elem, band_rows, kind)


def test_pair_schedule_benchmark_sizes():
    # the throughput channel and the above-cache channel, D2V37 FP32
    for kind in (ALTERNATE, SPLIT, TWIN):
        assert emulate(2048, 512, 37, 3, 3, 4, 0, kind)
        assert emulate(4096, 64, 37, 3, 3, 4, 0, kind)
        grid = grid_of(4096, 2048, *tile_shape(37, 3, 3, 4, kind), 0)
        assert grid[0] * grid[1] >= 256


def test_every_band_height_at_one_shape():
    for band_rows, elem, kind in itertools.product(range(1, 30), (4, 2), (ALTERNATE, SPLIT, TWIN)):
        emulate(100, 29, 37, 3, 3, elem, band_rows, kind)


def split_schedule_check(chunks, rr, HN, a, y0, y1, ny, PW, CW, rng):
    return _run_model(chunks, rr, HN, a, y0, y1, ny, PW, CW, rng, group_wait=True)


def _run_model(chunks, rr, HN, a, y0, y1, ny, PW, CW, rng, group_wait):
    """One random interleaving of the split schedule's waves, at the level of
    its LDS counters: every producer wave writes part of every row of its chunk
    and every consumer wave reads rows of its chunk. Checks that a consumer
    wave starts reading a chunk only when all its rows are complete in the ring
    and that no producer wave starts writing a slot that an unfinished reader
    still needs. Returns the number of events (the schedule always ends)."""
    nring = 2 * rr + 2 * HN
    need = [min(y0 + (k + 1) * rr + HN, y1 + HN, ny) for k in range(chunks)]
    rows_of = [list(range(a if k == 0 else need[k - 1], need[k])) for k in range(chunks)]
    reads_of = []
    for k in range(chunks):
        lo, hi = y0 + k * rr, min(y0 + (k + 1) * rr, y1)
        reads_of.append(sorted({min(max(j - e, 0), ny - 1) for j in range(lo, hi)
                                for e in range(-HN, HN + 1)}))
    slot = lambda j: (j - a) % nring  # noqa: E731
    content = {}          # slot -> (row, set of producer waves that finished writing it)
    writing = {}          # slot -> set of producer waves writing it now
    reading = {}          # slot -> {(consumer wave): row it needs}
    produced = consumed = 0
    # per-wave program counters: (chunk, stage)
    prog = {("p", w): [0, 0] for w in range(PW)}
    prog.update({("c", w): [0, 0] for w in range(CW)})
    events = 0
    while True:
        ready = []
        for (g, w), (k, st) in prog.items():
            if k >= chunks:
                continue
            if g == "p":
                if st == 0 and (k < 2 or consumed >= CW * (k - 1)):
                    ready.append((g, w))
                elif st in (1, 2) or (st == 3 and (not group_wait or produced >= PW * k)):
                    ready.append((g, w))
            else:
                if st == 0 and produced >= PW * (k + 1):
                    ready.append((g, w))
                elif st in (1, 2) or (st == 3 and (not group_wait or consumed >= CW * k)):
                    ready.append((g, w))
        if not ready:
            break
        g, w = ready[rng.integers(len(ready))]
        k, st = prog[(g, w)]
        events += 1
        if g == "p":
            if st == 0:                       # start writing chunk k
                for j in rows_of[k]:
                    s = slot(j)
                    for cw_, row in reading.get(s, {}).items():
                        assert row == j, ("overwrite while read", k, j, row)
                    writing.setdefault(s, set()).add(w)
                    if content.get(s, (None,))[0] != j:
                        content[s] = (j, set())
            elif st == 1:                     # finish writing
                for j in rows_of[k]:
                    s = slot(j)
                    writing[s].discard(w)
                    content[s][1].add(w)
            elif st == 3:
                produced += 1
            prog[(g, w)] = [k + 1, 0] if st == 3 else [k, st + 1]
        else:
            if st == 0:                       # start reading chunk k
                for j in reads_of[k]:
                    s = slot(j)
                    row, done = content.get(s, (None, set()))
                    assert row == j and len(done) == PW and not writing.get(s), ("stale", k, j)
                    reading.setdefault(s, {})[w] = j
            elif st == 1:
                for j in reads_of[k]:
                    reading[slot(j)].pop(w, None)
            elif st == 3:
                consumed += 1
            prog[(g, w)] = [k + 1, 0] if st == 3 else [k, st + 1]
    assert all(k >= chunks for k, _ in prog.values()), "a wave is stuck"
    return events


@pytest.mark.parametrize("rr,HN,y0,y1,ny,PW,CW", [
    (4, 3, 5, 10, 24, 3, 2), (4, 3, 0, 64, 512, 5, 4), (6, 3, 64, 128, 512, 7, 6),
    (2, 4, 3, 17, 17, 2, 1), (4, 3, 20, 24, 24, 5, 4), (8, 4, 0, 40, 40, 9, 8),
])
def test_split_schedule_random_interleavings(rr, HN, y0, y1, ny, PW, CW):
    rng = np.random.default_rng(rr * 1000 + y0)
    a = max(y0 - HN, 0)
    chunks = (y1 - y0 + rr - 1) // rr
    for _ in range(60):
        split_schedule_check(chunks, rr, HN, a, y0, y1, ny, PW, CW, rng)


def test_split_schedule_check_catches_a_wave_counted_early():
    """The check fails for the counting without the per-chunk wait (a wave may
    count chunk k before the others have counted chunk k - 1), as the first
    version of the kernel did: a planted mistake in the schedule model."""
    rng = np.random.default_rng(1)
    found = False
    for _ in range(200):
        try:
            _split_without_group_wait(3, 4, 3, 2, 5, 10, 24, 3, 2, rng)
        except AssertionError:
            found = True
            break
    assert found


def _split_without_group_wait(chunks, rr, HN, a, y0, y1, ny, PW, CW, rng):
    return _run_model(chunks, rr, HN, a, y0, y1, ny, PW, CW, rng, group_wait=False)


def twin_schedule_check(chunks, rr, HN, a, y0, y1, ny, PW, CW, rng, late_wait=True,
                        ring_wait=True):
    """One random interleaving of the two-producer-group schedule at the level
    of its LDS counters. Chunk k belongs to producer group k mod 2 as its
    (k // 2)-th chunk. A producer wave computes its chunk (no ring access),
    then, for k >= 2, waits for consumed >= CW (k - 1) before it writes the
    ring rows (late_wait; False moves the wait before the computation, which
    orders the same accesses), then waits until every wave of its group has
    counted the group's previous chunk and counts produced[g]. Consumers wait
    for produced[k mod 2] >= PW (k // 2 + 1). Checks as for the single group:
    no read of an incomplete or stale row, no write over a row an unfinished
    reader needs, and every wave reaches the end. ring_wait=False drops the
    ring wait (a planted mistake the check must catch)."""
    nring = 2 * rr + 2 * HN
    need = [min(y0 + (k + 1) * rr + HN, y1 + HN, ny) for k in range(chunks)]
    rows_of = [list(range(a if k == 0 else need[k - 1], need[k])) for k in range(chunks)]
    reads_of = []
    for k in range(chunks):
        lo, hi = y0 + k * rr, min(y0 + (k + 1) * rr, y1)
        reads_of.append(sorted({min(max(j - e, 0), ny - 1) for j in range(lo, hi)
                                for e in range(-HN, HN + 1)}))
    slot = lambda j: (j - a) % nring  # noqa: E731
    content, writing, reading = {}, {}, {}
    produced = [0, 0]
    consumed = 0
    # producer wave (g, w) runs chunks g, g + 2, ...; stages: 0 compute,
    # 1 start writing (ring wait), 2 finish writing, 3 count (group wait)
    prog = {("p", g, w): [g, 0] for g in range(2) for w in range(PW)}
    prog.update({("c", 0, w): [0, 0] for w in range(CW)})
    events = 0
    while True:
        ready = []
        for key, (k, st) in prog.items():
            if k >= chunks:
                continue
            if key[0] == "p":
                ring_free = k < 2 or consumed >= CW * (k - 1) or not ring_wait
                if st == 0 and (late_wait or ring_free):
                    ready.append(key)
                elif st == 1 and ring_free:
                    ready.append(key)
                elif st == 2 or (st == 3 and produced[key[1]] >= PW * (k // 2)):
                    ready.append(key)
            else:
                if st == 0 and produced[k % 2] >= PW * (k // 2 + 1):
                    ready.append(key)
                elif st in (1, 2) or (st == 3 and consumed >= CW * k):
                    ready.append(key)
        if not ready:
            break
        key = ready[rng.integers(len(ready))]
        k, st = prog[key]
        events += 1
        if key[0] == "p":
            w = (key[1], key[2])
            if st == 1:                       # start writing chunk k
                for j in rows_of[k]:
                    s = slot(j)
                    for row in reading.get(s, {}).values():
                        assert row == j, ("overwrite while read", k, j, row)
                    writing.setdefault(s, set()).add(w)
                    if content.get(s, (None,))[0] != j:
                        content[s] = (j, set())
            elif st == 2:                     # finish writing
                for j in rows_of[k]:
                    s = slot(j)
                    writing[s].discard(w)
                    content[s][1].add(w)
            elif st == 3:
                produced[key[1]] += 1
            prog[key] = [k + 2, 0] if st == 3 else [k, st + 1]
        else:
            w = key[2]
            if st == 0:                       # start reading chunk k
                g = k % 2
                for j in reads_of[k]:
                    s = slot(j)
                    row, done = content.get(s, (None, set()))
                    assert row == j and not writing.get(s), ("stale", k, j)
                    # every wave of the group that produced row j finished it
                    src = next(m for m in range(chunks) if j in rows_of[m])
                    assert {(src % 2, x) for x in range(PW)} <= done, ("incomplete", k, j)
                    reading.setdefault(s, {})[w] = j
            elif st == 1:
                for j in reads_of[k]:
                    reading[slot(j)].pop(w, None)
            elif st == 3:
                consumed += 1
            prog[key] = [k + 1, 0] if st == 3 else [k, st + 1]
    assert all(k >= chunks for k, _ in prog.values()), "a wave is stuck"
    return events


@pytest.mark.parametrize("rr,HN,y0,y1,ny,PW,CW", [
    (3, 3, 5, 10, 24, 3, 2), (3, 3, 0, 64, 512, 4, 3), (3, 3, 64, 128, 512, 4, 3),
    (2, 4, 3, 17, 17, 2, 1), (3, 3, 20, 24, 24, 4, 3), (4, 4, 0, 40, 40, 3, 2),
    (3, 3, 509, 512, 512, 4, 3), (3, 3, 0, 2, 2, 4, 3),
])
@pytest.mark.parametrize("late_wait", [True, False])
def test_twin_schedule_random_interleavings(rr, HN, y0, y1, ny, PW, CW, late_wait):
    rng = np.random.default_rng(rr * 1000 + y0 + late_wait)
    a = max(y0 - HN, 0)
    chunks = (y1 - y0 + rr - 1) // rr
    for _ in range(60):
        twin_schedule_check(chunks, rr, HN, a, y0, y1, ny, PW, CW, rng, late_wait)


def test_twin_schedule_check_catches_a_missing_ring_wait():
    """The check fails when a producer group writes its chunk without waiting
    for the consumers to free the ring rows (a planted mistake in the
    schedule model)."""
    rng = np.random.default_rng(5)
    found = False
    for _ in range(200):
        try:
            twin_schedule_check(6, 3, 3, 0, 0, 18, 18, 2, 2, rng, ring_wait=False)
        except AssertionError:
            found = True
            break
    assert found
