"""CPU model of the 7-point walker's LDS exchange (the z-march of the 3D passes):
for every tile of a grid, the four wavefronts' rows, the outer rows y0 - 1 and
y0 + 4 that wavefronts 0 and 3 form, the exchange slots they write and read,
and the rows their loads touch.  Checked at many plane sizes (rows per plane
not a multiple of 4, single rows, single planes):
  - every wavefront whose row lies in the plane receives rows y - 1 and y + 1
    of the same plane as its south and north neighbours, and zero outside
    the plane;
  - every slot written or read lies in the six-row buffer, and each slot is
    written by exactly one wavefront per plane;
  - every row a wavefront loads lies inside the plane and every plane inside
    the grid, including the wavefronts past the plane's last row;
  - the four wavefronts of a tile pass the same number of barriers;
  - in the split form of classic pass 1 (one vector row of the outer rows per
    wavefront), wavefronts 0 and 3 receive both vectors of rows y0 - 1 and
    y0 + 4, and every wavefront issues one outer load;
  - in the half-row form (half an outer row per wavefront), every buffer
    position is written once and wavefronts 0 and 3 read their own columns
    of rows y0 - 1 and y0 + 4.
The model follows the walker's index arithmetic step by step (tile ->
in-plane row, planes of the tile, clamped rows, slot numbers)."""
import pytest

WAVES = 4
SLOTS = WAVES + 2


def tiles_of(ny_plane, nz, planes):
    nty = (ny_plane + WAVES - 1) // WAVES
    ntz = (nz + planes - 1) // planes
    return nty, ntz


def wave_view(ty, tz, w, ny_plane, nz, planes):
    """The walker's per-wavefront quantities for tile (ty, tz)."""
    y = ty * WAVES + w
    z0 = tz * planes
    z1 = min(z0 + planes, nz)
    live = y < ny_plane
    yl = y if live else ny_plane - 1            # the row its loads read
    outer = w == 0 or w == WAVES - 1
    yo = y - 1 if w == 0 else y + 1
    has_o = outer and 0 <= yo < ny_plane
    yoc = yo if has_o else yl
    oslot = 0 if w == 0 else WAVES + 1
    return dict(y=y, z0=z0, z1=z1, live=live, yl=yl, outer=outer, has_o=has_o, yoc=yoc,
                oslot=oslot)


def run_tile(ty, tz, ny_plane, nz, planes):
    views = [wave_view(ty, tz, w, ny_plane, nz, planes) for w in range(WAVES)]
    z0, z1 = views[0]["z0"], views[0]["z1"]
    assert all(v["z0"] == z0 and v["z1"] == z1 for v in views)
    assert z0 < z1 <= nz
    barriers = [1] * WAVES  # the barrier at the walker's start
    for z in range(z0, z1):
        # loads of this step (rows in the plane, planes in the grid)
        for v in views:
            for row in (v["yl"], v["yoc"]):
                assert 0 <= row < ny_plane
            zmax = min(z1, nz - 1)
            for zz in (min(z + 2, zmax), min(z + 1, z1 - 1), max(z0 - 1, 0)):
                assert 0 <= zz < nz
        # writes into the exchange buffer: value = the row index or None (zero)
        buf = [[] for _ in range(SLOTS)]
        for w, v in enumerate(views):
            buf[w + 1].append(v["y"] if v["live"] else None)
            if v["outer"]:
                buf[v["oslot"]].append(v["yoc"] if v["has_o"] else None)
        for s in range(SLOTS):
            assert len(buf[s]) == 1, "slot %d written %d times" % (s, len(buf[s]))
        for w in range(WAVES):
            barriers[w] += 1
        # reads: south slot w, north slot w + 2
        for w, v in enumerate(views):
            south, north = buf[w][0], buf[w + 2][0]
            if not v["live"]:
                continue
            y = v["y"]
            assert south == (y - 1 if y > 0 else None)
            assert north == (y + 1 if y + 1 < ny_plane else None)
    assert len(set(barriers)) == 1
    return barriers[0]


@pytest.mark.parametrize("ny_plane", [1, 2, 3, 4, 5, 7, 8, 9, 13, 40, 64, 257])
@pytest.mark.parametrize("nz,planes", [(1, 1), (2, 8), (5, 8), (23, 8), (64, 32), (9, 4)])
def test_exchange_model(ny_plane, nz, planes):
    nty, ntz = tiles_of(ny_plane, nz, planes)
    rows_seen = set()
    for tz in range(ntz):
        for ty in range(nty):
            n = run_tile(ty, tz, ny_plane, nz, planes)
            assert n == 1 + min(planes, nz - tz * planes)
            for w in range(WAVES):
                y = ty * WAVES + w
                if y < ny_plane:
                    rows_seen.add((y, tz))
    # every in-plane row of every plane group is walked by exactly one wavefront
    assert rows_seen == {(y, tz) for y in range(ny_plane) for tz in range(ntz)}


def test_model_catches_a_wrong_slot():
    """A mistake in the slot arithmetic (north read from slot w + 1) is caught."""
    views = [wave_view(0, 0, w, 9, 4, 4) for w in range(WAVES)]
    buf = [None] * SLOTS
    for w, v in enumerate(views):
        buf[w + 1] = v["y"] if v["live"] else None
    wrong_north = buf[1 + 1]  # wavefront 1 reading slot w + 1: its own row
    assert wrong_north != views[1]["y"] + 1


def split_view(ty, w, ny_plane):
    """The split form of classic pass 1: wavefront w loads vector w & 1 of the
    tile's outer row y0 - 1 (w < 2) or y0 + 4 (w >= 2), clamped to a row of the
    plane when that row lies outside it."""
    y = ty * WAVES + w
    y0 = y - w
    yl = y if y < ny_plane else ny_plane - 1
    yo = y0 - 1 if w < 2 else y0 + WAVES
    yoc = yo if 0 <= yo < ny_plane else yl
    return dict(y0=y0, yo=yo, yoc=yoc, part=w & 1)


@pytest.mark.parametrize("ny_plane", [1, 2, 3, 4, 5, 7, 8, 9, 13, 40, 64, 257])
def test_split_outer_rows_model(ny_plane):
    nty = (ny_plane + WAVES - 1) // WAVES
    for ty in range(nty):
        views = [split_view(ty, w, ny_plane) for w in range(WAVES)]
        y0 = views[0]["y0"]
        # raw slot w holds (row, vector) = (yoc, part) of wavefront w
        raw = [(v["yoc"], v["part"]) for v in views]
        for v in views:
            assert 0 <= v["yoc"] < ny_plane
        # wavefront 0 joins slots 0 and 1: both vectors of row y0 - 1, when it exists
        if y0 > 0:
            assert raw[0] == (y0 - 1, 0) and raw[1] == (y0 - 1, 1)
        # wavefront 3 joins slots 2 and 3: both vectors of row y0 + 4, when it exists
        if y0 + WAVES < ny_plane:
            assert raw[2] == (y0 + WAVES, 0) and raw[3] == (y0 + WAVES, 1)
        # every wavefront issues exactly one outer-row load per plane
        assert len(raw) == WAVES


@pytest.mark.parametrize("ny_plane", [1, 2, 3, 4, 5, 7, 8, 9, 13, 40, 64, 257])
def test_half_outer_rows_model(ny_plane):
    """The half-row form: wavefront w loads columns 64 (w & 1) + lane of row
    y0 - 1 (w < 2) or y0 + 4 (w >= 2) into buffer position
    128 (w >> 1) + 64 (w & 1) + lane; wavefronts 0 and 3 then read their lane's
    two columns 2 lane, 2 lane + 1 from rows 0 and 1 of the buffer."""
    lanes, tile_cols = 64, 128
    nty = (ny_plane + WAVES - 1) // WAVES
    for ty in range(nty):
        buf = [None] * (2 * tile_cols)
        for w in range(WAVES):
            y = ty * WAVES + w
            y0 = y - w
            yl = y if y < ny_plane else ny_plane - 1
            yo = y0 - 1 if w < 2 else y0 + WAVES
            yoc = yo if 0 <= yo < ny_plane else yl
            assert 0 <= yoc < ny_plane
            for lane in range(lanes):
                col = (w & 1) * lanes + lane
                slot = (w >> 1) * tile_cols + (w & 1) * lanes + lane
                assert buf[slot] is None
                buf[slot] = (yoc, col)
        assert None not in buf
        y0 = ty * WAVES
        for lane in range(lanes):
            s0, s1 = buf[2 * lane], buf[2 * lane + 1]
            n0, n1 = buf[tile_cols + 2 * lane], buf[tile_cols + 2 * lane + 1]
            if y0 > 0:
                assert s0 == (y0 - 1, 2 * lane) and s1 == (y0 - 1, 2 * lane + 1)
            if y0 + WAVES < ny_plane:
                assert n0 == (y0 + WAVES, 2 * lane) and n1 == (y0 + WAVES, 2 * lane + 1)
