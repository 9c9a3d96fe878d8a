"""Host-side models of the step kernels' on-chip schedules (no GPU).

The step kernels keep each advected row in an LDS ring until it is collided
two rows later.  In a single-wavefront march each lane reads back only what
it wrote, so the ring only has to hold the row long enough; in the pair
launch (one wavefront advects, the other collides, one barrier per row) the
two wavefronts touch the ring between the same barriers, so the advector's
next write must never hit a slot the collider is still reading.

Model of one row iteration t of a chunk (rows y0 .. y1 - 1): the newest loaded
row is r = y0 - 4 + t, the advected row a = r - 2 goes to slot w(t), and the
collided row o = a - 2 is read from slot w(t - 2); rows are stored for
t >= 8 and o < y1.  Pair launch: the advector writes slot w(t) and its
density slot before barrier t; the collider reads both after barrier t, so
between barriers t and t + 1 the advector writes w(t + 1) while the collider
reads w(t) (density) and w(t - 2) (advected row).
"""
import pytest


def single_wave_reads(nslots, y0, y1):
    """Rows the single-wavefront march collides, as read back from its ring."""
    niter = ((y1 - y0) + 8 + 3) & ~3
    ring = [None] * nslots
    out = []
    for t in range(niter):
        a = y0 - 6 + t
        ring[t % nslots] = a
        o = a - 2
        got = ring[(t - 2) % nslots]
        if t >= 8 and o < y1:
            out.append((o, got))
    return out


@pytest.mark.parametrize("nslots", [3, 4])
def test_single_wave_ring_returns_each_row_two_iterations_later(nslots):
    for rows in range(1, 80):
        for y0 in (0, 5, 64):
            reads = single_wave_reads(nslots, y0, y0 + rows)
            assert [o for o, _ in reads] == list(range(y0, y0 + rows))
            assert all(o == got for o, got in reads)


def pair_conflicts(nslots, niter=64):
    """Barrier intervals in which the advector writes a ring slot that the
    collider reads in the same interval (a write-after-read race)."""
    bad = []
    for t in range(2, niter - 1):
        writes = {(t + 1) % nslots}                      # advector, iteration t + 1
        reads_rows = {(t - 2) % nslots}                   # collider, advected row o
        reads_density = {t % nslots}                      # collider, density of row a
        if writes & reads_rows or writes & reads_density:
            bad.append(t)
    return bad


def test_pair_launch_needs_four_ring_slots():
    """With three slots the advector's write of iteration t + 1 lands on the
    slot of row t - 2 that the collider reads after the same barrier; four
    slots keep writes and reads apart in every interval."""
    assert pair_conflicts(3)
    assert pair_conflicts(4) == []


# ---------------------------------------------------------------------------
# Persistent batched launch: which items an item of step s waits for, and
# that the ticket order always drains.

STRIP, HALO, REACH_Y = 56, 4, 4


def block_span(lo, hi, L, per, nblk, wrap):
    """Blocks of `per` (the last one ragged) of 0..L-1 that cover positions
    lo..hi, periodic or clipped (the kernel's rule, restated)."""
    if not wrap:
        lo, hi = max(lo, 0), min(hi, L - 1)
        first = lo // per
        return [first + k for k in range(hi // per - first + 1)]
    if hi - lo + 1 >= L:
        return list(range(nblk))
    lo, hi = lo % L, hi % L
    first, last = lo // per, hi // per
    count = min(last + nblk - first + 1, nblk) if lo > hi else last - first + 1
    return [(first + k) % nblk for k in range(count)]


def waits_of(Lx, Ly, rows, walls, strip, chunk):
    nstrips, nchunks = -(-Lx // STRIP), -(-Ly // rows)
    y0, y1 = chunk * rows, min(chunk * rows + rows, Ly)
    x0, x1 = strip * STRIP, min(strip * STRIP + STRIP, Lx)
    cs = block_span(y0 - REACH_Y, y1 + REACH_Y - 1, Ly, rows, nchunks, not walls)
    ss = block_span(x0 - HALO, x1 + HALO - 1, Lx, STRIP, nstrips, True)
    return {(c, s) for c in cs for s in ss}


def needed_by_brute_force(Lx, Ly, rows, walls, strip, chunk):
    """Items whose output nodes lie in the input of (strip, chunk): columns
    within HALO and rows within REACH_Y of its own, wrapped in x, wrapped in y
    unless walls (ghost rows belong to no item)."""
    nstrips = -(-Lx // STRIP)
    y0, y1 = chunk * rows, min(chunk * rows + rows, Ly)
    x0, x1 = strip * STRIP, min(strip * STRIP + STRIP, Lx)
    need = set()
    for y in range(y0 - REACH_Y, y1 + REACH_Y):
        if walls and (y < 0 or y >= Ly):
            continue
        yy = y % Ly
        for x in range(x0 - HALO, x1 + HALO):
            need.add((yy // rows, (x % Lx) // STRIP))
    assert all(0 <= s < nstrips for _, s in need)
    return need


@pytest.mark.parametrize("walls", [0, 1])
def test_persistent_waits_cover_exactly_the_overlapping_items(walls):
    """The kernel's span rule gives exactly the items whose outputs overlap
    an item's input, for ragged and tiny lattices (chunks and strips shorter
    than the reach, lattices smaller than the reach, one-item lattices)."""
    for Lx in (1, 3, 9, 56, 57, 60, 70, 112, 113, 200):
        for Ly in (1, 2, 5, 7, 9, 19, 50, 64, 66, 130):
            for rows in (1, 2, 3, 5, 8, 16, 64):
                nstrips, nchunks = -(-Lx // STRIP), -(-Ly // rows)
                for c in range(nchunks):
                    for s in range(nstrips):
                        assert waits_of(Lx, Ly, rows, walls, s, c) == \
                            needed_by_brute_force(Lx, Ly, rows, walls, s, c), (Lx, Ly, rows, c, s)


def test_persistent_waits_are_symmetric():
    """i waits for j exactly when j waits for i, so one wait covers both the
    reads of step s (outputs of step s - 1) and its writes (the buffer that
    the neighbours read in step s - 1)."""
    for Lx, Ly, rows, walls in ((70, 50, 5, 1), (57, 130, 16, 0), (9, 7, 5, 0), (200, 66, 8, 1)):
        nstrips, nchunks = -(-Lx // STRIP), -(-Ly // rows)
        for c in range(nchunks):
            for s in range(nstrips):
                for (c2, s2) in waits_of(Lx, Ly, rows, walls, s, c):
                    assert (c, s) in waits_of(Lx, Ly, rows, walls, s2, c2)


def test_persistent_tickets_always_drain():
    """Workers take tickets t = s * n + i in order and block until every
    item that t waits for has finished step s - 1.  Whatever the order in
    which blocked and running workers are served, every ticket completes:
    a ticket waits only for smaller tickets, all held by workers."""
    import random
    rng = random.Random(5)
    runs = [(70, 50, 5, 1), (9, 7, 5, 0), (57, 130, 16, 0)]
    items = []
    for r, (Lx, Ly, rows, walls) in enumerate(runs):
        for c in range(-(-Ly // rows)):
            for s in range(-(-Lx // STRIP)):
                items.append((r, c, s))
    index = {it: k for k, it in enumerate(items)}
    deps = [[index[(r, c2, s2)] for (c2, s2) in waits_of(*runs[r], s, c)] for (r, c, s) in items]
    n, nsteps = len(items), 6
    for workers in (1, 2, 3, 7, 64):
        done = [0] * n
        nxt, active = 0, []
        finished = 0
        while finished < n * nsteps:
            while len(active) < workers and nxt < n * nsteps:
                active.append(nxt)
                nxt += 1
            ready = [t for t in active if t // n == 0 or all(done[j] >= t // n for j in deps[t % n])]
            assert ready, "no worker can proceed"
            t = rng.choice(ready)
            active.remove(t)
            done[t % n] = t // n + 1
            finished += 1
        assert done == [nsteps] * n
