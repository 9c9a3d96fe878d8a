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
