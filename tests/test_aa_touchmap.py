"""Race-freedom and correctness of the in-place AA index maps (CPU, brute force).

The HIP kernel's even and odd steps are modelled here as maps from (node,
direction) to the (node, slot) each thread reads and writes, exactly as the
kernel's comments define them:
  even: read (x, i); write (x, opp i)   [+ wall term where x + c_i is a wall]
  odd : read (x - c_i, opp i), or (x, i) if x - c_i is a wall;
        write (x + c_i, i), or (x, opp i) if x + c_i is a wall.
On tiny lattices with random solid/wall tags we check that every (node, slot)
is touched by at most one thread per step (no race), that the odd step reads
exactly what the even step wrote, and that two AA steps of free streaming
(identity collision) reproduce the oracle's two-population push streaming.
"""
import numpy as np
import pytest

import oracle
from paper_2506_09242_amd import inputs


def _setup(q, shape, seed):
    nz, ny, nx = shape
    tags = inputs.random_tags(nx, ny, nz, seed=seed, solid_frac=0.25, wall_frac=0.1)
    c, w, opp = oracle.tables(q)
    fluid = (tags >= 1) & (tags <= 10)
    return tags, fluid, c, opp


def _nb(x, c, shape, sign):
    nz, ny, nx = shape
    return ((x[0] + sign * c[2]) % nz, (x[1] + sign * c[1]) % ny, (x[2] + sign * c[0]) % nx)


def _maps(q, shape, fluid, c, opp, parity):
    reads, writes = [], []
    for x in zip(*np.nonzero(fluid)):
        for i in range(q):
            if parity == 0:
                reads.append((x, i))
                writes.append((x, opp[i]))
            else:
                src = _nb(x, c[i], shape, -1)
                reads.append(((x, i) if not fluid[src] else (src, opp[i])))
                dst = _nb(x, c[i], shape, +1)
                writes.append(((x, opp[i]) if not fluid[dst] else (dst, i)))
    return reads, writes


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("shape,seed", [((3, 4, 5), 1), ((2, 3, 7), 2), ((4, 1, 3), 3), ((1, 2, 2), 4)])
def test_aa_maps_are_race_free_and_consistent(q, shape, seed):
    tags, fluid, c, opp = _setup(q, shape, seed)
    nf = int(fluid.sum())
    for parity in (0, 1):
        r, w = _maps(q, shape, fluid, c, opp, parity)
        assert len(set(r)) == len(r) == nf * q, "a slot is read twice in one step"
        assert len(set(w)) == len(w) == nf * q, "a slot is written twice in one step"
        # every touched slot belongs to a fluid node
        assert all(fluid[x] for x, _ in r) and all(fluid[x] for x, _ in w)
        # the step writes back exactly the slots it read: in place, no stray writes
        assert set(r) == set(w)
    # the odd step consumes what the even step produced
    r1, _ = _maps(q, shape, fluid, c, opp, 1)
    _, w0 = _maps(q, shape, fluid, c, opp, 0)
    assert set(r1) == set(w0)


def _aa_free_stream(q, shape, fluid, c, opp, f_nat, steps):
    """Apply `steps` AA steps with identity collision to natural-layout values and
    return the natural state (gathering after an odd step)."""
    a = f_nat.copy()  # slot array a[i][z][y][x]; non-fluid nodes hold garbage
    a[:, ~fluid] = np.nan
    for s in range(steps):
        parity = s % 2
        new = a.copy()
        for x in zip(*np.nonzero(fluid)):
            vals = []
            for i in range(q):
                if parity == 0:
                    vals.append(a[(i,) + x])
                else:
                    src = _nb(x, c[i], shape, -1)
                    vals.append(a[(i,) + x] if not fluid[src] else a[(opp[i],) + src])
            for i in range(q):
                if parity == 0:
                    new[(opp[i],) + x] = vals[i]
                else:
                    dst = _nb(x, c[i], shape, +1)
                    if fluid[dst]:
                        new[(i,) + dst] = vals[i]
                    else:
                        new[(opp[i],) + x] = vals[i]
        a = new
    if steps % 2 == 0:
        return a
    nat = np.zeros_like(a)
    for x in zip(*np.nonzero(fluid)):
        for i in range(q):
            src = _nb(x, c[i], shape, -1)
            nat[(i,) + x] = a[(i,) + x] if not fluid[src] else a[(opp[i],) + src]
    return nat


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("steps", [1, 2, 5])
def test_aa_free_streaming_matches_push(q, steps):
    shape = (3, 4, 5)
    tags, fluid, c, opp = _setup(q, shape, 9)
    # resting walls only: with identity collision the moving-wall term is the
    # one thing that differs between AA (applied at write time) and push
    tags = np.where(tags >= 16, 0, tags).astype(np.uint8)
    fluid = (tags >= 1) & (tags <= 10)
    rng = np.random.default_rng(steps)
    f0 = rng.uniform(0.5, 1.5, (q,) + shape) * fluid
    nz, ny, nx = shape
    o = oracle.Oracle(nx, ny, nz, q=q, tags=tags, free_streaming=True)
    o.f[:] = f0
    o.run(steps)
    aa = _aa_free_stream(q, shape, fluid, c, opp, f0, steps)
    assert np.array_equal(aa[:, fluid], o.f[:, fluid])


def _filler_writes(q, shape, fluid, c, opp, parity, sector, odd_fill):
    """(node, slot) targets of the step kernel's filler stores: a non-fluid node
    whose storage sector (`sector` consecutive node indices) holds a fluid node
    writes its own slots in the even step, and in the odd step slot 0 of itself
    and slot i of node x + (0, c_iy, c_iz) where that node is not fluid."""
    nz, ny, nx = shape
    flat = fluid.reshape(-1)
    out = []
    for n in range(flat.size):
        if flat[n]:
            continue
        a = n - n % sector
        if not flat[a:a + sector].any():
            continue
        x = (n // (nx * ny), (n // nx) % ny, n % nx)
        for i in range(q):
            if parity == 0:
                out.append((x, opp[i]))
            elif i == 0:
                out.append((x, 0))
            elif odd_fill:
                t = ((x[0] + c[i][2]) % nz, (x[1] + c[i][1]) % ny, x[2])
                if not fluid[t]:
                    out.append((t, i))
    return out


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("sector", [2, 4, 8])
@pytest.mark.parametrize("shape,seed", [((3, 4, 5), 1), ((2, 3, 7), 2), ((4, 5, 6), 5)])
def test_filler_stores_touch_only_dead_slots(q, sector, shape, seed):
    tags, fluid, c, opp = _setup(q, shape, seed)
    for parity in (0, 1):
        r, w = _maps(q, shape, fluid, c, opp, parity)
        live = set(r) | set(w)
        for odd_fill in (False, True):
            fw = _filler_writes(q, shape, fluid, c, opp, parity, sector, odd_fill)
            # never a fluid node's slot, and no slot written twice by fillers
            assert all(not fluid[x] for x, _ in fw)
            assert not (set(fw) & live)
            assert len(set(fw)) == len(fw)
    # even step: every slot of every sector that holds a fluid node is written
    nz, ny, nx = shape
    _, w0 = _maps(q, shape, fluid, c, opp, 0)
    written = set(w0) | set(_filler_writes(q, shape, fluid, c, opp, 0, sector, True))
    flat = fluid.reshape(-1)
    for a in range(0, flat.size, sector):
        if flat[a:a + sector].any():
            for n in range(a, min(a + sector, flat.size)):
                x = (n // (nx * ny), (n // nx) % ny, n % nx)
                assert all((x, i) in written for i in range(q))


def test_filler_completes_rows_next_to_x_walls():
    """A box with walls on the x faces: with odd-step fillers every sector of
    every row that holds fluid is written whole in both steps."""
    q, shape, sector = 19, (4, 4, 12), 4
    nz, ny, nx = shape
    fluid = np.ones(shape, bool)
    fluid[:, :, 0] = fluid[:, :, -1] = False
    c, w, opp = oracle.tables(q)
    for parity in (0, 1):
        _, wf = _maps(q, shape, fluid, c, opp, parity)
        written = set(wf) | set(_filler_writes(q, shape, fluid, c, opp, parity, sector, True))
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    assert all(((z, y, x), i) in written for i in range(q)), (parity, z, y, x)
