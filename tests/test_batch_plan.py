"""Host logic of the batched run: the work-item table and its dependency
lists (no GPU).

The persistent kernel runs items in ticket order (q-major, q = 2 n + stage
- 1) and lets an item start only when (a) the blocks in its dependency list
finished stage q-1 and (b) for stage 1 of step n > 0, every stage-2 block of
step n-1 of its box finished.  These tests check, from the stencil itself
(two cells in y, through the boundary rule), that the lists are exactly the
blocks an item reads from or is read by, and then run a randomised
discrete-event model of the queue to check that every row an item reads has
been written by the right producer and not yet overwritten.
"""
import random

import numpy as np
import pytest

import paper_1812_04135_amd as rs


def _cfg(nx, ny, ybc="reflect", xbc="periodic"):
    return {"ndim": 2, "n": [nx, ny], "dx": [1.0 / nx, 1.0 / ny], "gamma": 5.0 / 3.0, "xi": 4.0,
            "cfl": 0.4, "bc_lo": [xbc, ybc], "bc_hi": [xbc, ybc], "form": "pvs"}


def _mapped(k, n, ybc):
    # the boundary rule of the y axis, written out: periodic wraps, reflect
    # mirrors about the wall (ghost -1 is cell 0, ghost n is cell n-1)
    if ybc == "periodic":
        return k % n
    if k < 0:
        return -k - 1
    if k >= n:
        return 2 * n - k - 1
    return k


def _stencil_rows(r0, r1, n, ybc):
    return {_mapped(k, n, ybc) for k in range(r0 - 2, r1 + 2)}


BOXES = [
    [(16, 12, "reflect"), (70, 33, "reflect"), (130, 40, "periodic"), (200, 24, "reflect"),
     (64, 64, "periodic"), (37, 9, "periodic")],
    [(256, 100, "periodic"), (8, 4, "periodic"), (65, 17, "periodic"), (192, 8, "reflect"),
     (129, 257, "periodic"), (64, 33, "periodic")],
]
TILES = [[16, 16, 16, 16], [8, 24, 32, 8], [8, 8, 8, 8], [64, 40, 9, 256]]


def _plan(boxes, tiles):
    cfgs = [_cfg(nx, ny, ybc) for nx, ny, ybc in boxes]
    return rs.rsst_batch_plan(cfgs, tiles)


@pytest.mark.parametrize("boxes", BOXES)
@pytest.mark.parametrize("tiles", TILES)
def test_plan_blocks_tile_rows_and_deps_match_stencil(boxes, tiles):
    tab = _plan(boxes, tiles)
    assert tab.shape[1] == rs.BATCH_PLAN_COLS
    for b, (nx, ny, ybc) in enumerate(boxes):
        rows = tab[tab[:, 0] == b]
        assert list(rows[:, 1]) == list(range(len(rows)))
        # blocks cover [0, ny) once, in order, all but the last full
        assert rows[0, 2] == 0 and rows[-1, 3] == ny
        assert np.all(rows[1:, 2] == rows[:-1, 3])
        nwx = (nx + 63) // 64
        groups = 4 // nwx
        km = min(tiles[nwx - 1], ny)
        assert np.all(rows[:-1, 3] - rows[:-1, 2] == groups * km)
        owner = np.empty(ny, dtype=int)
        for p, r in enumerate(rows):
            owner[r[2]:r[3]] = p
        reads = [set(owner[list(_stencil_rows(r[2], r[3], ny, ybc))]) for r in rows]
        for p, r in enumerate(rows):
            want = set(reads[p]) | {o for o in range(len(rows)) if p in reads[o]}
            nd = r[4]
            got = list(r[5:5 + nd])
            assert got == sorted(want), (b, p, got, sorted(want))
            assert np.all(r[5 + nd:] == -1)


def test_plan_periodic_wrap_reaches_short_last_block():
    # ny = 33 with 16-row blocks: the last block is one row, so the first
    # block's stencil (rows -2, -1 -> 31, 32) reaches the last two blocks
    tab = _plan([(16, 33, "periodic")], [16, 16, 16, 16])
    # one wave per row: 4 strips of 16 rows per block -> a single block
    assert len(tab) == 1
    tab = _plan([(200, 33, "periodic")], [16, 16, 16, 16])
    assert [list(r[2:4]) for r in tab] == [[0, 16], [16, 32], [32, 33]]
    assert list(tab[0, 5:5 + tab[0, 4]]) == [0, 1, 2]
    assert list(tab[2, 5:5 + tab[2, 4]]) == [0, 1, 2]


def _simulate(boxes, tab, nsteps, nworkers, rng):
    """Discrete-event model of the ticket queue.  Returns the execution
    interval of every (q, item)."""
    nitem = len(tab)
    deps = [list(r[5:5 + r[4]]) for r in tab]
    base = {}
    for i, r in enumerate(tab):
        base.setdefault(int(r[0]), i)
    nblk = {b: int((tab[:, 0] == b).sum()) for b in base}
    total = 2 * nsteps * nitem
    end = {}
    free = [0.0] * nworkers
    for t in range(total):
        w = min(range(nworkers), key=lambda k: free[k])
        q, r = divmod(t, nitem)
        b = int(tab[r, 0])
        ready = free[w]
        if q > 0:
            for p in deps[r]:
                ready = max(ready, end[(q - 1, base[b] + p)])
        if q % 2 == 0 and q > 0:
            n = q // 2
            for p in range(nblk[b]):
                ready = max(ready, end[(2 * n - 1, base[b] + p)])
        dur = rng.uniform(0.5, 3.0)
        end[(q, r)] = ready + dur
        end[("start", q, r)] = ready
        free[w] = ready + dur
    return end


@pytest.mark.parametrize("boxes", BOXES)
@pytest.mark.parametrize("tiles", TILES[:3])
def test_queue_model_orders_every_read_after_its_write(boxes, tiles):
    """Every row read by an item was last written by the producer of the
    version it needs, and that producer's successor starts only after the
    reader ends (no overwrite while it may still read)."""
    tab = _plan(boxes, tiles)
    nsteps = 3
    rng = random.Random(1234)
    for nworkers in (1, 3, 17, 1000):
        ev = _simulate(boxes, tab, nsteps, nworkers, rng)
        nitem = len(tab)
        # writer of (buffer, box, row, version): U version n+1 by stage 2 of
        # step n, U1 version n by stage 1 of step n; U version 0 is the input
        owner = {}
        for i, r in enumerate(tab):
            for k in range(r[2], r[3]):
                owner[(int(r[0]), k)] = i

        def iv(q, i):
            return ev[("start", q, i)], ev[(q, i)]

        for q in range(2 * nsteps):
            n, st2 = q // 2, q % 2 == 1
            for i, r in enumerate(tab):
                b, ny, ybc = int(r[0]), boxes[int(r[0])][1], boxes[int(r[0])][2]
                s, e = iv(q, i)
                halo = _stencil_rows(r[2], r[3], ny, ybc)
                # stage 1 reads U_n (halo); stage 2 reads U1_n (halo) and U_n (own rows)
                reads = [("U1" if st2 else "U", k) for k in halo]
                if st2:
                    reads += [("U", k) for k in range(r[2], r[3])]
                for buf, k in reads:
                    j = owner[(b, k)]
                    if buf == "U":
                        wq, nq = 2 * n - 1, 2 * n + 1      # writer of U_n, writer of U_{n+1}
                    else:
                        wq, nq = 2 * n, 2 * n + 2          # writer of U1_n, writer of U1_{n+1}
                    if wq >= 0:
                        assert iv(wq, j)[1] <= s, (q, i, buf, k, "read before write")
                    if nq < 2 * nsteps and (nq, j) != (q, i):
                        assert iv(nq, j)[0] >= e, (q, i, buf, k, "overwritten while read")


def test_batch_takes_ideal_gas_boxes_only():
    cfgs = [_cfg(16, 12), dict(_cfg(20, 16), eos="vdw", eos_a=0.2, eos_b=0.1)]
    with pytest.raises(rs.RsstError) as e:
        rs.rsst_batch_plan(cfgs, [16, 16, 16, 16])
    assert e.value.code == -4  # RSST_E_UNSUPPORTED


def test_batch_takes_no_hydrostatic_walls():
    cfgs = [_cfg(16, 12), _cfg(20, 16, ybc="hydro")]
    with pytest.raises(rs.RsstError) as e:
        rs.rsst_batch_plan(cfgs, [16, 16, 16, 16])
    assert e.value.code == -4  # RSST_E_UNSUPPORTED
