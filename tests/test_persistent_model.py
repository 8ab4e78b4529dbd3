"""CPU model of the single-launch batch scheduler that is switched off.

That scheduler ran every pair and level of a batch as the tiles ("tasks") of
one persistent kernel: the host listed segments (one per pair, stage and
level: a pyramid reduce, the window statistics, the matching of a level) in
an order where every dependency comes first, numbered all tiles in that
order, and each resident workgroup took the next task number with an atomic
add, waited until the tile rows ("bands") it reads of its dependency segments
were complete (a band counter per tile row, bumped once per finished tile),
ran the tile and bumped its own band.  Two runs on the GPU hung and the
kernel was removed; this model rebuilds its task table and band waits with
the tile geometry that kernel used (reduce and statistics tiles 64 x 16,
matching tiles 128 x 8) and checks, on the CPU:

* every band a task waits on lies inside its dependency segment;
* every task of an awaited band has a smaller task number than the waiting
  task, so it was dequeued earlier by a running workgroup;
* the bands awaited, directly or through the tasks they wait on, cover every
  row each tile reads (rows derived from each tile's own stencil, not from
  the wait rule);
* a run of the scheduler with worker threads standing in for workgroups ends
  for any number of workers.
"""
import bisect
import threading

import pytest

RD_W, RD_H = 64, 16      # reduce output tile
ST_W, ST_H = 64, 16      # statistics tile
TILE_W, TILE_H1 = 128, 8  # matching tile
REDUCE, STATS, FULL, REFINE = range(4)


def level_dim(v, k):
    for _ in range(k):
        v = (v + 1) // 2
    return v


def cdiv(a, b):
    return -(-a // b)


class Seg:
    def __init__(self, typ, p, k, tx, ty, task0, band0, deps):
        self.type, self.pair, self.level = typ, p, k
        self.tiles_x, self.tiles_y = tx, ty
        self.task0, self.band0, self.deps = task0, band0, deps


def build_segments(pairs, n):
    """Segments in the removed scheduler's order: all reduces by level, all
    statistics, then the matching from each pair's coarsest level down."""
    segs, ntasks, nbands = [], 0, 0
    K = [k for _, _, k in pairs]
    Kmax = max(K)
    red, sta, mat = {}, {}, {}

    def add(typ, p, k, tx, ty, deps):
        nonlocal ntasks, nbands
        segs.append(Seg(typ, p, k, tx, ty, ntasks, nbands, [d for d in deps if d is not None]))
        ntasks += tx * ty
        nbands += ty
        return len(segs) - 1

    for k in range(1, Kmax):
        for p, (h0, w0, Kp) in enumerate(pairs):
            if k < Kp:
                h, w = level_dim(h0, k), level_dim(w0, k)
                red[p, k] = add(REDUCE, p, k, cdiv(w, RD_W), cdiv(h, RD_H), [red.get((p, k - 1))])
    for k in range(Kmax):
        for p, (h0, w0, Kp) in enumerate(pairs):
            if k < Kp:
                h, w = level_dim(h0, k), level_dim(w0, k)
                sta[p, k] = add(STATS, p, k, cdiv(w, ST_W), cdiv(h, ST_H), [red.get((p, k))])
    for d in range(Kmax):
        for p, (h0, w0, Kp) in enumerate(pairs):
            k = Kp - 1 - d
            if k < 0:
                continue
            h, w = level_dim(h0, k), level_dim(w0, k)
            coarsest = k == Kp - 1
            mat[p, k] = add(FULL if coarsest else REFINE, p, k, cdiv(w, TILE_W), cdiv(h, TILE_H1),
                            [sta[p, k], None if coarsest else mat[p, k + 1]])
    return segs, ntasks, nbands


def level_h(pairs, s):
    return level_dim(pairs[s.pair][0], s.level)


def dep_bands(pairs, s, d, ty, n):
    """The removed kernel's rule: the band range of dependency d that a task
    of s at tile row ty waits on."""
    if s.type == REDUCE:
        r0, r1, dh = 2 * RD_H * ty - 2, 2 * RD_H * ty + 2 * RD_H, RD_H
    elif s.type == STATS:
        r0, r1, dh = ST_H * ty - n, ST_H * ty + ST_H - 1 + n, RD_H
    elif d.type == STATS:
        r0, r1, dh = TILE_H1 * ty, TILE_H1 * ty + TILE_H1 - 1, ST_H
    else:
        r0, r1, dh = (TILE_H1 * ty) >> 1, (TILE_H1 * ty + TILE_H1 - 1) >> 1, TILE_H1
    Hd = level_h(pairs, d)
    return max(0, r0) // dh, min(Hd - 1, r1) // dh


def reads(pairs, s, ty, n):
    """Rows each tile reads from buffers other tiles write, from the tile's own
    stencil: {(buffer, pair, level): (first row, last row)}.  Level 0's image
    is the input (written by no tile)."""
    H = level_h(pairs, s)
    out = {}
    if s.type == REDUCE:  # 5-tap reduce of level k - 1, clamped reads
        Hp = level_dim(pairs[s.pair][0], s.level - 1)
        o0, o1 = RD_H * ty, min(H - 1, RD_H * ty + RD_H - 1)
        if s.level - 1 >= 1:
            out["img", s.pair, s.level - 1] = (max(0, 2 * o0 - 2), min(Hp - 1, 2 * o1 + 2))
    elif s.type == STATS:  # (2n+1)-row windows of its own rows
        y0, y1 = ST_H * ty, min(H - 1, ST_H * ty + ST_H - 1)
        if s.level >= 1:
            out["img", s.pair, s.level] = (max(0, y0 - n), min(H - 1, y1 + n))
    else:  # its own rows' statistics, its windows' image rows, the coarser map
        y0, y1 = TILE_H1 * ty, min(H - 1, TILE_H1 * ty + TILE_H1 - 1)
        out["stat", s.pair, s.level] = (y0, y1)
        if s.level >= 1:
            out["img", s.pair, s.level] = (max(0, y0 - n), min(H - 1, y1 + n))
        if s.type == REFINE:
            out["map", s.pair, s.level + 1] = (y0 >> 1, y1 >> 1)
    return out


def writer(s):
    """Buffer a segment's tiles write and the rows per band."""
    if s.type == REDUCE:
        return ("img", s.pair, s.level), RD_H
    if s.type == STATS:
        return ("stat", s.pair, s.level), ST_H
    return ("map", s.pair, s.level), TILE_H1


PAIR_SETS = {
    # the configurations' shapes: single pairs, the fwd+bwd batches, and odd sizes
    "configs": [(240, 320, 2), (992, 1436, 4), (540, 960, 4), (1988, 2880, 5)],
    "odd": [(1, 1, 1), (3, 70, 2), (33, 129, 3), (17, 17, 4), (130, 257, 3), (9, 600, 5)],
}


def _waits(pairs, segs, n):
    """(segment, tile row) -> list of (dependency segment, band lo, band hi)."""
    w = {}
    for si, s in enumerate(segs):
        for ty in range(s.tiles_y):
            w[si, ty] = [(di, *dep_bands(pairs, s, segs[di], ty, n)) for di in s.deps]
    return w


@pytest.mark.parametrize("key", sorted(PAIR_SETS))
@pytest.mark.parametrize("n", [3, 4, 5])
def test_awaited_bands_exist_and_come_earlier(key, n):
    pairs = PAIR_SETS[key]
    segs, ntasks, nbands = build_segments(pairs, n)
    waits = _waits(pairs, segs, n)
    for (si, ty), lst in waits.items():
        s = segs[si]
        first_task = s.task0 + ty * s.tiles_x
        for di, lo, hi in lst:
            d = segs[di]
            assert di < si
            assert 0 <= lo <= hi < d.tiles_y, (key, si, ty, di, lo, hi, d.tiles_y)
            last_awaited = d.task0 + (hi + 1) * d.tiles_x - 1
            assert last_awaited < first_task
    assert segs[-1].task0 + segs[-1].tiles_x * segs[-1].tiles_y == ntasks
    assert segs[-1].band0 + segs[-1].tiles_y == nbands


@pytest.mark.parametrize("key", sorted(PAIR_SETS))
@pytest.mark.parametrize("n", [3, 4, 5])
def test_awaited_bands_cover_every_row_read(key, n):
    pairs = PAIR_SETS[key]
    segs, _, _ = build_segments(pairs, n)
    waits = _waits(pairs, segs, n)
    producer = {writer(s)[0]: (si, writer(s)[1]) for si, s in enumerate(segs)}
    # bands complete before a tile of (segment, row) starts: the awaited bands
    # and, transitively, everything their tiles waited on
    memo = {}

    def closure(si, ty):
        if (si, ty) in memo:
            return memo[si, ty]
        done = set()
        for di, lo, hi in waits[si, ty]:
            for b in range(lo, hi + 1):
                if (di, b) not in done:
                    done.add((di, b))
                    done |= closure(di, b)
        memo[si, ty] = done
        return done

    for si, s in enumerate(segs):
        for ty in range(s.tiles_y):
            done = closure(si, ty)
            for buf, (r0, r1) in reads(pairs, s, ty, n).items():
                di, bh = producer[buf]
                for b in range(r0 // bh, r1 // bh + 1):
                    assert (di, b) in done, (key, s.type, s.pair, s.level, ty, buf, b)


@pytest.mark.parametrize("workers", [1, 3, 16, 64])
def test_scheduler_run_ends(workers):
    """Worker threads take task numbers from one counter, wait on their bands,
    then bump their own band, as the workgroups did; every run ends and every
    band reaches its count."""
    pairs = PAIR_SETS["configs"][:3] + PAIR_SETS["odd"]
    n = 4
    segs, ntasks, nbands = build_segments(pairs, n)
    waits = _waits(pairs, segs, n)
    task0s = [s.task0 for s in segs]
    counters = [0] * nbands
    cond = threading.Condition()
    head = [0]
    failed = []

    def work():
        while True:
            with cond:
                t = head[0]
                head[0] += 1
            if t >= ntasks:
                return
            si = bisect.bisect_right(task0s, t) - 1
            s = segs[si]
            ty = (t - s.task0) // s.tiles_x
            with cond:
                for di, lo, hi in waits[si, ty]:
                    d = segs[di]
                    for b in range(lo, hi + 1):
                        if not cond.wait_for(lambda: counters[d.band0 + b] >= d.tiles_x, timeout=30):
                            failed.append((t, di, b))
                            return
                counters[s.band0 + ty] += 1
                cond.notify_all()

    threads = [threading.Thread(target=work) for _ in range(workers)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not failed
    for s in segs:
        assert all(counters[s.band0 + b] == s.tiles_x for b in range(s.tiles_y))
