"""CPU replica of the persistent batching launch's work queue (k_multi.hip):
the phase-major item numbering, every wait and signal, and the index range
of every counter, workspace array and LDS slot each item touches, for the
six-index set of the GPU tests under every tile shape the autotuner can
pick.  A discrete-event schedule with 1 .. 8192 resident waves and random
item durations must drain (no wait left unsatisfied), every wait must be
satisfied by items numbered before the waiting one, and no access may leave
its allocation.  The replica follows the kernel's source text; it runs no
GPU code."""
import math
import random

import pytest

MULTI_CTR_TILES, MULTI_TILE_CTRS = 16, 5
PH = ["QH", "HIST", "THR", "TIE", "EMIT", "RR", "MERGE"]
RR_TILE_FLOATS = 64 * 36
KMAX_SPLIT = 64

# (n, d, m, L, nq, T) of the GPU test set; sub-dataset sizes follow the
# percentile partition (sizes differ by at most one)
SET = [(3000, 64, 8, 32, 70, 300), (1500, 33, 3, 16, 1, 1500), (5000, 128, 16, 64, 130, 700),
       (800, 20, 1, 48, 64, 9), (4100, 256, 16, 32, 5, 2000), (2200, 100, 7, 63, 200, 4000)]
K = 10


def cdiv(a, b):
    return -(-a // b)


def offsets(n, m):
    # sub-dataset j holds ranks [ceil(j n / m), ceil((j + 1) n / m))
    return [cdiv(j * n, m) for j in range(m + 1)]


def lay_out(chunk, slice_):
    """The plan's descriptors, allocation sizes and item numbering."""
    descs, tiles_before, q_before = [], 0, 0
    for (n, d, m, L, nq, T) in SET:
        Tq = min(T, n)
        off = offsets(n, m)
        maxsub = max(off[j + 1] - off[j] for j in range(m))
        sl = slice_
        if cdiv(Tq, sl) > KMAX_SPLIT:
            sl = cdiv(cdiv(Tq, KMAX_SPLIT), 64) * 64
        D = dict(n=n, d=d, m=m, L=L, W=1 if L <= 32 else 2, nq=nq, Tq=Tq, off=off, chunk=chunk,
                 nch=max(1, cdiv(maxsub, chunk)), slice=sl, nsplit=cdiv(Tq, sl),
                 tile_base=tiles_before, q_base=q_before, tiles=cdiv(nq, 64))
        tiles_before += D["tiles"]
        q_before += nq
        # workspace arrays (elements)
        D["size"] = dict(qcodes=nq * D["W"], ghist=D["tiles"] * m * (L + 1) * 64, ghthr=D["tiles"] * m * 64,
                         gtie=D["tiles"] * 4 * 64, gpstar=nq, cand=nq * Tq,
                         part=nq * D["nsplit"] * K if D["nsplit"] > 1 else 0,
                         gtheta=nq if D["nsplit"] > 1 else 0, codes=n * D["W"], R=m * (L + 1), inv=m * (L + 1),
                         At=d * L, Q=nq * d, Xl=n * cdiv(d, 8) * 8, perm=n, out=nq * K)
        descs.append(D)
    ntiles, nq_total = tiles_before, q_before
    ctr_words = MULTI_CTR_TILES + MULTI_TILE_CTRS * ntiles + 2 * nq_total
    seg, run = [], 0
    for ph in range(7):
        for D in descs:
            seg.append(run)
            c = [cdiv(D["nq"], 16), D["tiles"] * D["m"] * D["nch"], D["tiles"], D["nq"],
                 D["tiles"] * D["m"] * D["nch"], D["nq"] * D["nsplit"],
                 D["nq"] if D["nsplit"] > 1 else 0][ph]
            run += c
    seg.append(run)
    maxL = max(D["L"] for D in descs)
    lds = max((maxL + 1) * 64 * 4, RR_TILE_FLOATS * 4)
    return descs, seg, ntiles, nq_total, ctr_words, lds


class Bounds:
    def __init__(self, ctr_words, lds):
        self.ctr_words, self.lds = ctr_words, lds

    def ctr(self, i):
        assert 0 <= i < self.ctr_words, f"counter {i} outside {self.ctr_words}"
        return i

    @staticmethod
    def arr(D, name, lo, hi):  # [lo, hi) of array `name`
        assert 0 <= lo <= hi <= D["size"][name], f"{name}[{lo}:{hi}] outside {D['size'][name]}"

    def lds_bytes(self, hi):
        assert hi <= self.lds, f"LDS {hi} > {self.lds}"


def tile_ctr(B, D, tile, ph):
    return B.ctr(MULTI_CTR_TILES + (D["tile_base"] + tile) * MULTI_TILE_CTRS + ph)


def item_plan(B, D, ph, u, nq_total):
    """(waits, signals) of item u of phase ph of pair D, checking every index
    the kernel's item body forms.  waits: [(counter, need)]."""
    m, L, W, nch, k = D["m"], D["L"], D["W"], D["nch"], K
    L1, ctr_q = L + 1, MULTI_CTR_TILES + MULTI_TILE_CTRS * B.ntiles
    tq = lambda t: min(64, D["nq"] - t * 64)  # noqa: E731
    if ph == 0:  # QH: 16 queries
        q0, q1 = u * 16, min(D["nq"], u * 16 + 16)
        assert q0 < q1
        B.arr(D, "Q", q0 * D["d"], q1 * D["d"])
        B.arr(D, "At", 0, D["d"] * L)
        B.arr(D, "qcodes", q0 * W, q1 * W)
        if D["nsplit"] > 1:
            B.arr(D, "gtheta", q0, q1)
        return [], [tile_ctr(B, D, q0 >> 6, 0)]
    if ph in (1, 4):  # HIST / EMIT: (tile, sub-dataset, chunk)
        per_tile = m * nch
        tile, r = divmod(u, per_tile)
        j, c = divmod(r, nch)
        assert tile < D["tiles"] and j < m
        p0 = D["off"][j] + c * D["chunk"]
        p1 = min(D["off"][j + 1], p0 + D["chunk"])
        if p0 < p1:
            B.arr(D, "codes", p0 * W, p1 * W)
            B.arr(D, "qcodes", tile * 64 * W, (tile * 64 + tq(tile)) * W)
        if ph == 1:
            waits = [(tile_ctr(B, D, tile, 0), cdiv(tq(tile), 16))]
            if p0 < p1:
                B.lds_bytes(L1 * 64 * 4)
                B.arr(D, "ghist", ((tile * m + j) * L1) * 64, ((tile * m + j) * L1 + L1) * 64)
            return waits, [tile_ctr(B, D, tile, 1)]
        waits = [(tile_ctr(B, D, tile, 3), tq(tile))]
        if p0 < p1:
            B.arr(D, "ghthr", (tile * m + j) * 64, (tile * m + j) * 64 + 64)
            B.arr(D, "gtie", tile * 256, tile * 256 + 128)
            B.arr(D, "gpstar", tile * 64, tile * 64 + tq(tile))
            for q in range(tile * 64, tile * 64 + tq(tile)):
                B.ctr(ctr_q + D["q_base"] + q)
                # writes cand[q Tq + base + w] for w < min(cnt, Tq - base) only
                B.arr(D, "cand", q * D["Tq"], q * D["Tq"] + D["Tq"])
        return waits, [tile_ctr(B, D, tile, 4)]
    if ph == 2:  # THR: a tile
        tile = u
        P = m * L1
        B.arr(D, "ghist", tile * P * 64, (tile + 1) * P * 64)
        B.arr(D, "inv", 0, P)
        B.arr(D, "R", 0, m * L1)
        B.arr(D, "ghthr", tile * m * 64, (tile + 1) * m * 64)
        B.arr(D, "gtie", tile * 256, tile * 256 + 256)
        return [(tile_ctr(B, D, tile, 1), m * nch)], [tile_ctr(B, D, tile, 2)]
    if ph == 3:  # TIE: a query
        q = u
        tile = q >> 6
        B.arr(D, "gtie", tile * 256, tile * 256 + 192)
        B.arr(D, "gpstar", q, q + 1)
        B.arr(D, "codes", 0, D["n"] * W)  # some sub-dataset's range
        return [(tile_ctr(B, D, tile, 2), 1)], [tile_ctr(B, D, tile, 3)]
    if ph == 5:  # RR: a slice of a query's list
        q, split = divmod(u, D["nsplit"])
        B.ctr(ctr_q + D["q_base"] + q)
        cbeg = split * D["slice"]
        cend = min(D["Tq"], cbeg + D["slice"])
        assert cbeg < D["Tq"], "empty slice"
        B.arr(D, "cand", q * D["Tq"] + cbeg, q * D["Tq"] + cend)
        B.lds_bytes(RR_TILE_FLOATS * 4)
        waits = [(tile_ctr(B, D, q >> 6, 4), m * nch)]
        if D["nsplit"] == 1:
            B.arr(D, "out", q * k, q * k + k)
            return waits, []
        B.arr(D, "part", (q * D["nsplit"] + split) * k, (q * D["nsplit"] + split + 1) * k)
        return waits, [B.ctr(ctr_q + nq_total + D["q_base"] + q)]
    q = u  # MERGE
    B.arr(D, "part", q * D["nsplit"] * k, (q + 1) * D["nsplit"] * k)
    B.arr(D, "out", q * k, q * k + k)
    return [(B.ctr(ctr_q + nq_total + D["q_base"] + q), D["nsplit"])], []


def build_items(chunk, slice_):
    descs, seg, ntiles, nq_total, ctr_words, lds = lay_out(chunk, slice_)
    B = Bounds(ctr_words, lds)
    B.ntiles = ntiles
    nb = len(descs)
    items = []
    for w in range(seg[-1]):
        lo = max(i for i in range(len(seg) - 1) if seg[i] <= w)
        ph, b = divmod(lo, nb)
        items.append(item_plan(B, descs[b], ph, w - seg[lo], nq_total))
    return items, ctr_words


def schedule(items, ctr_words, waves, seed):
    """Discrete-event run of the work queue: `waves` resident waves take the
    next item number; a wave waits until each of its item's counters reaches
    its need, works for a random time, then signals.  Returns True when the
    queue drains."""
    rng = random.Random(seed)
    ctr = [0] * ctr_words
    total = len(items)
    head = 0
    # state of each wave: (item, ready time) or None once it has exited
    t = 0.0
    busy = {}  # wave -> (item, finish time) for items whose waits are satisfied
    waiting = {}  # wave -> item
    free = list(range(waves))
    done = 0
    steps = 0
    while done < total:
        steps += 1
        assert steps < 50 * total + 10 * waves, "no progress"
        # idle waves take the next numbers
        while free and head < total:
            wv = free.pop()
            waiting[wv] = head
            head += 1
        # waits satisfied now start working
        for wv, it in list(waiting.items()):
            if all(ctr[c] >= need for c, need in items[it][0]):
                busy[wv] = (it, t + rng.expovariate(1.0))
                del waiting[wv]
        if not busy:
            # every resident wave waits: only possible if some wait depends
            # on an item no wave has taken or can finish
            raise AssertionError(f"deadlock at item {min(waiting.values())} with {len(waiting)} waiting")
        wv, (it, t_end) = min(busy.items(), key=lambda kv: kv[1][1])
        t = t_end
        del busy[wv]
        for c in items[it][1]:
            ctr[c] += 1
        done += 1
        if head < total:
            free.append(wv)
    return ctr


@pytest.mark.parametrize("chunk", [4096, 16384, 65536])
@pytest.mark.parametrize("slice_", [512, 1024, 2048, 4096])
def test_persistent_queue_bounds_and_order(chunk, slice_):
    items, ctr_words = build_items(chunk, slice_)
    # every wait is on counters signalled only by items numbered before it,
    # and reaches exactly its need once they are done
    signals = {}
    for i, (_, sig) in enumerate(items):
        for c in sig:
            signals.setdefault(c, []).append(i)
    for i, (waits, _) in enumerate(items):
        for c, need in waits:
            src = signals.get(c, [])
            assert len(src) == need, f"item {i}: counter {c} gets {len(src)} signals, waits for {need}"
            assert all(s < i for s in src), f"item {i} waits on a later item"


@pytest.mark.parametrize("waves", [1, 3, 64, 8192])
def test_persistent_queue_drains(waves):
    items, ctr_words = build_items(16384, 1024)
    for seed in range(3):
        ctr = schedule(items, ctr_words, waves, seed)
        assert max(ctr) <= len(items)
