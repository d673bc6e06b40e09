"""A CPU model of the batch packing in k_tile_prep: greedy packing of a tile's pixels into
LDS batches of at most HAIR_PIXEL_CAPACITY fragments (Sec. 5.2, the per-pixel lists that the
shading pass orders, taken one batch of whole pixels at a time).

Every pixel t knows the next non-empty pixel at or after it (nxt) and the end of the batch that
would start at it (end: the longest run of whole pixels that fits, or t + 1 for a pixel deeper
than a batch).  The batch starts form the chain p_0 = nxt[0], p_{i+1} = nxt[end[p_i]].  A short
chain is followed by one lane; a long one is marked by pointer doubling over the tile's lanes:
jump[t] = nxt[end[t]], eight rounds of "a marked t marks jump[t], then jump[t] = jump[jump[t]]"
(a tile has at most 256 batches).  Within a round the lanes read the marks while others write
them; the model runs the lanes in random orders, which covers every interleaving's outcome since
an early-seen mark only spreads further along the same chain.  Both must mark the same pixels.
"""
import numpy as np
import pytest

P = 256   # pixels per tile


def _nxt_end(cnt, cap):
    off = np.zeros(P + 1, np.int64)
    off[1:] = np.cumsum(cnt)
    nxt = np.empty(P + 1, np.int64)
    end = np.empty(P, np.int64)
    for t in range(P):
        q = t
        while q < P and not off[q + 1] > off[t]:
            q += 1
        nxt[t] = q
        if cnt[t] > cap:
            end[t] = t + 1
        else:
            p1 = t + 1
            while p1 + 1 <= P and off[p1 + 1] - off[t] <= cap:
                p1 += 1
            end[t] = p1
    nxt[P] = P
    return nxt, end


def _serial(nxt, end):
    marks, p = set(), nxt[0]
    while p < P:
        marks.add(int(p))
        p = nxt[end[p]]
    return marks


def _doubling(nxt, end, rng, rounds=8):
    jump = np.empty(P + 1, np.int64)
    jump[:P] = nxt[end]
    jump[P] = P
    on = np.zeros(P + 1, bool)
    on[nxt[0]] = True
    for _ in range(rounds):
        j = jump.copy()
        for t in rng.permutation(P):   # racy reads of the marks, in some lane order
            if on[t]:
                on[j[t]] = True
        jump[:P] = j[j[:P]]
    return set(np.nonzero(on[:P])[0].tolist())


def _greedy(cnt, cap):
    """The packing written out directly: skip empty pixels, take whole pixels while they fit."""
    starts, p = set(), 0
    while p < P:
        while p < P and cnt[p] == 0:
            p += 1
        if p == P:
            break
        starts.add(p)
        if cnt[p] > cap:
            p += 1
            continue
        tot = 0
        while p < P and tot + cnt[p] <= cap:
            tot += cnt[p]
            p += 1
    return starts


def _cases(rng, cap):
    yield np.zeros(P, np.int64)
    yield np.full(P, cap, np.int64)                     # 256 batches: the longest chain
    yield np.full(P, cap + 1, np.int64)                 # every pixel deeper than a batch
    for trial in range(60):
        mode = trial % 4
        if mode == 0:
            yield rng.integers(0, 3 * cap // 256 + 1, P)
        elif mode == 1:
            yield rng.integers(0, cap // 8, P) * (rng.random(P) < 0.5)
        elif mode == 2:
            yield (rng.random(P) < 0.1) * rng.integers(cap // 2, 3 * cap, P)
        else:
            yield rng.integers(cap // 3, cap + 1, P)


@pytest.mark.parametrize("cap", [1536, 512])
def test_pointer_doubling_marks_the_greedy_batch_starts(cap):
    rng = np.random.default_rng(cap)
    for cnt in _cases(rng, cap):
        nxt, end = _nxt_end(cnt, cap)
        want = _greedy(cnt, cap)
        assert _serial(nxt, end) == want
        assert _doubling(nxt, end, rng) == want


def test_seven_rounds_miss_the_end_of_a_256_batch_chain():
    cap = 1536
    cnt = np.full(P, cap, np.int64)
    nxt, end = _nxt_end(cnt, cap)
    rng = np.random.default_rng(0)
    # lanes in increasing order let an early mark spread within a round, so run them in
    # decreasing order, the slowest spread
    class Rev:
        def permutation(self, n):
            return np.arange(n)[::-1]
    assert len(_doubling(nxt, end, Rev(), rounds=7)) == 128
    assert len(_doubling(nxt, end, Rev(), rounds=8)) == 256
    assert len(_doubling(nxt, end, rng, rounds=8)) == 256
