"""Host logic of the group dispatch orders (bhq_plan_order, CPU only):
every group is launched exactly once, the cost order is longest first,
and the XCD order cuts the groups into contiguous pieces of near-equal
cost, one per XCD, each sorted longest first inside windows (fixed-size
windows, then one tail window at the end of the piece)."""
import numpy as np
import pytest

from paper_1812_07313_amd import bhq


def _offsets(rng, ng, empty_frac=0.0):
    ni = rng.integers(1, 257, ng)
    ni[rng.random(ng) < empty_frac] = 0
    njp = rng.integers(0, 3000, ng)
    njc = rng.integers(0, 3000, ng)
    cat = lambda v: np.concatenate([[0], np.cumsum(v)]).astype(np.int64)
    cost = ni * (100 * njp + 265 * njc + 100)
    return cat(ni), cat(njp), cat(njc), cost


def test_cost_order_is_longest_first():
    rng = np.random.default_rng(3)
    i_off, jp_off, jc_off, cost = _offsets(rng, 1000)
    o = bhq.bhq_plan_order(i_off, jp_off, jc_off, bhq.ORDER_COST)
    assert sorted(o.tolist()) == list(range(1000))
    assert np.all(np.diff(cost[o]) <= 0)
    # ties keep the group order (stable)
    i_off = np.arange(0, 11, dtype=np.int64)
    z = np.zeros(11, dtype=np.int64)
    assert bhq.bhq_plan_order(i_off, z, z, bhq.ORDER_COST).tolist() == list(range(10))


def _windows(k, window, tail):
    """[start, end) of the windows of a piece of k groups."""
    body = max(k - tail, 0)
    w = [(s, min(body, s + window)) for s in range(0, body, window)]
    if body < k:
        w.append((body, k))
    return w


@pytest.mark.parametrize("ng,window,tail,xcds", [
    (1, 256, 1024, 8), (5, 256, 1024, 8), (1000, 256, 0, 8),
    (17914, 256, 1024, 8), (17914, 100, 333, 8), (3001, 7, 50, 3),
    (64, 1, 0, 1), (40000, 256, 1024, 8), (70000, 256, 1024, 8)])
def test_xcd_order_pieces_and_windows(ng, window, tail, xcds):
    rng = np.random.default_rng(ng + window)
    i_off, jp_off, jc_off, cost = _offsets(rng, ng, empty_frac=0.05)
    o = bhq.bhq_plan_order(i_off, jp_off, jc_off, bhq.ORDER_XCD, window, tail,
                           xcds)
    assert len(o) % xcds == 0
    real = o[o >= 0]
    assert sorted(real.tolist()) == list(range(ng))          # each group once
    assert len(o) <= xcds * ng
    total = cost.sum()
    prev_hi = -1
    for x in range(xcds):
        piece = o[x::xcds]
        k = int(np.sum(piece >= 0))
        assert np.all(piece[:k] >= 0) and np.all(piece[k:] == -1)  # padding last
        piece = piece[:k]
        if k == 0:
            continue
        # contiguous range of groups, after the previous piece's
        lo, hi = piece.min(), piece.max()
        assert hi - lo + 1 == k and lo == prev_hi + 1
        prev_hi = hi
        # windows: consecutive groups, each sorted longest first
        for s, e in _windows(k, window, tail):
            win = piece[s:e]
            assert sorted(win.tolist()) == list(range(lo + s, lo + e))
            assert np.all(np.diff(cost[win]) <= 0)
        # near-equal cost: within one group's cost of the even share
        assert abs(cost[piece].sum() - total / xcds) <= cost.max() + 1e-9 * total
    assert prev_hi == ng - 1
    # the slot count is set by the longest piece
    assert len(o) == xcds * max(int(np.sum(o[x::xcds] >= 0)) for x in range(xcds))


def test_xcd_order_small_hand_case():
    """4 groups of equal cost on 2 XCDs, window 1, no tail: groups 0,1 ->
    XCD 0 and 2,3 -> XCD 1, slots interleaved."""
    i_off = np.array([0, 1, 2, 3, 4])
    jp_off = np.array([0, 2, 4, 6, 8])
    jc_off = np.zeros(5, dtype=np.int64)
    o = bhq.bhq_plan_order(i_off, jp_off, jc_off, bhq.ORDER_XCD, 1, 0, 2)
    assert o.tolist() == [0, 2, 1, 3]
    # one heavy group takes a piece by itself; the other piece is padded
    jp_off = np.array([0, 100, 101, 102, 103])
    o = bhq.bhq_plan_order(i_off, jp_off, jc_off, bhq.ORDER_XCD, 256, 0, 2)
    assert o.tolist() == [0, 1, -1, 2, -1, 3]
    # a tail window sorts the end of the piece: costs 1*(k+1) rising
    i_off = np.arange(7)
    jp_off = np.concatenate([[0], np.cumsum(np.arange(1, 7))])
    jc_off = np.zeros(7, dtype=np.int64)
    o = bhq.bhq_plan_order(i_off, jp_off, jc_off, bhq.ORDER_XCD, 1, 3, 1)
    assert o.tolist() == [0, 1, 2, 5, 4, 3]


def test_plan_order_errors():
    i_off = np.array([0, 1, 2])
    z = np.zeros(3, dtype=np.int64)
    for mode, window, tail, xcds in ((2, 256, 0, 8), (1, 0, 0, 8),
                                     (1, 256, -1, 8), (1, 256, 0, 0),
                                     (1, 256, 0, 65), (1, (1 << 24) + 1, 0, 8),
                                     (1, 256, (1 << 24) + 1, 8)):
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_plan_order(i_off, z, z, mode, window, tail, xcds)
        assert ei.value.code == bhq.E_ARG
    with pytest.raises(bhq.BhqError) as ei:
        bhq.bhq_plan_order(np.array([0, 2, 1]), z, z)
    assert ei.value.code == bhq.E_RANGE
    with pytest.raises(bhq.BhqError) as ei:
        bhq.bhq_plan_order(np.array([1, 2, 3]), z, z)
    assert ei.value.code == bhq.E_RANGE
