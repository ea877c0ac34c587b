"""CPU checks of the queued single launch's work sequence (gbmc_queue_schedule,
host-only): every pass covers every tile once, the per-block completion counts
match the items, and a model of the launch's protocol drains for any number of
resident workgroups and any completion order.

The model follows the launch as the kernel implements it: workgroups take
tickets in order when they become resident, each of a workgroup's W waves runs
one of W consecutive items of the sequence, an item of pass p > 0 waits until
every block it touches is final in pass p - 1, and the item that completes a
block's count in a pass finalizes that block for the pass.  No GPU is used."""
import ctypes as C

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def lib():
    from paper_1803_09652_amd import _lib
    return _lib.load()


def _i32p(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def queue(lib, sizes, precision=0, tuning=None):
    off = np.ascontiguousarray(np.concatenate([[0], np.cumsum(sizes)]), dtype=np.int32)
    n = np.zeros(3, dtype=np.int32)
    nb = C.c_int32()
    tp = C.byref(tuning) if tuning is not None else None
    assert lib.gbmc_queue_schedule(len(sizes), _i32p(off), precision, tp, _i32p(n), None,
                                   C.byref(nb), None) == 0
    items = np.zeros(7 * int(n.sum()), dtype=np.int32)
    tot = np.zeros(3 * nb.value, dtype=np.int32)
    assert lib.gbmc_queue_schedule(len(sizes), _i32p(off), precision, tp, _i32p(n),
                                   _i32p(items), C.byref(nb), _i32p(tot)) == 0
    return n, items.reshape(-1, 7), nb.value, tot.reshape(3, -1)


def blocks_of(it):
    """Distinct batch blocks an item touches: its i blocks, then its j blocks."""
    _, _, b0, I0, I1, J0, J1 = (int(v) for v in it)
    return [b0 + I for I in range(I0, I1)] + [b0 + J for J in range(max(J0, I1), J1)]


SIZES = [1, 64, 65, 0, 200, 2500, 130, 129, 700]


@pytest.mark.parametrize("precision", [0, 1])
def test_sequence_covers_every_tile_once_per_pass_in_pass_order(lib, precision):
    n, items, nb, tot = queue(lib, SIZES, precision)
    assert items.shape[0] == n.sum()
    # sequence order: the descreening pass, then energy, then chain
    assert np.all(np.diff(items[:, 0]) >= 0)
    assert [int((items[:, 0] == p).sum()) for p in range(3)] == list(n)
    first = np.concatenate([[0], np.cumsum([(s + 63) // 64 for s in SIZES])])
    assert nb == first[-1]
    for p in range(3):
        seen = set()
        for it in items[items[:, 0] == p]:
            _, sys_, b0, I0, I1, J0, J1 = (int(v) for v in it)
            assert b0 == first[sys_]
            assert 0 <= I0 < I1 <= J1 and J0 >= I0 and J0 < J1
            for I in range(I0, I1):
                for J in range(J0, J1):
                    assert (sys_, I, J) not in seen
                    seen.add((sys_, I, J))
        want = {(b, I, J) for b, s in enumerate(SIZES)
                for I in range((s + 63) // 64) for J in range(I, (s + 63) // 64)}
        assert seen == want


@pytest.mark.parametrize("precision", [0, 1])
def test_block_totals_count_the_items_touching_each_block(lib, precision):
    n, items, nb, tot = queue(lib, SIZES, precision)
    want = np.zeros((3, nb), dtype=np.int64)
    for it in items:
        for X in blocks_of(it):
            want[it[0], X] += 1
    assert np.array_equal(tot, want)
    # every block has its diagonal tile in every pass, so every count is
    # reached and every wait of the next pass ends
    assert np.all(tot >= 1)


def test_first_two_passes_run_system_by_system_largest_first(lib):
    n, items, nb, tot = queue(lib, SIZES)
    for p in (0, 1):
        sy = items[items[:, 0] == p, 1]
        # contiguous runs of one system, in decreasing system size (stable)
        runs = [int(s) for k, s in enumerate(sy) if k == 0 or s != sy[k - 1]]
        assert len(runs) == len(set(runs))
        order = sorted((b for b, s in enumerate(SIZES) if s > 0), key=lambda b: -SIZES[b])
        assert runs == order
    # the chain pass: decreasing cost (half tiles) over the whole batch
    it = items[items[:, 0] == 2]
    cost = 2 * (it[:, 4] - it[:, 3]) * (it[:, 6] - it[:, 5]) - (it[:, 5] == it[:, 3])
    assert np.all(np.diff(cost) <= 0)


def simulate(items, tot, nb, W, slots, rng):
    """Runs the launch's protocol with `slots` resident workgroups of W waves;
    at every step one runnable wave (chosen at random) completes its item.
    Returns the completion step of every item and the step at which every block
    became final in every pass; fails on a deadlock."""
    n = items.shape[0]
    blk = [blocks_of(it) for it in items]
    # items of each pass touching each block, and the blocks each item still
    # waits for (those not final in the preceding pass)
    users = [[[] for _ in range(nb)] for _ in range(3)]
    for k in range(n):
        for X in blk[k]:
            users[items[k, 0]][X].append(k)
    pending = np.array([0 if items[k, 0] == 0 else len(blk[k]) for k in range(n)])
    cnt = np.zeros((3, nb), dtype=np.int64)
    final_at = np.full((3, nb), -1, dtype=np.int64)
    done_at = np.full(n, -1, dtype=np.int64)
    group_of = np.arange(n) // W
    left = np.bincount(group_of, minlength=(n + W - 1) // W)
    next_ticket, n_res = 0, 0
    resident, runnable = set(), set()
    step = 0
    while True:
        while n_res < slots and next_ticket * W < n:
            for k in range(next_ticket * W, min(n, next_ticket * W + W)):
                resident.add(k)
                if pending[k] == 0:
                    runnable.add(k)
            next_ticket += 1
            n_res += 1
        if not resident:
            break
        assert runnable, f"deadlock with {slots} workgroups of {W} waves at step {step}"
        cand = sorted(runnable)
        k = cand[rng.integers(len(cand))]
        p = items[k, 0]
        for X in blk[k]:
            cnt[p, X] += 1
            assert cnt[p, X] <= tot[p, X]
            if cnt[p, X] == tot[p, X]:
                assert final_at[p, X] < 0
                final_at[p, X] = step
                if p < 2:
                    for u in users[p + 1][X]:
                        pending[u] -= 1
                        if pending[u] == 0 and u in resident:
                            runnable.add(u)
        done_at[k] = step
        step += 1
        resident.discard(k)
        runnable.discard(k)
        left[group_of[k]] -= 1
        if left[group_of[k]] == 0:
            n_res -= 1
    assert np.all(done_at >= 0)
    assert np.all(final_at >= 0)
    return done_at, final_at


@pytest.mark.parametrize("W,slots", [(1, 1), (1, 3), (8, 1), (4, 2), (8, 5), (2, 1000)])
def test_protocol_drains_and_orders_the_passes(lib, W, slots):
    sizes = [1, 64, 65, 0, 200, 130, 129, 700]
    n, items, nb, tot = queue(lib, sizes)
    rng = np.random.default_rng(W * 1000 + slots)
    done_at, final_at = simulate(items, tot, nb, W, slots, rng)
    for k, it in enumerate(items):
        p = it[0]
        for X in blocks_of(it):
            # a block is final in a pass only after every item of that pass
            # touching it (its sums are complete) ...
            assert final_at[p, X] >= done_at[k]
            # ... and an item of the next pass runs only after its blocks are
            if p > 0:
                assert done_at[k] > final_at[p - 1, X]
    if W == 1 and slots == 1:
        # one wave at a time: the items complete in sequence order
        assert np.array_equal(done_at, np.arange(items.shape[0]))


def test_protocol_drains_on_an_uneven_batch(lib):
    # the first 8 system sizes of the 64-system uneven batch (500-20,000 atoms)
    sizes = [n for n, _, _ in synth.uneven_batch_sizes(8)]
    n, items, nb, tot = queue(lib, sizes)
    rng = np.random.default_rng(5)
    simulate(items, tot, nb, 8, 64, rng)


def test_queue_schedule_rejects_bad_input(lib):
    from paper_1803_09652_amd import _lib as L
    n = np.zeros(3, dtype=np.int32)
    nb = C.c_int32()
    off = np.array([0, 10, 5], dtype=np.int32)
    assert lib.gbmc_queue_schedule(2, _i32p(off), 0, None, _i32p(n), None, C.byref(nb),
                                   None) == L.GBMC_ERR_INVALID
    off = np.array([0, 10], dtype=np.int32)
    assert lib.gbmc_queue_schedule(1, _i32p(off), 7, None, _i32p(n), None, C.byref(nb),
                                   None) == L.GBMC_ERR_INVALID
    assert lib.gbmc_queue_schedule(1, _i32p(off), 0, None, None, None, C.byref(nb),
                                   None) == L.GBMC_ERR_INVALID
    off = np.array([0], dtype=np.int32)
    assert lib.gbmc_queue_schedule(0, _i32p(off), 0, None, _i32p(n), None, C.byref(nb),
                                   None) == 0
    assert list(n) == [0, 0, 0] and nb.value == 0
