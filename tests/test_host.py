"""Host-side logic that needs no GPU: the server's batch selection and the
seeded request generator."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1605_05236_amd import inputs
from paper_1605_05236_amd.serve import take_batch


def _queues(table, pending):
    q = {}
    for i in pending:
        q.setdefault(int(table[i]), []).append(int(i))
    return q


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("max_ops", [1, 50, 400, 20000, 1 << 30])
def test_take_batch_keeps_fifo_and_coalesces(seed, max_ops):
    rng = np.random.default_rng(seed)
    R = 1500  # pending sets beyond the first scan window (256 requests)
    table = rng.integers(0, 7 if seed % 2 else 300, R)
    kind = rng.integers(0, 3, R)
    n = rng.integers(0, 40, R)
    pending = np.sort(rng.choice(R, 1000, replace=False))
    rounds = 0
    order = []
    while pending.size:
        before = _queues(table, pending)
        taken, rest = take_batch(kind, table, n, pending, max_ops)
        assert taken.size >= 1 and taken[0] == pending[0]
        assert np.all(np.diff(taken) > 0) and np.all(np.diff(rest) > 0)
        assert np.array_equal(np.sort(np.concatenate([taken, rest])), pending)
        assert n[taken].sum() <= max_ops or taken.size == 1
        got = _queues(table, taken)
        for t, lst in got.items():
            q = before[t]
            assert lst == q[:len(lst)]  # a prefix of the table's queue
            assert len({int(kind[i]) for i in lst}) == 1  # one kind per table
            if max_ops >= n.sum():  # unbounded: the whole same-kind head run
                j = len(lst)
                assert j == len(q) or kind[q[j]] != kind[q[0]]
        if max_ops >= n.sum():
            assert set(got) == set(before)  # every table with work takes part
        order.extend(taken.tolist())
        pending = rest
        rounds += 1
    # per table, the requests ran in arrival order
    for t, lst in _queues(table, np.array(order)).items():
        assert lst == sorted(lst)


def test_request_stream_records_respect_their_ranges():
    bins = inputs.group_tables(3, 48, 7, 11)
    rs = inputs.RequestStream(4, bins, 4, 0.5, 41, max_ops=300)
    req = rs.take(2000)
    rec = rs.records_torch(req, device="cpu").numpy()
    off = np.concatenate([[0], np.cumsum(req["n"])])
    assert rec.size == off[-1]
    lk = []
    for i in range(2000):
        x, t = rec[off[i]:off[i + 1]], req["table"][i]
        if req["kind"][i] == 0:
            h = x < rs.miss_start
            assert np.all((x[h] >= rs.pre_start[t]) & (x[h] < rs.pre_start[t] + rs.half[t]))
            lk.append(x)
        elif req["kind"][i] == 2:
            assert np.all((x >= rs.pre_start[t] + rs.pre[t] // 2) & (x < rs.pre_start[t] + rs.pre[t]))
        else:
            assert np.all((x >= rs.fresh_start[t]) & (x < rs.fresh_start[t] + rs.fresh_cap[t]))
    writes = np.concatenate([rec[off[i]:off[i + 1]] for i in range(2000) if req["kind"][i]])
    assert np.unique(writes).size == writes.size  # no record inserted or deleted twice
    lk = np.concatenate(lk)
    assert abs((lk < rs.miss_start).mean() - 0.9) < 0.01
    # chunked generation (any split) gives the same records
    a = rs.records_torch(req, 0, 700, device="cpu").numpy()
    b = rs.records_torch(req, 700, 2000, device="cpu").numpy()
    assert np.array_equal(np.concatenate([a, b]), rec)


def test_payload_matches_key_stream():
    bins = inputs.group_tables(3, 8, 7, 9)
    rs = inputs.RequestStream(4, bins, 4, 0.5, 41, max_ops=64)
    req = rs.take(300)
    k, v, e = rs.payload(req, device="cpu", chunk_ops=500, pin=False)
    rec = rs.records_torch(req, device="cpu").numpy()
    total = rec.size
    kk, vv = inputs.keys_values(41, int(rec.max()) + 1)
    assert np.array_equal(k.numpy()[:total].view(np.uint64), kk[rec])
    assert np.array_equal(v.numpy()[:total].view(np.uint64), vv[rec])
    assert np.array_equal(e.numpy()[:total], (rec < rs.miss_start).astype(np.uint8))
    pk, pv = rs.prefill_payload(device="cpu", chunk_ops=333, pin=False)
    npre = int(rs.pre.sum())
    assert np.array_equal(pk.numpy()[:npre].view(np.uint64), kk[:npre] if kk.size >= npre
                          else inputs.keys_values(41, npre)[0])


# ---------------------------------------------------------------------------
# the torch image checker (used at full size on the GPU) agrees with the numpy
# checker on oracle images and catches the same planted faults
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme,B,d,ghost", [("queue", 4, 2, True), ("bfs", 8, 2, False),
                                              ("rattle", 1, 3, False),
                                              ("random_walk", 1, 4, False)])
def test_torch_checker_matches_numpy_checker(scheme, B, d, ghost):
    import checks
    import oracle
    n = 1 << 10
    load = 0.95 if B > 1 else 0.85
    keys, vals = inputs.keys_values(12, inputs.target_count(n, B, load),
                                    value_bits=32 if B == 1 else 64)
    o = oracle.OracleTable(n, B, d, scheme, ghost=ghost, hash_seed=77, rng_seed=78,
                           max_chain=1000, batch_ops=100)
    st = o.insert(keys, vals)["status"]
    img = o.export()
    rat = scheme == "rattle"
    stored = checks.check_invariants(img, n, B, d, 77, ghost=ghost, rattle=rat)
    assert checks.check_image_torch(img, n, B, d, 77, ghost=ghost, rattle=rat,
                                    device="cpu") == len(stored) == int((st == 1).sum())
    hb = checks.bins_of(keys[:500], n, d, 77)
    import torch
    ht = checks.bins_of_torch(torch.from_numpy(keys[:500].view(np.int64)), n, d, 77).numpy()
    assert np.array_equal(hb.astype(np.int64), ht)

    def planted(mutate):
        bad = {f: a.copy() for f, a in img.items()}
        mutate(bad)
        for fn in (lambda: checks.check_invariants(bad, n, B, d, 77, ghost=ghost, rattle=rat),
                   lambda: checks.check_image_torch(bad, n, B, d, 77, ghost=ghost, rattle=rat,
                                                    device="cpu")):
            with pytest.raises(AssertionError):
                fn()

    occ = np.nonzero(img["keys"] != checks.EMPTY)[0]
    empty = np.nonzero(img["keys"] == checks.EMPTY)[0]
    s0 = occ[0]
    others = [s for s in empty if s // B not in set(checks.bins_of(img["keys"][s0:s0 + 1], n, d,
                                                                   77)[0].tolist())]

    def move_out(bad):  # a key copied into a slot outside its bins
        bad["keys"][others[0]] = bad["keys"][s0]
        bad["keys"][s0] = checks.EMPTY

    def twice(bad):  # an unmarked second copy (in one of its own bins)
        hb0 = checks.bins_of(img["keys"][s0:s0 + 1], n, d, 77)[0]
        for bb in hb0.tolist():
            free = [s for s in range(bb * B, bb * B + B) if img["keys"][s] == checks.EMPTY]
            if free:
                bad["keys"][free[0]] = bad["keys"][s0]
                if rat:
                    bad["rattle"][free[0]] = 1 + hb0.tolist().index(bb)
                return
        bad["keys"][others[0]] = bad["keys"][s0]  # no room: falls back to a misplacement

    planted(move_out)
    planted(twice)
    if rat:
        def wrong_counter(bad):
            bad["rattle"][s0] = bad["rattle"][s0] % d + 1
        planted(wrong_counter)
    if ghost:
        def mark_single(bad):  # a duplicate mark with no twin
            s = next(x for x in occ if not (img["meta"][x // B] >> np.uint32(x % B)) & 1)
            bad["meta"][s // B] |= np.uint32(1 << (s % B))
        planted(mark_single)
