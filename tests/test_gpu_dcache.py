"""Device-resident cache stages (request / provision / assign on the GPU, then
the decode of the tasks they produce) against the CPU oracle.

Which request of a pair becomes its decode task and which slot it gets depend
on the order the device runs them, so the tests compare what is unique -- the
labels at every request's slot, the set of decoded pairs, the cache top and
the free-stack counts -- and check that the rest is valid: one slot per pair,
slots of distinct pairs disjoint and inside the cache, freed slots reused only
by pairs of their own size class."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

NEW, HIT, JOINED, FULL, INVALID = 0, 1, 2, 3, 4
NO_TASK = 0xFFFFFFFF
NO_SLOT = 0xFFFFFFFFFFFFFFFF


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_36898_amd as P
    vol = synth.voronoi_u32(256, 600, seed=21)
    c = oracle.encode_volume(vol, 5, nthreads=8)
    dv = P.DeviceVolume(c)
    return P, c, dv


class Batch:
    """One request call followed by the decode of the tasks it produced."""

    def __init__(self, P, dv, dc, plan, cache, cache_elems, ids, lods):
        import torch
        n = len(ids)
        self.ids = np.asarray(ids, np.uint32)
        self.lods = np.asarray(lods, np.uint8)
        d_ids = torch.from_numpy(self.ids.view(np.int32).copy()).cuda()
        d_lods = torch.from_numpy(self.lods.copy()).cuda()
        task = torch.full((n,), 7, dtype=torch.int32, device="cuda")
        slot = torch.full((n,), 7, dtype=torch.int64, device="cuda")
        state = torch.full((n,), 99, dtype=torch.int32, device="cuda")
        status = torch.full((n,), 99, dtype=torch.int32, device="cuda")
        stream = torch.cuda.current_stream()
        _say("dcache request + decode of", n, "requests")
        dc.request(stream, d_ids, d_lods, n, task, slot, state)
        plan.launch(stream, dv.tensor, task, d_lods, slot, n, cache, cache_elems, status)
        torch.cuda.synchronize()
        self.task = task.cpu().numpy().view(np.uint32)
        self.slot = slot.cpu().numpy().view(np.uint64)
        self.state = state.cpu().numpy()
        self.status = status.cpu().numpy()
        # decode tasks are exactly the NEW requests, with their own brick ids
        new = self.state == NEW
        assert np.array_equal(self.task[new], self.ids[new])
        assert (self.task[~new] == NO_TASK).all()
        assert (self.status[new] == 0).all() and (self.status[~new] == 1).all()
        assert (self.slot[(self.state == FULL) | (self.state == INVALID)] == NO_SLOT).all()

    def placed(self):
        """{(id, lod): slot} of the requests that got a slot; one slot per pair, one NEW per placed pair
        that was absent before (counted by the caller)."""
        m = {}
        for i in np.nonzero(np.isin(self.state, (NEW, HIT, JOINED)))[0]:
            k = (int(self.ids[i]), int(self.lods[i]))
            assert m.setdefault(k, int(self.slot[i])) == int(self.slot[i]), "pair %s got two slots" % (k,)
        return m


def _units(lod):
    return 1 << (3 * (5 - int(lod)))


def _check_disjoint(resident, cache_elems):
    iv = sorted((s, s + _units(l)) for (i, l), s in resident.items())
    for (a0, a1), (b0, b1) in zip(iv, iv[1:]):
        assert a1 <= b0, "slots overlap"
    assert all(0 <= a and b <= cache_elems for a, b in iv)


def _check_labels(c, cache, resident):
    import torch
    import paper_2609_36898_amd as P
    torch.cuda.synchronize()
    host = cache.cpu().numpy().view(np.uint32)
    keys = sorted(resident)
    ids = np.array([k[0] for k in keys], np.uint32)
    lods = np.array([k[1] for k in keys], np.uint8)
    offs, total = P.dense_offsets(np.full(len(keys), 5, np.uint8), lods)
    want, wst = oracle.decode_tasks(c, ids, lods, offs, total, 4, nthreads=8)
    assert (wst == 0).all()
    for k, o in zip(keys, offs):
        s, u = resident[k], _units(k[1])
        assert np.array_equal(host[s:s + u], want[int(o):int(o) + u]), "labels of pair %s differ" % (k,)


def _keys(rng, n, exclude=()):
    ex = set(exclude)
    out = []
    while len(out) < n:
        k = (int(rng.integers(0, 512)), int(rng.choice(6, p=[0.15, 0.2, 0.2, 0.15, 0.15, 0.15])))
        if k not in ex:
            ex.add(k)
            out.append(k)
    return out


def _requests(rng, keys, n):
    pick = rng.integers(0, len(keys), n)
    pick[:len(keys)] = np.arange(len(keys))  # every key at least once
    rng.shuffle(pick)
    return np.array([keys[p][0] for p in pick], np.uint32), np.array([keys[p][1] for p in pick], np.uint8)


def test_request_decode_free_reuse_and_full(env):
    import torch
    P, c, dv = env
    rng = np.random.default_rng(3)
    k1 = _keys(rng, 300)
    gone = [k1[i] for i in rng.permutation(len(k1))[:150]]
    k2 = _keys(rng, 120, exclude=k1)
    u1 = sum(_units(l) for _, l in k1)
    freed = np.bincount([5 - l for _, l in gone], minlength=7)
    new2 = np.bincount([5 - l for _, l in k2], minlength=7)
    growth = sum(max(0, int(new2[t]) - int(freed[t])) << (3 * t) for t in range(7))
    cache_elems = u1 + growth  # batch 2 fills the cache exactly
    cache = torch.zeros(cache_elems, dtype=torch.int32, device="cuda")
    dc = P.csgv.csgv_dcache(dv.info, dv.tensor, cache_elems, stack_cap=4096)
    plan = P.csgv_plan(dv.info, 4096)

    # batch 1: every pair absent, all fit; one NEW per pair, slots from the top
    ids, lods = _requests(rng, k1, 2000)
    b1 = Batch(P, dv, dc, plan, cache, cache_elems, ids, lods)
    res = b1.placed()
    assert set(res) == set(k1) and int((b1.state == NEW).sum()) == len(k1)
    top, counts = dc.query()
    assert top == u1 and (counts == 0).all()
    _check_disjoint(res, cache_elems)
    _check_labels(c, cache, res)

    # free half the pairs (with duplicates and pairs that are not resident)
    fids = np.array([k[0] for k in gone] * 2 + [k[0] for k in k2[:10]], np.uint32)
    flods = np.array([k[1] for k in gone] * 2 + [k[1] for k in k2[:10]], np.uint8)
    dc.free(None, torch.from_numpy(fids.view(np.int32).copy()).cuda(), torch.from_numpy(flods).cuda(), len(fids))
    top, counts = dc.query()
    assert top == u1 and np.array_equal(counts, freed)
    freed_slots = {t: sorted(res[k] for k in gone if 5 - k[1] == t) for t in range(7)}
    for k in gone:
        del res[k]

    # batch 2: new pairs pop the freed slots of their class first, then take the top up to the capacity;
    # kept pairs are hits and keep their labels
    keep = list(res)
    req_keys = k2 + [keep[i] for i in rng.permutation(len(keep))[:60]]
    ids, lods = _requests(rng, req_keys, 1500)
    b2 = Batch(P, dv, dc, plan, cache, cache_elems, ids, lods)
    got = b2.placed()
    assert set(got) == set(req_keys)
    assert int((b2.state == NEW).sum()) == len(k2)
    for k in keep:
        if k in got:
            assert got[k] == res[k]
    top, counts = dc.query()
    assert top == cache_elems
    assert np.array_equal(counts, np.maximum(freed - new2, 0))
    for t in range(7):
        from_stack = [got[k] for k in k2 if 5 - k[1] == t and got[k] < u1]
        assert len(from_stack) == min(int(new2[t]), int(freed[t]))
        assert set(from_stack) <= set(freed_slots[t])
    res.update({k: got[k] for k in k2})
    _check_disjoint(res, cache_elems)
    _check_labels(c, cache, res)

    # batch 3: the top is at the capacity; only classes with slots left on their stack get any,
    # the rest are FULL (joined requests of a FULL pair too); plus invalid requests
    k3 = _keys(rng, 80, exclude=list(res) + gone)
    ids, lods = _requests(rng, k3, 600)
    ids = np.concatenate([ids, np.array([512, 7, 3], np.uint32)])
    lods = np.concatenate([lods, np.array([0, 6, 200], np.uint8)])
    left = counts.copy()
    b3 = Batch(P, dv, dc, plan, cache, cache_elems, ids, lods)
    assert (b3.state[-3:] == INVALID).all()
    got = b3.placed()
    new3 = np.bincount([5 - l for _, l in k3], minlength=7)
    placed3 = np.bincount([5 - l for _, l in got], minlength=7)
    assert np.array_equal(placed3, np.minimum(new3, left))
    for k in k3:
        rows = (b3.ids == k[0]) & (b3.lods == k[1])
        if k in got:
            assert ((b3.state[rows] == NEW).sum() == 1) and not (b3.state[rows] == FULL).any()
        else:
            assert (b3.state[rows] == FULL).all()
    top, counts = dc.query()
    assert top >= cache_elems and np.array_equal(counts, left - placed3)
    res.update(got)
    _check_disjoint(res, cache_elems)
    _check_labels(c, cache, res)

    # reset: everything absent again, the top back at 0
    dc.reset()
    top, counts = dc.query()
    assert top == 0 and (counts == 0).all()
    ids, lods = _requests(rng, k1[:20], 20)
    b4 = Batch(P, dv, dc, plan, cache, cache_elems, ids, lods)
    assert (b4.state == NEW).all()
    _check_labels(c, cache, b4.placed())

    # overfull batch on an empty cache: pairs of every size race for the top at once; the ones that get
    # room must tile [0, top) with no overlap and no hole, the others are FULL
    dc.reset()
    k5 = _keys(rng, 400)
    ids, lods = _requests(rng, k5, 2400)
    b5 = Batch(P, dv, dc, plan, cache, cache_elems, ids, lods)
    got = b5.placed()
    assert 0 < len(got) < len(k5) and (b5.state == FULL).any()
    full_pairs = set(zip(b5.ids[b5.state == FULL].tolist(), b5.lods[b5.state == FULL].tolist()))
    assert not (full_pairs & set(got)), "a pair is FULL in one request and placed in another"
    top, counts = dc.query()
    assert top > cache_elems and (counts == 0).all()
    # the placed slots tile [0, their total) with no hole and no overlap
    _check_disjoint(got, cache_elems)
    assert max(s + _units(l) for (i, l), s in got.items()) == sum(_units(l) for _, l in got) <= cache_elems
    _check_labels(c, cache, got)
    dc.destroy()
    _say("dcache: 5 batches, reuse, full and overfull cache checked")


def test_mixed_brick_sides_use_size_classes():
    """32^3 and 64^3 bricks (u64 labels): a slot's size class is log2(side) - LOD, so a freed 64^3 LOD-1
    slot (32^3 elements) serves a 32^3 LOD-0 pair and never a 64^3 LOD-0 one."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_36898_amd as P
    n_b = 12
    l2 = np.array([6 if i % 2 == 0 else 5 for i in range(n_b)], np.uint8)
    bricks = [synth.uneven_brick_u64(1 << int(l2[i]), 23, i)[0].reshape(-1) for i in range(n_b)]
    c = oracle.encode_bricks(np.concatenate(bricks), l2, 8)
    dv = P.DeviceVolume(c)
    side = lambda i: int(l2[i])  # noqa: E731
    units = lambda i, l: 1 << (3 * (side(i) - int(l)))  # noqa: E731
    cache_elems = 3 * 64 ** 3
    cache = torch.zeros(cache_elems, dtype=torch.int64, device="cuda")
    dc = P.csgv.csgv_dcache(dv.info, dv.tensor, cache_elems, stack_cap=64)
    plan = P.csgv_plan(dv.info, 256)

    def batch(pairs):
        ids = np.array([p[0] for p in pairs], np.uint32)
        lods = np.array([p[1] for p in pairs], np.uint8)
        n = len(pairs)
        d_ids = torch.from_numpy(ids.view(np.int32).copy()).cuda()
        d_lods = torch.from_numpy(lods.copy()).cuda()
        task = torch.empty(n, dtype=torch.int32, device="cuda")
        slot = torch.empty(n, dtype=torch.int64, device="cuda")
        state = torch.empty(n, dtype=torch.int32, device="cuda")
        status = torch.empty(n, dtype=torch.int32, device="cuda")
        _say("mixed sides: request + decode of", n, "requests")
        dc.request(None, d_ids, d_lods, n, task, slot, state)
        plan.launch(None, dv.tensor, task, d_lods, slot, n, cache, cache_elems, status)
        torch.cuda.synchronize()
        st = state.cpu().numpy()
        sl = slot.cpu().numpy().view(np.uint64)
        ts = status.cpu().numpy()
        assert (ts[st == NEW] == 0).all()
        return st, sl

    def labels_ok(pairs, slots):
        ids = np.array([p[0] for p in pairs], np.uint32)
        lods = np.array([p[1] for p in pairs], np.uint8)
        offs, total = P.dense_offsets(l2[ids.astype(np.int64)], lods)
        want, wst = oracle.decode_tasks(c, ids, lods, offs, total, 8, nthreads=8)
        host = cache.cpu().numpy().view(np.uint64)
        assert (wst == 0).all()
        for (i, l), s, o in zip(pairs, slots, offs):
            u = units(i, l)
            assert np.array_equal(host[int(s):int(s) + u], want[int(o):int(o) + u]), "pair %d/%d" % (i, l)

    # a 64^3 brick at LOD 0 and LOD 1, a 32^3 brick at LOD 0 and LOD 1
    first = [(0, 0), (0, 1), (1, 0), (1, 1)]
    st, sl1 = batch(first)
    assert (st == NEW).all()
    assert dc.query()[0] == 64 ** 3 + 2 * 32 ** 3 + 16 ** 3
    labels_ok(first, sl1)
    # release the 64^3 LOD-1 slot (class 5, 32^3 elements) and the 32^3 LOD-1 slot (class 4)
    fids = torch.from_numpy(np.array([0, 1], np.int32)).cuda()
    flods = torch.from_numpy(np.array([1, 1], np.uint8)).cuda()
    dc.free(None, fids, flods, 2)
    top, counts = dc.query()
    assert counts[5] == 1 and counts[4] == 1 and counts.sum() == 2
    # class 5 (32^3 elements): a 32^3 brick at LOD 0 and a 64^3 brick at LOD 1 -- one pops the freed
    # 64^3 LOD-1 slot, the other takes the top; class 4: a 64^3 brick at LOD 2 pops the freed 32^3 LOD-1 slot
    second = [(3, 0), (2, 1), (4, 2)]
    st, sl = batch(second)
    assert (st == NEW).all()
    top2, counts2 = dc.query()
    assert (counts2 == 0).all() and top2 == top + 32 ** 3
    assert sorted(int(v) for v in sl[:2]) == sorted([int(sl1[1]), top])
    assert int(sl[2]) == int(sl1[3])
    keep = [first[0], first[2]] + second
    labels_ok(keep, [sl1[0], sl1[2]] + list(sl))
    dc.destroy()
    _say("dcache: mixed brick sides checked")
