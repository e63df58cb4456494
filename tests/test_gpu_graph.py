"""The three-call batch build (vf_batch_prepare, vf_batch_launch,
vf_batch_finish): the same structure as vf_batch_build, and a launch
captured into a HIP graph replays to the same structure, also on new keys
written into the captured buffers.  A replay whose values are too wide for
their b fails at finish and leaves the structure as it was."""
import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2503_18397_amd as vf
DEV = "cuda:0"
_NP = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}


def _shape(count, data_seed):
    # small instances (the one-wavefront kernel) and larger ones of every
    # cell width (the peel + band kernel)
    n, b = S.batch_shape(count, data_seed, lo=10, hi=30000, bits=(1, 4, 8, 16, 32, 64))
    n[: count // 2] = np.minimum(n[: count // 2], 120)
    n[:3] = [0, 1, 2]
    return n, b


def _inputs(n, b, data_seed):
    keys = S.member_keys(int(n.sum()), data_seed, device=DEV)
    vals = S.batch_values(n, b, data_seed, device=DEV)
    return keys, vals


def _state(bt, count):
    """Host copies of what a build decides: seeds, failures, all cells."""
    items = [bt.item(i) for i in range(count)]
    return ([it["local_seed"] for it in items], bt.failures,
            [bt.cells(i).cpu().clone() for i in range(count)])


def _same(a, c):
    assert a[0] == c[0]
    assert a[1] == c[1]
    for i, (x, y) in enumerate(zip(a[2], c[2])):
        assert torch.equal(x, y), i


def _oracle_check(bt, keys, vals, n, b, seed, sample):
    off = np.concatenate([[0], np.cumsum(n.astype(np.int64))])
    k_np = keys.cpu().numpy().view(np.uint64)
    v_np = vals.cpu().numpy().view(np.uint64)
    for i in sample:
        lo, hi = int(off[i]), int(off[i + 1])
        ob = O.build(k_np[lo:hi], v_np[lo:hi], b=int(b[i]), is_filter=False, h=0, seed=seed)
        it = bt.item(i)
        assert it["local_seed"] == (int(ob.t[0]) if ob.status == 0 else 255), i
        if ob.status == 0 and it["V"]:
            if it["packed"]:
                want = O.pack(ob.w[0], int(b[i]))
                got = bt.cells(i).cpu().numpy().view(np.uint64)
            else:
                want = ob.w[0].astype(_NP[it["cell_bytes"]])
                got = bt.cells(i).cpu().numpy().view(_NP[it["cell_bytes"]])
            assert np.array_equal(got, want), i


@pytest.mark.parametrize("packed", [False, True])
def test_prepared_build_equals_synchronous_build(packed):
    n, b = _shape(600, 41)
    keys, vals = _inputs(n, b, 41)
    print(f"[graph] prepared build packed={packed}, {n.size} instances", flush=True)
    ref = vf.Batch.build(keys, vals, n, b, seed=9, packed=packed)
    torch.cuda.synchronize()
    bt = vf.Batch.prepare(n, b, seed=9, device=DEV, packed=packed)
    with pytest.raises(vf.VFError):
        bt.query(torch.zeros(1, dtype=torch.int32, device=DEV), keys[:1])
    bt.launch(keys, vals)
    assert bt.finish() == ref.rc
    _same(_state(bt, n.size), _state(ref, n.size))
    assert bt.info["failed_shards"] == ref.info["failed_shards"]
    inst = torch.repeat_interleave(torch.arange(n.size, dtype=torch.int32, device=DEV),
                                   torch.as_tensor(n.astype(np.int64), device=DEV))
    assert torch.equal(bt.query(inst, keys), ref.query(inst, keys))
    ref.free()
    bt.free()


def test_graph_replays_match_eager_and_oracle():
    n, b = _shape(400, 57)
    count = n.size
    keys, vals = _inputs(n, b, 57)
    print(f"[graph] capture, {count} instances, {int(n.sum())} keys", flush=True)
    bt = vf.Batch.prepare(n, b, seed=3, device=DEV)
    # eager run first (loads the kernels), the reference for every replay
    bt.launch(keys, vals)
    assert bt.finish() == vf.VF_OK
    eager = _state(bt, count)
    _oracle_check(bt, keys, vals, n, b, 3, [3, 5, 200, 201, count - 1])

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        bt.launch(keys, vals)
    torch.cuda.synchronize()
    x = torch.arange(1 << 20, device=DEV, dtype=torch.float32)
    for r in range(3):
        print(f"[graph] replay {r}", flush=True)
        bt.structure.zero_()
        torch.cuda.synchronize()
        g.replay()
        assert bt.finish() == vf.VF_OK
        _same(_state(bt, count), eager)
        # eager work of the program between replays
        x = torch.sqrt(x + 1.0)
        torch.cuda.synchronize()

    # new keys and values written into the captured buffers
    keys2, vals2 = _inputs(n, b, 58)
    keys.copy_(keys2)
    vals.copy_(vals2)
    torch.cuda.synchronize()
    print("[graph] replay on new keys", flush=True)
    g.replay()
    assert bt.finish() == vf.VF_OK
    ref2 = vf.Batch.build(keys2, vals2, n, b, seed=3)
    torch.cuda.synchronize()
    built2 = _state(ref2, count)
    _same(_state(bt, count), built2)
    _oracle_check(bt, keys2, vals2, n, b, 3, [4, 6, 250, count - 2])
    ref2.free()

    # a value too wide for its instance: every build kernel of the replay
    # returns at once, finish reports it and the handle is unchanged
    before = bt.structure.clone()
    st_before = _state(bt, count)
    i = int(np.argmax((b < 32) & (n > 0)))
    off = int(np.sum(n[:i].astype(np.int64)))
    assert n[i] > 0 and b[i] < 32
    vals[off] = vals[off] | (1 << int(b[i]))
    torch.cuda.synchronize()
    print("[graph] replay with a value too wide", flush=True)
    g.replay()
    with pytest.raises(vf.VFError) as e:
        bt.finish()
    assert e.value.code == vf.VF_EINVAL
    assert torch.equal(bt.structure, before)
    _same(_state(bt, count), st_before)
    # fixed again: the replay builds
    vals.copy_(vals2)
    torch.cuda.synchronize()
    g.replay()
    assert bt.finish() == vf.VF_OK
    _same(_state(bt, count), built2)
    bt.free()


# ----------------------------------------------- sharded builds in three calls

def _oracle_fixed(keys, vals, b, is_filter, h, seed, cap):
    """The oracle's structure with every shard sized for cap keys."""
    import ctypes as C
    g = O.Geom()
    O.lib().orc_geometry(cap, h, 0, 0, -1, C.byref(g))
    return O.build(keys.cpu().numpy().view(np.uint64),
                   None if vals is None else vals.cpu().numpy().view(np.uint64),
                   b=b, is_filter=is_filter, h=h, seed=seed, geom=g)


def _same_as_oracle(st, ob, b):
    info = st.info
    assert (info["M"], info["V"], info["l"], info["sigma"]) == \
        (ob.geom["M"], ob.geom["V"], ob.geom["l"], ob.geom["sigma"])
    assert np.array_equal(st.local_seeds().cpu().numpy(), ob.t.astype(np.uint8))
    assert st.failures == ob.failures
    if info["packed"]:
        got = st.cells().cpu().numpy().view(np.uint64)
        assert np.array_equal(got, O.pack(ob.w.reshape(-1), b))
    else:
        cells = st.cells().cpu().numpy().view(_NP[info["cell_bytes"]])
        assert np.array_equal(cells, ob.w.astype(cells.dtype))


@pytest.mark.parametrize("is_filter,b,h,packed", [(True, 8, 4, False), (False, 12, 2, True)])
def test_prepared_sharded_build_equals_the_oracle(is_filter, b, h, packed):
    n = 1 << 18
    keys = S.member_keys(n, 61, device=DEV)
    vals = None if is_filter else S.values(n, b, 61, device=DEV)
    print(f"[graph] prepared sharded build filter={is_filter} b={b} h={h} packed={packed}",
          flush=True)
    st = vf.Structure.prepare(n, b=b, filter=is_filter, h=h, seed=4, packed=packed,
                              device=DEV)
    with pytest.raises(vf.VFError):
        st.query(keys[:1])
    st.launch(keys, vals)
    assert st.finish() == vf.VF_OK
    ob = _oracle_fixed(keys, vals, b, is_filter, h, 4, st.info["M"])
    _same_as_oracle(st, ob, b)
    q, _ = S.queries(keys, 20000, 62)
    got = st.query(q).cpu().numpy()
    if not is_filter:
        got = got.view(_NP[got.itemsize])
    assert np.array_equal(got.astype(np.uint64), O.query(ob, q.cpu().numpy().view(np.uint64)))
    st.free()


def test_captured_sharded_build_replays_and_reports_bad_input():
    n, b, h = 1 << 17, 12, 3
    keys = S.member_keys(n, 71, device=DEV)
    vals = S.values(n, b, 71, device=DEV)
    print("[graph] sharded build capture", flush=True)
    st = vf.Structure.prepare(n, b=b, filter=False, h=h, seed=2, device=DEV)
    st.launch(keys, vals)  # eager run first (loads the kernels)
    assert st.finish() == vf.VF_OK
    eager = (st.cells().cpu().clone(), st.local_seeds().cpu().clone(), st.failures)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        st.launch(keys, vals)
    torch.cuda.synchronize()
    x = torch.arange(1 << 20, device=DEV, dtype=torch.float32)
    for r in range(3):
        print(f"[graph] sharded replay {r}", flush=True)
        st.structure.zero_()
        torch.cuda.synchronize()
        g.replay()
        assert st.finish() == vf.VF_OK
        assert torch.equal(st.cells().cpu(), eager[0])
        assert torch.equal(st.local_seeds().cpu(), eager[1]) and st.failures == eager[2]
        x = torch.sqrt(x + 1.0)
        torch.cuda.synchronize()
    # new keys in the captured buffers: the oracle's structure for them
    # (keys of data seed 72 put 16 857 keys in one shard, above the bound of
    # 16 840: that build is refused, see the test below)
    keys2, vals2 = S.member_keys(n, 73, device=DEV), S.values(n, b, 73, device=DEV)
    keys.copy_(keys2)
    vals.copy_(vals2)
    torch.cuda.synchronize()
    g.replay()
    assert st.finish() == vf.VF_OK
    _same_as_oracle(st, _oracle_fixed(keys2, vals2, b, False, h, 2, st.info["M"]), b)
    # a value too wide: nothing is written, finish reports it
    before = st.structure.clone()
    vals[5] = vals[5] | (1 << b)
    torch.cuda.synchronize()
    g.replay()
    with pytest.raises(vf.VFError) as e:
        st.finish()
    assert e.value.code == vf.VF_EINVAL
    assert torch.equal(st.structure, before)
    st.free()


def test_prepared_build_with_a_bound_below_the_largest_shard_is_refused():
    n, h = 1 << 16, 4
    keys = S.member_keys(n, 81, device=DEV)
    st = vf.Structure.prepare(n, b=8, filter=True, h=h, max_shard=n >> h, device=DEV)
    before = st.structure.clone()
    st.launch(keys)
    with pytest.raises(vf.VFError) as e:
        st.finish()
    assert e.value.code == vf.VF_ENOSPC
    assert "above the bound" in vf.vf_last_error()
    assert torch.equal(st.structure, before)
    st.free()
