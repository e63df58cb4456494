"""Parity of batched builds (vf_batch_build, vf_batch_query) with the CPU
oracle.  Instance i of a batch must be exactly the unsharded structure the
oracle builds for its keys, values, width and the batch seed (h = 0): local
seed, failure record, every cell, and every queried value."""
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


def _batch_inputs(n, b, data_seed):
    total = int(np.sum(n))
    keys = S.member_keys(total, data_seed, device=DEV)
    vals = S.batch_values(n, b, data_seed, device=DEV)
    off = np.concatenate([[0], np.cumsum(n.astype(np.int64))])
    return keys, vals, off


def _check_instances(bt, keys, vals, n, b, off, seed, sample, tmax=255):
    k_np = keys.cpu().numpy().view(np.uint64)
    v_np = vals.cpu().numpy().view(np.uint64)
    fails = bt.failures
    for i in sample:
        lo, hi = int(off[i]), int(off[i + 1])
        ob = O.build(k_np[lo:hi], v_np[lo:hi], b=int(b[i]), is_filter=False, h=0, seed=seed,
                     tmax=tmax)
        it = bt.item(i)
        g = ob.geom
        assert (it["n"], it["l"], it["sigma"], it["V"], it["c_num"], it["c_den"]) == \
            (g["M"], g["l"], g["sigma"], g["V"], g["c_num"], g["c_den"]), i
        t = int(ob.t[0]) if ob.status == 0 else 255
        assert it["local_seed"] == min(t, 255), i
        assert [(a, c, d) for (s, a, c, d) in fails if s == i] == \
            [(a, c, d) for (s, a, c, d) in ob.failures], i
        if ob.status == 0:
            cells = bt.cells(i).cpu().numpy().view(_NP[it["cell_bytes"]])
            assert np.array_equal(cells, ob.w[0].astype(_NP[it["cell_bytes"]])), i


def test_small_batch_bit_exact():
    n, b = S.batch_shape(48, 11, lo=10, hi=20000)
    n[:4] = [0, 1, 2, 3]
    b[:6] = [1, 4, 8, 16, 32, 64]
    keys, vals, off = _batch_inputs(n, b, 11)
    print(f"[batch] {n.size} instances, {int(n.sum())} keys", flush=True)
    bt = vf.Batch.build(keys, vals, n, b, seed=5)
    torch.cuda.synchronize()
    assert bt.rc == vf.VF_OK
    info = bt.info
    assert info["S"] == n.size and info["n"] == int(n.sum()) and info["failed_shards"] == 0
    _check_instances(bt, keys, vals, n, b, off, 5, range(n.size))
    # every key answers its masked value in its instance; non-members
    # answer what the oracle answers
    inst = torch.as_tensor(np.repeat(np.arange(n.size), n.astype(np.int64)).astype(np.int32),
                           device=DEV)
    got = bt.query(inst, keys).cpu().numpy().view(np.uint64)
    mask = np.where(b >= 64, np.uint64(~np.uint64(0)),
                    (np.uint64(1) << b.astype(np.uint64)) - np.uint64(1))
    want = vals.cpu().numpy().view(np.uint64) & np.repeat(mask, n.astype(np.int64))
    assert np.array_equal(got, want)
    k_np = keys.cpu().numpy().view(np.uint64)
    for i in range(6, 12):
        neg = S.negative_keys(int(n[i]), 500, 11 + i, device=DEV)
        ob = O.build(k_np[off[i]:off[i + 1]], vals.cpu().numpy().view(np.uint64)[off[i]:off[i + 1]],
                     b=int(b[i]), is_filter=False, h=0, seed=5)
        qi = torch.full((500,), i, dtype=torch.int32, device=DEV)
        g2 = bt.query(qi, neg).cpu().numpy().view(np.uint64)
        assert np.array_equal(g2, O.query(ob, neg.cpu().numpy().view(np.uint64))), i
    # an instance index past the batch answers all ones
    bad = bt.query(torch.tensor([n.size], dtype=torch.int32, device=DEV), keys[:1])
    assert bad.cpu().numpy().view(np.uint64)[0] == np.uint64(~np.uint64(0))
    bt.free()


def test_batch_with_a_failing_instance_matches_the_oracle():
    """A duplicate key with two values makes its instance fail every local
    seed; the other instances are unaffected."""
    n = np.array([3000, 2500, 4000], dtype=np.uint64)
    b = np.array([8, 16, 4], dtype=np.int32)
    keys, vals, off = _batch_inputs(n, b, 23)
    keys[off[1] + 7] = keys[off[1] + 3]
    vals[off[1] + 7] = vals[off[1] + 3] ^ 1
    bt = vf.Batch.build(keys, vals, n, b, seed=2, tmax=3)
    torch.cuda.synchronize()
    assert bt.rc == vf.VF_EFAIL
    assert bt.info["failed_shards"] == 1
    assert [f for f in bt.failures if f[0] != 1] == []
    assert [f[1] for f in bt.failures] == [0, 1, 2]
    _check_instances(bt, keys, vals, n, b, off, 2, range(3), tmax=3)
    bt.free()


def test_batch_workload_sampled_instances_bit_exact():
    """The benchmark's batch: 100 000 instances of 10..50 000 keys with
    b in {1, 4, 8, 16, 32}; a sample of instances (largest, smallest and
    random ones) is rebuilt by the oracle, every member is queried."""
    n, b = S.batch_shape(100000, 2029)
    keys, vals, off = _batch_inputs(n, b, 2029)
    print(f"[batch] {n.size} instances, {int(n.sum())} keys", flush=True)
    bt = vf.Batch.build(keys, vals, n, b, seed=0)
    torch.cuda.synchronize()
    assert bt.rc == vf.VF_OK
    rng = np.random.default_rng(3)
    sample = sorted(set(rng.choice(n.size, 12, replace=False).tolist()
                        + [int(np.argmax(n)), int(np.argmin(n))]
                        + sorted({f[0] for f in bt.failures})[:2]))
    print(f"[batch] oracle on instances {sample}", flush=True)
    _check_instances(bt, keys, vals, n, b, off, 0, sample)
    inst = torch.repeat_interleave(torch.arange(n.size, dtype=torch.int32, device=DEV),
                                   torch.as_tensor(n.astype(np.int64), device=DEV))
    got = bt.query(inst, keys)
    bits = torch.as_tensor(b.astype(np.int64), device=DEV)[inst.long()]
    want = vals & ((torch.ones_like(bits) << bits) - 1)
    assert torch.equal(got, want)
    bt.free()
