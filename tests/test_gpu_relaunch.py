"""Parity of the whole-CU relaunch: a shard whose elimination window outgrows
its build workgroup's share of LDS is rebuilt by a second launch that has a
whole CU's LDS, from the local seed it had reached.  Capping the window
(vf_opts.max_window) forces that path on most shards; every local seed,
the failure record and every cell must still equal the oracle's."""
import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2503_18397_amd as vf
DEV = "cuda:0"


@pytest.mark.parametrize("n,h,b,cap", [(1 << 20, 4, 8, 64), (1 << 19, 3, 16, 128)])
def test_relaunched_filter_shards_equal_the_oracle(n, h, b, cap):
    print(f"[relaunch] filter n={n} h={h} b={b} max_window={cap}", flush=True)
    keys = S.member_keys(n, 201 + h, device=DEV)
    st = vf.Structure.build(keys, None, b=b, h=h, seed=4, max_window=cap)
    torch.cuda.synchronize()
    assert st.rc == vf.VF_OK
    info = st.info
    assert info["relaunched_shards"] > 0
    k_np = keys.cpu().numpy().view(np.uint64)
    ob = O.build(k_np, b=b, is_filter=True, h=h, seed=4)
    assert np.array_equal(st.local_seeds().cpu().numpy(), ob.t.astype(np.uint8))
    assert st.failures == ob.failures
    cells = st.cells().cpu().numpy().view({1: np.uint8, 2: np.uint16}[info["cell_bytes"]])
    assert np.array_equal(cells, ob.w.astype(cells.dtype))
    assert st.query(keys).min().item() == 1
    st.free()


def test_relaunched_function_shards_equal_the_oracle():
    n, h = 300000, 2
    print(f"[relaunch] function n={n} h={h}", flush=True)
    keys = S.member_keys(n, 233, device=DEV)
    vals = S.values(n, 8, 233, device=DEV)
    st = vf.Structure.build(keys, vals, b=8, h=h, seed=9, max_window=96)
    torch.cuda.synchronize()
    assert st.rc == vf.VF_OK and st.info["relaunched_shards"] > 0
    ob = O.build(keys.cpu().numpy().view(np.uint64), vals.cpu().numpy().view(np.uint64), b=8,
                 is_filter=False, h=h, seed=9)
    assert np.array_equal(st.local_seeds().cpu().numpy(), ob.t.astype(np.uint8))
    assert st.failures == ob.failures
    assert np.array_equal(st.cells().cpu().numpy(), ob.w.astype(np.uint8))
    assert torch.equal(st.query(keys).long(), vals)
    st.free()


def test_relaunched_batch_instances_equal_the_oracle():
    ns = np.array([30000, 5000, 12000, 700, 40000, 64, 2000], np.uint64)
    bs = np.array([8, 4, 16, 1, 8, 32, 4], np.int32)
    total = int(ns.sum())
    keys = S.member_keys(total, 301, device=DEV)
    vals = S.batch_values(ns, bs, 301, device=DEV)
    print(f"[relaunch] batch of {ns.size}", flush=True)
    bt = vf.Batch.build(keys, vals, ns, bs, seed=2, max_window=32)
    torch.cuda.synchronize()
    assert bt.rc == vf.VF_OK and bt.info["relaunched_shards"] > 0
    k_np = keys.cpu().numpy().view(np.uint64)
    v_np = vals.cpu().numpy().view(np.uint64)
    off = np.concatenate([[0], np.cumsum(ns.astype(np.int64))])
    np_of = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}
    for i in range(ns.size):
        lo, hi = int(off[i]), int(off[i + 1])
        ob = O.build(k_np[lo:hi], v_np[lo:hi], b=int(bs[i]), is_filter=False, h=0, seed=2)
        it = bt.item(i)
        assert it["local_seed"] == int(ob.t[0]), i
        assert [(a, c, d) for (s, a, c, d) in bt.failures if s == i] == \
            [(a, c, d) for (s, a, c, d) in ob.failures], i
        cells = bt.cells(i).cpu().numpy().view(np_of[it["cell_bytes"]])
        assert np.array_equal(cells, ob.w[0].astype(cells.dtype)), i
    bt.free()
