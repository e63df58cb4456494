"""Bit-array storage (vf_opts.packed: cells as one string of b-bit fields,
the storage of values of any width of section 5): the packed bits of every
shard or instance equal the oracle's cells packed the same way, and queries
read them back exactly."""
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


@pytest.mark.parametrize("b", [1, 4, 9, 17])
def test_packed_filter_equals_the_oracle(b):
    n, h, seed = 1 << 17, 3, 5
    print(f"[packed] filter b={b}", flush=True)
    keys = S.member_keys(n, 610 + b, device=DEV)
    st = vf.Structure.build(keys, None, b=b, h=h, seed=seed, packed=True)
    torch.cuda.synchronize()
    assert st.rc == vf.VF_OK and st.info["packed"] == 1
    ob = O.build(keys.cpu().numpy().view(np.uint64), b=b, is_filter=True, h=h, seed=seed)
    assert np.array_equal(st.local_seeds().cpu().numpy(), ob.t.astype(np.uint8))
    assert np.array_equal(st.cells().cpu().numpy().view(np.uint64), O.pack(ob.w.reshape(-1), b))
    q, _ = S.queries(keys, 1 << 18, 29)
    want = O.query(ob, q.cpu().numpy().view(np.uint64))
    assert np.array_equal(st.query(q).cpu().numpy().astype(np.uint64), want)
    assert np.array_equal(st.query_grouped(q).cpu().numpy().astype(np.uint64), want)
    # the same structure unpacked answers the same
    su = vf.Structure.build(keys, None, b=b, h=h, seed=seed)
    assert torch.equal(su.query(q), st.query(q))
    assert st.info["space_bits"] == su.info["space_bits"]
    st.free()
    su.free()


@pytest.mark.parametrize("b", [4, 33])
def test_packed_function_equals_the_oracle(b):
    n, h, seed = 50000, 2, 8
    print(f"[packed] function b={b}", flush=True)
    keys = S.member_keys(n, 640 + b, device=DEV)
    vals = S.values(n, b, 640 + b, device=DEV)
    st = vf.Structure.build(keys, vals, b=b, h=h, seed=seed, packed=True)
    torch.cuda.synchronize()
    assert st.rc == vf.VF_OK
    ob = O.build(keys.cpu().numpy().view(np.uint64), vals.cpu().numpy().view(np.uint64), b=b,
                 is_filter=False, h=h, seed=seed)
    assert np.array_equal(st.cells().cpu().numpy().view(np.uint64), O.pack(ob.w.reshape(-1), b))
    got = st.query(keys).cpu().numpy()
    got = got.view(_NP[got.itemsize]).astype(np.uint64)
    assert np.array_equal(got, vals.cpu().numpy().view(np.uint64))
    st.free()


def test_packed_batch_equals_the_oracle():
    ns = np.array([10, 63, 700, 5000, 23000, 3, 1, 0, 900], np.uint64)
    bs = np.array([1, 4, 9, 1, 4, 32, 17, 8, 64], np.int32)
    keys = S.member_keys(int(ns.sum()), 660, device=DEV)
    vals = S.batch_values(ns, bs, 660, device=DEV)
    print("[packed] batch", flush=True)
    bt = vf.Batch.build(keys, vals, ns, bs, seed=4, packed=True)
    torch.cuda.synchronize()
    assert bt.rc == vf.VF_OK
    k_np = keys.cpu().numpy().view(np.uint64)
    v_np = vals.cpu().numpy().view(np.uint64)
    off = np.concatenate([[0], np.cumsum(ns.astype(np.int64))])
    for i in range(ns.size):
        lo, hi = int(off[i]), int(off[i + 1])
        ob = O.build(k_np[lo:hi], v_np[lo:hi], b=int(bs[i]), is_filter=False, h=0, seed=4)
        it = bt.item(i)
        assert it["packed"] == 1 and it["local_seed"] == int(ob.t[0]), i
        got = bt.cells(i).cpu().numpy().view(np.uint64)
        assert np.array_equal(got, O.pack(ob.w[0], int(bs[i]))), i
    inst = torch.repeat_interleave(torch.arange(ns.size, dtype=torch.int32, device=DEV),
                                   torch.as_tensor(ns.astype(np.int64), device=DEV))
    assert torch.equal(bt.query(inst, keys), vals)
    bt.free()
