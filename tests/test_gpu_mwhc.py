"""Parity of the MWHC variant (section 4.1) with the oracle: 3-partite
hypergraphs, peel-only construction with local seeds, epsilon-cost
sharding; geometry, seeds, failure records (kind 2), cells and answers."""
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


def _check(st, ob):
    i = st.info
    g = ob.geom
    assert i["mwhc"] == 1
    assert (i["M"], i["h"], i["V"], i["c_num"], i["c_den"]) == \
        (g["M"], g["h"], g["V"], g["c_num"], g["c_den"])
    ts = st.local_seeds().cpu().numpy().astype(np.int64)
    ot = ob.t.astype(np.int64)
    ot[ot >= 255] = 255
    assert np.array_equal(ts[ob.shards], ot)
    assert st.failures == ob.failures
    cells = st.cells().cpu().numpy().view(_NP[i["cell_bytes"]])
    assert np.array_equal(cells[ob.shards], ob.w.astype(_NP[i["cell_bytes"]]))


@pytest.mark.parametrize("n,b,h,seed", [(1, 8, 0, 1), (5000, 16, 0, 2), (30000, 32, 2, 3)])
def test_mwhc_vfunc_bit_exact(n, b, h, seed):
    keys = S.member_keys(n, 400 + seed)
    vals = S.values(n, b, 400 + seed)
    st = vf.Structure.build(keys.to(DEV), vals.to(DEV), b=b, h=h, seed=seed, mwhc=True)
    torch.cuda.synchronize()
    ob = O.build(keys.numpy().view(np.uint64), vals.numpy().view(np.uint64), b=b,
                 is_filter=False, h=h, seed=seed, mwhc=True)
    assert (st.rc == vf.VF_OK) == (ob.status == 0)
    _check(st, ob)
    got = st.query(keys.to(DEV)).cpu().numpy().astype(np.uint64)
    assert np.array_equal(got & np.uint64((1 << b) - 1) if b < 64 else got,
                          vals.numpy().view(np.uint64))


def test_mwhc_vfilter_sharded_bit_exact():
    n, b, h = 1 << 18, 8, 3
    keys = S.member_keys(n, 431)
    st = vf.Structure.build(keys.to(DEV), None, b=b, h=h, seed=7, mwhc=True)
    torch.cuda.synchronize()
    ob = O.build(keys.numpy().view(np.uint64), b=b, is_filter=True, h=h, seed=7, mwhc=True)
    assert st.rc == vf.VF_OK and ob.status == 0
    _check(st, ob)
    neg = S.negative_keys(n, 100000, 431)
    got = st.query(neg.to(DEV)).cpu().numpy().astype(np.uint64)
    assert np.array_equal(got, O.query(ob, neg.numpy().view(np.uint64)))


def test_mwhc_duplicate_key_fails_every_seed_like_the_oracle():
    keys = S.member_keys(4000, 433)
    vals = S.values(4000, 8, 433)
    keys[7] = keys[3]
    st = vf.Structure.build(keys.to(DEV), vals.to(DEV), b=8, h=0, seed=1, tmax=3, mwhc=True)
    torch.cuda.synchronize()
    ob = O.build(keys.numpy().view(np.uint64), vals.numpy().view(np.uint64), b=8,
                 is_filter=False, h=0, seed=1, tmax=3, mwhc=True)
    assert st.rc == vf.VF_EFAIL and ob.status == 1
    assert st.failures == ob.failures and [f[2] for f in ob.failures] == [2, 2, 2]
