"""Parity of the back-substitution's LDS ring when it holds fewer columns
than a record reaches (vf_opts.ring_cols, a test option): vertices beyond
the ring are read from the cells, batches of 64 pivots that span half the
ring or more find their dependencies by binary search instead of through
the ring, and segments of every size use the ring.  Every local seed, the
failure record and every cell must still equal the oracle's."""
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


@pytest.mark.parametrize("is_filter,n,h,b,cols", [
    (True, 1 << 18, 2, 8, 64),      # s = 2^9: most gathers beyond the ring
    (True, 1 << 18, 2, 8, 256),     # some batches with, some without lane tags
    (False, 1 << 17, 1, 16, 64),    # 2-byte cells
    (False, 100000, 1, 32, 1024),   # 4-byte cells
])
def test_small_ring_equals_the_oracle(is_filter, n, h, b, cols):
    print(f"[ring] filter={is_filter} n={n} h={h} b={b} ring_cols={cols}", flush=True)
    keys = S.member_keys(n, 401 + cols, device=DEV)
    vals = None if is_filter else S.values(n, b, 401 + cols, device=DEV)
    st = vf.Structure.build(keys, vals, b=b, h=h, seed=6, ring_cols=cols)
    torch.cuda.synchronize()
    assert st.rc == vf.VF_OK
    info = st.info
    ob = O.build(keys.cpu().numpy().view(np.uint64),
                 None if is_filter else vals.cpu().numpy().view(np.uint64),
                 b=b, is_filter=is_filter, h=h, seed=6)
    assert np.array_equal(st.local_seeds().cpu().numpy(), ob.t.astype(np.uint8))
    assert st.failures == ob.failures
    cells = st.cells().cpu().numpy().view(_NP[info["cell_bytes"]])
    assert np.array_equal(cells, ob.w.astype(cells.dtype))
    got = st.query(keys)
    if is_filter:
        assert got.min().item() == 1
    else:
        # answers come back in a signed tensor of the cell width
        got_u = got.cpu().numpy().view(_NP[got.element_size()]).astype(np.uint64)
        assert np.array_equal(got_u, vals.cpu().numpy().view(np.uint64))
    st.free()


def test_small_ring_batch_equals_the_oracle():
    # segments from 2^2 to 2^9 vertices, all through a 64-column ring
    ns = np.array([30000, 5000, 12000, 700, 40000, 90, 2000, 300], np.uint64)
    bs = np.array([8, 4, 16, 1, 8, 32, 4, 16], np.int32)
    total = int(ns.sum())
    keys = S.member_keys(total, 431, device=DEV)
    vals = S.batch_values(ns, bs, 431, device=DEV)
    print(f"[ring] batch of {ns.size}, ring_cols=64", flush=True)
    bt = vf.Batch.build(keys, vals, ns, bs, seed=3, small=2, ring_cols=64)
    torch.cuda.synchronize()
    assert bt.rc == vf.VF_OK
    k_np = keys.cpu().numpy().view(np.uint64)
    v_np = vals.cpu().numpy().view(np.uint64)
    off = np.concatenate([[0], np.cumsum(ns.astype(np.int64))])
    for i in range(ns.size):
        lo, hi = int(off[i]), int(off[i + 1])
        ob = O.build(k_np[lo:hi], v_np[lo:hi], b=int(bs[i]), is_filter=False, h=0, seed=3)
        it = bt.item(i)
        assert it["local_seed"] == int(ob.t[0]), i
        assert [(a, c, d) for (s, a, c, d) in bt.failures if s == i] == \
            [(a, c, d) for (s, a, c, d) in ob.failures], i
        cells = bt.cells(i).cpu().numpy().view(_NP[it["cell_bytes"]])
        assert np.array_equal(cells, ob.w[0].astype(cells.dtype)), i
    bt.free()
