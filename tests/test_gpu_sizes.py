"""Shard sizes around the changes of the size rule, against the oracle:
shards above about 73 000 keys (whose duplicate-edge rule alone would ask
for 1024-vertex segments) and a largest shard just below 2^16 keys when the
planned bound on it is above 2^16 (the expansion factor is larger below
2^16, so the buffers must cover both sides)."""
import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2503_18397_amd as vf
DEV = "cuda:0"


def _sampled_parity(st, keys, h, b, seed, sample):
    ob = O.build(keys.cpu().numpy().view(np.uint64), b=b, is_filter=True, h=h, seed=seed,
                 shards=sample)
    i = st.info
    g = ob.geom
    assert (i["M"], i["l"], i["sigma"], i["V"], i["c_num"], i["c_den"]) == \
        (g["M"], g["l"], g["sigma"], g["V"], g["c_num"], g["c_den"])
    seeds = st.local_seeds().cpu().numpy()
    assert np.array_equal(seeds[ob.shards], ob.t.astype(np.uint8))
    assert [f for f in st.failures if f[0] in set(sample)] == ob.failures
    cells = st.cells()[torch.as_tensor(ob.shards.astype(np.int64), device=DEV)].cpu().numpy()
    assert np.array_equal(cells, ob.w.astype(np.uint8))
    assert st.query(keys).min().item() == 1


def test_shards_of_150k_keys_bit_exact():
    keys = S.member_keys(300000, 41, device=DEV)
    print("[sizes] n=300000 h=1", flush=True)
    st = vf.Structure.build(keys, None, b=8, h=1, seed=3)
    torch.cuda.synchronize()
    assert st.rc == vf.VF_OK and st.info["sigma"] == 9 and st.info["M"] > 140000
    _sampled_parity(st, keys, 1, 8, 3, [0, 1])


def test_largest_shard_below_a_power_of_two_with_a_bound_above_it():
    """Buffers are sized by the planning bound (here above 2^16) while the
    geometry follows the actual largest shard (below it)."""
    n = 8240421  # eps = 0.0175 gives h = 7: 128 shards of about 64 400 keys
    keys = S.member_keys(n, 43, device=DEV)
    sz = vf.vf_plan(n, 8, 0.0175, True)
    assert sz.h == 7 and sz.shard_cap >= 65536
    print("[sizes] n=8240421 eps=0.0175", flush=True)
    st = vf.Structure.build(keys, None, b=8, eps=0.0175, seed=1)
    torch.cuda.synchronize()
    assert st.rc == vf.VF_OK
    assert st.info["M"] < 65536 and (st.info["c_num"], st.info["c_den"]) == (1120, 1000)
    _sampled_parity(st, keys, 7, 8, 1, [0, 77, 127])
