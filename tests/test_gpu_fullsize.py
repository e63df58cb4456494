"""Parity at the benchmark's full size and launch configuration.

VFilter, b = 8, n = 2^27 keys, eps = 0.0175 (h = 11, 2048 shards of about
2^16 keys), build seed 0, data seed 2027 -- exactly what bench.py builds.
Shards are independent, so the oracle rebuilds a sample of them one by one
(including shards whose first attempts failed on the GPU) and the GPU's
geometry, local seeds, failure record, cells and query answers are compared
with it exactly; properties that hold at any size (every member answers 1,
the false-positive rate is 2^-b within a binomial bound) are checked on
everything.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2503_18397_amd as vf
DEV = "cuda:0"


def test_benchmark_workload_sampled_shards_bit_exact():
    n, data_seed, seed, eps, b = 1 << 27, 2027, 0, 0.0175, 8
    print("[fullsize] generating keys", flush=True)
    keys = S.member_keys(n, data_seed, device=DEV)
    print("[fullsize] gpu build", flush=True)
    st = vf.Structure.build(keys, None, b=b, eps=eps, seed=seed)
    torch.cuda.synchronize()
    assert st.rc == vf.VF_OK
    info = st.info
    assert info["h"] == 11 and info["S"] == 2048
    fails = st.failures
    failed = sorted({f[0] for f in fails})
    rng = np.random.default_rng(7)
    sample = sorted(set(rng.choice(2048, 5, replace=False).tolist() + failed[:3] + [0, 2047]))
    print(f"[fullsize] oracle build of shards {sample}", flush=True)
    keys_np = keys.cpu().numpy().view(np.uint64)
    ob = O.build(keys_np, b=b, is_filter=True, h=11, seed=seed, shards=sample)
    g = ob.geom
    assert (info["M"], info["l"], info["sigma"], info["V"], info["c_num"], info["c_den"]) == \
        (g["M"], g["l"], g["sigma"], g["V"], g["c_num"], g["c_den"])
    assert ob.status == 0
    seeds = st.local_seeds().cpu().numpy()
    assert np.array_equal(seeds[ob.shards], ob.t.astype(np.uint8))
    assert [f for f in fails if f[0] in set(sample)] == ob.failures
    cells = st.cells()[torch.as_tensor(ob.shards.astype(np.int64), device=DEV)].cpu().numpy()
    assert np.array_equal(cells, ob.w.astype(np.uint8))

    print("[fullsize] queries", flush=True)
    assert st.query(keys).min().item() == 1  # every member, all 2^27
    q, is_mem = S.queries(keys, 1 << 24, data_seed)
    ans = st.query(q).cpu().numpy()
    mem = is_mem.cpu().numpy()
    assert ans[mem].min() == 1
    N = int((~mem).sum())
    fp = int(ans[~mem].sum())
    p = 2.0 ** -b
    assert abs(fp - N * p) <= 5 * math.sqrt(N * p * (1 - p))
    want = O.query(ob, q.cpu().numpy().view(np.uint64))
    built = want != np.uint64(0xFFFFFFFFFFFFFFFF)  # queries falling in sampled shards
    assert built.sum() > 1000
    assert np.array_equal(ans[built].astype(np.uint64), want[built])

    print("[fullsize] grouped queries", flush=True)
    assert st.query_grouped(keys).min().item() == 1
    assert np.array_equal(st.query_grouped(q).cpu().numpy(), ans)
    # chunks of 2^22 queries, as in a workspace of a quarter of the queries
    ws = torch.empty(vf.vf_query_grouped_bytes(st.handle, 1 << 22), dtype=torch.uint8,
                     device=DEV)
    assert np.array_equal(st.query_grouped(q, workspace=ws).cpu().numpy(), ans)
