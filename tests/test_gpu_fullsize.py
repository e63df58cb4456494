"""Parity at the benchmark's full size and launch configuration.

VFilter, b = 8, n = 2^27 keys, eps = 0.0175 (h = 11, 2048 shards of about
2^16 keys), build seed 0, data seed 2027 -- exactly what bench.py builds.
The oracle rebuilds every shard (shards split over host threads), and the
GPU's geometry, every local seed, the whole failure record and every cell
are compared with it exactly; 2^24 mixed queries are compared element by
element, and so are the grouped answers of one chunk of 2^26 queries (the
benchmark's chunk: 1024 segments of exactly 2^16 queries, so positions up
to 65 535 in every segment); properties that hold at any size (every
member answers 1, the false-positive rate is 2^-b within a binomial bound)
are checked on everything.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2503_18397_amd as vf
DEV = "cuda:0"


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


def test_benchmark_workload_every_shard_bit_exact():
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
    print(f"[fullsize] oracle build of all 2048 shards on {_threads()} threads", flush=True)
    keys_np = keys.cpu().numpy().view(np.uint64)
    ob = O.build_threaded(keys_np, b=b, is_filter=True, h=11, seed=seed, threads=_threads())
    g = ob.geom
    assert (info["M"], info["l"], info["sigma"], info["V"], info["c_num"], info["c_den"]) == \
        (g["M"], g["l"], g["sigma"], g["V"], g["c_num"], g["c_den"])
    assert ob.status == 0
    assert np.array_equal(st.local_seeds().cpu().numpy(), ob.t.astype(np.uint8))
    assert fails == ob.failures and len(fails) > 100
    print("[fullsize] comparing all cells", flush=True)
    cells = st.cells().cpu().numpy()
    assert np.array_equal(cells, ob.w.astype(np.uint8))
    del cells

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
    assert np.array_equal(ans.astype(np.uint64), want)

    print("[fullsize] grouped queries: one chunk of 2^26", flush=True)
    assert st.query_grouped(keys).min().item() == 1
    assert np.array_equal(st.query_grouped(q).cpu().numpy(), ans)
    # the benchmark's chunk: 2^26 queries in one workspace
    q26, _ = S.queries(keys, 1 << 26, data_seed + 1)
    ws = torch.empty(vf.vf_query_grouped_bytes(st.handle, 1 << 26), dtype=torch.uint8,
                     device=DEV)
    got26 = st.query_grouped(q26, workspace=ws).cpu().numpy()
    q26_np = q26.cpu().numpy().view(np.uint64)
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(_threads()) as ex:
        want26 = np.concatenate(list(ex.map(lambda c: O.query(ob, c),
                                            np.array_split(q26_np, _threads()))))
    assert np.array_equal(got26.astype(np.uint64), want26)
    # chunks of 2^22 queries, as in a workspace of a quarter of the queries
    ws = torch.empty(vf.vf_query_grouped_bytes(st.handle, 1 << 22), dtype=torch.uint8,
                     device=DEV)
    assert np.array_equal(st.query_grouped(q, workspace=ws).cpu().numpy(), ans)
