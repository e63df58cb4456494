"""Queries grouped by shard (vf_query_grouped, vfilter_contains_grouped)
through the C ABI: every answer equals the CPU oracle's and the plain
query's, for every cell width, with cells in LDS and in global memory,
the MWHC hypergraph, one chunk and many chunks, and the argument errors."""
import ctypes as C

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


def _u64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def _queries(keys, n_neg, seed):
    neg = S.negative_keys(keys.numel(), n_neg, seed)
    return torch.cat([keys, neg])


def _check(st, ob, q, workspace=None):
    """Grouped answers == plain answers == oracle answers on q."""
    qd = q.to(DEV)
    dt = np.uint8 if st.is_filter else _NP[st.info["cell_bytes"]]
    got = st.query_grouped(qd, workspace=workspace).cpu().numpy().view(dt)
    plain = st.query(qd).cpu().numpy().view(dt)
    assert np.array_equal(got, plain)
    want = O.query(ob, _u64(q))
    assert np.array_equal(got.astype(np.uint64), want)


@pytest.mark.parametrize("n,b,h,seed", [
    (1, 8, 0, 1), (5000, 1, 0, 2), (40000, 8, 2, 3), (30000, 16, 2, 4), (20000, 32, 1, 5),
    (20000, 64, 1, 6), (200000, 8, 0, 7),
])
def test_vfunc_grouped_matches_oracle(n, b, h, seed):
    """Cell widths 1, 2, 4 and 8 bytes; (200000, h = 0) has 225K cells,
    more than LDS holds, which the grouped entry point answers with the
    plain gathers."""
    print(f"[grouped] vfunc n={n} b={b} h={h} seed={seed}", flush=True)
    keys = S.member_keys(n, 500 + seed)
    vals = S.values(n, b, 500 + seed)
    st = vf.Structure.build(keys.to(DEV), vals.to(DEV), b=b, h=h, seed=seed)
    assert st.rc == vf.VF_OK
    ob = O.build(_u64(keys), _u64(vals), b=b, is_filter=False, h=h, seed=seed)
    assert ob.status == 0
    _check(st, ob, _queries(keys, 3 * n + 7, 500 + seed))


@pytest.mark.parametrize("n,b,h,seed", [(1 << 17, 8, 3, 11), (100000, 4, 4, 12),
                                        (1 << 17, 8, 12, 14), (100000, 8, 13, 13)])
def test_vfilter_grouped_matches_oracle(n, b, h, seed):
    """h = 12 (4096 shards) is the largest shard count of the per-segment
    histograms (the scatter's LDS at its largest); h = 13 (8192 shards)
    takes the grouping for more shards: one shard counter per key."""
    print(f"[grouped] vfilter n={n} b={b} h={h} seed={seed}", flush=True)
    keys = S.member_keys(n, 600 + seed)
    st = vf.Structure.build(keys.to(DEV), None, b=b, h=h, seed=seed)
    assert st.rc == vf.VF_OK
    ob = O.build(_u64(keys), b=b, is_filter=True, h=h, seed=seed)
    q = _queries(keys, 200000, 600 + seed)
    _check(st, ob, q)
    assert st.query_grouped(keys.to(DEV)).min().item() == 1


def test_mwhc_grouped_matches_oracle():
    n, b, h, seed = 50000, 8, 2, 21
    print("[grouped] mwhc", flush=True)
    keys = S.member_keys(n, 700)
    vals = S.values(n, b, 700)
    st = vf.Structure.build(keys.to(DEV), vals.to(DEV), b=b, h=h, seed=seed, mwhc=True)
    assert st.rc == vf.VF_OK
    ob = O.build(_u64(keys), _u64(vals), b=b, is_filter=False, h=h, seed=seed, mwhc=True)
    _check(st, ob, _queries(keys, 50000, 700))


@pytest.mark.parametrize("chunk", [1, 999, 4096])
def test_many_chunks_give_the_same_answers(chunk):
    """A workspace of the per-shard part plus room for `chunk` keys (a few
    dozen more where the alignment leaves room): the queries are answered
    chunk by chunk."""
    n, b, h, seed = 30000, 8, 3, 31
    print(f"[grouped] chunk={chunk}", flush=True)
    keys = S.member_keys(n, 800)
    st = vf.Structure.build(keys.to(DEV), None, b=b, h=h, seed=seed)
    assert st.rc == vf.VF_OK
    ob = O.build(_u64(keys), b=b, is_filter=True, h=h, seed=seed)
    nq = 5000 if chunk == 1 else 100000
    q = _queries(keys[:nq // 2], nq - nq // 2, 800)
    # per-shard part + one key (8 B key, 4 B index, 1 B answer, each 256-aligned)
    fixed = vf.vf_query_grouped_bytes(st.handle, 1) - 768
    ws = torch.empty(fixed + 768 + 13 * chunk, dtype=torch.uint8, device=DEV)
    _check(st, ob, q, workspace=ws)


@pytest.mark.parametrize("b,reps,neg", [(8, 40, 3_000_000), (64, 320, 3_000_000)])
def test_large_chunk_matches_plain(b, reps, neg):
    """Millions of queries in one chunk: with b = 8 (5.6 million queries,
    687 segments of 8 200) the answers are placed through LDS windows; with
    b = 64 (24 million queries, 1024 segments of 23 400 and 183 KB windows,
    more than LDS holds) they are written straight to their places."""
    n, h, seed = 1 << 16, 2, 41
    print(f"[grouped] large chunk b={b}", flush=True)
    keys = S.member_keys(n, 1000)
    vals = S.values(n, b, 1000)
    st = vf.Structure.build(keys.to(DEV), vals.to(DEV), b=b, h=h, seed=seed)
    assert st.rc == vf.VF_OK
    q = torch.cat([keys.repeat(reps), S.negative_keys(n, neg, 1000)]).to(DEV)
    dt = _NP[st.info["cell_bytes"]]
    got = st.query_grouped(q).cpu().numpy().view(dt)
    assert np.array_equal(got, st.query(q).cpu().numpy().view(dt))
    assert np.array_equal(got[:n].astype(np.uint64), _u64(vals) & np.uint64(
        (1 << b) - 1 if b < 64 else 0xFFFFFFFFFFFFFFFF))
    ob = O.build(_u64(keys), _u64(vals), b=b, is_filter=False, h=h, seed=seed)
    tail = q[-20000:].cpu()
    assert np.array_equal(got[-20000:].astype(np.uint64), O.query(ob, _u64(tail)))


def test_grouped_argument_errors():
    n = 10000
    keys = S.member_keys(n, 900).to(DEV)
    vals = S.values(n, 8, 900).to(DEV)
    st = vf.Structure.build(keys, vals, b=8, h=1, seed=3)
    fl = vf.Structure.build(keys, None, b=8, h=1, seed=3)
    assert st.rc == vf.VF_OK and fl.rc == vf.VF_OK
    out = torch.empty(n, dtype=torch.uint8, device=DEV)
    need = vf.vf_query_grouped_bytes(st.handle, n)
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    lib = vf._lib
    k, o, w = keys.data_ptr(), out.data_ptr(), ws.data_ptr()
    # n = 0 does nothing
    assert lib.vf_query_grouped(st.handle, None, 0, None, None, 0, None) == vf.VF_OK
    # wrong kind of handle
    assert lib.vf_query_grouped(fl.handle, k, n, o, w, need, None) == vf.VF_EINVAL
    assert lib.vfilter_contains_grouped(st.handle, k, n, o, w, need, None) == vf.VF_EINVAL
    # null pointers, too small a workspace
    assert lib.vf_query_grouped(st.handle, k, n, o, None, need, None) == vf.VF_EINVAL
    assert lib.vf_query_grouped(st.handle, None, n, o, w, need, None) == vf.VF_EINVAL
    assert lib.vf_query_grouped(st.handle, k, n, o, w, 64, None) == vf.VF_ENOSPC
    # a workspace or keys not 8-byte aligned
    assert lib.vf_query_grouped(st.handle, k, n, o, w + 4, need - 4, None) == vf.VF_EINVAL
    assert lib.vf_query_grouped(st.handle, k + 4, n - 1, o, w, need, None) == vf.VF_EINVAL
    b = C.c_uint64(0)
    assert lib.vf_query_grouped_bytes(None, n, C.byref(b)) == vf.VF_EINVAL
    assert lib.vf_query_grouped_bytes(st.handle, n, None) == vf.VF_EINVAL
    # the out buffer is untouched by a rejected call, written by a good one
    out.fill_(0xAB)
    assert lib.vf_query_grouped(st.handle, k, n, o, w, 64, None) == vf.VF_ENOSPC
    torch.cuda.synchronize()
    assert out.min().item() == 0xAB
    assert lib.vf_query_grouped(st.handle, k, n, o, w, need, None) == vf.VF_OK
    torch.cuda.synchronize()
    assert torch.equal(out, vals.to(torch.uint8))
