"""Combined query launches (vf_query_multi): requests against several
structures (functions and filters, byte and packed cells, fuse and MWHC
graphs, sharded and not) answered by one launch per 16 requests give, for
every request, exactly what vf_query / vfilter_contains give alone, and the
oracle's answers on a sample; the serving loop merges waiting queries into
such launches with the same results."""
import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2503_18397_amd as vf
    from paper_2503_18397_amd.serve import Request, Server
DEV = "cuda:0"

# (kind, n, b, h, packed, mwhc)
_SHAPES = [("vfilter", 40000, 8, 2, False, False), ("vfilter", 30000, 5, 0, True, False),
           ("vfunc", 25000, 16, 1, False, False), ("vfunc", 20000, 33, 0, True, False),
           ("vfunc", 9000, 1, 0, True, False), ("vfilter", 12000, 8, 1, False, True),
           ("vfunc", 15000, 12, 0, False, True)]


def _structures():
    out = []
    for i, (kind, n, b, h, packed, mwhc) in enumerate(_SHAPES):
        keys = S.member_keys(n, 900 + i, device=DEV)
        vals = None if kind == "vfilter" else S.values(n, b, 900 + i, device=DEV)
        st = vf.Structure.build(keys, vals, b=b, h=h, seed=i, packed=packed, mwhc=mwhc)
        torch.cuda.synchronize()
        assert st.rc == vf.VF_OK, i
        out.append((st, keys, vals))
    return out


def _requests(structs, count, data_seed):
    rng = np.random.default_rng(data_seed)
    reqs = []
    for j in range(count):
        i = int(rng.integers(len(structs)))
        st, keys, _ = structs[i]
        n = [0, 1, 7, 300, 5000, 20000][j % 6]
        q, _ = S.queries(keys, max(n, 1), data_seed + j, member_share_per_256=128)
        reqs.append((i, q[:n].contiguous()))
    return reqs


def test_combined_launch_equals_single_queries_and_the_oracle():
    structs = _structures()
    reqs = _requests(structs, 37, 5)  # three launches: 16 + 16 + 5
    print(f"[multi] {len(reqs)} requests over {len(structs)} structures", flush=True)
    outs = vf.query_many([(structs[i][0], q) for i, q in reqs])
    torch.cuda.synchronize()
    for (i, q), got in zip(reqs, outs):
        want = structs[i][0].query(q)
        torch.cuda.synchronize()
        assert got.dtype == want.dtype and torch.equal(got, want), i
    # the oracle on one request per structure
    seen = set()
    for (i, q), got in zip(reqs, outs):
        if i in seen or q.numel() < 300:
            continue
        seen.add(i)
        kind, n, b, h, packed, mwhc = _SHAPES[i]
        st, keys, vals = structs[i]
        ob = O.build(keys.cpu().numpy().view(np.uint64),
                     None if vals is None else vals.cpu().numpy().view(np.uint64),
                     b=b, is_filter=kind == "vfilter", h=h, seed=i, mwhc=mwhc)
        want = O.query(ob, q.cpu().numpy().view(np.uint64))
        g = got.cpu().numpy()
        g = g if kind == "vfilter" else g.view({1: np.uint8, 2: np.uint16, 4: np.uint32,
                                                8: np.uint64}[g.itemsize])
        assert np.array_equal(g.astype(np.uint64), want), i


def test_combined_launch_rejects_a_batch_handle():
    n = np.array([100, 200], np.uint64)
    b = np.array([8, 8], np.int32)
    keys = S.member_keys(300, 77, device=DEV)
    bt = vf.Batch.build(keys, S.batch_values(n, b, 77, device=DEV), n, b)
    out = torch.empty(10, dtype=torch.uint8, device=DEV)
    with pytest.raises(vf.VFError) as e:
        vf.vf_query_multi([(bt.handle, keys[:10], out)])
    assert e.value.code == vf.VF_EINVAL
    bt.free()


def test_served_burst_of_queries_is_merged_with_the_same_results():
    structs = _structures()
    reqs = _requests(structs, 40, 11)
    alone = [structs[i][0].query(q).cpu() for i, q in reqs]
    srv = Server(slots=1)
    # the structures are resident: register them as finished builds
    for i, (st, keys, _) in enumerate(structs):
        r = Request(i, "vfilter", keys)
        r.result = st
        srv.sched.built[i] = r
    sub = [Request(100 + j, "query", q, target=i) for j, (i, q) in enumerate(reqs)]
    with srv.sched.cv:  # all arrive together: they wait and are merged
        for r in sub:
            srv.submit(r)
    st_ = srv.drain(timeout=60)
    srv.close()
    print("[multi] served", st_.summary(), "merged launches", srv.merged_launches, flush=True)
    assert st_.summary()["errors"] == 0
    assert srv.merged_launches >= 2
    for r, want in zip(sub, alone):
        assert torch.equal(r.result.cpu(), want)
