"""The allocation-free grouped filter query (vfilter_contains_grouped_noalloc,
for callers that cannot allocate) against the entry point it varies,
vfilter_contains_grouped with a caller workspace: bit-identical answers on
two calls in a row, the second with a smaller input (the static workspace
keeps the first call's contents), on structures with few and many shards."""
import pytest
import torch

import synthetic as S

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2503_18397_amd as vf
DEV = "cuda:0"


@pytest.mark.parametrize("n,h,b,q1,q2", [
    (1 << 20, 4, 8, 6_000_000, 100_003),   # 16 shards: two chunks of the array
    (1 << 22, 11, 8, 5_000_000, 777),      # 2048 shards: per-segment tables
    (1 << 18, 13, 4, 500_000, 65_537),     # 8192 shards: per-key scatter path
])
def test_noalloc_matches_grouped_with_workspace(n, h, b, q1, q2):
    print(f"[noalloc] n={n} h={h} b={b} q={q1},{q2}", flush=True)
    keys = S.member_keys(n, 91 + h, device=DEV)
    st = vf.Structure.build(keys, None, b=b, h=h, seed=7)
    assert st.rc == vf.VF_OK
    for q, ds in ((q1, 11), (q2, 12)):
        qs, _ = S.queries(keys, q, ds)
        out_na = torch.full((q,), 7, dtype=torch.uint8, device=DEV)
        vf.vfilter_contains_grouped_noalloc(st.handle, qs, out_na)
        want = st.query_grouped(qs)
        torch.cuda.synchronize()
        assert torch.equal(out_na, want)
        assert torch.equal(out_na, st.query(qs))
    # members always answer 1
    out = torch.zeros(n, dtype=torch.uint8, device=DEV)
    vf.vfilter_contains_grouped_noalloc(st.handle, keys, out)
    torch.cuda.synchronize()
    assert int(out.min()) == 1
    st.free()


def test_noalloc_rejects_a_function_handle():
    keys = S.member_keys(1000, 5, device=DEV)
    vals = S.values(1000, 8, 5, device=DEV)
    st = vf.Structure.build(keys, vals, b=8, h=0, seed=1)
    out = torch.zeros(1000, dtype=torch.uint8, device=DEV)
    with pytest.raises(vf.VFError) as e:
        vf.vfilter_contains_grouped_noalloc(st.handle, keys, out)
    assert e.value.code == vf.VF_EINVAL
    st.free()
