"""Building from keys in host memory (vfilter_build_host): the chunked
copy-and-count path gives the same structure as building from the same keys
on the device, and sampled shards match the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2503_18397_amd as vf
DEV = "cuda:0"


def test_host_streamed_build_equals_device_build():
    n, h, b, seed = 1 << 24, 8, 8, 4
    keys_dev = S.member_keys(n, 51, device=DEV)
    keys_host = torch.empty(n, dtype=torch.int64, pin_memory=True)
    keys_host.copy_(keys_dev)
    opts = vf.vf_default_opts(h=h)
    sz = vf.vf_plan(n, b, 0.0, True, opts)
    extra = (8 * n + 255) // 256 * 256
    ws = torch.empty(sz.workspace_bytes + extra, dtype=torch.uint8, device=DEV)
    st = torch.empty(sz.structure_bytes, dtype=torch.uint8, device=DEV)
    print("[stream] host build, 2^22-key chunks", flush=True)
    rc, hh = vf.vfilter_build_host(keys_host, b, 0.0, seed, opts, ws, st, chunk=1 << 22)
    torch.cuda.synchronize()
    assert rc == vf.VF_OK
    with pytest.raises(vf.VFError):  # the workspace must hold the device copy too
        vf.vfilter_build_host(keys_host, b, 0.0, seed, opts, ws[: sz.workspace_bytes], st)
    ref = vf.Structure.build(keys_dev, None, b=b, h=h, seed=seed)
    torch.cuda.synchronize()
    ih, ir = vf.vf_info(hh), ref.info
    for f in ("M", "l", "sigma", "V", "n_failures", "failed_shards"):
        assert ih[f] == ir[f], f
    nb = ir["S"] * ir["V"]
    assert torch.equal(st[:nb], ref.cells().view(-1))
    assert vf.vf_failures(hh) == ref.failures
    out = torch.empty(n, dtype=torch.uint8, device=DEV)
    vf.vfilter_contains(hh, keys_dev, out)
    assert out.min().item() == 1
    sample = [0, 97, 255]
    ob = O.build(keys_host.numpy().view(np.uint64), b=b, is_filter=True, h=h, seed=seed,
                 shards=sample)
    cells = ref.cells()[torch.as_tensor(sample, device=DEV)].cpu().numpy()
    assert np.array_equal(cells, ob.w.astype(np.uint8))
    vf.vf_free(hh)
