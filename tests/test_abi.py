"""CPU checks of the C-ABI library: it loads, exports every function that
include/vf.h declares, and its host-side planning agrees with the paper's
formulas (no GPU compute is called here)."""
import ctypes as C
import math
import os
import re
import subprocess

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "vf.h")
LIB = os.path.join(ROOT, "paper_2503_18397_amd", "libvf.so")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const\s+char)\s+\**\s*(vf\w*|vfilter\w*)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("vf_plan", "vf_build", "vf_query", "vfilter_build", "vfilter_contains",
                 "vf_info", "vf_failures", "vf_free", "vf_default_opts"):
        assert want in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (python -m paper_2503_18397_amd.build)"
    out = subprocess.check_output(["nm", "-D", "--defined-only", LIB], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    lib = C.CDLL(LIB)
    for name in _declared():
        assert name in exported, name
        assert hasattr(lib, name)


def test_binding_exports_the_same_names():
    import paper_2503_18397_amd as vf
    for name in _declared():
        assert hasattr(vf, name), name


def test_plan_uses_eq_logballsbins_and_sizes_the_cells():
    import paper_2503_18397_amd as vf
    for n, eps in [(1 << 27, 0.0175), (10**6, 0.001), (1 << 20, 0.05), (5000, 0.5)]:
        s = vf.vf_plan(n, 8, eps, True, None)
        assert s.h == O.shard_bits_eps(n, eps)
        S = 1 << s.h
        g = O.geometry(s.shard_cap, s.h)
        assert s.structure_bytes >= S * g["V"]  # one byte per cell at b = 8
        assert s.shard_cap >= n / S
    s = vf.vf_plan(1 << 27, 8, 0.0175, True, None)
    assert s.h == 11 and s.shard_cap < 1.05 * (1 << 16)


def test_plan_rejects_bad_arguments():
    import paper_2503_18397_amd as vf
    for b in (0, 65):
        with pytest.raises(vf.VFError) as e:
            vf.vf_plan(1000, b, 0.01, True, None)
        assert e.value.code == vf.VF_EINVAL
    with pytest.raises(vf.VFError):
        vf.vf_plan(1000, 8, 0.0, True, None)  # no eps and no h
    with pytest.raises(vf.VFError):
        vf.vf_plan(1000, 8, 0.01, True, vf.vf_default_opts(tmax=0))
    with pytest.raises(vf.VFError):
        vf.vf_plan(1000, 8, 0.01, True, vf.vf_default_opts(h=25))
    # the ring test option: a power of two from 64 to 2048, or 0
    for bad in (32, 100, 4096):
        with pytest.raises(vf.VFError) as e:
            vf.vf_plan(1 << 16, 8, 0.0175, True, vf.vf_default_opts(h=2, ring_cols=bad))
        assert e.value.code == vf.VF_EINVAL
    for good in (0, 64, 2048):
        vf.vf_plan(1 << 16, 8, 0.0175, True, vf.vf_default_opts(h=2, ring_cols=good))


def test_host_allocation_failure_is_vf_enomem():
    """A host allocation the library cannot make is reported as VF_ENOMEM
    (never as VF_EINVAL, never as an exception crossing the C ABI).  A
    batch of 2^32 - 1 instances needs 256 GiB of host descriptors; under an
    8 GiB address-space limit that allocation fails before any instance
    array is read."""
    code = r"""
import ctypes as C, resource, sys
resource.setrlimit(resource.RLIMIT_AS, (8 << 30, 8 << 30))
lib = C.CDLL(sys.argv[1])
n = (C.c_uint64 * 1)(10)
b = (C.c_int32 * 1)(8)
out = (C.c_uint64 * 4)()
rc = lib.vf_batch_plan(C.c_uint64((1 << 32) - 1), n, b, None, out)
print(rc)
"""
    r = subprocess.run(["python3", "-c", code, LIB], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert int(r.stdout.strip().splitlines()[-1]) == -6  # VF_ENOMEM
    import paper_2503_18397_amd as vf
    assert vf.VF_ENOMEM == -6


def test_plain_library_keeps_no_stage_clocks():
    """The stage clocks exist only in the profiling build; the plain library
    says so (no device call is made)."""
    import paper_2503_18397_amd as vf
    assert vf._lib.vf_stage_clocks(None, 0, 1) == vf.VF_EINVAL
    assert vf._lib.vf_stage_clocks(None, 0, 0) == vf.VF_EINVAL


def test_split_calls_reject_null_arguments_before_any_device_call():
    """The three-call builds and the combined query check their arguments
    on the host (VF_EINVAL) before they touch a device."""
    import paper_2503_18397_amd as vf
    L = vf._lib
    h = C.c_void_p()
    assert L.vf_build_prepare(0, 0, 8, 0.0, 1, 0, None, None, 0, None, 0, C.byref(h)) == \
        vf.VF_EINVAL
    assert L.vf_build_prepare(1000, 0, 8, 0.0, 1, 0, None, None, 0, None, 0, None) == vf.VF_EINVAL
    assert L.vf_build_launch(None, None, None, None) == vf.VF_EINVAL
    assert L.vf_build_finish(None, None) == vf.VF_EINVAL
    assert L.vf_batch_launch(None, None, None, None) == vf.VF_EINVAL
    assert L.vf_batch_finish(None, None) == vf.VF_EINVAL
    assert L.vf_query_multi(None, 1, None) == vf.VF_EINVAL
    assert L.vf_query_multi(None, 0, None) == vf.VF_OK  # nothing to answer
    bad = (vf.QueryReq * 1)()
    assert L.vf_query_multi(bad, 1, None) == vf.VF_EINVAL  # null handle
