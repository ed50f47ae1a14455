"""CPU-only checks of the C-ABI library: it loads, exports every function that
include/pmf.h declares, and its host-side validation works without a GPU."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(pmf_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1509_06004_amd import pmf
    return pmf.load_library()


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("pmf_create", "pmf_solve_batch", "pmf_extract_cut", "pmf_destroy"):
        assert n in names


def test_header_is_plain_c_and_cxx(tmp_path):
    """The header compiles as C99 and as C++ (callers from either language)."""
    import subprocess
    src = tmp_path / "use.c"
    src.write_text('#include "pmf.h"\nint main(void) { pmf_options o; pmf_default_options(&o); return (int)o.tile_w; }\n')
    for cmd in (["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-I", os.path.dirname(HEADER), str(src)],
                ["g++", "-std=c++17", "-Wall", "-Werror", "-fsyntax-only", "-x", "c++", "-I", os.path.dirname(HEADER),
                 str(src)]):
        subprocess.run(cmd, check=True)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n


def test_strerror_and_defaults(lib):
    from paper_1509_06004_amd import pmf
    assert pmf.pmf_strerror(0) == "ok"
    assert "headroom" in pmf.pmf_strerror(pmf.PMF_EOVERFLOW)
    assert pmf.pmf_strerror(999) == "unknown status"
    o = pmf.pmf_default_options()
    assert o.tile_w in (32, 64) and o.tile_w * o.tile_h == 1024
    assert o.inner_iters > 0 and o.sweeps_per_relabel > 0 and o.max_supersteps > 0


def _fake(W=10, H=7, K=4, L=3, ptr=0x1000):
    from paper_1509_06004_amd import pmf
    return pmf.InstanceC(W, H, K, L, ptr, ptr, ptr, 0, 0, ptr)


def test_host_validation(lib):
    from paper_1509_06004_amd import pmf
    assert pmf.pmf_check_instances([_fake(), _fake(K=8)]) == (pmf.PMF_OK, -1)
    bad = [_fake(), _fake(K=6)]
    assert pmf.pmf_check_instances(bad) == (pmf.PMF_EINVAL, 1)
    assert pmf.pmf_check_instances([_fake(W=0)])[0] == pmf.PMF_EINVAL
    assert pmf.pmf_check_instances([_fake(L=0)])[0] == pmf.PMF_EINVAL
    assert pmf.pmf_check_instances([_fake(ptr=0)])[0] == pmf.PMF_EINVAL
    assert pmf.pmf_check_instances([_fake(W=1 << 15, H=1 << 15)])[0] == pmf.PMF_EINVAL
    assert pmf.pmf_check_instances([])[0] == pmf.PMF_OK


def test_null_handle_is_rejected(lib):
    from paper_1509_06004_amd import pmf
    assert pmf.pmf_solve_batch(None, [_fake()], 0x10, 0) == pmf.PMF_EINVAL
    assert pmf.pmf_extract_cut(None, 0, 0, 0x10) == pmf.PMF_EINVAL
    assert pmf.pmf_destroy(None) == pmf.PMF_EINVAL
    assert pmf.load_library().pmf_get_trace(None, None, 0) == -pmf.PMF_EINVAL


def test_query_bytes_scales_with_size(lib):
    from paper_1509_06004_amd import pmf
    small = pmf.pmf_query_bytes([_fake(64, 64, 4, 1)])
    big = pmf.pmf_query_bytes([_fake(500, 375, 4, 20)])
    eight = pmf.pmf_query_bytes([_fake(500, 375, 8, 20)])
    assert 0 < small < big < eight
    px = 500 * 375
    # state: K+3 int32 planes + uint16 mask word + L uint8 masks per pixel,
    # and 128 inbox words per 32x32 tile at K = 4, 384 at K = 8
    tiles = 16 * 12
    assert big >= px * ((4 + 3) * 4 + 2 + 20) + tiles * 128 * 4
    assert eight >= px * ((8 + 3) * 4 + 2 + 20) + tiles * 384 * 4
    with pytest.raises(pmf.PmfError):
        pmf.pmf_query_bytes([_fake(K=5)])


def test_to_device_share_never_returns_another_arrays_copy():
    """A share dict carried over calls holds each uploaded array with its
    copy; an entry under the id of a new object but for another array (ids of
    dead objects are reused) is not taken for the new one."""
    import torch
    from paper_1509_06004_amd import pmf, workload
    inst = workload.config0()[0]
    share = {}
    first = pmf.to_device([inst], device="cpu", share=share)[0]
    assert torch.equal(first.lambdas, torch.from_numpy(inst.lambdas))
    again = pmf.to_device([inst], device="cpu", share=share)[0]
    assert again.lambdas is first.lambdas  # same object: one copy
    other = inst.with_lambdas(inst.lambdas + 1)
    share[id(other.lambdas)] = (object(), torch.zeros(3, dtype=torch.int32))  # a stale entry under its id
    got = pmf.to_device([other], device="cpu", share=share)[0]
    assert torch.equal(got.lambdas, torch.from_numpy(other.lambdas))
