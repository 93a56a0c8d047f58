"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: these tests run without a GPU)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT, gpu_available

HEADER_DIR = os.path.join(ROOT, "include")


def declared_functions():
    names = set()
    for fn in os.listdir(HEADER_DIR):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fn)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        names |= set(re.findall(r"\b(kh_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("kh_create", "kh_destroy", "kh_count", "kh_count_multi_k",
                     "kh_table_info", "kh_table_export", "kh_table_free",
                     "kh_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_1809_07014_amd as kh
    lib = kh.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_library_is_built_for_gfx950():
    from paper_1809_07014_amd import build
    assert build.ARCH == "gfx950"
    assert os.path.exists(build.SO)
    # the device code object inside the library names its target
    data = open(build.SO, "rb").read()
    assert b"gfx950" in data


def test_null_arguments_are_rejected():
    import paper_1809_07014_amd as kh
    lib = kh.load()
    p = kh.Params()
    lib.kh_default_params(ctypes.byref(p), 21)
    assert (p.k, p.min_count, p.qual_offset, p.qual_cutoff) == (21, 2, 33, 20)
    out = ctypes.c_void_p()
    rs = kh.ReadsStruct(None, None, None, 0, 0)
    assert lib.kh_count(None, ctypes.byref(rs), ctypes.byref(p), None,
                        ctypes.byref(out)) == kh.KH_EINVAL
    assert b"NULL" in lib.kh_last_error()
    assert lib.kh_table_info(None, None, None, None, None) == kh.KH_EINVAL
    assert lib.kh_table_free(None) == kh.KH_OK


@pytest.mark.skipif(gpu_available(), reason="checks the no-GPU error path")
def test_create_without_gpu_fails_loudly():
    import paper_1809_07014_amd as kh
    with pytest.raises(kh.KHError) as e:
        kh.Context(0)
    assert e.value.code == kh.KH_EDEVICE
    with pytest.raises(kh.KHError) as e:
        kh.release_cached(0)
    assert e.value.code == kh.KH_EDEVICE


def test_default_tuning():
    import paper_1809_07014_amd as kh
    assert kh.default_tuning() == dict(load_factor=0.5, bloom_bits=2, bloom_lanes=4,
                                       count_lanes=2, tiles_per_block=8, aggregate=0,
                                       tails_overlap=1, partitioned=1)


def test_owner_of_matches_oracle_partition():
    """The library's key-space partition (host side) and the oracle's shard
    function are written independently from the same published definition."""
    import numpy as np
    import oracle
    import paper_1809_07014_amd as kh
    rng = np.random.default_rng(5)
    for W in (1, 2, 3, 4):
        for S in (2, 5, 8, 1000):
            for _ in range(50):
                key = rng.integers(0, 2**63, size=W, dtype=np.uint64) * np.uint64(2) + \
                    rng.integers(0, 2, size=W, dtype=np.uint64)
                assert kh.owner_of(key, S) == oracle.shard_of(key, S)
    assert kh.owner_of(np.array([7], np.uint64), 1) == 0


def test_create_needs_both_allocator_hooks(kh):
    """kh_create refuses one allocator hook without the other before it
    touches a device."""
    import ctypes
    lib = kh.load()
    h = ctypes.c_void_p()
    one = kh._allocator_hooks((lambda n, d: 0, lambda p, n, d: None))
    assert lib.kh_create(ctypes.byref(h), 0, 0, one[0], None, None) == kh.KH_EINVAL
    assert lib.kh_create(ctypes.byref(h), 0, 0, None, one[1], None) == kh.KH_EINVAL
    assert not h.value
    assert b"alloc_fn" in lib.kh_last_error()


def test_allocator_hook_marshalling(kh):
    """The Python side of the allocator hooks: addresses pass through, an
    allocator that raises reports no memory (NULL), frees see the size."""
    seen = []

    def alloc(n, d):
        if n > 1000:
            raise MemoryError("too big")
        return 0x1000 + n

    def free(p, n, d):
        seen.append((p, n, d))

    a, f, user = kh._allocator_hooks((alloc, free))
    assert user is None
    assert a(64, 0, None) == 0x1000 + 64
    assert not a(5000, 0, None)  # NULL
    f(0x1040, 64, 3, None)
    assert seen == [(0x1040, 64, 3)]
    assert kh._allocator_hooks(None) == (None, None, None)


def test_header_is_plain_c(tmp_path):
    """include/kmerhip.h compiles as strict C99 and as C++ (no torch or C++
    types cross the boundary)."""
    import os
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    src = tmp_path / "use.c"
    src.write_text('#include "kmerhip.h"\nint main(void) { kh_ctx *c = 0; (void)c; return 0; }\n')
    for extra in (["-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror"],
                  ["-x", "c++", "-std=c++17", "-Wall", "-Werror"]):
        r = subprocess.run([gcc, "-fsyntax-only", "-I" + inc] + extra + [str(src)],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
