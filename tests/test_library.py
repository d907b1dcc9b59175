"""CPU-only checks of the boundary: libskis.so builds for gfx950, loads, and exports every
function include/skis.h declares; the product package neither imports the oracle nor
falls back to the CPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "skis.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(skis_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    from paper_1709_03565_amd import build, skis
    if not os.path.exists(skis.LIB_PATH):
        build.build()
    return skis.LIB_PATH


def test_header_declares_the_boundary():
    names = _declared()
    for want in ["skis_build_sketch", "skis_estimate", "skis_greedy_max_cover", "skis_preprocess",
                 "skis_sketch_export", "skis_sketch_free", "skis_last_error"]:
        assert want in names


def test_library_exports_every_declared_symbol(libpath):
    L = ctypes.CDLL(libpath)
    for name in _declared():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (skis_\w+)", out))
    assert set(_declared()) <= exported
    from paper_1709_03565_amd import skis
    assert set(skis.EXPORTED) == set(_declared())


def test_library_targets_gfx950(libpath):
    # the embedded device code object names its target
    assert b"amdgcn-amd-amdhsa--gfx950" in open(libpath, "rb").read()


def test_default_options_and_errors_without_gpu(libpath):
    from paper_1709_03565_amd import skis
    o = skis.default_options()
    assert o.slots_per_block == 4 and o.visited_threshold == 192 and o.threads_per_block == 64
    assert o.quads_per_lane == 1
    assert o.build_inverse_index == 1
    L = skis.lib()
    h = ctypes.c_void_p()
    # argument checks happen before any device work
    assert L.skis_build_sketch(0, 0, None, None, None, 10, 1, None, None, ctypes.byref(h)) == skis.SKIS_EINVAL
    assert b"n must be positive" in L.skis_last_error()
    assert L.skis_build_sketch(5, -1, None, None, None, 10, 1, None, None, ctypes.byref(h)) == skis.SKIS_EINVAL
    assert L.skis_estimate(None, 1, None, None, None, None, None) == skis.SKIS_EINVAL
    assert L.skis_greedy_max_cover(None, 1, None, None, None, None, None) == skis.SKIS_EINVAL


def test_product_code_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_1709_03565_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f), errors="ignore").read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "skis_oracle" not in text and "ora_" not in text, f


def test_bench_kernel_names_match_the_library_table():
    # bench.py names the first-tier kernel (for the roofline and the counter lookup) from
    # its own copy of the (threads, slots, visited) -> (hash size, item capacity) table
    import re
    import bench
    src = open(os.path.join(ROOT, "paper_1709_03565_amd", "csrc", "skis_sample.hip")).read()
    table = src[src.index("kTier0[] = {"):src.index("};", src.index("kTier0[] = {"))]
    rows = re.findall(r"\{(\d+), (\d+), (\d+), (\d+), k_sample<(\d+), (\d+), (\d+), (\d+), (\d+), (\d+), 0>\}",
                      table)
    assert len(rows) >= 10
    for r in rows:
        th, sl, vi, pl, th2, sl2, vi2, hcap, icap, pl2 = map(int, r)
        assert (th, sl, vi, pl) == (th2, sl2, vi2, pl2)
        name = bench.tier_kernel_names(dict(threads_per_block=th, slots_per_block=sl, visited_threshold=vi,
                                            quads_per_lane=pl))[0]
        assert name == "k_sample<%d, %d, %d, %d, %d, %d, 0>" % (th, sl, vi, hcap, icap, pl)
    # the later tiers' names as the library instantiates them
    names = bench.tier_kernel_names({})
    mid = re.search(r"kTierMidV\[\] = \{\s*\{64, 1, 1024, \d, (k_sample<[^>]*>)\}", src).group(1)
    assert names[1] == mid
    assert "kTierHash = %s;" % names[2].replace("6144", "TIERH_RCAP").replace("8192", "TIERH_HCAP") in src
    assert "kTierGlobal = k_sample<TIERG_BLOCK, TIERG_SLOTS, 1, 1, 8 * TIERG_BLOCK, 2, 3>;" in src
    assert names[3] == "k_sample<1024, 1, 1, 1, 8192, 2, 3>" and "constexpr int TIERG_BLOCK = 1024;" in src
    assert "constexpr int TIERH_RCAP = 6144;" in src and "constexpr int TIERH_HCAP = 8192;" in src
