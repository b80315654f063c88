"""C-ABI library: loads, exports every symbol the header declares, and
rejects bad arguments before touching the GPU (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lindblad.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) - {"defined"})


@pytest.fixture(scope="module")
def L():
    from paper_2603_18052_amd import lindblad
    return lindblad.lib()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("lindblad_liouvillian", "lindblad_propagator", "lindblad_propagate", "grape_gradient",
              "lindblad_generators", "lindblad_propagate_baseline", "lindblad_batch_run",
              "lb_workspace_create", "lb_workspace_destroy", "lindblad_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2603_18052_amd import lindblad
    assert set(declared_functions()) <= set(lindblad.SYMBOLS)


def test_validation_errors_without_gpu(L):
    from paper_2603_18052_amd import lindblad as lb
    assert L.lindblad_liouvillian(0, None, 0, None, None, None) == lb.ESHAPE
    assert "d must be" in lb.last_error()
    assert L.lindblad_liouvillian(3, None, 0, None, None, None) == lb.EINVAL
    assert L.lindblad_liouvillian(3, 1, 70, 1, 1, None) == lb.ESHAPE
    assert L.lindblad_generators(0, 1, 1, 1, 1, 1, 1, None) == lb.ESHAPE
    assert L.lindblad_generators(9, -1, 1, 1, 1, 1, 1, None) == lb.ESHAPE
    dts = (ctypes.c_double * 1)(0.5)
    assert L.lindblad_propagator(0, 1, 1, dts, 0.25, 1, None, None, None, None) == lb.ESHAPE
    assert L.lindblad_propagator(9, 0, 1, dts, 0.25, 1, None, None, None, None) == lb.ESHAPE
    assert L.lindblad_propagator(9, 1, None, dts, 0.25, 1, None, None, None, None) == lb.EINVAL
    assert L.lindblad_propagator(9, 1, 1, dts, 0.0, 1, None, None, None, None) == lb.EINVAL
    bad = (ctypes.c_double * 1)(float("nan"))
    assert L.lindblad_propagator(9, 1, 1, bad, 0.25, 1, None, None, None, None) == lb.EINVAL
    assert L.lindblad_propagate(9, 1, 0, 0, 1, 1, None, None) == lb.ESHAPE
    assert L.lindblad_propagate(9, 1, 0, 1, 1, -1, None, None) == lb.EINVAL
    assert L.lindblad_propagate(9, 1, 9, 1, 1, 1, None, None) == lb.EINVAL
    assert L.lindblad_propagate(9, 1, 8, 1, 1, 1, None, None) == lb.EINVAL  # past the last precision
    assert L.lindblad_propagate(9, None, 0, 1, 1, 1, None, None) == lb.EINVAL
    assert L.lindblad_propagate_baseline(5000, 1, 1, 1, 1, None, None) == lb.ESHAPE


def test_workspace_lifecycle(L):
    h = ctypes.c_void_p()
    assert L.lb_workspace_create(1 << 20, ctypes.byref(h)) == 0
    assert L.lb_workspace_bytes(h) == 0
    assert L.lb_workspace_destroy(h) == 0
    assert L.lb_workspace_create(1 << 20, None) == -1


def test_chain_variant_lists_and_rule(L):
    """Host-side variant bookkeeping: which kernels exist for a shape, the
    built-in choice, and the tuning table (no kernel runs)."""
    from paper_2603_18052_amd import lindblad as lb
    # d = 3: every FP64 family that handles n = 9
    v = lb.chain_variants(9, "c128", 1)
    assert v[:3] == [100, 150, 200]  # baseline, its graph-replayed twin, wave
    assert [x for x in v if x // 100 == 3] == [301, 302, 303]  # KS = 3 k steps
    assert {501, 502, 551, 552, 1104, 1154, 1108, 1158, 1101, 1151, 1102, 1152} <= set(v) and 600 not in v
    assert 600 in lb.chain_variants(9, "c64", 1000) and 100 not in lb.chain_variants(9, "c64", 1)
    assert lb.chain_variant(9, "c128", 1) == 200
    # d = 9 headline: fused with the smallest k split giving at most 32 units
    v = lb.chain_variants(81, "c128", 4096)
    assert [x for x in v if x // 100 == 3] == [306, 308, 311]
    assert 800 in v and 800 in lb.chain_variants(96, "c64", 16) and 800 not in lb.chain_variants(85, "c128", 16)
    assert {1000, 1001, 1002, 1003} <= set(v) and 1003 in lb.chain_variants(81, "c64", 16)
    assert 1002 not in lb.chain_variants(82, "c128", 16)
    assert 200 not in v
    assert lb.chain_variant(81, "c128", 4096) == 1002  # rows/columns 0..79 on MFMA, 80 on the VALU
    assert lb.chain_variant(84, "c128", 4096) == 800  # SIMD-balanced layout
    assert lb.chain_variant(81, "c128", 64) == 100  # little work per step: plain matvec
    assert lb.chain_variant(81, "c64", 64) == 1003
    assert lb.chain_variant(100, "c64", 64) == 308
    assert lb.chain_variant(16, "c64", 4096) == 200
    # d = 27: no fused variant; GEMM from 16 states, matvec below
    assert not [x for x in lb.chain_variants(729, "c128", 64) if x // 100 == 3]
    assert lb.chain_variant(729, "c128", 64) == 501
    assert lb.chain_variant(729, "c128", 1024) == 1101  # ring LDS-tiled GEMM: 16 x 16 tiles fill the chip
    assert lb.chain_variant(729, "c64", 1024) == 1101
    assert lb.chain_variant(729, "c128", 512) == 502  # 128 tiles: the small-tile GEMM
    assert lb.chain_variant(729, "c128", 1) == 100
    assert lb.chain_variant(729, "c64", 1) == 600
    assert 100 not in lb.chain_variants(729, "c64", 64)
    # BF16 precisions
    assert lb.chain_variants(81, "bf16_sliced", 16) == [400, 700, 750, 1200, 1250, 1201, 1251, 1202, 1252]
    assert lb.chain_variants(729, "bf16_sliced", 16) == [700, 750, 1200, 1250, 1201, 1251, 1202, 1252]
    assert [lb.variant_name(x) for x in (150, 552, 306, 800, 1000, 1001, 1002, 1003, 1104, 1158)] == [
        "baseline+graph", "gemm(w2)+graph", "fused(k6)", "fused_balanced", "fused_tail", "fused_tail(w16)",
        "fused_tail(tiles)", "fused_tail(tiles+presum)", "gemm_tiled(w4)", "gemm_tiled(w8)+graph"]
    assert [lb.variant_name(x) for x in (1200, 1201, 1251)] == [
        "planes_tiled", "planes_tiled(ring)", "planes_tiled(ring)+graph"]
    assert [lb.variant_name(x) for x in (1300, 1301, 1302, 1500, 1553)] == [
        "i8_fused(w8)", "i8_fused(w4)", "i8_fused(w8+progress)", "i8_gemm(96x64)", "i8_gemm(96x32 pair)+graph"]
    assert lb.chain_variant(729, "bf16_hilo", 16) == 1202
    assert lb.chain_variant(729, "bf16_sliced", 1024) == 1202  # ring plane GEMM (256 tiles: no k split)
    # fixed point: one wavefront per state for n <= 16, else the per-row matvec (and its graph twin)
    assert lb.chain_variants(9, "q15", 1) == [900, 901, 951, 1400]
    assert lb.chain_variants(729, "q15", 3) == [901, 951]
    assert lb.chain_variant(81, "q15", 16) == 1400  # the INT8-core kernel up to n = 96
    assert lb.chain_variant(729, "q15", 16) == 901
    # Q1.31 and the INT8-digit chain: one fused INT8-core kernel each, n <= 96
    assert lb.chain_variants(9, "q31", 1) == [1400] and lb.chain_variants(97, "q31", 1) == []
    assert lb.chain_variants(81, "i8_sliced", 4096) == [1300, 1301, 1302, 1500, 1550, 1501, 1551, 1502, 1552, 1503, 1553]
    assert lb.chain_variant(96, "i8_sliced", 1) == 1300
    # past the fused limit: 96 x 32 tiles two to a CU (1503) while they give
    # 240 or more workgroups, else 64 x 16 (1502)
    assert lb.chain_variants(729, "i8_sliced", 64) == [1500, 1550, 1501, 1551, 1502, 1552, 1503, 1553]
    assert lb.chain_variant(729, "i8_sliced", 1024) == 1503 and lb.chain_variant(729, "i8_sliced", 480) == 1503
    assert lb.chain_variant(729, "i8_sliced", 448) == 1502 and lb.chain_variant(729, "i8_sliced", 1) == 1502
    # the Hermitian-coordinate form: the fused kernels for n = d^2 <= 192 only
    i8v = [1300, 1301, 1302, 1500, 1550, 1501, 1551, 1502, 1552, 1503, 1553]
    assert lb.chain_variants(81, "i8_herm", 4096) == i8v and lb.chain_variant(81, "i8_herm", 1) == 1300
    assert lb.chain_variants(169, "i8_herm", 16) == i8v and lb.chain_variants(1, "i8_herm", 1) == i8v
    assert lb.chain_variants(82, "i8_herm", 16) == [] and lb.chain_variant(82, "i8_herm", 16) == 0
    # past n = 192 the per-step GEMM on the n x n step, the embedding's tile rule on n rows
    assert lb.chain_variants(196, "i8_herm", 16) == [1500, 1550, 1501, 1551, 1502, 1552, 1503, 1553]
    assert lb.chain_variant(729, "i8_herm", 1024) == 1503 and lb.chain_variant(729, "i8_herm", 64) == 1502
    # tuning table: set, read back, reject a variant the shape lacks, clear
    lb.tune_set(81, "c128", 4096, 502)
    assert lb.chain_variant(81, "c128", 4096) == 502
    with pytest.raises(lb.LindbladError):
        lb.tune_set(81, "c128", 4096, 200)
    lb.tune_set(81, "c128", 4096, 0)
    assert lb.chain_variant(81, "c128", 4096) == 1002
    cnt = ctypes.c_int()
    assert L.lindblad_chain_variants(0, 0, 1, None, 0, ctypes.byref(cnt)) == lb.ESHAPE
    assert L.lindblad_chain_variants(9, 8, 1, None, 0, ctypes.byref(cnt)) == lb.EINVAL
    assert L.lindblad_chain_variants(9, 0, 1, None, 0, ctypes.byref(cnt)) == 0 and cnt.value == 18
    assert L.lindblad_propagate_variant(9, 1, 0, 1, 1, 5, 999, None, None) == lb.EINVAL
    assert L.lindblad_tune(9, 1, 0, 1, 1, 0, 1, None, None, None, None) == lb.EINVAL


def test_c_client_compiles_against_the_header(tmp_path):
    """include/lindblad.h is plain C: the C client in tests/c builds with gcc
    -std=c99 and links against liblindblad.so (it runs in the GPU tests)."""
    import subprocess
    from paper_2603_18052_amd import lindblad
    lindblad.lib()
    pkg = os.path.join(ROOT, "paper_2603_18052_amd")
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", "/opt/rocm/include", os.path.join(ROOT, "tests", "c", "abi_client.c"), "-o",
           str(tmp_path / "abi_client"), "-L", pkg, "-llindblad", "-L", "/opt/rocm/lib", "-lamdhip64"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_expmv_params_meet_the_remainder_bound():
    """lindblad_expmv_params (host only): every sub-step satisfies
    e^{2r} r^{m+1} / (m+1)! <= 2^-53 with r = a / s <= 4, and bad norms fail."""
    import math
    from paper_2603_18052_amd import lindblad as lb
    assert lb.expmv_params(0.0) == (1, 1)
    for a in (1e-6, 0.3, 1.0, 4.0, 13.0, 26.5, 100.0, 1e4):
        s, m = lb.expmv_params(a)
        r = a / s
        assert s >= 1 and 1 <= m <= 80 and r <= 4.0 + 1e-12
        assert 2 * r + (m + 1) * math.log(r) - math.lgamma(m + 2) <= -53 * math.log(2) + 1e-9, (a, s, m)
    s1, m1 = lb.expmv_params(13.0)
    assert s1 * m1 <= 13 * 18  # never worse than theta = 1 (18 terms, 13 sub-steps)
    for bad in (-1.0, float("inf"), float("nan"), 1e12):
        with pytest.raises(lb.LindbladError):
            lb.expmv_params(bad)
