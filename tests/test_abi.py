"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function the header declares, and rejects bad arguments without a device."""

import ctypes
import os
import re

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            txt = open(os.path.join(inc, fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(cmaes_[a-z_]+)\s*\(", txt))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("cmaes_create", "cmaes_generation", "cmaes_restart_ipop", "cmaes_state",
                     "cmaes_destroy", "cmaes_set_state", "cmaes_generation_with_z", "cmaes_ask",
                     "cmaes_tell", "cmaes_set_objective", "cmaes_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2409_11765_amd as P
    lib = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layouts_match_header():
    import paper_2409_11765_amd.binding as B
    # int32 x4, int64, double x7, stream pointer, two function pointers, the
    # allocator context and two int32 (variant) -> 120 bytes on x86-64
    assert ctypes.sizeof(B.CmaesOptions) == 4 * 4 + 8 + 8 * 7 + 8 + 3 * 8 + 8
    assert B.CmaesOptions.dev_malloc.offset == 88 and B.CmaesOptions.alloc_ctx.offset == 104
    assert B.CmaesState.m.offset == 4 * 4 + 8 * 3 + 8 * 2 + 4 + 4 + 4 + 4


def test_default_options_and_errors_without_device():
    import paper_2409_11765_amd as P
    o = P.cmaes_default_options()
    assert (o.precision, o.k_max, o.box_lo, o.box_hi, o.f_target) == (1, 256, -4.0, 4.0, 1e-8)
    with pytest.raises(P.CmaesError):
        P.cmaes_create(0, 10, 1.0, 1)          # n < 1
    with pytest.raises(P.CmaesError):
        P.cmaes_create(5, 1, 1.0, 1)           # lambda < 2
    with pytest.raises(P.CmaesError):
        P.cmaes_create(5, 10, -1.0, 1)         # sigma0 <= 0
    assert isinstance(P.cmaes_last_error(), str)


def test_gemm_tile_table_without_device():
    import paper_2409_11765_amd as P
    assert P.cmaes_gemm_config_count() == 7
    tiles = [P.cmaes_gemm_config_info(c) for c in range(7)]
    assert tiles[0] == (128, 128, 16)
    for bm, bn, bk in tiles:
        # 4 waves in a 2 x 2 grid of 32 x 32 MFMA blocks; float4 staging
        assert bm % 64 == 0 and bn % 64 == 0 and bk in (16, 32)
    assert len(set(tiles)) == 7
    assert any(bm == bn for bm, bn, _ in tiles)
    with pytest.raises(P.CmaesError):
        P.cmaes_gemm_config_info(7)
    with pytest.raises(P.CmaesError):
        P.cmaes_gemm_config_info(-1)


def test_syrk_split_plan_without_device():
    import paper_2409_11765_amd as P
    # headline covariance update (n = 1000, mu = 3072): 128-tiles, two 4-wave
    # workgroups per CU, or one 8-wave workgroup per CU for 128 x 128 x 32
    assert P.cmaes_syrk_plan(0, 1000, 3072) == (36, 224, 14)
    assert P.cmaes_syrk_plan(4, 1000, 3072) == (36, 448, 7)
    for cfg in (0, 4, 5, 6):
        bm = P.cmaes_gemm_config_info(cfg)[0]
        for n, K in [(1, 1), (10, 5), (40, 64), (200, 4864), (1000, 3072), (2000, 2048), (97, 33)]:
            tiles, kspan, splits = P.cmaes_syrk_plan(cfg, n, K)
            tm = -(-n // bm)
            assert tiles == tm * (tm + 1) // 2
            # the splits cover [0, K) exactly once, none of them empty
            assert kspan % 32 == 0 and splits >= 1
            assert (splits - 1) * kspan < K <= splits * kspan
    for bad in [(1, 100, 100), (3, 100, 100), (7, 100, 100), (0, 0, 10), (0, 10, 0)]:
        with pytest.raises(P.CmaesError):
            P.cmaes_syrk_plan(*bad)


def test_krep_status_layout():
    import paper_2409_11765_amd.binding as B
    assert ctypes.sizeof(B.KrepStatus) == 4 * 4 + 8 * 3
    assert B.KrepStatus.lockstep_generations.offset == 16


def test_ctypes_layouts_equal_the_c_compilers(tmp_path):
    """The binding's structure layouts equal what a C compiler makes of the
    header (gcc on the host)."""
    import shutil
    import subprocess
    import paper_2409_11765_amd.binding as B
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stddef.h>
#include <stdio.h>
#include "cmaes_mi355x.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(cmaes_options_t), offsetof(cmaes_options_t, stream),
         offsetof(cmaes_options_t, dev_malloc), offsetof(cmaes_options_t, alloc_ctx),
         offsetof(cmaes_options_t, variant), sizeof(cmaes_state_t),
         offsetof(cmaes_state_t, m), offsetof(cmaes_state_t, order), sizeof(cmaes_krep_status_t));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(B.CmaesOptions), B.CmaesOptions.stream.offset, B.CmaesOptions.dev_malloc.offset,
            B.CmaesOptions.alloc_ctx.offset, B.CmaesOptions.variant.offset, ctypes.sizeof(B.CmaesState),
            B.CmaesState.m.offset,
            B.CmaesState.order.offset, ctypes.sizeof(B.KrepStatus)]
    assert got == want
