"""Checks of the gfx950 assembly the library is built from (no GPU needed).

Two MFMA placements gave wrong results on the device: result registers that
partially overlap the accumulator input, and a global store of a result
reached through a branch right after the MFMA (the store read a partly
written tile). The build refuses both; these tests pin the checks."""
import os

import pytest

from paper_2112_01579_amd import build as B


def test_partial_overlap_detector():
    bad = "\tv_mfma_f32_16x16x4_f32 v[84:87], v84, v82, v[86:89]\n"
    same = "\tv_mfma_f32_16x16x4_f32 v[8:11], v83, v79, v[8:11]\n"
    apart = "\tv_mfma_f32_16x16x32_f16 v[8:11], v[32:35], v[36:39], v[12:15]\n"
    zero = "\tv_mfma_f32_16x16x4_f32 v[86:89], v79, v80, 0\n"
    agpr = "\tv_mfma_f32_16x16x16_f16 a[0:3], v[30:31], v[38:39], a[2:5]\n"
    fn = "_Zkernel:\n"
    assert B.mfma_partial_overlaps(fn + bad) == [("_Zkernel", bad.strip())]
    assert B.mfma_partial_overlaps(fn + same + apart + zero) == []
    assert len(B.mfma_partial_overlaps(agpr)) == 1


def test_early_vmem_read_detector():
    body = [
        "_Zk:",
        "\tv_mfma_f32_16x16x4_f32 v[8:11], v8, v9, v[84:87]",
        "\ts_cbranch_vccnz .LBB3_110",
        "\tglobal_load_dwordx4 v[80:83], v[12:13], off",
        "\ts_waitcnt vmcnt(0)",
        "\ts_nop 6",
        "\tv_add_f32_e32 v11, v11, v83",
        ".LBB3_110:",
        "\tglobal_store_dwordx4 v[12:13], v[8:11], off",
        "\ts_endpgm",
    ]
    bad = B.mfma_early_vmem_reads("\n".join(body))
    assert len(bad) == 1 and "global_store" in bad[0][2]
    # enough wait states on every path: accepted
    padded = body[:2] + ["\ts_nop 7", "\ts_nop 7", "\ts_nop 3"] + body[2:]
    assert B.mfma_early_vmem_reads("\n".join(padded)) == []
    # a load into the result registers does not read them: accepted
    load = body[:2] + ["\tglobal_load_dwordx4 v[8:11], v[12:13], off", "\ts_endpgm"]
    assert B.mfma_early_vmem_reads("\n".join(load)) == []
    # a chain: the first result is overwritten by the next MFMA, whose own
    # result is padded: accepted
    chain = body[:2] + ["\tv_mfma_f32_16x16x4_f32 v[8:11], v1, v2, v[8:11]", "\ts_nop 7", "\ts_nop 3"] + body[2:]
    assert B.mfma_early_vmem_reads("\n".join(chain)) == []


def test_built_kernels_have_no_partial_mfma_overlap():
    files = B.device_asm_files()
    if not files:
        pytest.skip("library not built in this tree")
    n_mfma = 0
    for path in files:
        with open(path) as fh:
            text = fh.read()
        n_mfma += text.count("v_mfma")
        assert B.mfma_partial_overlaps(text) == [], os.path.basename(path)
        assert B.mfma_early_vmem_reads(text) == [], os.path.basename(path)
    assert n_mfma > 1000
