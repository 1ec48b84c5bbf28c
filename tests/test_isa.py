"""Checks of the gfx950 assembly the library is built from (no GPU needed).

A global store of an MFMA result reached through a branch right after the
MFMA was issued without the wait states the result needs and wrote partly
stale tiles on the device. The build refuses such code; these tests pin the
check."""
import os

import pytest

from paper_2112_01579_amd import build as B


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


def test_built_kernels_read_mfma_results_late_enough():
    files = B.device_asm_files()
    if not files:
        pytest.skip("library not built in this tree")
    n_mfma = 0
    for path in files:
        with open(path) as fh:
            text = fh.read()
        n_mfma += text.count("v_mfma")
        assert B.mfma_early_vmem_reads(text) == [], os.path.basename(path)
    assert n_mfma > 1000
