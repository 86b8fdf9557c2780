"""The build's check on generated gfx950 code: a join of an exec-narrowing
branch must restore exec before any vector work (CPU only)."""
import glob
import os

import pytest

from paper_2604_07372_amd import asmcheck

BAD = """_Zkernel:
\ts_and_saveexec_b64 s[0:1], s[70:71]
\ts_cbranch_execz .LBB0_224
\tglobal_load_dword v227, v[6:7], off offset:20
.LBB0_224:
\ts_waitcnt vmcnt(0)
\tscratch_store_dword off, v227, off offset:140
\tv_mov_b32_e32 v97, v30
\ts_or_b64 exec, exec, s[0:1]
\ts_endpgm
"""

GOOD = """_Zkernel:
\ts_and_saveexec_b64 s[0:1], vcc
\ts_cbranch_execz .LBB0_18
\tglobal_load_dword v9, v[6:7], off
.LBB0_18:
\ts_or_b64 exec, exec, s[0:1]
\tv_mov_b32_e32 v97, v30
\ts_and_saveexec_b64 s[2:3], vcc
\ts_cbranch_execz .LBB0_19
\tv_mov_b32_e32 v1, 0
.LBB0_19:
\tv_writelane_b32 v134, s24, 11
\ts_or_b64 exec, exec, s[2:3]
\ts_cbranch_execz .LBB0_20
\ts_branch .LBB0_21
.LBB0_20:
\tv_mov_b32_e32 v5, v6
.LBB0_21:
\ts_endpgm
"""


ELSE = """_Zkernel:
\ts_and_saveexec_b64 s[6:7], vcc
\ts_xor_b64 s[6:7], exec, s[6:7]
\ts_cbranch_execz .LBB0_7
\tv_mov_b32_e32 v1, 1
.LBB0_7:
\ts_andn2_saveexec_b64 s[0:1], s[6:7]
\tv_mov_b64_e32 v[6:7], 0
\ts_or_b64 exec, exec, s[0:1]
\ts_endpgm
"""

ELSE_LATE = """_Zkernel:
\ts_and_saveexec_b64 s[6:7], vcc
\ts_xor_b64 s[6:7], exec, s[6:7]
\ts_cbranch_execz .LBB0_7
\tv_mov_b32_e32 v1, 1
.LBB0_7:
\tv_mov_b32_e32 v9, v1
\ts_andn2_saveexec_b64 s[0:1], s[6:7]
\tv_mov_b64_e32 v[6:7], 0
\ts_or_b64 exec, exec, s[0:1]
\ts_endpgm
"""


def test_accepts_the_else_branch_of_an_if_else():
    # the join block switches exec to the else lanes before its vector work
    assert asmcheck.find_masked_joins(ELSE) == []
    # but a copy placed before that switch still runs under the then-mask
    found = asmcheck.find_masked_joins(ELSE_LATE)
    assert len(found) == 1 and found[0][2][0].startswith("v_mov_b32_e32 v9")


def test_flags_copies_before_the_exec_restore():
    found = asmcheck.find_masked_joins(BAD)
    assert len(found) == 1
    func, line, extra = found[0]
    assert func == "_Zkernel" and extra[0].startswith("scratch_store_dword")
    assert any(x.startswith("v_mov_b32") for x in extra)


def test_accepts_restore_first_lane_ops_and_full_exec_guards():
    # restore right after the join; v_writelane ignores exec; an execz branch
    # with no narrowing before it (full exec) is not a join of a divergent if
    assert asmcheck.find_masked_joins(GOOD) == []


def test_built_device_code_is_clean():
    build = os.path.join(os.path.dirname(asmcheck.__file__), "_build")
    files = glob.glob(os.path.join(build, "*-hip-amdgcn-amd-amdhsa-gfx950.s"))
    if not files:
        pytest.skip("no device assembly in _build (library not built here)")
    assert asmcheck.check_files(files) == []
