"""The persistent solver once hung on the GPU because workgroup barriers sat inside control flow
that the compiler had laid out as divergent (exec-masked): a wave with an empty mask skipped a
region the others executed, and the barriers no longer matched.  Every barrier-enclosing branch is
now decided by a wave-uniform value (readfirstlane).  This CPU test keeps it that way: it compiles
the library's device code for gfx950 and checks, by a control-flow analysis of the assembly, that
no barrier (and no call into a function with barriers) runs under a narrowed execution mask.  The
analysis is itself checked on planted kernels: a barrier under a lane-dependent branch or in the
else arm of a lane-dependent if / else (must be flagged), and a barrier under a uniform branch or
after the join of a lane-dependent if / else (must pass)."""
import os
import shutil

import pytest

from barrier_audit import audit, compile_to_asm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1905_10574_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc (cross-compiles, no GPU)")

PLANTED = r"""
#include <hip/hip_runtime.h>
__global__ void __launch_bounds__(256) k_bad(double *x, int n)
{
    __shared__ double s[256];
    s[threadIdx.x] = x[threadIdx.x];
    if ((int)threadIdx.x < n) {            // lane-dependent: an exec-masked region
        __syncthreads();
        x[threadIdx.x] = s[255 - threadIdx.x];
    }
}
__global__ void __launch_bounds__(256) k_bad_else(double *x, int n)
{
    __shared__ double s[256];
    s[threadIdx.x] = x[threadIdx.x];
    if ((int)threadIdx.x < n) {            // lane-dependent if / else, barrier in the else arm
        x[threadIdx.x] = s[threadIdx.x] * 2.0;
    } else {
        __syncthreads();
        x[threadIdx.x] = s[255 - threadIdx.x];
    }
}
__global__ void __launch_bounds__(256) k_good_else(double *x, int n)
{
    __shared__ double s[256];
    s[threadIdx.x] = x[threadIdx.x];
    double v;
    if ((int)threadIdx.x < n) v = s[threadIdx.x] * 2.0 + x[n];   // lane-dependent if / else,
    else v = s[255 - threadIdx.x] - x[2 * n];                     // the barrier after the join
    __syncthreads();
    x[threadIdx.x] = v + s[(threadIdx.x + 1) & 255];
}
__global__ void __launch_bounds__(256) k_good(double *x, int n)
{
    __shared__ double s[256];
    s[threadIdx.x] = x[threadIdx.x];
    const int u = __builtin_amdgcn_readfirstlane((int)x[0] > n ? 1 : 0);
    if (u) {                                // wave-uniform: a scalar branch
        __syncthreads();
        x[threadIdx.x] = s[255 - threadIdx.x];
    }
}
"""


def test_audit_flags_a_barrier_under_divergent_control_flow(tmp_path):
    src = tmp_path / "planted.hip"
    src.write_text(PLANTED)
    found = audit(compile_to_asm(str(src), str(tmp_path / "planted.s")))
    bad = [f for f in found if "k_bad" in f[0] and "k_bad_else" not in f[0]]
    bad_else = [f for f in found if "k_bad_else" in f[0]]
    good = [f for f in found if "k_good" in f[0]]
    assert bad, "the planted divergent barrier was not found"
    assert bad_else, "the planted barrier in an else arm was not found"
    assert not good, good


# If / else as the compiler lays it out when the then arm holds a nested region: the else lanes are
# kept in a second register (s_xor_b64), the else arm entered with s_andn2_saveexec_b64 into a
# third, and that third register closes the whole if / else.
IFELSE = """
f_join:
\ts_and_saveexec_b64 s[0:1], vcc
\ts_xor_b64 s[2:3], exec, s[0:1]
\ts_cbranch_execz .LBB0_3
\ts_and_saveexec_b64 s[0:1], s[6:7]
\ts_cbranch_execz .LBB0_2
\tv_mov_b32 v0, 1
.LBB0_2:
\ts_or_b64 exec, exec, s[0:1]
.LBB0_3:
\ts_andn2_saveexec_b64 s[4:5], s[2:3]
\ts_cbranch_execz .LBB0_5
\tv_mov_b32 v0, 2
{else_arm}
.LBB0_5:
\ts_or_b64 exec, exec, s[4:5]
\ts_barrier
\ts_endpgm
.Lfunc_end0:
"""


# A register that held a copy of exec and was then overwritten (here by a lane compare) no longer
# restores the full mask: exec set from it is narrowed, and the barrier after it must be flagged.
STALE = """
f_stale:
\ts_mov_b64 s[0:1], exec
\tv_cmp_gt_i32_e64 s[0:1], s8, v4
\ts_mov_b64 exec, s[0:1]
\ts_barrier
\ts_endpgm
.Lfunc_end0:
"""


def test_audit_drops_overwritten_exec_copies():
    found = audit(STALE)
    assert len(found) == 1 and found[0][2] == "s_barrier"
    assert not audit(STALE.replace("\tv_cmp_gt_i32_e64 s[0:1], s8, v4\n", ""))


def test_audit_follows_the_two_register_else_arm():
    assert not audit(IFELSE.format(else_arm="\tv_mov_b32 v1, 2"))
    found = audit(IFELSE.format(else_arm="\ts_barrier"))
    assert len(found) == 1 and found[0][2] == "s_barrier"


@pytest.mark.parametrize("src", ["solver.hip", "extras.hip", "noalloc.hip"])
def test_library_barriers_run_with_full_masks(tmp_path, src):
    asm = compile_to_asm(os.path.join(CSRC, src), str(tmp_path / (src + ".s")))
    found = audit(asm)
    assert "s_barrier" in asm or src != "solver.hip"
    assert not found, "\n".join(f"{f} {b}: {s} (open: {r})" for f, b, s, r in found[:20])
