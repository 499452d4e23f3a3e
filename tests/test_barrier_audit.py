"""The persistent solver once hung on the GPU because workgroup barriers sat inside control flow
that the compiler had laid out as divergent (exec-masked): a wave with an empty mask skipped a
region the others executed, and the barriers no longer matched.  Every barrier-enclosing branch is
now decided by a wave-uniform value (readfirstlane).  This CPU test keeps it that way: it compiles
the library's device code for gfx950 and checks, by a control-flow analysis of the assembly, that
no barrier (and no call into a function with barriers) runs under a narrowed execution mask.  The
analysis is itself checked on two planted kernels, one with a barrier under a lane-dependent branch
(must be flagged) and one under a uniform branch (must pass)."""
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
    bad = [f for f in audit(compile_to_asm(str(src), str(tmp_path / "planted.s"))) if "k_bad" in f[0]]
    good = [f for f in audit(compile_to_asm(str(src), str(tmp_path / "planted2.s"))) if "k_good" in f[0]]
    assert bad, "the planted divergent barrier was not found"
    assert not good, good


@pytest.mark.parametrize("src", ["solver.hip", "extras.hip", "noalloc.hip"])
def test_library_barriers_run_with_full_masks(tmp_path, src):
    asm = compile_to_asm(os.path.join(CSRC, src), str(tmp_path / (src + ".s")))
    found = audit(asm)
    assert "s_barrier" in asm or src != "solver.hip"
    assert not found, "\n".join(f"{f} {b}: {s} (open: {r})" for f, b, s, r in found[:20])
