"""The compiled kernels never hold a workgroup barrier inside a loop that
lanes leave one by one (paper_2206_13574_amd/asm_check.py).  That shape
livelocks a persistent kernel: with a per-query early exit in front of the
queue fetch (thread 0's atomic, a barrier, everyone reads the slot), the
compiler sends every lane but thread 0 straight back to the barrier to
re-read the same slot while thread 0 waits outside the loop.  The checker is
pinned on a small kernel written both ways."""
import os

import pytest

from paper_2206_13574_amd import asm_check, build

_BAD = r"""
#include <hip/hip_runtime.h>
__global__ __launch_bounds__(256) void k_persistent(int* queue, const int* val, int* out, int n) {
    __shared__ int slot;
    for (;;) {
        if (threadIdx.x == 0) slot = atomicAdd(queue, 1);
        __syncthreads();
        const int r = __builtin_amdgcn_readfirstlane(slot);
        __syncthreads();
        if (r >= n) break;
        const int v = val[r];
        if (v < 0) {                      // a query to skip: early exit to the loop head
            if (threadIdx.x == 0) out[r] = -1;
            continue;
        }
        atomicAdd(out + r, v + (int)threadIdx.x);
        __syncthreads();
    }
}
"""

_GOOD = r"""
#include <hip/hip_runtime.h>
__global__ __launch_bounds__(256) void k_persistent(int* queue, const int* val, int* out, int n) {
    __shared__ int slot;
    for (;;) {
        if (threadIdx.x == 0) slot = atomicAdd(queue, 1);
        __syncthreads();
        const int r = __builtin_amdgcn_readfirstlane(slot);
        __syncthreads();
        if (r >= n) break;
        const int v = __builtin_amdgcn_readfirstlane(val[r]);
        if (v < 0) {                      // skipped, but through the common loop tail
            if (threadIdx.x == 0) out[r] = -1;
        } else {
            atomicAdd(out + r, v + (int)threadIdx.x);
        }
        __syncthreads();
    }
}
"""


def _flags(tmp_path, src):
    p = tmp_path / "k.hip"
    p.write_text(src)
    return {k: v for k, v in asm_check.check_asm(asm_check.device_asm(str(p))).items() if v}


def test_checker_flags_an_early_exit_in_a_persistent_loop(tmp_path):
    assert _flags(tmp_path, _BAD), "the checker must flag the early-exit form"
    assert not _flags(tmp_path, _GOOD)


@pytest.mark.parametrize("src", [s for s in build.sources() if s.endswith(".hip")], ids=os.path.basename)
def test_library_kernels_have_no_barrier_in_a_lane_exit_loop(src):
    flagged = {k: v for k, v in asm_check.check_asm(asm_check.device_asm(src)).items() if v}
    assert not flagged, flagged
