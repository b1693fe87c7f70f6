"""Walk-length tracking (Algorithm 4, the learned pass, the trace dump) adds
no per-entry loop over the active lanes to the alignment kernel.

Updating a workgroup-wide maximum from every recorded entry with an LDS
atomic compiles, through the compiler's atomic optimizer, into a loop over
the wave's active lanes before a single atomic: several instructions per
lane for every entry, which made the tracked instantiations take about
twice as long as the exact one on the same work.  Each lane now keeps its
maxima in registers, reduced once per score.  The check: in the gfx950
assembly (paper_2206_13574_amd/asm_check.py), every tracked instantiation
holds no more such lane loops nested five or more loops deep (the per-entry
loops: query, attempt, score, batch or round, and below) than the exact
instantiation of the same width, whose deep lane loops sit on the end test's
rare paths.  Pinned on the kernel's earlier form, which fails it."""
import os
import re

import pytest

from paper_2206_13574_amd import asm_check, build

_SRC = [s for s in build.sources() if s.endswith("gwfa_kernels.hip")][0]
_DEEP = 5


def _deep_counts(text):
    out = {}
    for name, lines in asm_check._functions(text):
        m = re.search(r"k_alignILi(\d+)ELi(\d)E", name)
        if m:
            out[(int(m.group(1)), int(m.group(2)))] = sum(d >= _DEEP for _, d in asm_check.lane_loops(lines))
    return out


@pytest.fixture(scope="module")
def counts():
    return _deep_counts(asm_check.device_asm(_SRC))


def test_every_instantiation_is_checked(counts):
    assert sorted(counts) == [(b, m) for b in (64, 128, 256, 512) for m in range(4)]


def test_tracked_instantiations_add_no_deep_lane_loops(counts):
    for (block, mode), n in counts.items():
        assert n <= counts[(block, 0)], (block, mode, n, counts[(block, 0)])


def test_checker_flags_per_entry_atomics(tmp_path):
    """The earlier form (two LDS atomics per recorded entry) fails the check."""
    src = open(_SRC).read()
    new = """        lmax.x = max(lmax.x, i + W);
        lmax.y = max(lmax.y, i);"""
    assert new in src
    src = src.replace(new, """        atomicMax(&S.amax, i + W);
        atomicMax(&S.imax, i);""")
    p = tmp_path / "gwfa_kernels.hip"
    p.write_text(src)
    c = _deep_counts(asm_check.device_asm(str(p)))
    assert all(c[(b, m)] > c[(b, 0)] for b in (64, 128, 256, 512) for m in (1, 2, 3))
