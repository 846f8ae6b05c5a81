"""dawn_sssp_noalloc: the single-source call that takes its workspace from the
library's fixed per-device scratch array instead of allocating.  Its result
must equal dawn_sssp's (the allocating entry point it mirrors) bit for bit, on
calls in a row whose graphs shrink, so that a call starts correctly on the
scratch contents the previous, larger call left behind.  Each launch mix the
plain call can take is covered: one workgroup (small graphs), the persistent
launch, and step launches followed by the persistent launch."""
import numpy as np
import pytest

import graphgen
from gpu_helpers import announce, assert_sssp_matches, to_np

pytestmark = pytest.mark.gpu


def _pair(dawn, csr, s):
    import torch
    ref = dawn.sssp(csr, s)
    out = torch.full((csr.n,), 7, dtype=ref.dtype, device=ref.device)   # garbage start
    dawn.sssp_noalloc(csr, s, out)
    torch.cuda.synchronize()
    return to_np(ref), to_np(out)


def _run_sequence(dawn, graphs, tag):
    for i, g in enumerate(graphs):
        csr = dawn.Csr.from_graph(g)
        need = dawn.sssp_workspace_bytes(g.n, g.m)
        assert need <= dawn.NOALLOC_SCRATCH_BYTES
        for s in graphgen.pick_sources(g, 2, 40 + i):
            announce("noalloc", tag, "call", i, "n", g.n, "m", g.m, "source", int(s))
            ref, got = _pair(dawn, csr, int(s))
            assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), \
                f"{tag} call {i} source {s}: differs from dawn_sssp"
            assert_sssp_matches(g, int(s), got, tag=f"{tag} call {i}")


def test_noalloc_equals_plain_u32_shrinking(dawn):
    big = graphgen.rmat(17, 16, 7, weights="u32", wlo=1, whi=255)    # persistent launch
    small = graphgen.er(1000, 8000, 1, weights="u32", wlo=1, whi=100)  # one workgroup
    _run_sequence(dawn, [big, small], "u32")


def test_noalloc_equals_plain_f32_shrinking(dawn):
    big = graphgen.grid(512, 512, 0.01, 3, weights="f32unit")
    small = graphgen.grid(40, 40, 0.01, 2, weights="f32unit")
    _run_sequence(dawn, [big, small], "f32")


def test_noalloc_equals_plain_step_launches(dawn):
    prev = dawn.set_tuning(mode=1, step_launches=6)
    try:
        big = graphgen.rmat(18, 16, 9, weights="u32", wlo=1, whi=255)
        mid = graphgen.rmat(14, 8, 10, weights="u32", wlo=1, whi=255)
        _run_sequence(dawn, [big, mid], "mode1")
    finally:
        dawn.set_tuning(**prev)

