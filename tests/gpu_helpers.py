"""Shared helpers of the GPU parity tests (compare the HIP path with the oracle)."""
import sys

import numpy as np

import oracle

INF32 = 0xFFFFFFFF


def announce(*parts):
    """Name the case on the real stderr before a GPU step (survives capture)."""
    sys.__stderr__.write("[gpu-case] " + " ".join(str(p) for p in parts) + "\n")
    sys.__stderr__.flush()


def to_np(t):
    return t.detach().cpu().numpy()


def assert_sssp_matches(g, s, got, ref=None, check_invariants=True, tag=""):
    """Bit-exact for u32; for f32 bit-exact against the fp32-fold oracle and
    within 2^-22 * hops(v) * d64(v) of the fp64 oracle (INF exact)."""
    got = np.asarray(got)
    if g.wtype == "u32":
        if ref is None:
            ref, _ = oracle.sssp(g, s, "u32")
        got = got.view(np.uint32)
        bad = np.nonzero(got != ref)[0]
        assert bad.size == 0, (f"{tag} source {s}: {bad.size} mismatches, first v={bad[0]} "
                               f"gpu={got[bad[0]]} ref={ref[bad[0]]}")
    else:
        got = got.view(np.float32)
        d32, h32 = oracle.sssp(g, s, "f32fold") if ref is None else ref
        bad = np.nonzero(got.view(np.uint32) != d32.view(np.uint32))[0]
        assert bad.size == 0, (f"{tag} source {s}: {bad.size} fp32-fold mismatches, first "
                               f"v={bad[0]} gpu={got[bad[0]]!r} ref={d32[bad[0]]!r}")
        d64, h64 = oracle.sssp(g, s, "f64")
        viol = oracle.f32_tolerance_violations(g, s, got, d64, h64, d32, h32)
        assert viol.size == 0, f"{tag} source {s}: tolerance violated at {viol[:5]}"
    if check_invariants:
        rc, v = oracle.check(g, s, got)
        assert rc == 0, f"{tag} source {s}: invariant V{rc} fails at vertex {v}"
