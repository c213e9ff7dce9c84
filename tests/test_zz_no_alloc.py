"""glt_count_noalloc (no device allocation during the call; fixed per-device scratch) against
glt_count, bit-exact, through the C ABI: two calls in a row, the second on a smaller graph,
per-edge and global, and a graph too large for the scratch refused with a clear error."""
import sys

import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def say(msg):
    sys.__stderr__.write(f"[gpu-case] {msg}\n")
    sys.__stderr__.flush()


def _dev(rp, col):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(rp)).cuda(),
            torch.from_numpy(np.ascontiguousarray(col, dtype=np.int32)).cuda())


def test_noalloc_matches_count_twice_then_smaller():
    import torch

    import paper_1608_05138_amd as glt
    ctx = glt.Context(0)
    try:
        graphs = [("chung-lu-20000", 20000, gg.chung_lu(20000, 200000, 2.1, 19999.0, 8)),
                  ("er-1000", 1000, gg.er(1000, 10000, 160805138)),
                  ("clique-on-noise", 2300, None)]
        rng = np.random.default_rng(3)
        lo, hi = gg.er_pairs(2300, 6000, rng)
        iu = np.triu_indices(700, 1)   # out-degrees up to 699: global-memory bitmap rows
        a = np.concatenate([lo, iu[0]]); b = np.concatenate([hi, iu[1]])
        key = np.unique(np.minimum(a, b) * 2300 + np.maximum(a, b))
        graphs[2] = ("clique700-noise", 2300, gg.csr_from_pairs(2300, key // 2300, key % 2300))
        for name, n, (rp, col) in graphs:
            rpt, ct = _dev(rp, col)
            m = col.size // 2
            for per_edge in (True, False):
                say(f"noalloc {name} per_edge={per_edge}")
                X0, pe0 = ctx.count(rpt, ct, n=n, per_edge=per_edge)
                out = torch.full((13, m), -1, dtype=torch.int64, device="cuda") if per_edge else None
                X1, pe1 = ctx.count_noalloc(rpt, ct, n=n, per_edge=per_edge, out=out)
                torch.cuda.synchronize()
                assert X1 == X0, name
                if per_edge:
                    assert torch.equal(pe1, pe0), name
        # the scratch holds one call's workspace: a graph beyond it is refused, not truncated
        n = 200000
        rp, col = gg.chung_lu(n, 2000000, 2.5, float(n - 1), 5)
        rpt, ct = _dev(rp, col)
        say("noalloc refuses a graph beyond the scratch")
        with pytest.raises(glt.GltError) as ei:
            ctx.count_noalloc(rpt, ct, n=n)
        assert ei.value.status == -6 and "scratch" in str(ei.value)
        # host inputs are refused by the binding and by the library
        with pytest.raises(ValueError):
            ctx.count_noalloc(rp, col, n=n)
        # the handle and the scratch still work afterwards
        n2, (rp2, col2) = gg.cycle(9)
        rpt2, ct2 = _dev(rp2, col2)
        X, _ = ctx.count_noalloc(rpt2, ct2, n=n2)
        assert X[0] == 9 and X[11] == 9
    finally:
        ctx.close()
