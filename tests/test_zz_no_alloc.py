"""The allocation-free densification plan (gs_densify_plan_noalloc) against
gs_densify_plan with a workspace: bit-identical maps and row counts on two
calls in a row, the second with fewer parents (the shared device scratch then
holds the first call's larger contents), and host-side rejection of sizes
beyond its limit."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2507_20239_amd import gsmi

pytestmark = pytest.mark.gpu

NOALLOC_MAX = 1 << 23


def _masks(rng, n):
    split = (rng.random(n) < 0.05).astype(np.uint8)
    clone = ((rng.random(n) < 0.08) & (split == 0)).astype(np.uint8)
    prune = (rng.random(n) < 0.02).astype(np.uint8)
    return [torch.from_numpy(m).cuda() for m in (split, clone, prune)]


@pytest.mark.parametrize("sizes", [(3_000_000, 1_000_003), (NOALLOC_MAX, 5)])
def test_noalloc_plan_matches_workspace_plan(sizes):
    rng = np.random.default_rng(11)
    cap = 2 * max(sizes)
    src = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    kind = torch.full((cap,), 255, dtype=torch.uint8, device="cuda")
    n_out = torch.zeros(1, dtype=torch.int64, device="cuda")
    for n in sizes:
        print("noalloc plan n=%d" % n, flush=True)
        s, c, p = _masks(rng, n)
        want_src, want_kind, m = gsmi.densify_plan(s, c, p)
        gsmi.densify_plan_noalloc(s, c, p, src, kind, n_out)
        torch.cuda.synchronize()
        assert int(n_out.item()) == m
        assert torch.equal(src[:m], want_src) and torch.equal(kind[:m], want_kind)
        # the map itself: a pruned parent emits nothing, a split or clone two rows
        cnt = torch.bincount(src[:m].long(), minlength=n)
        want_cnt = torch.where(p.bool(), 0, torch.where((s | c).bool(), 2, 1))
        assert torch.equal(cnt, want_cnt)


def test_noalloc_plan_empty_and_oversized():
    n_out = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    e = torch.empty(0, dtype=torch.uint8, device="cuda")
    src = torch.empty(1, dtype=torch.int32, device="cuda")
    kind = torch.empty(1, dtype=torch.uint8, device="cuda")
    gsmi.densify_plan_noalloc(e, e, e, src, kind, n_out)
    torch.cuda.synchronize()
    assert int(n_out.item()) == 0
    L = gsmi.lib()
    fake = ctypes.c_void_p(256)
    st = L.gs_densify_plan_noalloc(fake, fake, fake, NOALLOC_MAX + 1, fake, fake, 10, fake, None)
    assert st == gsmi.GS_ERR_INVALID and b"at most" in L.gs_last_error()
