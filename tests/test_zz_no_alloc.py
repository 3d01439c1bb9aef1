"""The allocation-free curvature product (wf_hvp_noalloc) through the C-ABI: the same
result as wf_hvp on two calls in a row (the second smaller), no device allocation by the
call, and a clear error for a batch that does not fit its scratch array."""
import numpy as np
import pytest

from paper_1810_00503_amd import workloads as WL
from tests.gpu_util import make_problem, random_half

pytestmark = pytest.mark.gpu


def _case(lib, torch, wl, batch, seed, dtype="f32"):
    prob = make_problem(lib, torch, wl, dtype)
    rng = np.random.default_rng(seed)
    p = np.stack([random_half(rng, wl.ncomp, wl.n) for _ in range(batch)])
    pt = torch.tensor(p, dtype=prob.cdtype, device="cuda:0")
    return prob, pt


def test_noalloc_hvp_matches_hvp_on_consecutive_calls(lib):
    import torch
    cases = [(WL.shear_workload(256, 31, nbands_e=4, nbands_b=4), 3, "f32"),
             (WL.density_workload(64, 32, nbands=4), 1, "f32"),
             (WL.cmb_workload(96, 33, nbands=5), 2, "f64")]
    for wl, batch, dtype in cases:
        print(f"[hvp_noalloc n={wl.n} ncomp={wl.ncomp} batch={batch} {dtype}]", flush=True)
        prob, pt = _case(lib, torch, wl, batch, 7 + wl.n, dtype)
        out = torch.full_like(pt, float("nan"))
        lib.wf_hvp_noalloc(prob, pt, out)
        ref = lib.wf_hvp(prob, pt)
        torch.cuda.synchronize()
        # the same kernels with the same tiles: bit for bit
        assert torch.equal(out, ref)
        assert bool(torch.isfinite(torch.view_as_real(out)).all())


def test_noalloc_hvp_allocates_nothing(lib):
    import torch
    print("[hvp_noalloc allocation]", flush=True)
    cx = lib.Context(0)
    try:
        wl = WL.shear_workload(512, 41, nbands_e=3, nbands_b=3)
        prob, pt = _case(lib, torch, wl, 4, 5)
        out = torch.empty_like(pt)
        # a first call of the same shape on the new context (code objects load lazily)
        lib.wf_hvp_noalloc(prob, pt, out, ctx=cx)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for _ in range(3):
            lib.wf_hvp_noalloc(prob, pt, out, ctx=cx)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        # wf_hvp on the same context grows its workspace (3 vectors of 2 MiB per map here):
        # the measurement sees an allocation of that size
        ref = lib.wf_hvp(prob, pt, ctx=cx)
        torch.cuda.synchronize()
        free2 = torch.cuda.mem_get_info()[0]
        assert free0 - free1 < 2 * 2 ** 20, (free0, free1)
        assert free1 - free2 >= 16 * 2 ** 20, (free1, free2)
        assert torch.equal(out, ref)
    finally:
        cx.close()


def test_noalloc_hvp_rejects_batches_beyond_its_scratch(lib):
    import torch
    print("[hvp_noalloc limit]", flush=True)
    wl = WL.cmb_workload(1024, 51, nbands=4)
    prob, pt = _case(lib, torch, wl, 6, 3)
    with pytest.raises(lib.WFError) as e:
        lib.wf_hvp_noalloc(prob, pt, torch.empty_like(pt))
    assert e.value.code == -1 and "scratch" in str(e.value)
    # one map of that size fits and still matches
    out = torch.empty_like(pt[:1])
    lib.wf_hvp_noalloc(prob, pt[:1], out)
    torch.cuda.synchronize()
    assert torch.equal(out, lib.wf_hvp(prob, pt[:1]))
